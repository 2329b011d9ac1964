"""The serving runtime's host logic on the CPU: its source compiled against
host stand-ins for HIP and for the search (tests/serve_stub), driven through
admission with small and large device budgets, one or many spectra per
launch, host and device spectra, and a ring that wraps."""

import os
import shutil
import subprocess

import pytest

from conftest import ROOT

STUB = os.path.join(ROOT, "tests", "serve_stub")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not installed")
    d = tmp_path_factory.mktemp("serve")
    out = d / "drive"
    # the runtime's source next to the stand-in header, so that its
    # #include "internal.hpp" resolves to the stand-in
    shutil.copy(os.path.join(ROOT, "paper_2406_15186_amd", "csrc", "serve.hip"), d / "serve.cpp")
    shutil.copy(os.path.join(STUB, "internal.hpp"), d / "internal.hpp")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I", os.path.join(ROOT, "include"),
           str(d / "serve.cpp"), os.path.join(STUB, "stub_search.cpp"),
           os.path.join(STUB, "drive.cpp"), "-o", str(out)]
    subprocess.run(cmd, check=True)
    return str(out)


# spectra are drawn up to the whole budget in size (about two fit on
# average), so admission waits for room and the ring wraps constantly
@pytest.mark.parametrize("budget,max_batch,nreq,seed", [
    (1 << 20, 256, 50, 1),     # many spectra per launch
    (1 << 20, 1, 50, 2),       # one spectrum per launch
    (1 << 20, 3, 300, 3),
    (1 << 21, 1, 300, 4),
    (1 << 21, 7, 400, 5),
])
def test_every_request_completes_once(driver, budget, max_batch, nreq, seed):
    r = subprocess.run([driver, str(budget), str(max_batch), str(nreq), str(seed)],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.startswith(f"ok {nreq}")


# edges: 1 = requests of the largest size a budget that is not a multiple of
# the ring's 256-byte placement admits (each must still be served); 2 =
# searches that fail on the device (their count word carries the failure
# code), which must come back as PULSCAN_EHIP while the rest are served
@pytest.mark.parametrize("budget,max_batch,nreq,seed,edges", [
    ((1 << 20) + 100, 3, 100, 6, 1),
    ((1 << 20) + 8, 1, 60, 7, 1),
    (1 << 20, 4, 200, 8, 2),
    ((1 << 21) + 200, 256, 150, 9, 3),
])
def test_ring_edge_and_device_failures(driver, budget, max_batch, nreq, seed, edges):
    r = subprocess.run([driver, str(budget), str(max_batch), str(nreq), str(seed), str(edges)],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.startswith(f"ok {nreq}")


# admission by free device memory: a budget of 0 takes half of what is free
# (rounded down to the ring's 256-byte placement); a budget beyond what is free
# (with the server's own candidate buffers) is refused; a device short of
# room for another set's scratch (under 256 MiB free) serves one set at a time
@pytest.mark.parametrize("free_mib,budget,status,expect", [
    (1024, 0, 0, 512 << 20),
    (1000, 0, 0, 500 << 20),
    (256, 1 << 30, -2, 0),
    (100, 64 << 20, -2, 0),       # 64 MiB of spectra + 64 MiB of candidate buffers
])
def test_budget_from_free_device_memory(driver, free_mib, budget, status, expect):
    env = dict(os.environ, PULSCAN_STUB_FREE_MIB=str(free_mib))
    r = subprocess.run([driver, str(budget), "4", "0", "1"], capture_output=True, text=True,
                       timeout=60, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.split() == ["create", str(status), "budget", str(expect)]


def test_low_free_memory_serves_one_set_at_a_time(driver):
    env = dict(os.environ, PULSCAN_STUB_FREE_MIB="200")
    r = subprocess.run([driver, str(1 << 20), "3", "120", "11"], capture_output=True, text=True,
                       timeout=60, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.startswith("ok 120")
