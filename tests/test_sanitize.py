"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The FP64 oracle (driven through every entry point by tests/sanitize/
oracle_drive.c) and the serving runtime's host logic (serve.hip against the
host stand-ins of tests/serve_stub) are built with -fsanitize=address,undefined
and no recovery, so any out-of-bounds access, use after free, leak, signed
overflow, misaligned or null access ends the run with a report and a non-zero
status.  ThreadSanitizer is not used: this toolchain's runtime does not follow
the condition-variable waits with a timeout that libstdc++ makes
(pthread_cond_clockwait), and reports the serving runtime's correctly locked
accesses as races."""

import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_drive"
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", *SAN, "-fopenmp",
           os.path.join(ROOT, "tests", "sanitize", "oracle_drive.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=ENV)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith("ok "), r.stdout[-2000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]


@pytest.fixture(scope="module")
def serve_driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not installed")
    stub = os.path.join(ROOT, "tests", "serve_stub")
    d = tmp_path_factory.mktemp("serve_san")
    # the runtime's source next to the stand-in header (see test_serve_logic)
    shutil.copy(os.path.join(ROOT, "paper_2406_15186_amd", "csrc", "serve.hip"), d / "serve.cpp")
    shutil.copy(os.path.join(stub, "internal.hpp"), d / "internal.hpp")
    out = d / "drive"
    cmd = ["g++", "-std=c++17", *SAN, "-pthread", "-I", os.path.join(ROOT, "include"),
           str(d / "serve.cpp"), os.path.join(stub, "stub_search.cpp"),
           os.path.join(stub, "drive.cpp"), "-o", str(out)]
    subprocess.run(cmd, check=True)
    return str(out)


@pytest.mark.parametrize("budget,max_batch,nreq,seed,edges", [
    (1 << 20, 256, 50, 1, 0),
    (1 << 20, 3, 300, 3, 0),
    (1 << 21, 7, 400, 5, 0),
    ((1 << 20) + 100, 5, 200, 6, 3),
])
def test_serving_runtime_under_address_and_undefined_sanitizers(serve_driver, budget, max_batch,
                                                                nreq, seed, edges):
    r = subprocess.run([serve_driver, str(budget), str(max_batch), str(nreq), str(seed),
                        str(edges)],
                       capture_output=True, text=True, timeout=120, env=ENV)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith(f"ok {nreq}")
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
