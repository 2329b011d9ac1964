"""GPU checks of the serving runtime: spectra submitted one by one (device-
resident or in pinned host memory) come back with the candidates the plain
search finds for them, and the oracle's, in any admission grouping the
device budget forces, with ordered timestamps."""

import ctypes
import time

import numpy as np
import pytest

import synth
from gpu_helpers import compare_candidates, say, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2406_15186_amd as pk
    pk.lib()
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    import torch
    assert torch.cuda.is_available()
    c = pk.Context(0)
    yield c
    c.close()


def spectra(oracle_lib, count, seed=31):
    rng = np.random.default_rng(seed)
    wl = synth.workload("plain_2e16")
    out = []
    for s in range(count):
        n = int(rng.integers(1 << 15, 1 << 17))
        x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, spawn=40 + s, nbins=n)
        out.append((x, int(rng.choice([32, 64, 100]))))
    return out


def drain(srv, want, timeout_s=60.0):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < want:
        assert time.time() < t_end, f"only {len(got)} of {want} results"
        for r in srv.pulscan_server_poll(wait_ms=50):
            got[r[0]] = r
    return got


@pytest.mark.parametrize("budget_spectra,max_batch", [(1000, 256), (3, 256), (1000, 1)])
def test_served_results_match_plain_searches(ctx, pk, oracle_lib, budget_spectra, max_batch):
    specs = spectra(oracle_lib, 12)
    dev = [to_device(x) for x, _ in specs]
    host = []
    for x, _ in specs:
        nbytes = x.nbytes
        p = pk.pulscan_host_alloc(nbytes)
        ctypes.memmove(p, x.ctypes.data, nbytes)
        host.append(p)
    budget = budget_spectra * max(x.nbytes for x, _ in specs)
    srv = pk.Server(0, hbm_budget=budget, max_batch=max_batch, chunk=1024, sigma_thresh=6.0)
    try:
        tickets = {}
        for i, ((x, z), d) in enumerate(zip(specs, dev)):
            on_dev = i % 2 == 0
            ptr = d.data_ptr() if on_dev else host[i]
            t = srv.pulscan_server_submit(ptr, x.shape[0], z, on_dev)
            tickets[t] = i
        res = drain(srv, len(specs))
        pending, completed, batches, used = srv.pulscan_server_stats()
        assert pending == 0 and completed == len(specs) and used == 0
        if max_batch == 1 or budget_spectra < len(specs):
            assert batches > 1
        say(f"served {completed} spectra in {batches} launches (budget {budget_spectra} spectra)")
        for t, (tk, status, total, ts, tb, td, cands) in res.items():
            i = tickets[t]
            assert status == pk.PULSCAN_OK, (i, status)
            assert ts <= tb <= td
            ref, rc = ctx.pulscan_search_ex(dev[i], specs[i][1], 1024, 6.0)
            assert total == rc == len(cands)
            assert (cands == ref).all(), i
            if i < 2:
                # one device-resident and one host spectrum against the oracle
                x, z = specs[i]
                orc = oracle_lib.search(x, z, 1024, 6.0, tables=True)
                compare_candidates(cands, orc, orc.P, float(x.shape[0] * z), 6.0, oracle_lib,
                                   f"served {'device' if i % 2 == 0 else 'host'} spectrum {i}")
    finally:
        srv.close()
        for p in host:
            pk.pulscan_host_free(p)


def test_server_rejects_unsearchable_spectra(pk):
    import torch
    srv = pk.Server(0, chunk=1024)
    try:
        d = torch.zeros((512, 2), dtype=torch.float32, device="cuda")
        with pytest.raises(pk.PulscanError) as e:
            srv.pulscan_server_submit(d.data_ptr(), 512, 64, True)   # shorter than a chunk
        assert e.value.status == pk.PULSCAN_EINVAL
        with pytest.raises(pk.PulscanError):
            srv.pulscan_server_submit(d.data_ptr(), 4096, 5000, True)  # zmax beyond 4096
    finally:
        srv.close()


def test_budget_from_free_device_memory(pk, oracle_lib):
    # hbm_budget = 0: half the device memory free at creation; a budget beyond
    # the free memory is refused; the derived budget serves spectra
    import torch
    free0, total = torch.cuda.mem_get_info()
    with pytest.raises(pk.PulscanError) as e:
        pk.Server(0, hbm_budget=int(total) + (1 << 30))
    assert e.value.status == pk.PULSCAN_ENOMEM
    srv = pk.Server(0, hbm_budget=0, max_batch=8, chunk=1024, sigma_thresh=6.0)
    try:
        b = srv.pulscan_server_budget()
        free1, _ = torch.cuda.mem_get_info()
        say(f"server budget {b / 2**30:.1f} GiB of {free0 / 2**30:.1f} GiB free")
        assert b % 256 == 0
        assert 0.4 * free0 <= b <= 0.5 * free0 + (64 << 20)
        sp = spectra(oracle_lib, 3, seed=57)
        ds = [to_device(x) for x, _ in sp]
        tickets = [srv.pulscan_server_submit(d.data_ptr(), d.shape[0], z, True)
                   for d, (_, z) in zip(ds, sp)]
        got = drain(srv, len(tickets))
        assert sorted(got) == sorted(tickets)
        assert all(r[1] == pk.PULSCAN_OK for r in got.values())
    finally:
        srv.close()
