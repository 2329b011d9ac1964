"""GPU checks of the batched path (many spectra of uneven lengths in one
fused launch): graph capture and replay against eager calls, the chunk and
tile autotuner, and sampled parity of a DM-trial batch against the FP64
oracle."""

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


def small_batch(oracle_lib, nspec=6, seed=11):
    rng = np.random.default_rng(seed)
    wl = synth.workload("plain_2e16")
    xs, zs = [], []
    for s in range(nspec):
        n = int(rng.integers(20000, 70000))
        x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, spawn=s, nbins=n)
        xs.append(x)
        zs.append(int(rng.choice([16, 32, 64])))
    return xs, zs


@pytest.mark.parametrize("numharm,best,fp16", [(1, False, False), (3, True, False), (1, False, True)])
def test_graph_replays_match_eager(ctx, pk, oracle_lib, numharm, best, fp16):
    """A graph-mode batched call replays its captured launches; every replay,
    with eager work and synchronisations in between and new data in the same
    buffers, matches an eager call."""
    import torch
    xs, zs = small_batch(oracle_lib)
    ds = [to_device(x) for x in xs]
    eager_opts = pk.make_opts(numharm=numharm, best_per_chunk=best, power_fp16=fp16)
    graph_opts = pk.make_opts(numharm=numharm, best_per_chunk=best, graph=True, power_fp16=fp16)
    cap = sum(pk.worst_count(d.shape[0], z, 256, numharm) for d, z in zip(ds, zs))
    for rep in range(4):
        if rep == 2:
            # new contents in the same device buffers: a replay must see them
            for s, d in enumerate(ds):
                y, _ = synth.make_spectrum(synth.workload("plain_2e16"), oracle_lib.power_for_sigma,
                                           spawn=100 + s, nbins=d.shape[0])
                d.copy_(torch.from_numpy(y).to("cuda"))
        ref, rc, _ = ctx.pulscan_search_batched(ds, zs, 256, 6.0, capacity=cap, opts=eager_opts)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
        got, gc, _ = ctx.pulscan_search_batched(ds, zs, 256, 6.0, capacity=cap, opts=graph_opts)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert gc == rc and len(got) == len(ref), rep
        assert (got == ref).all(), rep
        say(f"graph replay {rep}: {gc} candidates")


def test_graph_is_recaptured_after_other_calls(ctx, pk, oracle_lib):
    """Calls with other arguments (that grow the context's buffers and refill
    its thresholds) in between do not leave a stale graph behind."""
    xs, zs = small_batch(oracle_lib, nspec=3, seed=5)
    ds = [to_device(x) for x in xs]
    go = pk.make_opts(graph=True)
    a, na, _ = ctx.pulscan_search_batched(ds, zs, 256, 6.0, opts=go)
    wl = synth.workload("plain_2e23")
    big, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=1 << 21)
    ctx.pulscan_search_ex(to_device(big), 200, 1024, 5.5)
    b, nb, _ = ctx.pulscan_search_batched(ds, zs, 256, 6.0, opts=go)
    c, nc, _ = ctx.pulscan_search_batched(ds, zs, 256, 6.0, opts=go)
    ref, nr, _ = ctx.pulscan_search_batched(ds, zs, 256, 6.0)
    assert na == nb == nc == nr
    assert (a == ref).all() and (b == ref).all() and (c == ref).all()


def test_graph_plain_search_on_a_stream(ctx, pk, oracle_lib):
    import torch
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    ref, rc = ctx.pulscan_search_ex(d, 64, 256, 6.0)
    s = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(s):
            got, gc = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(graph=True, stream=s))
        torch.cuda.synchronize()
        assert gc == rc and (got == ref).all(), rep


def test_autotuned_chunk_is_reported_and_consistent(ctx, pk, oracle_lib):
    xs, zs = small_batch(oracle_lib, nspec=4, seed=8)
    ds = [to_device(x) for x in xs]
    got, n, used = ctx.pulscan_search_batched(ds, zs, 0, 6.0)
    assert used in (256, 1024, 4096)
    ref, nr, u2 = ctx.pulscan_search_batched(ds, zs, used, 6.0)
    assert u2 == used and nr == n and (ref == got).all()
    # a second call with the same signature reuses the choice
    again, n3, u3 = ctx.pulscan_search_batched(ds, zs, 0, 6.0)
    assert u3 == used and n3 == n and (again == got).all()
    say(f"autotuned chunk {used}, {n} candidates")


@pytest.mark.parametrize("chunk", [1024, 256])
def test_dm_trial_batch_sampled_parity(ctx, pk, oracle_lib, chunk):
    """A batch of 64 DM-trial spectra of 2^16..2^19 bins with per-spectrum zmax
    in {64, 128, 200} and 0-5 tones each (the batched workload's recipe at a
    size the oracle checks quickly), searched in one launch; three spectra
    are compared with the oracle and all spectra's candidates are ordered.
    With chunk 256 the batch has more than 4096 tiles, so the counts are
    scanned by the two-level scan after the bank kernel."""
    wls = synth.batched_workload(nspec=64, n_lo=1 << 16, n_hi=1 << 19, seed=3)
    xs = []
    for w in wls:
        x, _ = synth.make_spectrum(w, oracle_lib.power_for_sigma)
        xs.append(x)
    ds = [to_device(x) for x in xs]
    zs = [w.zmax for w in wls]
    got, n, used = ctx.pulscan_search_batched(ds, zs, chunk, 6.0)
    assert n == len(got) and used == chunk
    keys = [(int(c["spectrum"]), int(c["chunk"]), int(c["width"])) for c in got]
    assert keys == sorted(keys)
    for s in (0, 17, 63):
        orc = oracle_lib.search(xs[s], zs[s], chunk, 6.0, tables=True)
        nt = float(xs[s].shape[0] * zs[s])
        compare_candidates(got[got["spectrum"] == s], orc, orc.P, nt, 6.0, oracle_lib,
                           label=f"batch spectrum {s}")


def test_plain_search_with_many_tiles(ctx, pk, oracle_lib):
    """2^21 bins in 64-bin chunks: over 8000 tiles, scanned in two levels."""
    wl = synth.workload("plain_2e23")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=1 << 21)
    got, n = ctx.pulscan_search_ex(to_device(x), 200, 64, 6.0)
    assert n == len(got) > 0
    orc = oracle_lib.search(x, 200, 64, 6.0, tables=True)
    compare_candidates(got, orc, orc.P, float(len(x) * 200), 6.0, oracle_lib, "many tiles")
    again, n2 = ctx.pulscan_search_ex(to_device(x), 200, 64, 6.0)
    assert n2 == n and (again == got).all()
