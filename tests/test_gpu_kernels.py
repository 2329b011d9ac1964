"""The two bank kernels give the same bits.

The tiled kernel (one workgroup per tile) and the streaming kernel
(persistent workgroups over contiguous block ranges) normalise with the same
operations and sum every boxcar in the same canonical FP32 order, so the
library may pick either per launch.  Candidate lists, dense per-chunk tables
and normalised powers are compared byte for byte, forcing each kernel in turn
on the same spectra: the small and the paper-scale shapes, ragged lengths,
logarithmic width sampling, the dense route and a batch.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import say, to_device

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


def spectrum(oracle_lib, n, Z, C, seed, tones=3, red=0.0):
    wl = synth.Workload(f"kern_{seed}", n, Z, C, 6.0, seed, tones, None, (1, min(Z - 1, 60)),
                        (8.0, 15.0), (1000, max(1001, n - Z - 2)), red_frac=red)
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=n)
    return x


def both(ctx, pk, fn):
    out = []
    for k in (pk.PULSCAN_KERNEL_TILED, pk.PULSCAN_KERNEL_STREAM):
        ctx.pulscan_ctx_set_kernel(k)
        out.append(fn())
    ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_AUTO)
    return out


CASES = [
    # n, zmax, chunk, options
    (1 << 16, 64, 256, {}),
    (1 << 16, 64, 256, {"dense": True}),
    ((1 << 18) + 37, 200, 1024, {}),
    ((1 << 18) + 37, 200, 1024, {"dense": True}),
    (1 << 20, 200, 1024, {"width_search": 1}),
    ((1 << 19) + 4099, 300, 1024, {}),
    (300000, 32, 256, {"norm_block": 1024}),
]


@pytest.mark.parametrize("n,Z,C,kw", CASES)
def test_kernels_give_identical_candidates(ctx, pk, oracle_lib, n, Z, C, kw):
    x = spectrum(oracle_lib, n, Z, C, seed=n % 97 + Z, red=0.01)
    d = to_device(x)
    say(f"kernels n={n} Z={Z} C={C} {kw}")
    opts = pk.make_opts(**kw)
    (a, na), (b, nb) = both(ctx, pk, lambda: ctx.pulscan_search_ex(d, Z, C, 6.0, opts=opts))
    assert na == nb and na > 0
    assert a.tobytes() == b.tobytes(), "tiled and streaming kernels differ"


@pytest.mark.parametrize("n,Z,C", [(1 << 16, 64, 256), ((1 << 18) + 37, 200, 1024)])
def test_kernels_give_identical_tables(ctx, pk, oracle_lib, n, Z, C):
    x = spectrum(oracle_lib, n, Z, C, seed=5 + Z)
    d = to_device(x)
    (ta, tb) = both(ctx, pk, lambda: [t.cpu().numpy() for t in ctx.pulscan_debug_tables(d, Z, C)
                                      if t is not None])
    assert len(ta) == len(tb) >= 2
    for i, (u, v) in enumerate(zip(ta, tb)):
        assert u.tobytes() == v.tobytes(), i


def test_kernels_give_identical_batches(ctx, pk, oracle_lib):
    xs = [spectrum(oracle_lib, n, z, 1024, seed=40 + s)
          for s, (n, z) in enumerate([(1 << 17, 64), (200001, 200), (1 << 18, 128)])]
    ds = [to_device(x) for x in xs]
    zs = [64, 200, 128]
    (a, na, ca), (b, nb, cb) = both(ctx, pk, lambda: ctx.pulscan_search_batched(ds, zs, 1024, 6.0))
    assert na == nb and ca == cb == 1024
    assert a.tobytes() == b.tobytes()
    # and every spectrum of the batch as its own search
    parts = []
    for s, (d, z) in enumerate(zip(ds, zs)):
        g, _ = ctx.pulscan_search_ex(d, z, 1024, 6.0)
        g["spectrum"] = s
        parts.append(g)
    assert np.concatenate(parts).tobytes() == a.tobytes()


def test_set_kernel_rejects_unknown_values(ctx, pk):
    with pytest.raises(pk.PulscanError) as e:
        ctx.pulscan_ctx_set_kernel(7)
    assert e.value.status == pk.PULSCAN_EINVAL


def test_heavily_flagged_tiles_match_the_dense_route(ctx, pk, oracle_lib):
    # one trial and a 1-sigma threshold put the thresholds just above the
    # mean, so the pruning bound flags nearly every lane and the tiles switch
    # to the dense evaluation: the candidates stay those of the dense route
    # and of the other kernel, byte for byte
    n, Z, C = (1 << 18) + 333, 200, 1024
    x = spectrum(oracle_lib, n, Z, C, seed=77)
    d = to_device(x)
    say("heavily flagged tiles")
    low = pk.make_opts(ntrials=1.0)
    ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_TILED)
    try:
        a, na = ctx.pulscan_search_ex(d, Z, C, 1.0, opts=low)
        b, nb = ctx.pulscan_search_ex(d, Z, C, 1.0, opts=pk.make_opts(ntrials=1.0, dense=True))
    finally:
        ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_AUTO)
    assert na == nb and na > 10000
    assert a.tobytes() == b.tobytes()
    (c, nc), (e, ne) = both(ctx, pk, lambda: ctx.pulscan_search_ex(d, Z, C, 1.0, opts=low))
    assert nc == ne == na
    assert c.tobytes() == e.tobytes() == a.tobytes()


def test_mixed_zmax_batch_matches_each_search(ctx, pk, oracle_lib):
    # a batch mixing small and large zmax, whose ranges the streaming
    # kernel's workgroups take in an order that depends on their speed: the
    # candidates are those of the tiled kernel and of every spectrum searched
    # alone
    shapes = [(1 << 17, 8), (150001, 300), (1 << 17, 16), (90000, 300), (70001, 8)]
    xs = [spectrum(oracle_lib, n, z, 1024, seed=90 + s, red=0.01) for s, (n, z) in enumerate(shapes)]
    ds = [to_device(x) for x in xs]
    zs = [z for _, z in shapes]
    say("mixed zmax batch")
    (a, na, ca), (b, nb, cb) = both(ctx, pk, lambda: ctx.pulscan_search_batched(ds, zs, 1024, 6.0))
    assert na == nb > 0 and ca == cb == 1024
    assert a.tobytes() == b.tobytes()
    parts = []
    for s, (d, z) in enumerate(zip(ds, zs)):
        g, _ = ctx.pulscan_search_ex(d, z, 1024, 6.0)
        g["spectrum"] = s
        parts.append(g)
    assert np.concatenate(parts).tobytes() == a.tobytes()


def test_ranges_taken_in_turn_give_the_same_candidates(ctx, pk):
    # a batch long enough (64 spectra of 2^20..2^23 bins, about 2.9e8) for
    # the streaming kernel to cut it into several ranges per workgroup, which
    # workgroups take from a counter in an order that varies between runs:
    # the candidates stay those of the tiled kernel, of a second run, and of
    # every spectrum searched alone
    import torch
    wls = synth.batched_workload(nspec=64, seed=11)

    def tone_power(A, w, nt):
        return float(ctx.pulscan_threshold_table(w, A, nt)[w - 1])

    xs = [synth.make_spectrum_device(w, tone_power)[0] for w in wls]
    zs = [w.zmax for w in wls]
    torch.cuda.synchronize()
    say(f"ranges taken in turn: {sum(w.nbins for w in wls)} bins")
    ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_STREAM)
    try:
        a, na, _ = ctx.pulscan_search_batched(xs, zs, 1024, 6.0)
        b, nb, _ = ctx.pulscan_search_batched(xs, zs, 1024, 6.0)
        ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_TILED)
        c, nc, _ = ctx.pulscan_search_batched(xs, zs, 1024, 6.0)
    finally:
        ctx.pulscan_ctx_set_kernel(pk.PULSCAN_KERNEL_AUTO)
    assert na == nb == nc > 0
    assert a.tobytes() == b.tobytes() == c.tobytes()
    parts = []
    for s, (d, z) in enumerate(zip(xs, zs)):
        g, _ = ctx.pulscan_search_ex(d, z, 1024, 6.0)
        g["spectrum"] = s
        parts.append(g)
    assert np.concatenate(parts).tobytes() == a.tobytes()
    del xs
    torch.cuda.empty_cache()
