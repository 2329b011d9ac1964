"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances (gpu_helpers): boxcar powers within a relative 1e-5; candidate
(chunk, width) sets identical except entries within 1e-4 sigma of the
threshold (listed); sigma within 1e-3; argmax bins identical except near
ties; integer-valued powers bit-exact.
"""

import numpy as np
import pytest

import synth
from gpu_helpers import compare_candidates, compare_tables, say, to_device

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


def nchunks(n, C):
    return (n + C - 1) // C


# ------------------------------------------------------------ thresholds --

@pytest.mark.parametrize("n,Z,ws", [(1 << 16, 64, 0), (1 << 23, 200, 0), (1 << 20, 128, 1),
                                    (5000, 1, 0)])
def test_threshold_table_matches_oracle(ctx, oracle_lib, n, Z, ws):
    say(f"thresholds n={n} Z={Z} ws={ws}")
    searched = [w for w in range(1, Z + 1) if oracle_lib.width_is_searched(w, Z, ws)]
    nt = float(n * max(len(searched), 1))
    T = ctx.pulscan_threshold_table(Z, 6.0, nt, ws)
    for w in range(1, Z + 1):
        if w not in searched:
            assert np.isposinf(T[w - 1])
            continue
        t = oracle_lib.power_for_sigma(6.0, w, nt)
        # the smallest FP32 value not below the FP64 threshold
        assert float(T[w - 1]) >= t * (1 - 1e-12)
        assert float(np.nextafter(T[w - 1], np.float32(-np.inf))) < t * (1 + 1e-12)


# ------------------------------------------------- bank on given powers --

BANK_CASES = [
    (4096, 64, 256), (5000, 200, 1024), (1000, 1, 64), (777, 77, 64), (65536 + 123, 200, 1024),
    (3000, 256, 256), (2048, 16, 128), (10000, 37, 192), (8192 + 5, 300, 4096), (300, 300, 64),
]


@pytest.mark.parametrize("n,Z,C", BANK_CASES)
def test_bank_from_power_integer_exact(ctx, oracle_lib, n, Z, C):
    """Integer powers sum exactly in FP32: M and I must equal the oracle's."""
    say(f"bank_from_power int n={n} Z={Z} C={C}")
    rng = np.random.default_rng(n * 7 + Z)
    P = rng.integers(0, 20, n).astype(np.float32)
    M, I = ctx.pulscan_debug_bank_from_power(to_device(P), Z, C)
    Mo, Io = oracle_lib.chunk_maxima(P.astype(np.float64), Z, C)
    Mg = M.cpu().numpy().astype(np.float64)
    Ig = I.cpu().numpy().view(np.uint32).astype(np.int64)
    Ig[Ig == 0xFFFFFFFF] = -1
    np.testing.assert_array_equal(Mg, Mo)
    np.testing.assert_array_equal(Ig, Io)


@pytest.mark.parametrize("n,Z,C", BANK_CASES[:6])
def test_bank_from_power_float(ctx, oracle_lib, n, Z, C):
    say(f"bank_from_power float n={n} Z={Z} C={C}")
    rng = np.random.default_rng(n + 3 * Z)
    P = rng.exponential(2.0, n).astype(np.float32)
    M, I = ctx.pulscan_debug_bank_from_power(to_device(P), Z, C)
    Mo, Io = oracle_lib.chunk_maxima(P.astype(np.float64), Z, C)
    err, ties = compare_tables(M.cpu().numpy(), I.cpu().numpy(), Mo, Io, P.astype(np.float64),
                               f"float n={n}")
    say(f"  max rel err {err:.2e}, near-tie argmax differences {ties}")


# ------------------------------------------------ normalisation + tables --

TABLE_CASES = [
    ("plain_2e16", None, None, None),
    ("plain_2e16", 65536 + 100, 64, 256),     # ragged tail: last block uses the last 256 bins
    ("plain_2e16", 1 << 14, 200, 1024),
    ("plain_2e16", 1 << 12, 32, 64),
    ("plain_2e16", 8192, 128, 4096),
]


@pytest.mark.parametrize("name,n,Z,C", TABLE_CASES)
def test_tables_with_normalisation(ctx, oracle_lib, name, n, Z, C):
    wl = synth.workload(name)
    n = n or wl.nbins
    Z = Z or wl.zmax
    C = C or wl.chunk
    say(f"tables {name} n={n} Z={Z} C={C}")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=n)
    M, I, P, S = ctx.pulscan_debug_tables(to_device(x), Z, C)
    orc = oracle_lib.search(x, Z, C, 6.0, tables=True)
    _, _, st = oracle_lib.normalise(x, C, oracle_lib.NORM_MOM)
    Sg = S.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(Sg, st, rtol=2e-6, atol=1e-6)
    Pg = P.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(Pg, orc.P, rtol=1e-5, atol=1e-5)
    err, ties = compare_tables(M.cpu().numpy(), I.cpu().numpy(), orc.M, orc.I, orc.P, name)
    say(f"  max rel err {err:.2e}, near-tie argmax differences {ties}")


# --------------------------------------------------------- full searches --

def _search_case(ctx, oracle_lib, x, Z, C, sigma=6.0, label="", **kw):
    say(f"search {label} n={len(x)} Z={Z} C={C}")
    cands, count = ctx.pulscan_search_ex(to_device(x), Z, C, sigma, **kw)
    assert count == len(cands)
    orc = oracle_lib.search(x, Z, C, sigma, tables=True)
    nt = float(len(x) * Z)
    compare_candidates(cands, orc, orc.P, nt, sigma, oracle_lib, label)
    return cands, orc


def test_search_plain_2e16(ctx, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, tones = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    cands, orc = _search_case(ctx, oracle_lib, x, wl.zmax, wl.chunk, label="plain_2e16")
    assert len(cands) > 20


def test_search_plain_2e23(ctx, oracle_lib):
    """The paper-scale spectrum: 2^23 bins, red-noise ramp, 50 tones, Z = 200."""
    wl = synth.workload("plain_2e23")
    x, tones = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    cands, orc = _search_case(ctx, oracle_lib, x, wl.zmax, wl.chunk, label="plain_2e23")
    say(f"  {len(cands)} candidates")
    assert len(cands) > 100


# the last two are the largest zmax that the 64 KiB of LDS per workgroup
# admit with FP32 power: 2048, with 1024-bin chunks and blocks (one-block
# tiles, two halo blocks) and with 4096-bin chunks and blocks
@pytest.mark.parametrize("n,Z,C", [(1 << 14, 1, 256), (1 << 14, 256, 256), (256, 64, 256),
                                   (1024 + 64, 64, 1024), (20000, 100, 64),
                                   (3 * 1024 + 517, 2048, 1024), (2 * 4096 + 333, 2048, 4096)])
def test_search_edge_shapes(ctx, oracle_lib, n, Z, C):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=n)
    _search_case(ctx, oracle_lib, x, Z, C, label=f"edge n={n} Z={Z} C={C}")


def test_search_degenerate_blocks(ctx, oracle_lib):
    """Constant and all-zero blocks (MAD = 0 -> normalised to 0) next to a
    huge-dynamic-range block."""
    rng = np.random.default_rng(77)
    n, C = 4096, 256
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    x[0:256] = 3.0 + 1.0j          # constant block
    x[256:512] = 0                 # zero block
    x[1024:1280] *= np.float32(1e3)
    x[1030] = 5e4 + 5e4j           # a huge outlier
    _search_case(ctx, oracle_lib, x, 64, C, label="degenerate")


def test_search_pure_noise_is_quiet(ctx, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, None, spawn=5)
    cands, count = ctx.pulscan_search_ex(to_device(x), wl.zmax, wl.chunk, wl.sigma)
    assert count == 0


@pytest.mark.parametrize("zmax,widths", [(64, [2, 3, 5, 9, 17, 33, 64]),
                                          (100, [2, 3, 5, 9, 17, 33, 65, 100])])
def test_log2_width_search(ctx, pk, oracle_lib, zmax, widths):
    """Logarithmic z sampling (z = 1, 2, 4, ... z-max): the searched widths,
    the trial count and the candidates match the oracle's."""
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    opts = pk.make_opts(width_search=pk.PULSCAN_W_LOG2)
    cands, count = ctx.pulscan_search_ex(to_device(x), zmax, wl.chunk, wl.sigma, opts=opts)
    orc = oracle_lib.search(x, zmax, wl.chunk, wl.sigma, tables=True,
                            width_search=oracle_lib.W_LOG2)
    nt = float(wl.nbins * len(widths))
    compare_candidates(cands, orc, orc.P, nt, wl.sigma, oracle_lib, f"log2 zmax {zmax}")
    assert set(cands["width"].tolist()) <= set(widths)
    assert zmax in set(orc.cands["width"].tolist())  # the endpoint finds something here
    T = ctx.pulscan_threshold_table(zmax, wl.sigma, nt, width_search=pk.PULSCAN_W_LOG2)
    assert [w for w in range(1, zmax + 1) if np.isfinite(T[w - 1])] == widths


# ------------------------------------------------------- API behaviours --

def test_overflow_returns_true_count_and_canonical_prefix(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    full, count = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
    assert count > 5
    part, count2 = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma, capacity=5)
    assert count2 == count and len(part) == 5
    assert (part == full[:5]).all()
    # a zero-capacity call still reports the count
    none, count3 = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma, capacity=0)
    assert count3 == count and len(none) == 0


def test_invalid_arguments(ctx, pk):
    import torch
    x = torch.zeros(4096, dtype=torch.complex64, device="cuda")
    bad = [
        (dict(zmax=0, chunk=256), pk.PULSCAN_EINVAL),
        (dict(zmax=10, chunk=0), pk.PULSCAN_EINVAL),
        (dict(zmax=5000, chunk=256), pk.PULSCAN_EINVAL),              # zmax > nbins
        (dict(zmax=10, chunk=8192), pk.PULSCAN_EINVAL),               # block > nbins
        (dict(zmax=10, chunk=128), pk.PULSCAN_EINVAL),                # MoM block not 4^k
        (dict(zmax=10, chunk=100, opts=pk.make_opts(norm_block=64)), pk.PULSCAN_EUNSUPPORTED),
        (dict(zmax=10, chunk=4096, opts=pk.make_opts(norm=pk.PULSCAN_NORM_EXACT)),
         pk.PULSCAN_EUNSUPPORTED),                                    # exact: blocks <= 1024
        (dict(zmax=10, chunk=512, opts=pk.make_opts(norm=pk.PULSCAN_NORM_EXACT)),
         pk.PULSCAN_EUNSUPPORTED),                                    # exact: 64 lanes x 4^k
        (dict(zmax=10, chunk=16), pk.PULSCAN_EUNSUPPORTED),           # valid 4^k, below 64
        (dict(zmax=10, chunk=256, opts=pk.make_opts(ntrials=0.5)), pk.PULSCAN_EINVAL),
        (dict(zmax=10, chunk=256, opts=pk.make_opts(width_search=7)), pk.PULSCAN_EINVAL),
    ]
    for kw, expect in bad:
        with pytest.raises(pk.PulscanError) as ei:
            ctx.pulscan_search_ex(x, sigma_thresh=6.0, **kw)
        assert ei.value.status == expect, (kw, ei.value.status)
    with pytest.raises(pk.PulscanError) as ei:
        ctx.pulscan_search_ex(x, 10, 256, float("nan"))
    assert ei.value.status == pk.PULSCAN_EINVAL


def test_chunk_320_with_block_64_is_supported(ctx, pk, oracle_lib):
    """A chunk that is a multiple of 64 but not a power of 4, with its own block."""
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=1 << 14)
    opts = pk.make_opts(norm_block=64)
    cands, _ = ctx.pulscan_search_ex(to_device(x), 50, 320, 6.0, opts=opts)
    orc = oracle_lib.search(x, 50, 320, 6.0, norm_block=64, tables=True)
    compare_candidates(cands, orc, orc.P, float(len(x) * 50), 6.0, oracle_lib, "chunk320")


def test_deterministic_repeats(ctx, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    first, _ = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
    for _ in range(10):
        again, _ = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
        assert again.tobytes() == first.tobytes()


def test_plain_entry_point_matches_ctx(pk, ctx, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    a, na = pk.pulscan_search(d, wl.zmax, wl.chunk, wl.sigma)
    b, nb = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
    assert na == nb and a.tobytes() == b.tobytes()


def test_async_device_output(ctx, pk, oracle_lib):
    import torch
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    ref, n_ref = ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
    cap = 4096
    buf = torch.zeros(cap * pk.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream()
    opts = pk.make_opts(async_=True, stream=s)
    ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma, capacity=cap, opts=opts,
                          out_device=buf, count_device=cnt)
    torch.cuda.synchronize()
    n = int(cnt.item())
    assert n == n_ref
    got = buf.cpu().numpy()[:n * pk.CANDIDATE_DTYPE.itemsize].view(pk.CANDIDATE_DTYPE)
    assert got.tobytes() == ref.tobytes()


def test_batched_matches_plain(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    shapes = [(1 << 16, 64), (50000, 200), (1 << 14, 128), (70001, 37), (4096, 1), (33333, 200)]
    specs, zs, refs = [], [], []
    for s, (n, Z) in enumerate(shapes):
        x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, spawn=s, nbins=n)
        d = to_device(x)
        specs.append(d)
        zs.append(Z)
        r, _ = ctx.pulscan_search_ex(d, Z, 1024, 6.0)
        r = r.copy()
        r["spectrum"] = s
        refs.append(r)
    say(f"batched {len(shapes)} spectra")
    got, count, used = ctx.pulscan_search_batched(specs, zs, 1024, 6.0)
    assert used == 1024
    ref = np.concatenate(refs)
    assert count == len(ref)
    assert got.tobytes() == ref.tobytes()
    # and one spectrum of the batch against the oracle directly
    x1 = specs[1].cpu().numpy()
    orc = oracle_lib.search(x1, 200, 1024, 6.0, tables=True)
    sub = got[got["spectrum"] == 1]
    compare_candidates(sub, orc, orc.P, float(50000 * 200), 6.0, oracle_lib, "batched[1]")


def test_kernel_timing_records_launches(ctx, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    ctx.pulscan_ctx_kernel_time()
    ctx.pulscan_ctx_set_timing(True)
    for _ in range(3):
        ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
    ms, k = ctx.pulscan_ctx_kernel_time()
    ctx.pulscan_ctx_set_timing(False)
    assert k == 3 and ms > 0
    # every 4th launch: the first, the fifth and the ninth of ten
    ctx.pulscan_ctx_set_timing(4)
    for _ in range(10):
        ctx.pulscan_search_ex(d, wl.zmax, wl.chunk, wl.sigma)
    ms, k = ctx.pulscan_ctx_kernel_time()
    ctx.pulscan_ctx_set_timing(0)
    assert k == 3 and ms > 0
    with pytest.raises(Exception):
        ctx.pulscan_ctx_set_timing(-1)


# ------------------------------------------------- pruning is exact --------

def _pruned_vs_dense(ctx, pk, x, Z, C, sigma=6.0, label=""):
    d = to_device(x)
    a, na = ctx.pulscan_search_ex(d, Z, C, sigma)
    b, nb = ctx.pulscan_search_ex(d, Z, C, sigma, opts=pk.make_opts(dense=True))
    assert na == nb, (label, na, nb)
    assert a.tobytes() == b.tobytes(), label
    return na


@pytest.mark.parametrize("name", ["plain_2e16", "plain_2e23"])
def test_pruned_equals_dense_workloads(ctx, pk, oracle_lib, name):
    wl = synth.workload(name)
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    say(f"pruned vs dense {name}")
    n = _pruned_vs_dense(ctx, pk, x, wl.zmax, wl.chunk, wl.sigma, name)
    assert n > 0


def test_pruned_equals_dense_near_threshold(ctx, pk, oracle_lib):
    """Many seeds with tones whose matched boxcar sits near the threshold, so
    many per-chunk maxima fall just either side of it."""
    import dataclasses
    base = synth.workload("plain_2e16")
    wl = dataclasses.replace(base, n_tones=40, z_choices=None, z_range=(1, 200), A_range=(5.5, 6.5),
                             r_range=(0, (1 << 16) - 202))
    total = 0
    for spawn in range(12):
        x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, spawn=spawn)
        for Z, C in ((64, 256), (200, 1024), (130, 64)):
            total += _pruned_vs_dense(ctx, pk, x, Z, C, 6.0, f"seed {spawn} Z={Z} C={C}")
    say(f"  {total} candidates compared")
    assert total > 0


def test_pruned_at_tile_edges_and_spectrum_end(ctx, pk, oracle_lib):
    """Wide tones straddling every tile boundary and ending at the last bin:
    the pruning bound must hold across halos and the spectrum's end."""
    rng = np.random.default_rng(99)
    for n, Z, C in ((3 * 4096 + 777, 200, 1024), (2 * 4096 + 300, 64, 256), (5000, 150, 64)):
        x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
        for edge in list(range(4096, n, 4096)) + [n]:
            for w, amp in ((190, 1.6), (30, 3.0), (5, 6.0)):
                lo = max(edge - w // 2, 0) if edge < n else n - w
                x[lo:lo + w] += np.complex64(amp)
        _pruned_vs_dense(ctx, pk, x, Z, C, 6.0, f"edges n={n} Z={Z} C={C}")
        cands, _ = ctx.pulscan_search_ex(to_device(x), Z, C, 6.0)
        orc = oracle_lib.search(x, Z, C, 6.0, tables=True)
        compare_candidates(cands, orc, orc.P, float(n * Z), 6.0, oracle_lib, f"edges n={n}")
        assert len(cands) > 0


def test_pruned_equals_dense_batched(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    specs, zs = [], []
    for s, (n, Z) in enumerate([(1 << 16, 64), (50000, 200), (70001, 37), (4096, 1)]):
        x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, spawn=s, nbins=n)
        specs.append(to_device(x))
        zs.append(Z)
    a, na, _ = ctx.pulscan_search_batched(specs, zs, 1024, 6.0)
    b, nb, _ = ctx.pulscan_search_batched(specs, zs, 1024, 6.0, opts=pk.make_opts(dense=True))
    assert na == nb and a.tobytes() == b.tobytes()
