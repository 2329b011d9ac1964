"""GPU parity of the search variants: harmonic summing (section 2.3),
r-block output (section 2.4) and the best candidate per chunk, each through
the C ABI against the FP64 oracle (or, where the variant only reorganises
the same candidates, against the library's own plain output)."""

import numpy as np
import pytest

import synth
from gpu_helpers import SIGMA_ATOL, SIGMA_BAND, compare_candidates, say, to_device

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


def stage_parity(ctx, pk, oracle, x, Z, C, sigma, numharm, label, **kw):
    n = x.shape[0]
    d = to_device(x)
    got, cnt = ctx.pulscan_search_ex(d, Z, C, sigma, opts=pk.make_opts(numharm=numharm, **kw))
    assert cnt == len(got)
    orc = oracle.search(x, Z, C, sigma, tables=True, numharm=numharm)
    for H in range(1, numharm + 1):
        S = orc.P if H == 1 else oracle.harmonic_sum(orc.P, H)
        M, I = oracle.chunk_maxima(S, Z, C)
        sub = oracle.SearchResult(orc.cands[orc.cands["harm"] == H], M, I)
        compare_candidates(got[got["harmonics"] == H], sub, S, float((n // H) * Z), sigma,
                           oracle, label=f"{label} H={H}", dofmul=H * (H + 1) // 2)
    keys = [(int(c["harmonics"]), int(c["chunk"]), int(c["width"])) for c in got]
    assert keys == sorted(keys), f"{label}: not in (stage, chunk, width) order"
    say(f"{label}: {len(got)} candidates, per stage {np.bincount(got['harmonics'])[1:].tolist()}")
    return got


@pytest.mark.parametrize("nbins,Z,C,numharm,sig", [(1 << 16, 64, 256, 1, None),
                                                   (1 << 18, 200, 1024, 1, None),
                                                   (1 << 16, 64, 256, 4, None),
                                                   (1 << 16, 64, 256, 1, 0.5)])
def test_candidate_sigma_at_gpu_power(ctx, pk, oracle_lib, nbins, Z, C, numharm, sig):
    """Every candidate's significance against the oracle's at the candidate's
    own FP32 power, dof and trial count: only the significance arithmetic
    (and the FP32 rounding of the reported value) differs, so they agree far
    more closely than the search-level tolerance.  A threshold of 0.5 sigma
    makes nearly every chunk maximum a candidate, so the reported values
    run from the small significances near the Gaussian's centre (where the
    inversion starts without its tail terms) to the tones'."""
    wl = synth.workload("plain_2e16")
    sig = wl.sigma if sig is None else sig
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=nbins)
    got, cnt = ctx.pulscan_search_ex(to_device(x), Z, C, sig,
                                     opts=pk.make_opts(numharm=numharm))
    assert cnt == len(got) > 0
    worst = worst_lp = 0.0
    for c in got:
        H = int(c["harmonics"])
        nt = float((nbins // H) * Z)
        dof = int(c["width"]) * H * (H + 1) // 2
        ref = oracle_lib.candidate_sigma(float(c["power"]), dof, nt)
        worst = max(worst, abs(float(c["sigma"]) - ref) / max(1.0, abs(ref)))
        # the log probability of section 2.6 the significance comes from
        ref_lp = oracle_lib.log_p_corrected(float(c["power"]), dof, nt)
        worst_lp = max(worst_lp, abs(float(c["logp"]) - ref_lp) / max(1.0, abs(ref_lp)))
    say(f"sigma at GPU power n={nbins} Z={Z} H<={numharm} threshold {sig}: {len(got)} candidates "
        f"(sigma {float(got['sigma'].min()):.2f}..{float(got['sigma'].max()):.2f}), "
        f"max relative difference {worst:.2e}, log p {worst_lp:.2e}")
    assert worst <= 2e-6
    assert worst_lp <= 2e-6
    if sig < 1.0:
        assert float(got["sigma"].min()) < 2.0


@pytest.mark.parametrize("nbins,Z,C,numharm", [(1 << 16, 64, 256, 4), ((1 << 16) + 123, 64, 256, 3),
                                               (1 << 20, 200, 1024, 4), (5000, 16, 64, 8)])
def test_harmonic_stages_match_oracle(ctx, pk, oracle_lib, nbins, Z, C, numharm):
    wl = synth.workload("plain_2e16")
    say(f"harmonics nbins={nbins} Z={Z} C={C} numharm={numharm}")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=nbins)
    got = stage_parity(ctx, pk, oracle_lib, x, Z, C, wl.sigma, numharm, f"harm n={nbins}")
    assert len(got) > 0


def test_harmonic_pruned_equals_dense(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    a, na = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(numharm=4))
    b, nb = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(numharm=4, dense=True))
    assert na == nb and (a == b).all()


def test_harmonic_batched_equals_plain(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    xs = [synth.make_spectrum(wl, oracle_lib.power_for_sigma, spawn=s, nbins=n)[0]
          for s, n in ((0, 1 << 16), (1, 40000), (2, 50001))]
    ds = [to_device(x) for x in xs]
    opts = pk.make_opts(numharm=3)
    got, cnt, used = ctx.pulscan_search_batched(ds, [64, 32, 48], 256, 6.0, opts=opts)
    assert used == 256 and cnt == len(got)
    parts = []
    for s, (d, z) in enumerate(zip(ds, [64, 32, 48])):
        g, _ = ctx.pulscan_search_ex(d, z, 256, 6.0, opts=opts)
        g["spectrum"] = s
        parts.append(g)
    ref = np.concatenate(parts)
    assert len(ref) == len(got) and (ref == got).all()


@pytest.mark.parametrize("numharm,rb", [(1, 1000), (1, 256), (2, 4096)])
def test_rblock_matches_the_oracle(ctx, pk, oracle_lib, numharm, rb):
    """R-Block (section 2.4): the GPU's reported block indices against the
    oracle's R-Block search of the same spectrum."""
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    got, _ = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(numharm=numharm, rblock=rb))
    exact, _ = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(numharm=numharm))
    orc = oracle_lib.search(x, 64, 256, 6.0, numharm=numharm, rblock=rb)
    orc_exact = oracle_lib.search(x, 64, 256, 6.0, numharm=numharm)
    key = lambda c: (int(c["harmonics"] if "harmonics" in c.dtype.names else c["harm"]),
                     int(c["chunk"]), int(c["width"]))
    g = {key(c): c for c in got}
    ge = {key(c): c for c in exact}
    o = {key(c): c for c in orc.cands}
    oe = {key(c): c for c in orc_exact.cands}
    # candidates away from the threshold are the oracle's
    for k in set(g) ^ set(o):
        s = float(o[k]["sigma"]) if k in o else float(g[k]["sigma"])
        assert abs(s - 6.0) < 1e-3, (k, s)
    assert len(set(g) & set(o)) > 0
    for k in set(g) & set(o):
        assert abs(float(g[k]["power"]) - o[k]["power"]) <= 1e-5 * o[k]["power"], k
        if int(ge[k]["bin"]) == int(oe[k]["bin"]):  # same argmax: same block
            assert int(g[k]["bin"]) == int(o[k]["bin"]), k
        assert int(g[k]["bin"]) == int(ge[k]["bin"]) // rb, k


def test_rblock_reports_block_indices(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    a, _ = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(numharm=2))
    b, _ = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(numharm=2, rblock=1000))
    assert len(a) == len(b) > 0
    np.testing.assert_array_equal(b["bin"], a["bin"] // 1000)
    for f in ("spectrum", "width", "power", "sigma", "chunk", "harmonics"):
        np.testing.assert_array_equal(a[f], b[f])


def best_of(c):
    """Per (spectrum, stage, chunk) run of a canonical list: the highest sigma,
    the first on ties."""
    out = []
    i = 0
    while i < len(c):
        j = i
        key = (c[i]["spectrum"], c[i]["harmonics"], c[i]["chunk"])
        b = i
        while j < len(c) and (c[j]["spectrum"], c[j]["harmonics"], c[j]["chunk"]) == key:
            if c[j]["sigma"] > c[b]["sigma"]:
                b = j
            j += 1
        out.append(c[b])
        i = j
    return np.array(out, dtype=c.dtype) if out else c[:0]


@pytest.mark.parametrize("numharm", [1, 3])
def test_best_per_chunk(ctx, pk, oracle_lib, numharm):
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    full, _ = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(numharm=numharm))
    best, cnt = ctx.pulscan_search_ex(d, 64, 256, 6.0,
                                      opts=pk.make_opts(numharm=numharm, best_per_chunk=True))
    assert cnt == len(best) > 0
    ref = best_of(full)
    assert len(ref) == len(best) and (ref == best).all()
    # against the oracle: each kept chunk's sigma is the oracle's best there
    orc = oracle_lib.search(x, 64, 256, 6.0, numharm=numharm).cands
    groups = {}
    for c in orc:
        k = (int(c["harm"]), int(c["chunk"]))
        groups[k] = max(groups.get(k, -np.inf), float(c["sigma"]))
    kept = {(int(c["harmonics"]), int(c["chunk"])): float(c["sigma"]) for c in best}
    for k, s in kept.items():
        if k not in groups:
            assert abs(s - 6.0) < 10 * SIGMA_BAND, k
            continue
        assert abs(s - groups[k]) <= 2 * SIGMA_ATOL, (k, s, groups[k])
    for k in set(groups) - set(kept):
        assert abs(groups[k] - 6.0) < SIGMA_BAND, k


def test_best_per_chunk_async_device_output(ctx, pk, oracle_lib):
    import torch
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    ref, rc = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(best_per_chunk=True,
                                                                          numharm=2))
    cap = pk.worst_count(d.shape[0], 64, 256, 2)
    buf = torch.zeros(cap * pk.CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        o = pk.make_opts(best_per_chunk=True, numharm=2, async_=True, stream=s)
        ctx.pulscan_search_ex(d, 64, 256, 6.0, capacity=cap, opts=o, out_device=buf,
                              count_device=cnt)
    s.synchronize()
    n = int(cnt.item())
    assert n == rc
    got = buf.cpu().numpy()[:n * pk.CANDIDATE_DTYPE.itemsize].view(pk.CANDIDATE_DTYPE)
    assert (got == ref).all()


def test_variant_options_are_validated(ctx, pk):
    import torch
    d = torch.zeros((4096, 2), dtype=torch.float32, device="cuda")
    for kw in ({"numharm": 17}, {"numharm": -1}, {"rblock": -5}):
        o = pk.make_opts(**kw)
        with pytest.raises(pk.PulscanError) as e:
            ctx.pulscan_search_ex(d, 16, 256, 6.0, opts=o)
        assert e.value.status == pk.PULSCAN_EINVAL


# ----------------------------------------------------- FP16 power storage --

# FP16 storage rounds each power to 11 bits (relative 2^-11 = 4.9e-4); a
# boxcar of them is within that of its FP32 sum, and the re-check makes every
# decision within 0.5 sigma of the threshold on FP32 power.  The reported
# power of a candidate is then within 1e-3 of the oracle's maximum (a
# re-checked one is the FP32 power at the FP16 argmax, a near tie at most), its
# sigma within 0.05, and the candidate sets differ at most in entries whose
# oracle sigma is within 0.05 of the threshold.
POWER16_RTOL = 1e-3
SIGMA16_ATOL = 0.05
BAND16 = 0.05


def fp16_diff(got, orc, sigma, label):
    g = {(int(c["harmonics"]), int(c["chunk"]), int(c["width"])): c for c in got}
    o = {(int(c["harm"]), int(c["chunk"]), int(c["width"])): c for c in orc.cands}
    only_o = set(o) - set(g)
    only_g = set(g) - set(o)
    for k in only_o:
        assert abs(float(o[k]["sigma"]) - sigma) < BAND16, (label, "missing", k, o[k])
    for k in only_g:
        assert abs(float(g[k]["sigma"]) - sigma) < BAND16, (label, "extra", k, g[k])
    rel = 0.0
    for k in set(g) & set(o):
        a, b = g[k], o[k]
        r = abs(float(a["power"]) - b["power"]) / b["power"]
        rel = max(rel, r)
        assert r <= POWER16_RTOL, (label, k, a, b)
        assert abs(float(a["sigma"]) - b["sigma"]) <= SIGMA16_ATOL, (label, k, a, b)
    say(f"{label}: {len(g)} candidates, set difference {len(only_o)} missing / {len(only_g)} "
        f"extra, max relative boxcar error {rel:.2e}")
    return len(only_o), len(only_g), rel


@pytest.mark.parametrize("nbins,Z,C,numharm", [(1 << 16, 64, 256, 1), (1 << 20, 200, 1024, 1),
                                               (1 << 18, 64, 1024, 3)])
def test_fp16_power_matches_oracle(ctx, pk, oracle_lib, nbins, Z, C, numharm):
    wl = synth.workload("plain_2e23")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=nbins)
    d = to_device(x)
    got, n = ctx.pulscan_search_ex(d, Z, C, 6.0,
                                   opts=pk.make_opts(power_fp16=True, numharm=numharm))
    assert n == len(got) > 0
    keys = [(int(c["harmonics"]), int(c["chunk"]), int(c["width"])) for c in got]
    assert keys == sorted(keys)
    orc = oracle_lib.search(x, Z, C, 6.0, numharm=numharm)
    fp16_diff(got, orc, 6.0, f"fp16 n={nbins} numharm={numharm}")


def test_fp16_pruned_equals_dense_and_batched(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    xs = [synth.make_spectrum(wl, oracle_lib.power_for_sigma, spawn=s, nbins=n)[0]
          for s, n in ((0, 1 << 16), (1, 50000))]
    ds = [to_device(x) for x in xs]
    a, na = ctx.pulscan_search_ex(ds[0], 64, 256, 6.0, opts=pk.make_opts(power_fp16=True))
    b, nb = ctx.pulscan_search_ex(ds[0], 64, 256, 6.0,
                                  opts=pk.make_opts(power_fp16=True, dense=True))
    assert na == nb and (a == b).all()
    got, n, _ = ctx.pulscan_search_batched(ds, [64, 48], 256, 6.0,
                                           opts=pk.make_opts(power_fp16=True))
    c, _ = ctx.pulscan_search_ex(ds[1], 48, 256, 6.0, opts=pk.make_opts(power_fp16=True))
    c["spectrum"] = 1
    ref = np.concatenate([a, c])
    assert n == len(ref) and (got == ref).all()


def test_fp16_admits_the_largest_chunk(ctx, pk, oracle_lib):
    """A 16384-bin chunk (with 1024-bin normalisation blocks) needs more LDS
    than a workgroup has with FP32 power and fits with FP16: one 16384-bin
    tile, its 17 blocks normalised by 8 waves (two or three each)."""
    n = 2 * 16384 + 123
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=n)
    d = to_device(x)
    with pytest.raises(pk.PulscanError) as e:
        ctx.pulscan_search_ex(d, 200, 16384, 6.0, opts=pk.make_opts(norm_block=1024))
    assert e.value.status == pk.PULSCAN_EUNSUPPORTED
    got, cnt = ctx.pulscan_search_ex(d, 200, 16384, 6.0,
                                     opts=pk.make_opts(norm_block=1024, power_fp16=True))
    assert cnt == len(got) > 0
    orc = oracle_lib.search(x, 200, 16384, 6.0, norm_block=1024)
    fp16_diff(got, orc, 6.0, f"fp16 n={n} C=16384")


def test_fp16_admits_the_largest_zmax(ctx, pk, oracle_lib):
    """zmax 4096 with 1024-bin chunks needs about 72 KiB of LDS per
    workgroup with FP32 power (its 64-bit maxima and thresholds alone
    48 KiB), so it is refused; with FP16 power it fits."""
    n = 5 * 1024 + 517
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=n)
    d = to_device(x)
    with pytest.raises(pk.PulscanError) as e:
        ctx.pulscan_search_ex(d, 4096, 1024, 6.0)
    assert e.value.status == pk.PULSCAN_EUNSUPPORTED
    got, cnt = ctx.pulscan_search_ex(d, 4096, 1024, 6.0, opts=pk.make_opts(power_fp16=True))
    assert cnt == len(got) > 0
    orc = oracle_lib.search(x, 4096, 1024, 6.0)
    fp16_diff(got, orc, 6.0, f"fp16 n={n} Z=4096")


def test_fp16_unsupported_with_4096_blocks(ctx, pk):
    import torch
    d = torch.zeros((1 << 14, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(pk.PulscanError) as e:
        ctx.pulscan_search_ex(d, 64, 4096, 6.0, opts=pk.make_opts(power_fp16=True))
    assert e.value.status == pk.PULSCAN_EUNSUPPORTED


# ------------------------------------------- exact median normalisation --

@pytest.mark.parametrize("n,Z,C", [(1 << 16, 64, 256), (65536 + 100, 64, 256), (1 << 14, 200, 1024),
                                   (1 << 12, 32, 64)])
def test_exact_normalisation_tables(ctx, pk, oracle_lib, n, Z, C):
    """Exact median / MAD per block (the CPU version's, section 2.5) against
    the oracle's EXACT mode: statistics, normalised power and the dense
    per-chunk maxima."""
    from gpu_helpers import compare_tables
    wl = synth.workload("plain_2e16")
    x, _ = synth.make_spectrum(wl, oracle_lib.power_for_sigma, nbins=n)
    opts = pk.make_opts(norm=pk.PULSCAN_NORM_EXACT)
    M, I, P, S = ctx.pulscan_debug_tables(to_device(x), Z, C, opts=opts)
    _, _, st = oracle_lib.normalise(x, C, oracle_lib.NORM_EXACT)
    np.testing.assert_allclose(S.cpu().numpy().astype(np.float64), st, rtol=2e-6, atol=1e-6)
    orc = oracle_lib.search(x, Z, C, 6.0, mode=oracle_lib.NORM_EXACT, tables=True)
    np.testing.assert_allclose(P.cpu().numpy().astype(np.float64), orc.P, rtol=1e-5, atol=1e-5)
    err, ties = compare_tables(M.cpu().numpy(), I.cpu().numpy(), orc.M, orc.I, orc.P, "exact")
    say(f"exact tables n={n}: max rel err {err:.2e}, near ties {ties}")


def test_exact_median_with_repeated_values(ctx, pk, oracle_lib):
    """Blocks full of ties (quantised amplitudes) and constant blocks (MAD 0)."""
    rng = np.random.default_rng(12)
    n = 1 << 14
    x = np.round(rng.standard_normal((n, 2)) * 2).astype(np.float32) / 2
    x[1024:2048] = 3.0
    x[5000:5300, 0] = -1.5
    xc = x.view(np.complex64).reshape(n)
    opts = pk.make_opts(norm=pk.PULSCAN_NORM_EXACT)
    M, I, P, S = ctx.pulscan_debug_tables(to_device(xc), 16, 256, opts=opts)
    _, _, st = oracle_lib.normalise(xc, 256, oracle_lib.NORM_EXACT)
    np.testing.assert_array_equal(S.cpu().numpy().astype(np.float64), st)
    orc = oracle_lib.search(xc, 16, 256, 6.0, mode=oracle_lib.NORM_EXACT, tables=True)
    np.testing.assert_allclose(P.cpu().numpy().astype(np.float64), orc.P, rtol=1e-5, atol=1e-5)


def test_exact_search_matches_oracle(ctx, pk, oracle_lib):
    wl = synth.workload("plain_2e16")
    x, tones = synth.make_spectrum(wl, oracle_lib.power_for_sigma)
    d = to_device(x)
    got, n = ctx.pulscan_search_ex(d, 64, 256, 6.0, opts=pk.make_opts(norm=pk.PULSCAN_NORM_EXACT))
    orc = oracle_lib.search(x, 64, 256, 6.0, mode=oracle_lib.NORM_EXACT, tables=True)
    compare_candidates(got, orc, orc.P, float(len(x) * 64), 6.0, oracle_lib, "exact search")
    # every injected tone is found with the exact median (unlike the MoM,
    # whose statistics a wide tone inflates)
    for t in tones:
        near = got[(got["bin"] >= t.r0 - t.z - 1) & (got["bin"] <= t.r0 + t.z + 1)]
        assert len(near) > 0, t
