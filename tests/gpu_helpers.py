"""Shared helpers of the GPU parity tests: running the library, running the
oracle on the same seeded input, and comparing the two under the stated
tolerances."""

import sys

import numpy as np

# Boxcar powers: FP32 sums of up to zmax FP32 terms against FP64.  The bound
# the search is held to is a relative 1e-5.
POWER_RTOL = 1e-5
# Significance of matched candidates (FP64 on both sides, from powers that
# differ by at most POWER_RTOL).
SIGMA_ATOL = 1e-3
# Entries this close to the threshold may fall on either side.
SIGMA_BAND = 1e-4
# A different argmax bin is accepted when the oracle's own boxcar at the GPU's
# bin is within this relative distance of the oracle's maximum (a near tie).
TIE_RTOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def boxcar_at(P, i, w):
    return float(np.sum(P[int(i):int(i) + int(w)], dtype=np.float64))


def compare_candidates(gpu, orc, P, ntrials, sigma_thresh, oracle_mod, label="", dofmul=1):
    """Compare GPU candidates with the oracle's SearchResult (tables=True).

    P is the searched series: the power, or harmonic stage H, whose width-w
    boxcars have 2 w dofmul degrees of freedom with dofmul = H(H+1)/2.
    Returns the list of (chunk, width) entries accepted only because they
    sit within SIGMA_BAND of the threshold.
    """
    g = {(int(c["chunk"]), int(c["width"])): c for c in gpu}
    o = {(int(c["chunk"]), int(c["width"])): c for c in orc.cands}
    banded = []
    for k in set(o) - set(g):
        s = float(o[k]["sigma"])
        assert abs(s - sigma_thresh) < SIGMA_BAND, f"{label} oracle-only candidate {k} sigma {s}"
        banded.append(k)
    for k in set(g) - set(o):
        c, w = k
        s = oracle_mod.candidate_sigma(orc.M[c, w - 1], w * dofmul, ntrials)
        assert abs(s - sigma_thresh) < SIGMA_BAND, f"{label} gpu-only candidate {k} sigma {s}"
        banded.append(k)
    for k in set(g) & set(o):
        a, b = g[k], o[k]
        c, w = k
        assert abs(float(a["power"]) - b["power"]) <= POWER_RTOL * b["power"], (label, k, a, b)
        assert abs(float(a["sigma"]) - b["sigma"]) <= SIGMA_ATOL, (label, k, a, b)
        if int(a["bin"]) != int(b["bin"]):
            assert int(a["bin"]) + w <= len(P), (label, k, a)
            y = boxcar_at(P, a["bin"], w)
            assert y >= (1 - TIE_RTOL) * b["power"], (label, "argmax", k, a, b, y)
    # canonical order
    keys = [(int(c["spectrum"]), int(c["chunk"]), int(c["width"])) for c in gpu]
    assert keys == sorted(keys), f"{label} not in canonical order"
    if banded:
        say(f"{label}: {len(banded)} entries within {SIGMA_BAND} sigma of the threshold: {sorted(banded)}")
    return banded


def compare_tables(Mg, Ig, orc_M, orc_I, P, label=""):
    """Dense per-chunk maxima: M within POWER_RTOL, I equal or a near tie."""
    Mg = np.asarray(Mg, dtype=np.float64)
    Ig = np.asarray(Ig).view(np.uint32).astype(np.int64)
    none_o = orc_I < 0
    none_g = Ig == 0xFFFFFFFF
    assert (none_o == none_g).all(), f"{label} windows that fit differ"
    assert np.isneginf(Mg[none_g]).all()
    ok = ~none_o
    rel = np.abs(Mg[ok] - orc_M[ok]) / np.maximum(np.abs(orc_M[ok]), 1e-30)
    assert rel.max(initial=0.0) <= POWER_RTOL, f"{label} max rel err {rel.max()}"
    diff = np.argwhere(ok & (Ig != orc_I))
    for c, wi in diff:
        y = boxcar_at(P, Ig[c, wi], wi + 1)
        assert y >= (1 - TIE_RTOL) * orc_M[c, wi], (label, c, wi + 1, Ig[c, wi], orc_I[c, wi])
    return rel.max(initial=0.0), len(diff)
