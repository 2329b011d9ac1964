"""Seeded complex Fourier spectra: white noise, a red-noise ramp, boxcar tones.

The noise model is the paper's additive white Gaussian noise: every bin is
x = a + jb with a, b ~ N(0, 1) (section 2.1.2, the equation defining the
complex spectrum X).  The paper's own inputs were SIGPROC ``fake``
filterbanks turned into PRESTO ``.fft`` files (section 3.2); those files are
not available, and these seeded spectra stand in for them.

A drifting tone of drift z occupies bins r0 .. r0+z (z + 1 bins, the width
of the unit boxcar that matches it, section 2.2.3).  Each of its bins gets
alpha * exp(i phi_k) added, with phi_k uniform on [0, 2 pi).  Its strength
is given as a Gaussian-equivalent significance A: alpha^2 is chosen so that
the expected boxcar power of the matched width w equals the power whose
Bonferroni-corrected significance is A, i.e.
    w * (2 + alpha^2) = tone_power(A, w, ntrials).
``tone_power`` is supplied by the caller; nothing here evaluates the
chi-square or normal distributions.

Random streams: numpy PCG64 seeded through SeedSequence(seed).  In a batch,
spectrum s draws its length, zmax and tone count from child s of
SeedSequence(batch_seed) and its data from its own seed
batch_seed * 1000003 + s.  Within one spectrum the draws are, in order: the
tone parameters, the noise (one (n, 2) float32 standard-normal draw), then
the tone phases.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np

ToneGen = Callable[[float, int, float], float]


@dataclasses.dataclass
class Tone:
    r0: int          # first bin of the tone
    z: int           # drift in bins: the tone covers z + 1 bins
    A: float         # target significance (Gaussian-equivalent sigma)
    alpha2: float = 0.0   # per-bin added power |alpha|^2 (filled by inject_tones)


@dataclasses.dataclass
class Workload:
    name: str
    nbins: int
    zmax: int
    chunk: int
    sigma: float
    seed: int
    n_tones: int
    z_choices: Optional[Sequence[int]]   # explicit drifts (one tone each), or None
    z_range: tuple                        # inclusive (lo, hi) when z_choices is None
    A_range: tuple                        # (lo, hi), uniform
    r_range: tuple                        # inclusive (lo, hi) of r0
    red_frac: float = 0.0                 # fraction of bins under the 1/f ramp


def rng_for(seed: int, spawn: Optional[int] = None) -> np.random.Generator:
    """PCG64 generator for ``seed`` (and child ``spawn`` of it, if given)."""
    ss = np.random.SeedSequence(seed)
    if spawn is not None:
        ss = ss.spawn(spawn + 1)[spawn]
    return np.random.Generator(np.random.PCG64(ss))


def white_noise(n: int, rng: np.random.Generator) -> np.ndarray:
    """n complex64 bins with independent N(0, 1) real and imaginary parts."""
    x = rng.standard_normal((n, 2), dtype=np.float32)
    return x.view(np.complex64).reshape(n)


def red_ramp(x: np.ndarray, frac: float) -> np.ndarray:
    """Scale bins k < K = floor(frac * n) by sqrt(K / max(k, 1)) in place.

    Power then falls as 1/k over the first K bins and meets the white level
    at k = K: a stand-in for low-frequency red noise.
    """
    n = x.shape[0]
    K = int(np.floor(frac * n))
    if K > 0:
        k = np.arange(K, dtype=np.float64)
        scale = np.sqrt(K / np.maximum(k, 1.0)).astype(np.float32)
        x[:K] *= scale
    return x


def draw_tones(rng: np.random.Generator, wl: Workload, n_tones: Optional[int] = None,
               nbins: Optional[int] = None) -> List[Tone]:
    """Tone parameters for workload ``wl`` (r0, z, A), drawn from ``rng``.

    r0 is drawn from wl.r_range, capped so a tone of drift 200 still fits in
    ``nbins`` (default wl.nbins)."""
    n = wl.nbins if nbins is None else int(nbins)
    count = wl.n_tones if n_tones is None else n_tones
    if wl.z_choices is not None:
        zs = [int(z) for z in wl.z_choices][:count]
        count = len(zs)
    else:
        zs = [int(z) for z in rng.integers(wl.z_range[0], wl.z_range[1] + 1, size=count)]
    r_hi = min(wl.r_range[1], n - 202)
    r_lo = min(wl.r_range[0], max(r_hi, 0))
    r0s = rng.integers(r_lo, max(r_hi, r_lo) + 1, size=count)
    As = rng.uniform(wl.A_range[0], wl.A_range[1], size=count)
    return [Tone(int(r), z, float(a)) for r, z, a in zip(r0s, zs, As)]


def inject_tones(x: np.ndarray, tones: Sequence[Tone], rng: np.random.Generator,
                 zmax: int, ntrials: float, tone_power: ToneGen) -> np.ndarray:
    """Add each tone's constant-amplitude, random-phase bins to ``x`` in place.

    The matched width is w = min(z + 1, zmax); alpha^2 = max(T - 2w, 0) / w
    with T = tone_power(A, w, ntrials).
    """
    n = x.shape[0]
    for t in tones:
        w = min(t.z + 1, zmax)
        T = float(tone_power(t.A, w, ntrials))
        t.alpha2 = max(T - 2.0 * w, 0.0) / w
        lo, hi = t.r0, min(t.r0 + t.z + 1, n)
        phi = rng.uniform(0.0, 2.0 * np.pi, size=hi - lo)
        amp = np.float32(np.sqrt(t.alpha2))
        x[lo:hi] += (amp * np.exp(1j * phi)).astype(np.complex64)
    return x


def make_spectrum(wl: Workload, tone_power: Optional[ToneGen], spawn: Optional[int] = None,
                  nbins: Optional[int] = None, n_tones: Optional[int] = None):
    """Build one spectrum of workload ``wl``.

    Returns (x, tones): x is complex64 of length nbins (default wl.nbins).
    With ``tone_power`` None no tones are injected (pure noise, plus the
    ramp if the workload has one).
    """
    rng = rng_for(wl.seed, spawn)
    n = wl.nbins if nbins is None else int(nbins)
    tones = draw_tones(rng, wl, n_tones, n) if tone_power is not None else []
    x = white_noise(n, rng)
    if wl.red_frac > 0:
        red_ramp(x, wl.red_frac)
    if tones:
        ntrials = float(n) * wl.zmax
        inject_tones(x, tones, rng, wl.zmax, ntrials, tone_power)
    return x, tones


WORKLOADS = {
    # 2^16 bins, three tones of drift 10, 40, 60 at r0 in 1e3..6e4, 8-15 sigma.
    "plain_2e16": Workload("plain_2e16", 1 << 16, 64, 256, 6.0, 1, 3, (10, 40, 60), (1, 200),
                           (8.0, 15.0), (1000, 60000)),
    # 2^23 bins, 1/f ramp over the first 1 %, 50 tones of drift 1..200, 5-20 sigma.
    "plain_2e23": Workload("plain_2e23", 1 << 23, 200, 1024, 6.0, 2, 50, None, (1, 200),
                           (5.0, 20.0), (1000, (1 << 23) - 202), red_frac=0.01),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def batched_workload(nspec: int = 512, n_lo: int = 1 << 20, n_hi: int = 1 << 23,
                     seed: int = 3, zchoices=(64, 128, 200), sigma: float = 6.0):
    """Per-spectrum (nbins, zmax, n_tones) of a batch of DM-trial spectra.

    Spectrum s draws from child s of SeedSequence(seed): nbins uniform on
    [n_lo, n_hi], zmax uniform over ``zchoices``, 0-5 tones (drift 1..200,
    5-20 sigma).  Returns a list of Workload objects (chunk left 0: chosen
    by the caller).
    """
    out = []
    for s in range(nspec):
        rng = rng_for(seed, s)
        n = int(rng.integers(n_lo, n_hi + 1))
        z = int(zchoices[int(rng.integers(0, len(zchoices)))])
        k = int(rng.integers(0, 6))
        out.append(Workload(f"batch{seed}_{s}", n, z, 0, sigma, seed * 1000003 + s, k, None,
                            (1, 200), (5.0, 20.0), (1000, max(1001, n - 202))))
    return out


def make_spectrum_device(wl: Workload, tone_power: Optional[ToneGen], device="cuda",
                         nbins: Optional[int] = None):
    """The same recipe as make_spectrum, generated on a GPU for batches too
    large to build on the host: the N(0, 1) noise comes from torch's seeded
    device generator (seed wl.seed), tone parameters and phases from the
    numpy stream of make_spectrum.  The values differ from make_spectrum's;
    a test that needs the oracle copies the spectrum back.  Returns a
    float32 (n, 2) device tensor and the tones."""
    import torch
    rng = rng_for(wl.seed)
    n = wl.nbins if nbins is None else int(nbins)
    tones = draw_tones(rng, wl, nbins=n) if tone_power is not None else []
    g = torch.Generator(device=device)
    g.manual_seed(int(wl.seed))
    x = torch.randn((n, 2), generator=g, device=device, dtype=torch.float32)
    if wl.red_frac > 0:
        K = int(np.floor(wl.red_frac * n))
        if K > 0:
            k = np.arange(K, dtype=np.float64)
            sc = torch.from_numpy(np.sqrt(K / np.maximum(k, 1.0)).astype(np.float32)).to(device)
            x[:K] *= sc[:, None]
    if tones:
        ntrials = float(n) * wl.zmax
        for t in tones:
            w = min(t.z + 1, wl.zmax)
            T = float(tone_power(t.A, w, ntrials))
            t.alpha2 = max(T - 2.0 * w, 0.0) / w
            lo, hi = t.r0, min(t.r0 + t.z + 1, n)
            phi = rng.uniform(0.0, 2.0 * np.pi, size=hi - lo)
            amp = np.float32(np.sqrt(t.alpha2))
            add = np.stack([amp * np.cos(phi), amp * np.sin(phi)], axis=1).astype(np.float32)
            x[lo:hi] += torch.from_numpy(add).to(device)
    return x, tones
