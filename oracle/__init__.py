"""FP64 CPU oracle for the boxcar search (ctypes over ``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  It shares no code with
the GPU library and never imports it.  See ``oracle.c`` for the paper
passages each function follows.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NORM_MOM = 0
NORM_EXACT = 1
MAD_SCALE = 1.482602218505602


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-D_GNU_SOURCE",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cand(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int64), ("bin", ctypes.c_int64), ("width", ctypes.c_int32),
                ("harm", ctypes.c_int32), ("power", ctypes.c_double), ("sigma", ctypes.c_double),
                ("logp", ctypes.c_double)]


CAND_DTYPE = np.dtype([("chunk", np.int64), ("bin", np.int64), ("width", np.int32),
                       ("harm", np.int32), ("power", np.float64), ("sigma", np.float64),
                       ("logp", np.float64)])
assert CAND_DTYPE.itemsize == ctypes.sizeof(_Cand)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        i64 = ctypes.c_int64
        L.oracle_med4.restype = ctypes.c_double
        L.oracle_med4.argtypes = [ctypes.c_double] * 4
        L.oracle_mom.restype = ctypes.c_double
        L.oracle_mom.argtypes = [dp, i64, dp]
        L.oracle_exact_median.restype = ctypes.c_double
        L.oracle_exact_median.argtypes = [dp, i64, dp]
        L.oracle_normalise.restype = ctypes.c_int
        L.oracle_normalise.argtypes = [fp, i64, i64, ctypes.c_int, dp, dp, dp]
        L.oracle_power.restype = None
        L.oracle_power.argtypes = [dp, dp, i64, dp]
        L.oracle_boxcar.restype = None
        L.oracle_boxcar.argtypes = [dp, i64, ctypes.c_int, dp]
        L.oracle_chunk_maxima.restype = None
        L.oracle_chunk_maxima.argtypes = [dp, i64, ctypes.c_int, i64, dp,
                                          ctypes.POINTER(ctypes.c_int64)]
        for name in ("oracle_log_sf_chi2_2w",):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_int]
        for name in ("oracle_log_norm_sf", "oracle_sigma_from_logp"):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_double]
        for name in ("oracle_log_p_corrected", "oracle_candidate_sigma"):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
        L.oracle_power_for_sigma.restype = ctypes.c_double
        L.oracle_power_for_sigma.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
        L.oracle_search.restype = i64
        L.oracle_search.argtypes = [fp, i64, ctypes.c_int, i64, ctypes.c_double, i64, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_int, i64, ctypes.POINTER(_Cand), dp,
                                    ctypes.POINTER(ctypes.c_int64), dp]
        L.oracle_search_harm.restype = i64
        L.oracle_search_harm.argtypes = [fp, i64, ctypes.c_int, i64, ctypes.c_double, i64,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         i64, i64, ctypes.POINTER(_Cand), dp,
                                         ctypes.POINTER(ctypes.c_int64), dp]
        L.oracle_width_is_searched.restype = ctypes.c_int
        L.oracle_width_is_searched.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_rblock_index.restype = i64
        L.oracle_rblock_index.argtypes = [i64, i64]
        L.oracle_harmonic_sum.restype = i64
        L.oracle_harmonic_sum.argtypes = [dp, i64, ctypes.c_int, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _as_spec(spec):
    """complex64 array -> contiguous float32 (n, 2) view."""
    s = np.ascontiguousarray(spec)
    if s.dtype == np.complex64:
        s = s.view(np.float32).reshape(-1, 2)
    s = np.ascontiguousarray(s, dtype=np.float32).reshape(-1, 2)
    return s


def med4(a, b, c, d) -> float:
    return lib().oracle_med4(a, b, c, d)


def mom(x) -> float:
    x = _as_f64(x)
    work = np.empty_like(x)
    return lib().oracle_mom(_dptr(x), x.size, _dptr(work))


def exact_median(x) -> float:
    x = _as_f64(x)
    work = np.empty_like(x)
    return lib().oracle_exact_median(_dptr(x), x.size, _dptr(work))


def normalise(spec, block: int, mode: int = NORM_MOM):
    """(re', im', stats[nblocks, 4]) in FP64; stats = med_re, mad_re, med_im, mad_im."""
    s = _as_spec(spec)
    n = s.shape[0]
    re = np.empty(n)
    im = np.empty(n)
    nb = (n + block - 1) // block
    st = np.empty((nb, 4))
    rc = lib().oracle_normalise(s.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, block, mode,
                                _dptr(re), _dptr(im), _dptr(st))
    if rc != 0:
        raise ValueError("oracle_normalise rejected its arguments")
    return re, im, st


def power(re, im):
    re = _as_f64(re)
    im = _as_f64(im)
    P = np.empty_like(re)
    lib().oracle_power(_dptr(re), _dptr(im), re.size, _dptr(P))
    return P


def boxcar(P, w: int):
    P = _as_f64(P)
    n = P.size
    Y = np.empty(max(n - w + 1, 0))
    if Y.size:
        lib().oracle_boxcar(_dptr(P), n, w, _dptr(Y))
    return Y


def chunk_maxima(P, zmax: int, chunk: int):
    """(M[nchunks, zmax], I[nchunks, zmax]) per-chunk maxima and argmax."""
    P = _as_f64(P)
    n = P.size
    nc = (n + chunk - 1) // chunk
    M = np.empty((nc, zmax))
    I = np.empty((nc, zmax), dtype=np.int64)
    lib().oracle_chunk_maxima(_dptr(P), n, zmax, chunk, _dptr(M),
                              I.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return M, I


def harmonic_sum(P, H: int):
    """Stage-H harmonic sum S_H (floor(n / H) values) of a power series."""
    P = _as_f64(P)
    S = np.empty(max(P.size // max(H, 1), 0))
    m = lib().oracle_harmonic_sum(_dptr(P), P.size, int(H), _dptr(S) if S.size else
                                  ctypes.cast(None, ctypes.POINTER(ctypes.c_double)))
    return S[:m]


def log_sf_chi2_2w(x: float, w: int) -> float:
    return lib().oracle_log_sf_chi2_2w(float(x), int(w))


def log_norm_sf(s: float) -> float:
    return lib().oracle_log_norm_sf(float(s))


def sigma_from_logp(lp: float) -> float:
    return lib().oracle_sigma_from_logp(float(lp))


def log_p_corrected(power: float, w: int, ntrials: float) -> float:
    return lib().oracle_log_p_corrected(float(power), int(w), float(ntrials))


def candidate_sigma(power: float, w: int, ntrials: float) -> float:
    return lib().oracle_candidate_sigma(float(power), int(w), float(ntrials))


def power_for_sigma(sigma: float, w: int, ntrials: float) -> float:
    return lib().oracle_power_for_sigma(float(sigma), int(w), float(ntrials))


class SearchResult:
    def __init__(self, cands, M=None, I=None, P=None):
        self.cands = cands
        self.M = M
        self.I = I
        self.P = P


W_ALL = 0
W_LOG2 = 1


def width_is_searched(w: int, zmax: int, width_search: int = W_ALL) -> bool:
    """Is width w of a 1..zmax bank searched for candidates (section 4.1.3)?"""
    return bool(lib().oracle_width_is_searched(int(w), int(zmax), int(width_search)))


def rblock_index(b: int, rblock: int) -> int:
    """The location an R-Block search reports for window start b (section 2.4)."""
    return int(lib().oracle_rblock_index(int(b), int(rblock)))


def search(spec, zmax: int, chunk: int, sigma: float, norm_block: int = 0, mode: int = NORM_MOM,
           ntrials: float = 0.0, tables: bool = False, cap: int = None,
           width_search: int = W_ALL, numharm: int = 1, rblock: int = 0) -> SearchResult:
    """Full search of one spectrum; candidates in (stage, chunk, width) order.
    With numharm > 1 the harmonic stages H = 1..numharm are searched and each
    candidate carries its stage in ``harm``; tables are those of stage 1.
    With rblock > 0 each candidate's ``bin`` is its r-block index (R-Block)."""
    s = _as_spec(spec)
    n = s.shape[0]
    nc = (n + chunk - 1) // chunk
    if cap is None:
        cap = sum(((n // H) + chunk - 1) // chunk for H in range(1, max(numharm, 1) + 1)) * zmax
    out = np.zeros(max(cap, 1), dtype=CAND_DTYPE)
    M = I = P = None
    mp = ip = pp = None
    if tables:
        M = np.empty((nc, zmax))
        I = np.empty((nc, zmax), dtype=np.int64)
        P = np.empty(n)
        mp, ip, pp = _dptr(M), I.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(P)
    cnt = lib().oracle_search_harm(s.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, zmax,
                                   chunk, sigma, norm_block, mode, ntrials, width_search,
                                   max(int(numharm), 1), int(rblock), cap,
                                   out.ctypes.data_as(ctypes.POINTER(_Cand)), mp, ip, pp)
    if cnt < 0:
        raise ValueError("oracle_search rejected its arguments")
    return SearchResult(out[:min(cnt, cap)].copy(), M, I, P)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(t: int) -> None:
    lib().oracle_set_num_threads(int(t))
