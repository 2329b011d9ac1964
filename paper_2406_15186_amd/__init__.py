"""Python binding of the MI355X boxcar-search library (``libpulscan.so``).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  Device memory and streams come from PyTorch tensors and
streams.  The names follow the C ABI declared in ``include/pulscan.h``.

There is no fallback: if the library has not been built, importing the
binding's functions raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpulscan.so")

PULSCAN_OK = 0
PULSCAN_EINVAL = -1
PULSCAN_ENOMEM = -2
PULSCAN_EOVERFLOW = -3
PULSCAN_EHIP = -4
PULSCAN_EUNSUPPORTED = -5
PULSCAN_NORM_MOM = 0
PULSCAN_NORM_EXACT = 1
PULSCAN_W_ALL = 0
PULSCAN_W_LOG2 = 1
PULSCAN_KERNEL_STREAM = 0
PULSCAN_KERNEL_TILED = 1
PULSCAN_KERNEL_AUTO = 2
# count_device values of an asynchronous search that failed on the device
PULSCAN_COUNT_LOST = 0xFFFFFFFFFFFFFFFF
PULSCAN_COUNT_POOL_FULL = 0xFFFFFFFFFFFFFFFE


class pulscan_candidate(ctypes.Structure):
    _fields_ = [("spectrum", ctypes.c_uint32), ("bin", ctypes.c_uint32),
                ("width", ctypes.c_uint32), ("power", ctypes.c_float),
                ("sigma", ctypes.c_float), ("chunk", ctypes.c_uint32),
                ("harmonics", ctypes.c_uint32), ("logp", ctypes.c_float)]


CANDIDATE_DTYPE = np.dtype([("spectrum", np.uint32), ("bin", np.uint32), ("width", np.uint32),
                            ("power", np.float32), ("sigma", np.float32), ("chunk", np.uint32),
                            ("harmonics", np.uint32), ("logp", np.float32)])


class pulscan_candidates(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("capacity", ctypes.c_uint64),
                ("count", ctypes.c_uint64), ("on_device", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("count_device", ctypes.c_void_p)]


class pulscan_opts(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_int32), ("norm_block", ctypes.c_int32),
                ("ntrials", ctypes.c_double), ("width_search", ctypes.c_int32),
                ("async_", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("dense", ctypes.c_int32), ("numharm", ctypes.c_int32),
                ("best_per_chunk", ctypes.c_int32), ("rblock", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("power_fp16", ctypes.c_int32)]


class pulscan_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_batch", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("sigma_thresh", ctypes.c_float),
                ("max_candidates", ctypes.c_uint32), ("opts", pulscan_opts)]


class pulscan_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32),
                ("count", ctypes.c_uint32), ("total", ctypes.c_uint64),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("candidates", ctypes.c_void_p)]


assert ctypes.sizeof(pulscan_server_config) == 80
assert ctypes.sizeof(pulscan_result) == 56
assert ctypes.sizeof(pulscan_candidate) == 32 == CANDIDATE_DTYPE.itemsize
assert ctypes.sizeof(pulscan_candidates) == 40
assert ctypes.sizeof(pulscan_opts) == 56

# every function the header declares: name -> (restype, argtypes)
_vp, _sz, _i, _f, _d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_float, ctypes.c_double
SIGNATURES = {
    "pulscan_strerror": (ctypes.c_char_p, [_i]),
    "pulscan_opts_default": (None, [ctypes.POINTER(pulscan_opts)]),
    "pulscan_ctx_create": (_i, [ctypes.POINTER(_vp), _i]),
    "pulscan_ctx_destroy": (None, [_vp]),
    "pulscan_search": (_i, [_vp, _sz, _i, _i, _f, ctypes.POINTER(pulscan_candidates)]),
    "pulscan_search_ex": (_i, [_vp, _vp, _sz, _i, _i, _f, ctypes.POINTER(pulscan_opts),
                               ctypes.POINTER(pulscan_candidates)]),
    "pulscan_search_batched": (_i, [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint64),
                                    ctypes.POINTER(ctypes.c_int32), _i, _f,
                                    ctypes.POINTER(pulscan_opts),
                                    ctypes.POINTER(pulscan_candidates), ctypes.POINTER(_i)]),
    "pulscan_debug_tables": (_i, [_vp, _vp, _sz, _i, _i, ctypes.POINTER(pulscan_opts), _vp, _vp,
                                  _vp, _vp]),
    "pulscan_debug_bank_from_power": (_i, [_vp, _vp, _sz, _i, _i, _vp, _vp]),
    "pulscan_threshold_table": (_i, [_vp, _i, _f, _d, _i, ctypes.POINTER(ctypes.c_float)]),
    "pulscan_ctx_set_timing": (_i, [_vp, _i]),
    "pulscan_ctx_kernel_time": (_i, [_vp, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_uint64)]),
    "pulscan_ctx_set_kernel": (_i, [_vp, _i]),
    "pulscan_ctx_last_kernel": (_i, [_vp, ctypes.POINTER(_i)]),
    "pulscan_ctx_set_spin": (_i, [_vp, ctypes.c_uint32]),
    "pulscan_search_noalloc": (_i, [_vp, ctypes.c_size_t, _i, _i, _f, ctypes.POINTER(pulscan_opts),
                                    ctypes.POINTER(pulscan_candidates)]),
    "pulscan_server_config_default": (None, [ctypes.POINTER(pulscan_server_config)]),
    "pulscan_server_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(pulscan_server_config)]),
    "pulscan_server_destroy": (None, [_vp]),
    "pulscan_server_submit": (ctypes.c_int64, [_vp, _vp, ctypes.c_uint64, ctypes.c_int32,
                                               ctypes.c_int32]),
    "pulscan_server_poll": (_i, [_vp, ctypes.POINTER(pulscan_result), _i, _i]),
    "pulscan_server_stats": (_i, [_vp] + [ctypes.POINTER(ctypes.c_uint64)] * 4),
    "pulscan_server_budget": (_i, [_vp, ctypes.POINTER(ctypes.c_uint64)]),
    "pulscan_host_alloc": (_i, [ctypes.POINTER(_vp), ctypes.c_uint64]),
    "pulscan_host_free": (None, [_vp]),
}

_lib = None


class PulscanError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = lib().pulscan_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})" if where else f"{msg} ({status})")


def lib() -> ctypes.CDLL:
    """The loaded library.  Raises if it has not been built.

    torch is imported first: the library then binds to the HIP runtime torch
    has already loaded, so the process holds a single runtime and device
    pointers and streams from torch are valid in the library's calls.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2406_15186_amd.build` (hipcc, gfx950)")
        import torch  # noqa: F401  (load torch's HIP runtime before ours binds)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str, allow_overflow: bool = False) -> int:
    if status == PULSCAN_OK or (allow_overflow and status == PULSCAN_EOVERFLOW):
        return status
    raise PulscanError(status, where)


def _spectrum_ptr(spectrum) -> tuple:
    """(device pointer, nbins) of a complex64 (n,) or float32 (n, 2) CUDA tensor."""
    import torch
    if not isinstance(spectrum, torch.Tensor) or not spectrum.is_cuda:
        raise TypeError("spectrum must be a CUDA (HIP) torch tensor")
    if not spectrum.is_contiguous():
        raise ValueError("spectrum must be contiguous")
    if spectrum.dtype == torch.complex64:
        n = spectrum.numel()
    elif spectrum.dtype == torch.float32 and spectrum.dim() == 2 and spectrum.shape[1] == 2:
        n = spectrum.shape[0]
    else:
        raise TypeError("spectrum must be complex64 (n,) or float32 (n, 2)")
    return spectrum.data_ptr(), n


def pulscan_opts_default() -> pulscan_opts:
    o = pulscan_opts()
    lib().pulscan_opts_default(ctypes.byref(o))
    return o


def worst_count(nbins: int, zmax: int, chunk: int, numharm: int = 1) -> int:
    """Most candidates one spectrum can yield: one per (stage, chunk, width)."""
    if chunk <= 0 or zmax <= 0:
        return 0
    return sum(((nbins // H) + chunk - 1) // chunk for H in range(1, max(numharm, 1) + 1)) * zmax


def make_opts(norm: int = PULSCAN_NORM_MOM, norm_block: int = 0, ntrials: float = 0.0,
              width_search: int = PULSCAN_W_ALL, async_: bool = False, stream=None,
              dense: bool = False, numharm: int = 1, best_per_chunk: bool = False,
              rblock: int = 0, graph: bool = False, power_fp16: bool = False) -> pulscan_opts:
    o = pulscan_opts_default()
    o.norm, o.norm_block, o.ntrials = norm, norm_block, ntrials
    o.width_search, o.async_, o.dense = width_search, int(bool(async_)), int(bool(dense))
    o.numharm, o.best_per_chunk, o.rblock = int(numharm), int(bool(best_per_chunk)), int(rblock)
    o.graph = int(bool(graph))
    o.power_fp16 = int(bool(power_fp16))
    if stream is not None:
        o.stream = stream if isinstance(stream, int) else stream.cuda_stream
    return o


def pulscan_search_noalloc(spectrum, zmax: int, chunk: int, sigma_thresh: float, out_device,
                           capacity: Optional[int] = None, opts: Optional[pulscan_opts] = None,
                           count_device=None) -> int:
    """The no-allocation search of one device spectrum into ``out_device`` (a
    CUDA uint8 tensor of capacity*32 bytes).  Returns the true count (0 for
    an asynchronous call, whose count goes to ``count_device``)."""
    ptr, n = _spectrum_ptr(spectrum)
    if opts is None:
        opts = pulscan_opts_default()
    if capacity is None:
        capacity = out_device.numel() // CANDIDATE_DTYPE.itemsize
    out = pulscan_candidates()
    out.data = out_device.data_ptr()
    out.on_device = 1
    out.capacity = capacity
    if count_device is not None:
        out.count_device = count_device.data_ptr()
    st = lib().pulscan_search_noalloc(ptr, n, zmax, chunk, sigma_thresh, ctypes.byref(opts),
                                      ctypes.byref(out))
    _check(st, "pulscan_search_noalloc", allow_overflow=True)
    return int(out.count)


class Context:
    """A library context (``pulscan_ctx``) on one HIP device."""

    def __init__(self, device: int = 0):
        self._ctx = ctypes.c_void_p()
        _check(lib().pulscan_ctx_create(ctypes.byref(self._ctx), device), "pulscan_ctx_create")
        self.device = device

    def close(self):
        if self._ctx:
            lib().pulscan_ctx_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._ctx

    # -- searches ---------------------------------------------------------
    def pulscan_search_ex(self, spectrum, zmax: int, chunk: int, sigma_thresh: float,
                          capacity: Optional[int] = None, opts: Optional[pulscan_opts] = None,
                          out_device=None, count_device=None):
        """Search one spectrum.  Returns (candidates, true_count).

        Host output by default (a numpy structured array of CANDIDATE_DTYPE).
        With ``out_device`` (a CUDA uint8 tensor of capacity*32 bytes) the
        candidates stay on the device and the array returned is None.
        """
        ptr, n = _spectrum_ptr(spectrum)
        if opts is None:
            opts = pulscan_opts_default()
        if capacity is None:
            capacity = worst_count(n, zmax, chunk, opts.numharm)
        out = pulscan_candidates()
        host = None
        if out_device is not None:
            out.data = out_device.data_ptr()
            out.on_device = 1
        else:
            host = np.zeros(max(capacity, 1), dtype=CANDIDATE_DTYPE)
            out.data = host.ctypes.data
        out.capacity = capacity
        if count_device is not None:
            out.count_device = count_device.data_ptr()
        st = lib().pulscan_search_ex(self._ctx, ptr, n, zmax, chunk, sigma_thresh,
                                     ctypes.byref(opts), ctypes.byref(out))
        _check(st, "pulscan_search_ex", allow_overflow=True)
        if host is None:
            return None, int(out.count)
        return host[:min(int(out.count), capacity)].copy(), int(out.count)

    def pulscan_search_batched(self, spectra: Sequence, zmax: Sequence[int], chunk: int,
                               sigma_thresh: float, capacity: Optional[int] = None,
                               opts: Optional[pulscan_opts] = None, out_device=None,
                               count_device=None):
        """Search several spectra in one launch.  Returns (candidates, true_count, chunk_used)."""
        ns = len(spectra)
        ptrs = (ctypes.c_void_p * ns)()
        ns_arr = (ctypes.c_uint64 * ns)()
        zs = (ctypes.c_int32 * ns)()
        if opts is None:
            opts = pulscan_opts_default()
        cap_auto = 0
        for i, (s, z) in enumerate(zip(spectra, zmax)):
            p, n = _spectrum_ptr(s)
            ptrs[i], ns_arr[i], zs[i] = p, n, int(z)
            cap_auto += worst_count(n, int(z), max(chunk, 64), opts.numharm)
        if capacity is None:
            capacity = cap_auto
        out = pulscan_candidates()
        host = None
        if out_device is not None:
            out.data = out_device.data_ptr()
            out.on_device = 1
        else:
            host = np.zeros(max(capacity, 1), dtype=CANDIDATE_DTYPE)
            out.data = host.ctypes.data
        out.capacity = capacity
        if count_device is not None:
            out.count_device = count_device.data_ptr()
        used = ctypes.c_int(0)
        st = lib().pulscan_search_batched(self._ctx, ns, ptrs, ns_arr, zs, chunk, sigma_thresh,
                                          ctypes.byref(opts), ctypes.byref(out), ctypes.byref(used))
        _check(st, "pulscan_search_batched", allow_overflow=True)
        if host is None:
            return None, int(out.count), used.value
        return host[:min(int(out.count), capacity)].copy(), int(out.count), used.value

    # -- parity helpers ---------------------------------------------------
    def pulscan_debug_tables(self, spectrum, zmax: int, chunk: int,
                             opts: Optional[pulscan_opts] = None, want_power: bool = True,
                             want_stats: bool = True):
        """Dense per-chunk maxima (M, I), and optionally power and block stats, as CUDA tensors."""
        import torch
        ptr, n = _spectrum_ptr(spectrum)
        if opts is None:
            opts = pulscan_opts_default()
        block = opts.norm_block if opts.norm_block > 0 else chunk
        nc = (n + chunk - 1) // chunk
        dev = spectrum.device
        M = torch.empty((nc, zmax), dtype=torch.float32, device=dev)
        I = torch.empty((nc, zmax), dtype=torch.int32, device=dev)
        P = torch.empty(n, dtype=torch.float32, device=dev) if want_power else None
        S = torch.empty(((n + block - 1) // block, 4), dtype=torch.float32, device=dev) \
            if want_stats else None
        torch.cuda.synchronize(dev)
        st = lib().pulscan_debug_tables(self._ctx, ptr, n, zmax, chunk, ctypes.byref(opts),
                                        M.data_ptr(), I.data_ptr(),
                                        P.data_ptr() if P is not None else None,
                                        S.data_ptr() if S is not None else None)
        _check(st, "pulscan_debug_tables")
        return M, I, P, S   # I holds uint32 bit patterns (0xFFFFFFFF: no window)

    def pulscan_debug_bank_from_power(self, power, zmax: int, chunk: int):
        """(M, I) of the bank run directly on a CUDA float32 power tensor."""
        import torch
        if power.dtype != torch.float32 or not power.is_cuda or not power.is_contiguous():
            raise TypeError("power must be a contiguous CUDA float32 tensor")
        n = power.numel()
        nc = (n + chunk - 1) // chunk
        M = torch.empty((nc, zmax), dtype=torch.float32, device=power.device)
        I = torch.empty((nc, zmax), dtype=torch.int32, device=power.device)
        torch.cuda.synchronize(power.device)
        st = lib().pulscan_debug_bank_from_power(self._ctx, power.data_ptr(), n, zmax, chunk,
                                                 M.data_ptr(), I.data_ptr())
        _check(st, "pulscan_debug_bank_from_power")
        return M, I

    def pulscan_threshold_table(self, zmax: int, sigma_thresh: float, ntrials: float,
                                width_search: int = PULSCAN_W_ALL) -> np.ndarray:
        T = np.zeros(zmax, dtype=np.float32)
        st = lib().pulscan_threshold_table(self._ctx, zmax, sigma_thresh, ntrials, width_search,
                                           T.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        _check(st, "pulscan_threshold_table")
        return T

    # -- timing -----------------------------------------------------------
    def pulscan_ctx_set_timing(self, enable=True):
        """Bracket every N-th bank launch with HIP events: True or 1 times every
        launch, N > 1 every N-th, False or 0 none."""
        _check(lib().pulscan_ctx_set_timing(self._ctx, int(enable)), "pulscan_ctx_set_timing")

    def pulscan_ctx_last_kernel(self) -> int:
        """The bank kernel of the last launch (PULSCAN_KERNEL_STREAM or _TILED; -1 before)."""
        k = ctypes.c_int(-1)
        _check(lib().pulscan_ctx_last_kernel(self._ctx, ctypes.byref(k)), "pulscan_ctx_last_kernel")
        return int(k.value)

    def pulscan_ctx_set_kernel(self, kernel: int):
        """PULSCAN_KERNEL_AUTO (default), PULSCAN_KERNEL_STREAM or PULSCAN_KERNEL_TILED."""
        _check(lib().pulscan_ctx_set_kernel(self._ctx, int(kernel)), "pulscan_ctx_set_kernel")

    def pulscan_ctx_set_spin(self, polls: int):
        """Polls of a cross-workgroup word before the streaming kernel gives up."""
        _check(lib().pulscan_ctx_set_spin(self._ctx, int(polls)), "pulscan_ctx_set_spin")

    def pulscan_ctx_kernel_time(self):
        """(summed milliseconds, launches) of bank kernels since the last call."""
        ms = ctypes.c_double(0.0)
        k = ctypes.c_uint64(0)
        _check(lib().pulscan_ctx_kernel_time(self._ctx, ctypes.byref(ms), ctypes.byref(k)),
               "pulscan_ctx_kernel_time")
        return ms.value, k.value


class Server:
    """The serving runtime (``pulscan_server``): submit spectra as they arrive,
    poll finished results with their timestamps."""

    def __init__(self, device: int = 0, hbm_budget: int = 4 << 30, max_batch: int = 256,
                 chunk: int = 1024, sigma_thresh: float = 6.0, max_candidates: int = 1 << 20,
                 opts: Optional[pulscan_opts] = None):
        cfg = pulscan_server_config()
        lib().pulscan_server_config_default(ctypes.byref(cfg))
        cfg.hbm_budget, cfg.max_batch, cfg.chunk = hbm_budget, max_batch, chunk
        cfg.sigma_thresh, cfg.max_candidates = sigma_thresh, max_candidates
        if opts is not None:
            cfg.opts = opts
        self._srv = ctypes.c_void_p()
        _check(lib().pulscan_server_create(ctypes.byref(self._srv), device, ctypes.byref(cfg)),
               "pulscan_server_create")
        self._res = (pulscan_result * 1024)()

    def close(self):
        if self._srv:
            lib().pulscan_server_destroy(self._srv)
            self._srv = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pulscan_server_submit(self, ptr: int, nbins: int, zmax: int, on_device: bool) -> int:
        """Queue a spectrum by address (device pointer, or pinned/host pointer)."""
        t = lib().pulscan_server_submit(self._srv, ptr, nbins, zmax, int(bool(on_device)))
        if t < 0:
            raise PulscanError(int(t), "pulscan_server_submit")
        return int(t)

    def pulscan_server_poll(self, wait_ms: int = 0, max_results: int = 1024):
        """Finished results: list of (ticket, status, total, t_submit, t_start,
        t_done, candidates array)."""
        k = lib().pulscan_server_poll(self._srv, self._res, min(max_results, 1024), wait_ms)
        _check(k if k < 0 else 0, "pulscan_server_poll")
        out = []
        for r in self._res[:k]:
            c = np.zeros(r.count, dtype=CANDIDATE_DTYPE)
            if r.count:
                ctypes.memmove(c.ctypes.data, r.candidates, r.count * CANDIDATE_DTYPE.itemsize)
            out.append((r.ticket, r.status, r.total, r.t_submit, r.t_start, r.t_done, c))
        return out

    def pulscan_server_budget(self) -> int:
        """The server's budget in bytes (as configured, or half the free
        device memory at creation for hbm_budget = 0)."""
        b = ctypes.c_uint64()
        _check(lib().pulscan_server_budget(self._srv, ctypes.byref(b)), "pulscan_server_budget")
        return int(b.value)

    def pulscan_server_stats(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().pulscan_server_stats(self._srv, *[ctypes.byref(x) for x in v]),
               "pulscan_server_stats")
        return tuple(int(x.value) for x in v)


def pulscan_host_alloc(nbytes: int) -> int:
    p = ctypes.c_void_p()
    _check(lib().pulscan_host_alloc(ctypes.byref(p), nbytes), "pulscan_host_alloc")
    return int(p.value)


def pulscan_host_free(ptr: int) -> None:
    lib().pulscan_host_free(ctypes.c_void_p(ptr))


def pulscan_search(spectrum, zmax: int, chunk: int, sigma_thresh: float,
                   capacity: Optional[int] = None):
    """The plain call on the library's default context: (candidates, true_count)."""
    ptr, n = _spectrum_ptr(spectrum)
    if capacity is None:
        capacity = worst_count(n, zmax, chunk)
    host = np.zeros(max(capacity, 1), dtype=CANDIDATE_DTYPE)
    out = pulscan_candidates()
    out.data = host.ctypes.data
    out.capacity = capacity
    st = lib().pulscan_search(ptr, n, zmax, chunk, sigma_thresh, ctypes.byref(out))
    _check(st, "pulscan_search", allow_overflow=True)
    return host[:min(int(out.count), capacity)].copy(), int(out.count)


def pulscan_strerror(status: int) -> str:
    return lib().pulscan_strerror(status).decode()
