"""MI355X (gfx950) phase-space Monte Carlo: Python binding of ``libhydra_phsp.so``.

Raubold-Lynch N-body phase-space generation and integration (arXiv:1711.05683,
sec. 4.2).  Every step of the computation runs in the HIP library; this module
only marshals arguments: torch tensors provide device memory and the current
HIP stream, and the C ABI declared in ``include/hydra_phsp.h`` is called through
ctypes with raw device pointers.  There is no CPU fallback: if the library has
not been built (``python -m paper_1711_05683_amd.build``) every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

from . import build as _build

LIB_PATH = _build.LIB_PATH
NMAX = 10
STATS = 4

OK, EINVAL, EKINEMATICS, ENOMEM, EDEVICE, EAGAIN, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6

_lib = None


class PhspError(RuntimeError):
    """A non-OK status returned by the C ABI."""

    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


def _declare(lib):
    c = ctypes
    d, i, u32, u64, vp = c.c_double, c.c_int, c.c_uint32, c.c_uint64, c.c_void_p
    dp = c.POINTER(c.c_double)
    lib.hydra_phsp_generate.argtypes = [d, dp, i, dp, vp, u64, u64, u64, u32, u64, vp, u64, vp, vp, vp]
    lib.hydra_phsp_generate.restype = i
    lib.hydra_phsp_generate_mixed.argtypes = lib.hydra_phsp_generate.argtypes
    lib.hydra_phsp_generate_mixed.restype = i
    lib.hydra_phsp_integrate_async.argtypes = [d, dp, i, u64, u64, u32, u64, vp, vp]
    lib.hydra_phsp_integrate_async.restype = i
    lib.hydra_phsp_integrate.argtypes = [d, dp, i, u64, u64, u32, u64, dp, dp, vp]
    lib.hydra_phsp_integrate.restype = i
    lib.hydra_phsp_strerror.argtypes = [i]
    lib.hydra_phsp_strerror.restype = c.c_char_p
    lib.hydra_phsp_last_error.argtypes = []
    lib.hydra_phsp_last_error.restype = c.c_char_p
    lib.hydra_phsp_abi_version.argtypes = []
    lib.hydra_phsp_abi_version.restype = i
    lib.hydra_phsp_selftest_sortnet.argtypes = []
    lib.hydra_phsp_selftest_sortnet.restype = i
    lib.hydra_phsp_release.argtypes = []
    lib.hydra_phsp_release.restype = i
    lib.hydra_phsp_timing_enable.argtypes = [i]
    lib.hydra_phsp_timing_enable.restype = i
    lib.hydra_phsp_timing_reset.argtypes = []
    lib.hydra_phsp_timing_reset.restype = i
    lib.hydra_phsp_timing_read.argtypes = [dp, c.POINTER(c.c_uint64)]
    lib.hydra_phsp_timing_read.restype = i


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1711_05683_amd.build` (no CPU fallback exists)")
        handle = ctypes.CDLL(LIB_PATH)
        _declare(handle)
        _lib = handle
    return _lib


def _check(status: int):
    if status != OK:
        msg = lib().hydra_phsp_last_error().decode(errors="replace")
        raise PhspError(status, msg or lib().hydra_phsp_strerror(status).decode())


def _masses(masses: Sequence[float]):
    n = len(masses)
    arr = (ctypes.c_double * max(n, 1))(*[float(m) for m in masses])
    return arr, n


def _stream_handle(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def generate(parent_mass: float, masses: Sequence[float], nevents: int, *, seed: int = 42,
             stream_id: int = 0, event_offset: int = 0, parent_p4: Optional[Sequence[float]] = None,
             parent_dev: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
             weights: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None,
             want_stats: bool = True, mixed: bool = False, device=None,
             stream: Optional[torch.cuda.Stream] = None):
    """Generate events on the GPU (asynchronous on the current stream).

    Returns ``(p4, weights, stats)``: ``p4`` is ``[N, 4, ld]`` (float64, or float32
    when ``mixed``), ``weights`` is ``[nevents]`` float64 and ``stats`` holds
    ``(n, mean, M2, sigma)`` of the weights (None unless ``want_stats``).
    ``parent_p4`` is one (E, px, py, pz) applied to all events; ``parent_dev`` a
    ``[4, ld_parent]`` float64 device tensor of per-event parents."""
    m, n = _masses(masses)
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    dtype = torch.float32 if mixed else torch.float64
    if out is None:
        out = torch.empty((n, 4, max(nevents, 1)), dtype=dtype, device=dev)
    if weights is None:
        weights = torch.empty(max(nevents, 1), dtype=torch.float64, device=dev)
    if stats is None and want_stats:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    if out.dtype != dtype or not out.is_contiguous() or out.dim() != 3 or out.shape[:2] != (n, 4):
        raise ValueError(f"out must be a contiguous [{n}, 4, ld] {dtype} tensor")
    if weights.dtype != torch.float64 or not weights.is_contiguous():
        raise ValueError("weights must be a contiguous float64 tensor")
    ld = out.shape[2]
    p4h = None
    if parent_p4 is not None:
        p4h = (ctypes.c_double * 4)(*[float(x) for x in parent_p4])
    ldp = 0
    if parent_dev is not None:
        if parent_dev.dtype != torch.float64 or parent_dev.dim() != 2 or parent_dev.shape[0] != 4 \
                or not parent_dev.is_contiguous():
            raise ValueError("parent_dev must be a contiguous [4, ld_parent] float64 tensor")
        ldp = parent_dev.shape[1]
    fn = lib().hydra_phsp_generate_mixed if mixed else lib().hydra_phsp_generate
    _check(fn(parent_mass, m, n, p4h, _dptr(parent_dev), ldp, nevents, seed, stream_id, event_offset,
              _dptr(out), ld, _dptr(weights), _dptr(stats), _stream_handle(stream)))
    return out, weights, stats


def integrate_async(parent_mass: float, masses: Sequence[float], nevents: int, *, seed: int = 42,
                    stream_id: int = 0, event_offset: int = 0, stats: Optional[torch.Tensor] = None,
                    device=None, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Integral without storage; returns the device stats tensor (n, mean, M2, sigma)."""
    m, n = _masses(masses)
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if stats is None:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    _check(lib().hydra_phsp_integrate_async(parent_mass, m, n, nevents, seed, stream_id, event_offset,
                                            _dptr(stats), _stream_handle(stream)))
    return stats


def integrate(parent_mass: float, masses: Sequence[float], nevents: int, *, seed: int = 42,
              stream_id: int = 0, event_offset: int = 0,
              stream: Optional[torch.cuda.Stream] = None):
    """Synchronous integral: returns (mean, sigma) as Python floats."""
    m, n = _masses(masses)
    mean = ctypes.c_double()
    sigma = ctypes.c_double()
    _check(lib().hydra_phsp_integrate(parent_mass, m, n, nevents, seed, stream_id, event_offset,
                                      ctypes.byref(mean), ctypes.byref(sigma), _stream_handle(stream)))
    return mean.value, sigma.value


def status_of(fn_name: str, *args) -> int:
    """Raw status of a C-ABI call (for validation tests)."""
    return getattr(lib(), fn_name)(*args)


def selftest_sortnet() -> bool:
    return lib().hydra_phsp_selftest_sortnet() == OK


def release():
    _check(lib().hydra_phsp_release())


def timing_enable(on: bool = True):
    """Bracket every main-kernel launch with HIP events on its stream."""
    _check(lib().hydra_phsp_timing_enable(1 if on else 0))
    _check(lib().hydra_phsp_timing_reset())


def timing_read():
    """(total kernel milliseconds, launches) since the last timing_enable/reset."""
    ms = ctypes.c_double()
    k = ctypes.c_uint64()
    _check(lib().hydra_phsp_timing_read(ctypes.byref(ms), ctypes.byref(k)))
    return ms.value, k.value
