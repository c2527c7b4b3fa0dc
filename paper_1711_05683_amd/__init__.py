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
    lib.hydra_phsp_generate_noalloc.argtypes = lib.hydra_phsp_generate.argtypes
    lib.hydra_phsp_generate_noalloc.restype = i
    lib.hydra_phsp_generate_chain.argtypes = [d, dp, i, i, dp, i, u64, u64, u32, u32, u64, vp, u64, vp, vp,
                                              vp, u64, vp, vp, vp]
    lib.hydra_phsp_generate_chain.restype = i
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
    lib.hydra_phsp_set_events_per_thread.argtypes = [i, i]
    lib.hydra_phsp_set_events_per_thread.restype = i
    lib.hydra_phsp_set_unweight_chunks.argtypes = [i]
    lib.hydra_phsp_set_unweight_chunks.restype = i
    lib.hydra_phsp_stats_merge.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.hydra_phsp_stats_merge.restype = i
    lib.hydra_phsp_events_per_thread.argtypes = [i, i, i]
    lib.hydra_phsp_events_per_thread.restype = i
    lib.hydra_phsp_timing_enable.argtypes = [i]
    lib.hydra_phsp_timing_enable.restype = i
    lib.hydra_phsp_timing_reset.argtypes = []
    lib.hydra_phsp_timing_reset.restype = i
    lib.hydra_phsp_timing_read.argtypes = [dp, c.POINTER(c.c_uint64)]
    lib.hydra_phsp_timing_read.restype = i
    lib.hydra_phsp_generate_unweighted.argtypes = [d, dp, i, dp, u64, u64, u32, u64, d, vp, u64, vp, vp, vp, vp]
    lib.hydra_phsp_generate_unweighted.restype = i
    lib.hydra_phsp_integrate_model.argtypes = [d, dp, i, vp, i, u64, u64, u32, u64, vp, vp, vp]
    lib.hydra_phsp_integrate_model.restype = i
    lib.hydra_phsp_generate_unweighted_model.argtypes = [d, dp, i, vp, i, u64, u64, u32, u64, d, vp, u64, vp,
                                                         vp, vp, vp]
    lib.hydra_phsp_generate_unweighted_model.restype = i
    lib.hydra_phsp_generate_unweighted_user_model.argtypes = [vp, d, dp, dp, i, u64, u64, u32, u64, d, vp, u64,
                                                              vp, vp, vp, vp]
    lib.hydra_phsp_generate_unweighted_user_model.restype = i
    lib.hydra_phsp_user_model_create.argtypes = [c.c_char_p, i, c.POINTER(vp)]
    lib.hydra_phsp_user_model_create.restype = i
    lib.hydra_phsp_user_model_destroy.argtypes = [vp]
    lib.hydra_phsp_user_model_destroy.restype = i
    lib.hydra_phsp_user_model_daughters.argtypes = [vp]
    lib.hydra_phsp_user_model_daughters.restype = i
    lib.hydra_phsp_integrate_user_model.argtypes = [vp, d, dp, dp, i, u64, u64, u32, u64, vp, vp, vp]
    lib.hydra_phsp_integrate_user_model.restype = i
    lib.hydra_phsp_vegas_iteration.argtypes = [vp, i, vp, u64, u64, u32, vp, vp, vp, vp]
    lib.hydra_phsp_vegas_iteration.restype = i
    lib.hydra_phsp_vegas_refine.argtypes = [i, i, vp, vp, d]
    lib.hydra_phsp_vegas_refine.restype = i
    lib.hydra_phsp_vegas.argtypes = [vp, i, u64, i, i, d, u64, vp, dp, dp, dp, vp]
    lib.hydra_phsp_vegas.restype = i
    lib.hydra_phsp_user_integrand_create.argtypes = [c.c_char_p, i, c.POINTER(vp)]
    lib.hydra_phsp_user_integrand_create.restype = i
    lib.hydra_phsp_user_integrand_destroy.argtypes = [vp]
    lib.hydra_phsp_user_integrand_destroy.restype = i
    lib.hydra_phsp_vegas_user_iteration.argtypes = [vp, dp, dp, dp, i, i, vp, u64, u64, u32, vp, vp, vp, vp]
    lib.hydra_phsp_vegas_user_iteration.restype = i
    lib.hydra_phsp_vegas_user.argtypes = [vp, dp, dp, dp, i, i, u64, i, i, d, u64, vp, dp, dp, dp, vp]
    lib.hydra_phsp_vegas_user.restype = i
    lib.hydra_phsp_probe_write.argtypes = [vp, u64, i, vp, u64, i, vp]
    lib.hydra_phsp_probe_write.restype = i
    lib.hydra_phsp_probe_philox.argtypes = [u64, i, u64, u32, vp, vp]
    lib.hydra_phsp_probe_philox.restype = i


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1711_05683_amd.build` (no CPU fallback exists)")
        handle = ctypes.CDLL(LIB_PATH)
        _declare(handle)
        _declare_batch(handle)
        _declare_serve(handle)
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


def _check_buf(t: Optional[torch.Tensor], name: str, dtype, min_numel: int):
    """Reject a caller buffer the C ABI cannot check itself: wrong dtype, not
    contiguous, or fewer than ``min_numel`` elements (the kernels would write
    past its end).  Runs before any device is touched."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor")
    if t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} elements, {min_numel} needed")


def _launch_device(device=None, stream: Optional[torch.cuda.Stream] = None) -> torch.device:
    """The device the library will launch on: the stream's, else the current one.
    A ``device`` argument must name that device (the library launches on the
    current device; make another one current with ``torch.cuda.device``)."""
    cur = torch.device("cuda", torch.cuda.current_device())
    if stream is not None and torch.device(stream.device) != cur:
        raise ValueError(f"stream is on {stream.device}, the current device is {cur}")
    if device is not None:
        d = torch.device(device)
        if d.type != "cuda" or (d.index is not None and d.index != cur.index):
            raise ValueError(f"device {d} is not the current device {cur}")
    return cur


def _resident(device=None, stream: Optional[torch.cuda.Stream] = None, **bufs) -> torch.device:
    """Check that every given buffer lives in device memory of the launch device
    and return that device (host tensors are rejected before any device query)."""
    for name, t in bufs.items():
        if t is not None and not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA (device) tensor, got one on {t.device}")
    dev = _launch_device(device, stream)
    for name, t in bufs.items():
        if t is not None and t.device != dev:
            raise ValueError(f"{name} is on {t.device}, the launch device is {dev}")
    return dev


def aligned_ld(nevents: int) -> int:
    """Leading dimension for an SoA output of ``nevents`` events: a multiple of 32
    elements, so every column starts on a 128-byte line (FP64 and FP32) and each
    wave's stores cover whole lines.  Columns that start mid-line make the stores
    partial-line writes, which cost up to ~40% of the write bandwidth on MI355X."""
    return (max(nevents, 1) + 31) // 32 * 32


def generate(parent_mass: float, masses: Sequence[float], nevents: int, *, seed: int = 42,
             stream_id: int = 0, event_offset: int = 0, parent_p4: Optional[Sequence[float]] = None,
             parent_dev: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
             weights: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None,
             want_stats: bool = True, mixed: bool = False, noalloc: bool = False, device=None,
             stream: Optional[torch.cuda.Stream] = None):
    """Generate events on the GPU (asynchronous on the current stream).

    Returns ``(p4, weights, stats)``: ``p4`` is ``[N, 4, ld]`` (float64, or float32
    when ``mixed``; when ``out`` is not given, a ``[N, 4, nevents]`` view of a buffer
    with ``aligned_ld(nevents)`` columns), ``weights`` is ``[nevents]`` float64 and ``stats`` holds
    ``(n, mean, M2, sigma)`` of the weights (None unless ``want_stats``).
    ``parent_p4`` is one (E, px, py, pz) applied to all events; ``parent_dev`` a
    ``[4, ld_parent]`` float64 device tensor of per-event parents.  ``noalloc``
    calls ``hydra_phsp_generate_noalloc`` (the library allocates nothing; pass
    ``out``, ``weights`` and ``stats`` to keep the binding from allocating)."""
    m, n = _masses(masses)
    dtype = torch.float32 if mixed else torch.float64
    if out is not None and (not isinstance(out, torch.Tensor) or out.dtype != dtype or not out.is_contiguous()
                            or out.dim() != 3 or tuple(out.shape[:2]) != (n, 4)):
        raise ValueError(f"out must be a contiguous [{n}, 4, ld] {dtype} tensor")
    _check_buf(weights, "weights", torch.float64, nevents)
    _check_buf(stats, "stats", torch.float64, STATS)
    if parent_dev is not None:
        if not isinstance(parent_dev, torch.Tensor) or parent_dev.dtype != torch.float64 or parent_dev.dim() != 2 \
                or parent_dev.shape[0] != 4 or not parent_dev.is_contiguous():
            raise ValueError("parent_dev must be a contiguous [4, ld_parent] float64 tensor")
        if parent_dev.shape[1] < nevents:
            raise ValueError(f"parent_dev has {parent_dev.shape[1]} events per row, {nevents} needed")
    dev = _resident(device, stream, out=out, weights=weights, stats=stats, parent_dev=parent_dev)
    own_out = out is None
    if own_out:
        out = torch.empty((n, 4, aligned_ld(nevents)), dtype=dtype, device=dev)
    if weights is None:
        weights = torch.empty(max(nevents, 1), dtype=torch.float64, device=dev)
    if stats is None and want_stats:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    ld = out.shape[2]
    p4h = None
    if parent_p4 is not None:
        p4h = (ctypes.c_double * 4)(*[float(x) for x in parent_p4])
    ldp = 0
    if parent_dev is not None:
        ldp = parent_dev.shape[1]
    fn = lib().hydra_phsp_generate_mixed if mixed else lib().hydra_phsp_generate
    if noalloc:
        if mixed:
            raise ValueError("the allocation-free entry point is FP64 only")
        fn = lib().hydra_phsp_generate_noalloc
    _check(fn(parent_mass, m, n, p4h, _dptr(parent_dev), ldp, nevents, seed, stream_id, event_offset,
              _dptr(out), ld, _dptr(weights), _dptr(stats), _stream_handle(stream)))
    if own_out:
        out = out[:, :, :max(nevents, 1)]
    return out, weights, stats


def generate_chain(parent_mass: float, masses: Sequence[float], chained: int, masses2: Sequence[float],
                   nevents: int, *, seed: int = 42, stream_id: int = 0, stream_id2: int = 1, event_offset: int = 0,
                   out: Optional[torch.Tensor] = None, weights: Optional[torch.Tensor] = None,
                   stats: Optional[torch.Tensor] = None, out2: Optional[torch.Tensor] = None,
                   weights2: Optional[torch.Tensor] = None, stats2: Optional[torch.Tensor] = None,
                   want_stats: bool = True, device=None, stream: Optional[torch.cuda.Stream] = None):
    """A sequential decay in one launch (asynchronous): the first stage at rest,
    then daughter ``chained`` of every event decays into ``masses2`` (at most 4
    daughters) with counter stream ``stream_id2``.  The same result as
    ``generate`` twice, the second call with ``parent_dev=p4[chained]``.
    Returns ``(p4, weights, stats, p4_2, weights2, stats2)``; outputs not given
    are allocated on the line grid (``aligned_ld(nevents)`` columns) and
    returned as ``[N, 4, nevents]`` views."""
    m, n = _masses(masses)
    m2, n2 = _masses(masses2)
    for o, k, name in ((out, n, "out"), (out2, n2, "out2")):
        if o is not None and (not isinstance(o, torch.Tensor) or o.dtype != torch.float64 or not o.is_contiguous()
                              or o.dim() != 3 or tuple(o.shape[:2]) != (k, 4) or o.shape[2] < nevents):
            raise ValueError(f"{name} must be a contiguous [{k}, 4, ld >= nevents] float64 tensor")
    for b, name in ((weights, "weights"), (weights2, "weights2")):
        _check_buf(b, name, torch.float64, nevents)
    for b, name in ((stats, "stats"), (stats2, "stats2")):
        _check_buf(b, name, torch.float64, STATS)
    dev = _resident(device, stream, out=out, weights=weights, stats=stats, out2=out2, weights2=weights2,
                    stats2=stats2)
    views = []
    if out is None:
        out = torch.empty((n, 4, aligned_ld(nevents)), dtype=torch.float64, device=dev)
        views.append(0)
    if out2 is None:
        out2 = torch.empty((n2, 4, aligned_ld(nevents)), dtype=torch.float64, device=dev)
        views.append(1)
    if weights is None:
        weights = torch.empty(max(nevents, 1), dtype=torch.float64, device=dev)
    if weights2 is None:
        weights2 = torch.empty(max(nevents, 1), dtype=torch.float64, device=dev)
    if want_stats:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev) if stats is None else stats
        stats2 = torch.empty(STATS, dtype=torch.float64, device=dev) if stats2 is None else stats2
    _check(lib().hydra_phsp_generate_chain(parent_mass, m, n, int(chained), m2, n2, nevents, seed, stream_id,
                                           stream_id2, event_offset, _dptr(out), out.shape[2], _dptr(weights),
                                           _dptr(stats), _dptr(out2), out2.shape[2], _dptr(weights2),
                                           _dptr(stats2), _stream_handle(stream)))
    if 0 in views:
        out = out[:, :, :max(nevents, 1)]
    if 1 in views:
        out2 = out2[:, :, :max(nevents, 1)]
    return out, weights, stats, out2, weights2, stats2


def _unweighted_buffers(n: int, ntrials: int, capacity, want_events, want_index, device, stream, out, index,
                        counts, w_max_out):
    """Check or allocate the outputs of an unweighted sample; returns
    (out, index, counts, w_max_out, ld)."""
    cap = aligned_ld(ntrials) if capacity is None else int(capacity)
    if out is not None and (not isinstance(out, torch.Tensor) or out.dtype != torch.float64
                            or not out.is_contiguous() or out.dim() != 3 or tuple(out.shape[:2]) != (n, 4)):
        raise ValueError(f"out must be a contiguous [{n}, 4, capacity] float64 tensor")
    if index is not None:
        _check_buf(index, "index", torch.int64, 1)
        if index.dim() != 1:
            raise ValueError("index must be a one-dimensional int64 tensor")
    if out is not None and index is not None and index.shape[0] != out.shape[2]:
        raise ValueError("index must have one entry per output column")
    _check_buf(counts, "counts", torch.int64, 2)
    _check_buf(w_max_out, "w_max_out", torch.float64, 1)
    dev = _resident(device, stream, out=out, index=index, counts=counts, w_max_out=w_max_out)
    if out is None and want_events:
        out = torch.empty((n, 4, max(cap, 1)), dtype=torch.float64, device=dev)
    idx = index
    if idx is None and want_index:
        idx = torch.empty(out.shape[2] if out is not None else max(cap, 1), dtype=torch.int64, device=dev)
    if counts is None:
        counts = torch.empty(2, dtype=torch.int64, device=dev)
    wm = w_max_out if w_max_out is not None else torch.empty(1, dtype=torch.float64, device=dev)
    ld = out.shape[2] if out is not None else (idx.shape[0] if idx is not None else 0)
    return out, idx, counts, wm, ld


def generate_unweighted(parent_mass: float, masses: Sequence[float], ntrials: int, *, seed: int = 42,
                        stream_id: int = 0, event_offset: int = 0, w_max: float = 0.0,
                        parent_p4: Optional[Sequence[float]] = None, capacity: Optional[int] = None,
                        want_events: bool = True, want_index: bool = False, device=None,
                        stream: Optional[torch.cuda.Stream] = None, out: Optional[torch.Tensor] = None,
                        index: Optional[torch.Tensor] = None, counts: Optional[torch.Tensor] = None,
                        w_max_out: Optional[torch.Tensor] = None):
    """Hit-or-miss unweighted sample from ``ntrials`` weighted trials (asynchronous).

    Trial g is kept when v_g * w_max < w_g (``w_max`` = 0: the largest trial
    weight).  Returns ``(p4, index, counts, w_max_used)``: ``p4`` an
    ``[N, 4, capacity]`` float64 buffer whose first ``counts[0]`` columns are the
    kept events in trial order (None unless ``want_events``), ``index`` their
    global indices (int64, None unless ``want_index``), ``counts`` a device int64
    pair (kept, trials with w > w_max) and ``w_max_used`` a device scalar.  Read
    ``counts`` after synchronizing the stream.  ``out``, ``index``, ``counts`` and
    ``w_max_out`` may be given (contiguous, of those shapes and dtypes) to reuse
    buffers; ``capacity`` is then ``out``'s (or ``index``'s) last dimension."""
    m, n = _masses(masses)
    out, idx, counts, wm, ld = _unweighted_buffers(n, ntrials, capacity, want_events, want_index, device, stream,
                                                   out, index, counts, w_max_out)
    p4h = None
    if parent_p4 is not None:
        p4h = (ctypes.c_double * 4)(*[float(x) for x in parent_p4])
    _check(lib().hydra_phsp_generate_unweighted(parent_mass, m, n, p4h, ntrials, seed, stream_id, event_offset,
                                                float(w_max), _dptr(out), ld, _dptr(idx), _dptr(counts),
                                                _dptr(wm), _stream_handle(stream)))
    return out, idx, counts, wm


class BreitWigner(ctypes.Structure):
    """``hydra_phsp_breit_wigner``: a relativistic Breit-Wigner factor in the
    invariant mass of daughters (i, j)."""
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32), ("mass", ctypes.c_double),
                ("width", ctypes.c_double)]


def integrate_model(parent_mass: float, masses: Sequence[float], nevents: int, resonances=(), *, seed: int = 42,
                    stream_id: int = 0, event_offset: int = 0, values: Optional[torch.Tensor] = None,
                    want_values: bool = False, stats: Optional[torch.Tensor] = None, device=None,
                    stream: Optional[torch.cuda.Stream] = None):
    """Integral of |A|^2 over phase space, |A|^2 = prod of Breit-Wigner intensities
    given as (i, j, mass, width) tuples (asynchronous).  Returns ``(stats, values)``:
    the device stats (n, mean, M2, sigma) of w |A|^2 and, when asked, the per-event
    values."""
    m, n = _masses(masses)
    _check_buf(values, "values", torch.float64, nevents)
    _check_buf(stats, "stats", torch.float64, STATS)
    dev = _resident(device, stream, values=values, stats=stats)
    arr, k = _bw_array(resonances)
    if values is None and want_values:
        values = torch.empty(max(nevents, 1), dtype=torch.float64, device=dev)
    if stats is None:
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    _check(lib().hydra_phsp_integrate_model(parent_mass, m, n, ctypes.cast(arr, ctypes.c_void_p), k, nevents,
                                            seed, stream_id, event_offset, _dptr(values), _dptr(stats),
                                            _stream_handle(stream)))
    return stats, values


def _bw_array(resonances):
    k = len(resonances)
    arr = (BreitWigner * max(k, 1))(*[BreitWigner(int(a), int(b), float(c), float(d)) for a, b, c, d in resonances])
    return arr, k


def generate_unweighted_model(parent_mass: float, masses: Sequence[float], ntrials: int, resonances=(), *,
                              seed: int = 42, stream_id: int = 0, event_offset: int = 0, w_max: float = 0.0,
                              capacity: Optional[int] = None, want_events: bool = True, want_index: bool = False,
                              device=None, stream: Optional[torch.cuda.Stream] = None,
                              out: Optional[torch.Tensor] = None, index: Optional[torch.Tensor] = None,
                              counts: Optional[torch.Tensor] = None, w_max_out: Optional[torch.Tensor] = None):
    """Hit-or-miss sample of the Breit-Wigner model (parent at rest): trial g is
    kept when v_g * w_max < w_g |A|^2(g) (``w_max`` = 0: the largest w |A|^2).
    Arguments and results as for generate_unweighted."""
    m, n = _masses(masses)
    arr, k = _bw_array(resonances)
    out, idx, counts, wm, ld = _unweighted_buffers(n, ntrials, capacity, want_events, want_index, device, stream,
                                                   out, index, counts, w_max_out)
    _check(lib().hydra_phsp_generate_unweighted_model(parent_mass, m, n, ctypes.cast(arr, ctypes.c_void_p), k,
                                                      ntrials, seed, stream_id, event_offset, float(w_max),
                                                      _dptr(out), ld, _dptr(idx), _dptr(counts), _dptr(wm),
                                                      _stream_handle(stream)))
    return out, idx, counts, wm


USER_PARAMS = 16


class UserModel:
    """A user intensity compiled at run time: ``source`` is HIP device code that
    defines ``double hydra_phsp_user_intensity(const double* e, const double* px,
    const double* py, const double* pz, const double* par)`` for ``n_daughters``
    daughters (see include/hydra_phsp_model.h).  Compilation needs no GPU; a source
    that does not compile raises PhspError with the compiler's log."""

    def __init__(self, source: str, n_daughters: int):
        self._h = None
        h = ctypes.c_void_p()
        _check(lib().hydra_phsp_user_model_create(source.encode(), int(n_daughters), ctypes.byref(h)))
        self._h = h
        self.n = int(n_daughters)

    def integrate(self, parent_mass: float, masses: Sequence[float], nevents: int, params: Sequence[float] = (),
                  *, seed: int = 42, stream_id: int = 0, event_offset: int = 0,
                  values: Optional[torch.Tensor] = None, want_values: bool = False,
                  stats: Optional[torch.Tensor] = None, device=None, stream: Optional[torch.cuda.Stream] = None):
        """As integrate_model, with the user's intensity and parameters (at most
        USER_PARAMS).  Returns ``(stats, values)``."""
        m, n, par = self._params(masses, params)
        _check_buf(values, "values", torch.float64, nevents)
        _check_buf(stats, "stats", torch.float64, STATS)
        dev = _resident(device, stream, values=values, stats=stats)
        if values is None and want_values:
            values = torch.empty(max(nevents, 1), dtype=torch.float64, device=dev)
        if stats is None:
            stats = torch.empty(STATS, dtype=torch.float64, device=dev)
        _check(lib().hydra_phsp_integrate_user_model(self._h, parent_mass, m, par, len(params), nevents, seed,
                                                     stream_id, event_offset, _dptr(values), _dptr(stats),
                                                     _stream_handle(stream)))
        return stats, values

    def _params(self, masses, params):
        if self._h is None:
            raise ValueError("the model was destroyed")
        m, n = _masses(masses)
        if n != self.n:
            raise ValueError(f"the model has {self.n} daughters, {n} masses given")
        if len(params) > USER_PARAMS:
            raise ValueError(f"at most {USER_PARAMS} parameters")
        return m, n, (ctypes.c_double * max(len(params), 1))(*[float(x) for x in params])

    def generate_unweighted(self, parent_mass: float, masses: Sequence[float], ntrials: int,
                            params: Sequence[float] = (), *, seed: int = 42, stream_id: int = 0,
                            event_offset: int = 0, w_max: float = 0.0, capacity: Optional[int] = None,
                            want_events: bool = True, want_index: bool = False, device=None,
                            stream: Optional[torch.cuda.Stream] = None, out: Optional[torch.Tensor] = None,
                            index: Optional[torch.Tensor] = None, counts: Optional[torch.Tensor] = None,
                            w_max_out: Optional[torch.Tensor] = None):
        """Hit-or-miss sample of the user's intensity (parent at rest): trial g
        is kept when v_g * w_max < w_g * intensity(g).  Arguments and results as
        for generate_unweighted."""
        m, n, par = self._params(masses, params)
        out, idx, counts, wm, ld = _unweighted_buffers(n, ntrials, capacity, want_events, want_index, device,
                                                       stream, out, index, counts, w_max_out)
        _check(lib().hydra_phsp_generate_unweighted_user_model(self._h, parent_mass, m, par, len(params), ntrials,
                                                               seed, stream_id, event_offset, float(w_max),
                                                               _dptr(out), ld, _dptr(idx), _dptr(counts),
                                                               _dptr(wm), _stream_handle(stream)))
        return out, idx, counts, wm

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(lib().hydra_phsp_user_model_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


VEGAS_DMAX = 16


class GaussBox(ctypes.Structure):
    """``hydra_phsp_gauss_box``: the product-of-Gaussians integrand over a box."""
    _fields_ = [("dim", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lo", ctypes.c_double * VEGAS_DMAX), ("hi", ctypes.c_double * VEGAS_DMAX),
                ("mean", ctypes.c_double * VEGAS_DMAX), ("sigma", ctypes.c_double * VEGAS_DMAX)]


def gauss_box(lo, hi, mean, sigma) -> GaussBox:
    f = GaussBox()
    f.dim = len(lo)
    for k in range(len(lo)):
        f.lo[k], f.hi[k], f.mean[k], f.sigma[k] = float(lo[k]), float(hi[k]), float(mean[k]), float(sigma[k])
    return f


def vegas_iteration(f: GaussBox, grid: torch.Tensor, calls: int, *, seed: int = 42, iteration: int = 0,
                    want_hist: bool = True, want_values: bool = False, stream: Optional[torch.cuda.Stream] = None):
    """One VEGAS iteration on the device grid ([dim, bins+1] float64, asynchronous).
    Returns (stats, hist or None, values or None) as device tensors."""
    if not isinstance(grid, torch.Tensor) or grid.dtype != torch.float64 or not grid.is_contiguous() \
            or grid.dim() != 2 or grid.shape[0] != f.dim:
        raise ValueError("grid must be a contiguous [dim, bins+1] float64 tensor")
    bins = grid.shape[1] - 1
    dev = _resident(None, stream, grid=grid)
    stats = torch.empty(STATS, dtype=torch.float64, device=dev)
    hist = torch.empty((f.dim, bins), dtype=torch.float64, device=dev) if want_hist else None
    vals = torch.empty(max(calls, 1), dtype=torch.float64, device=dev) if want_values else None
    _check(lib().hydra_phsp_vegas_iteration(ctypes.byref(f), bins, _dptr(grid), calls, seed, iteration, _dptr(stats),
                                            _dptr(hist), _dptr(vals), _stream_handle(stream)))
    return stats, hist, vals


class UserIntegrand:
    """A VEGAS integrand compiled at run time: ``source`` is HIP device code that
    defines ``double hydra_phsp_user_integrand(const double* x, const double* par)``
    over ``dim`` coordinates (see include/hydra_phsp_vegas.h).  Compilation needs
    no GPU; a source that does not compile raises PhspError with the log."""

    def __init__(self, source: str, dim: int):
        self._h = None
        h = ctypes.c_void_p()
        _check(lib().hydra_phsp_user_integrand_create(source.encode(), int(dim), ctypes.byref(h)))
        self._h = h
        self.dim = int(dim)

    def _box(self, lo, hi, params):
        if self._h is None:
            raise ValueError("the integrand was destroyed")
        if len(lo) != self.dim or len(hi) != self.dim:
            raise ValueError(f"the integrand has {self.dim} dimensions")
        if len(params) > USER_PARAMS:
            raise ValueError(f"at most {USER_PARAMS} parameters")
        D = ctypes.c_double
        return ((D * self.dim)(*map(float, lo)), (D * self.dim)(*map(float, hi)),
                (D * max(len(params), 1))(*map(float, params)))

    def iteration(self, lo, hi, grid: torch.Tensor, calls: int, params=(), *, seed: int = 42, iteration: int = 0,
                  want_hist: bool = True, want_values: bool = False, stream: Optional[torch.cuda.Stream] = None):
        """One iteration on the device grid ([dim, bins+1] float64, asynchronous);
        returns (stats, hist or None, values or None) as device tensors."""
        lo_a, hi_a, par = self._box(lo, hi, params)
        if grid.dtype != torch.float64 or not grid.is_contiguous() or grid.dim() != 2 or grid.shape[0] != self.dim:
            raise ValueError("grid must be a contiguous [dim, bins+1] float64 tensor")
        bins = grid.shape[1] - 1
        dev = _resident(None, stream, grid=grid)
        stats = torch.empty(STATS, dtype=torch.float64, device=dev)
        hist = torch.empty((self.dim, bins), dtype=torch.float64, device=dev) if want_hist else None
        vals = torch.empty(max(calls, 1), dtype=torch.float64, device=dev) if want_values else None
        _check(lib().hydra_phsp_vegas_user_iteration(self._h, lo_a, hi_a, par, len(params), bins, _dptr(grid), calls,
                                                     seed, iteration, _dptr(stats), _dptr(hist), _dptr(vals),
                                                     _stream_handle(stream)))
        return stats, hist, vals

    def vegas(self, lo, hi, calls: int, iterations: int, params=(), *, warmup: int = 0, bins: int = 50,
              alpha: float = 1.5, seed: int = 42, grid=None, stream: Optional[torch.cuda.Stream] = None):
        """The whole integration (synchronous): (result, error, chi2/dof, final grid [dim, bins+1])."""
        import numpy as np
        lo_a, hi_a, par = self._box(lo, hi, params)
        g = np.ascontiguousarray(grid if grid is not None else
                                 np.tile(np.arange(bins + 1) / bins, (self.dim, 1)), dtype=np.float64)
        res, err, chi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().hydra_phsp_vegas_user(self._h, lo_a, hi_a, par, len(params), g.shape[1] - 1, calls, warmup,
                                           iterations, alpha, seed, g.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(res), ctypes.byref(err), ctypes.byref(chi),
                                           _stream_handle(stream)))
        return res.value, err.value, chi.value, g

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(lib().hydra_phsp_user_integrand_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def vegas_refine(grid, hist, alpha: float = 1.5):
    """Refined copy of a host grid ([dim, bins+1] numpy float64) from a host histogram."""
    import numpy as np
    g = np.array(grid, dtype=np.float64, copy=True, order="C")
    h = np.ascontiguousarray(hist, dtype=np.float64)
    _check(lib().hydra_phsp_vegas_refine(g.shape[0], g.shape[1] - 1, g.ctypes.data, h.ctypes.data, float(alpha)))
    return g


def vegas(f: GaussBox, calls: int, iterations: int, *, warmup: int = 0, bins: int = 50, alpha: float = 1.5,
          seed: int = 42, grid=None, stream: Optional[torch.cuda.Stream] = None):
    """VEGAS integration (synchronous): returns (result, error, chi2/dof, final grid [dim, bins+1])."""
    import numpy as np
    g = np.zeros((f.dim, bins + 1), dtype=np.float64) if grid is None else np.array(grid, dtype=np.float64)
    if grid is None:
        g[:] = np.arange(bins + 1) / bins
    res, err, chi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().hydra_phsp_vegas(ctypes.byref(f), bins, calls, warmup, iterations, float(alpha), seed,
                                  g.ctypes.data, ctypes.byref(res), ctypes.byref(err), ctypes.byref(chi),
                                  _stream_handle(stream)))
    return res.value, err.value, chi.value, g


PROBE_SPAN = 1024


def probe_write(out: torch.Tensor, weights: torch.Tensor, nevents: int, *, events_per_thread: int = 1,
                stream: Optional[torch.cuda.Stream] = None):
    """Streaming-write probe (asynchronous): the generator's store pattern with
    constant data.  ``out`` is a contiguous ``[C, ld]`` float64 tensor (``[N, 4, ld]``
    of a generate call may be passed flattened); column c gets the value c and
    ``weights`` gets -1 for events < ``nevents``."""
    if not isinstance(out, torch.Tensor) or out.dtype != torch.float64 or not out.is_contiguous() or out.dim() < 2:
        raise ValueError("out must be a contiguous [C, ld] (or [N, 4, ld]) float64 tensor")
    _check_buf(weights, "weights", torch.float64, nevents)
    ld = out.shape[-1]
    cols = out.numel() // max(ld, 1)
    _resident(None, stream, out=out, weights=weights)
    _check(lib().hydra_phsp_probe_write(_dptr(out), ld, cols, _dptr(weights), nevents, events_per_thread,
                                        _stream_handle(stream)))


def probe_philox(nevents: int, calls_per_event: int, *, seed: int = 42, stream_id: int = 0,
                 fold: Optional[torch.Tensor] = None, device=None, stream: Optional[torch.cuda.Stream] = None):
    """Philox probe (asynchronous): returns the int32 tensor of per-block
    exclusive-or folds of every Philox word the generator's events would draw
    (``PROBE_SPAN`` events per block)."""
    blocks = (nevents + PROBE_SPAN - 1) // PROBE_SPAN
    _check_buf(fold, "fold", torch.int32, blocks)
    dev = _resident(device, stream, fold=fold)
    if fold is None:
        fold = torch.empty(max(blocks, 1), dtype=torch.int32, device=dev)
    _check(lib().hydra_phsp_probe_philox(nevents, calls_per_event, seed, stream_id, _dptr(fold),
                                         _stream_handle(stream)))
    return fold


def integrate_async(parent_mass: float, masses: Sequence[float], nevents: int, *, seed: int = 42,
                    stream_id: int = 0, event_offset: int = 0, stats: Optional[torch.Tensor] = None,
                    device=None, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Integral without storage; returns the device stats tensor (n, mean, M2, sigma)."""
    m, n = _masses(masses)
    _check_buf(stats, "stats", torch.float64, STATS)
    dev = _resident(device, stream, stats=stats)
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


def set_events_per_thread(path: int, ept: int):
    """Events per thread for path 0 (integrate), 1 (FP64) or 2 (mixed); 0 = default."""
    _check(lib().hydra_phsp_set_events_per_thread(path, ept))


def stats_merge(a, b):
    """Statistics (n, mean, M2, sigma) of the union of two disjoint event sets
    from theirs (host values: sequences, or tensors on any device, which are
    copied to the host).  Returns a list of four floats."""
    def rec(x, name):
        if isinstance(x, torch.Tensor):
            x = x.detach().to("cpu", torch.float64).reshape(-1).tolist()
        x = [float(v) for v in x]
        if len(x) < 3:
            raise ValueError(f"{name} needs n, mean and M2")
        return (ctypes.c_double * STATS)(*(x + [0.0] * STATS)[:STATS])
    ra, rb = rec(a, "a"), rec(b, "b")
    out = (ctypes.c_double * STATS)()
    _check(lib().hydra_phsp_stats_merge(ctypes.addressof(ra), ctypes.addressof(rb), ctypes.addressof(out)))
    return list(out)


def set_unweight_chunks(chunks: int):
    """Pipeline depth of unweighted calls that store events (0 = default, 1 = no overlap)."""
    _check(lib().hydra_phsp_set_unweight_chunks(chunks))


def events_per_thread(path: int, n_daughters: int, per_event_parents: bool = False,
                      off_line_grid: bool = False) -> int:
    """Events per thread of the next launch on path 0 (integrate), 1 (FP64) or 2 (mixed);
    ``off_line_grid``: for outputs whose columns do not start on 128-byte lines."""
    r = lib().hydra_phsp_events_per_thread(path, n_daughters, int(per_event_parents) | (2 if off_line_grid else 0))
    _check(min(r, 0))
    return r


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


# ----------------------------------------------------------------- batched ----

class ChannelDesc(ctypes.Structure):
    """``hydra_phsp_channel`` (include/hydra_phsp_batch.h)."""
    _fields_ = [("parent_mass", ctypes.c_double), ("masses", ctypes.c_double * NMAX),
                ("n_daughters", ctypes.c_int32), ("stream_id", ctypes.c_uint32),
                ("nevents", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("event_offset", ctypes.c_uint64), ("p4_out_dev", ctypes.c_void_p),
                ("ld", ctypes.c_uint64), ("weights_dev", ctypes.c_void_p),
                ("stats_dev", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """``hydra_phsp_tuning``: events per thread (0 = per class, as a single-channel call),
    persistent blocks per CU (0 = default),
    tile schedule (0 static stride, 1 dynamic, 2 one block per tile, 3 one launch
    over every tile at one event per thread, 4 one persistent launch over every
    tile at each N's default) and the
    number of streams the class kernels are spread over (0 or 1 = one)."""
    _fields_ = [("ept", ctypes.c_int32), ("grid_per_cu", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("streams", ctypes.c_int32)]


def _declare_batch(lib):
    c = ctypes
    i, vp = c.c_int, c.c_void_p
    chp = c.POINTER(ChannelDesc)
    tp = c.POINTER(Tuning)
    lib.hydra_phsp_batch_run.argtypes = [chp, i, tp, vp, c.POINTER(c.c_int)]
    lib.hydra_phsp_batch_run.restype = i
    lib.hydra_phsp_plan_create.argtypes = [chp, i, tp, c.POINTER(c.c_void_p)]
    lib.hydra_phsp_plan_create.restype = i
    lib.hydra_phsp_plan_launch.argtypes = [vp, vp]
    lib.hydra_phsp_plan_launch.restype = i
    lib.hydra_phsp_plan_destroy.argtypes = [vp]
    lib.hydra_phsp_plan_destroy.restype = i
    lib.hydra_phsp_plan_info.argtypes = [vp, c.POINTER(c.c_uint64), c.POINTER(c.c_uint64)]
    lib.hydra_phsp_plan_info.restype = i
    lib.hydra_phsp_autotune.argtypes = [chp, i, vp, tp, c.POINTER(c.c_double)]
    lib.hydra_phsp_autotune.restype = i


def channel(parent_mass: float, masses: Sequence[float], nevents: int, *, seed: int = 42,
            stream_id: int = 0, event_offset: int = 0, out: Optional[torch.Tensor] = None,
            weights: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None) -> ChannelDesc:
    """Describe one batch channel; out/weights None together = integrate-only.
    The buffers must live on the device the batch will run on (the current one
    when the batch is enqueued or its plan created)."""
    n = len(masses)
    if out is not None and (not isinstance(out, torch.Tensor) or out.dtype != torch.float64
                            or not out.is_contiguous() or out.dim() != 3 or tuple(out.shape[:2]) != (n, 4)):
        raise ValueError(f"out must be a contiguous [{n}, 4, ld] float64 tensor")
    if out is not None and out.shape[2] < nevents:
        raise ValueError(f"out has ld {out.shape[2]} < nevents {nevents}")
    _check_buf(weights, "weights", torch.float64, nevents)
    _check_buf(stats, "stats", torch.float64, STATS)
    if any(t is not None for t in (out, weights, stats)):
        _resident(None, None, out=out, weights=weights, stats=stats)
    d = ChannelDesc()
    d.parent_mass = float(parent_mass)
    for k, mk in enumerate(masses):
        d.masses[k] = float(mk)
    d.n_daughters = len(masses)
    d.stream_id = stream_id
    d.nevents = nevents
    d.seed = seed
    d.event_offset = event_offset
    d.p4_out_dev = None if out is None else out.data_ptr()
    d.ld = 0 if out is None else out.shape[-1]
    d.weights_dev = None if weights is None else weights.data_ptr()
    d.stats_dev = None if stats is None else stats.data_ptr()
    return d


def _channel_array(chans):
    arr = (ChannelDesc * len(chans))(*chans)
    return arr


def _tuning(ept=0, grid_per_cu=0, schedule=0, streams=0):
    t = Tuning()
    t.ept = ept
    t.grid_per_cu = grid_per_cu
    t.schedule = schedule
    t.streams = streams
    return t


def batch_run(chans, *, ept: int = 0, grid_per_cu: int = 0, schedule: int = 0, streams: int = 0,
              stream=None):
    """Enqueue one batch (all channels; one launch per (daughter count, mode) class)."""
    L = lib()
    arr = _channel_array(chans)
    bad = ctypes.c_int(-1)
    t = _tuning(ept, grid_per_cu, schedule, streams)
    st = L.hydra_phsp_batch_run(arr, len(chans), ctypes.byref(t), _stream_handle(stream), ctypes.byref(bad))
    if st != OK:
        msg = L.hydra_phsp_last_error().decode(errors="replace")
        raise PhspError(st, f"channel {bad.value}: {msg}")


class Plan:
    """A batch captured into a HIP graph; launch() replays it."""

    def __init__(self, chans, *, ept: int = 0, grid_per_cu: int = 0, schedule: int = 0, streams: int = 0):
        L = lib()
        arr = _channel_array(chans)
        t = _tuning(ept, grid_per_cu, schedule, streams)
        h = ctypes.c_void_p()
        _check(L.hydra_phsp_plan_create(arr, len(chans), ctypes.byref(t), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().hydra_phsp_plan_launch(self._h, _stream_handle(stream)))

    def info(self):
        nt, g = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().hydra_phsp_plan_info(self._h, ctypes.byref(nt), ctypes.byref(g)))
        return nt.value, g.value

    def destroy(self):
        if self._h:
            _check(lib().hydra_phsp_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune(chans, stream=None):
    """(ept, grid_per_cu, schedule, streams, ms) of the fastest launch shape for this batch."""
    t = Tuning()
    ms = ctypes.c_double()
    _check(lib().hydra_phsp_autotune(_channel_array(chans), len(chans), _stream_handle(stream),
                                     ctypes.byref(t), ctypes.byref(ms)))
    return t.ept, t.grid_per_cu, t.schedule, t.streams, ms.value


# ----------------------------------------------------------------- serving ----

class RequestDesc(ctypes.Structure):
    """``hydra_phsp_request`` (include/hydra_phsp_serve.h)."""
    _fields_ = [("parent_mass", ctypes.c_double), ("masses", ctypes.c_double * NMAX),
                ("n_daughters", ctypes.c_int32), ("integrate_only", ctypes.c_int32),
                ("nevents", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("stream_id", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ServerCounters(ctypes.Structure):
    """``hydra_phsp_server_counters``."""
    _fields_ = [("bytes_in_use", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64), ("ticks", ctypes.c_uint64),
                ("finished", ctypes.c_uint64), ("budget_stalls", ctypes.c_uint64), ("active_stalls", ctypes.c_uint64),
                ("queue_wait_max_s", ctypes.c_double), ("queue_wait_sum_s", ctypes.c_double)]


class ResultDesc(ctypes.Structure):
    """``hydra_phsp_result``."""
    _fields_ = [("status", ctypes.c_int32), ("n_daughters", ctypes.c_int32),
                ("nevents", ctypes.c_uint64), ("mean", ctypes.c_double), ("sigma", ctypes.c_double),
                ("p4_dev", ctypes.c_void_p), ("weights_dev", ctypes.c_void_p),
                ("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


def _declare_serve(lib):
    c = ctypes
    i, vp, u64 = c.c_int, c.c_void_p, c.c_uint64
    lib.hydra_phsp_server_create.argtypes = [u64, u64, i, c.POINTER(c.c_void_p)]
    lib.hydra_phsp_server_submit.argtypes = [vp, c.POINTER(RequestDesc), c.POINTER(u64)]
    lib.hydra_phsp_server_step.argtypes = [vp]
    lib.hydra_phsp_server_completed.argtypes = [vp, c.POINTER(u64), i]
    lib.hydra_phsp_server_poll.argtypes = [vp, u64, c.POINTER(ResultDesc)]
    lib.hydra_phsp_server_release.argtypes = [vp, u64]
    lib.hydra_phsp_server_drain.argtypes = [vp]
    lib.hydra_phsp_server_replay.argtypes = [vp, c.POINTER(RequestDesc), c.POINTER(c.c_double), i,
                                             c.POINTER(c.c_double), c.POINTER(c.c_double),
                                             c.POINTER(u64)]
    lib.hydra_phsp_server_stats.argtypes = [vp, c.POINTER(u64), c.POINTER(u64), c.POINTER(u64),
                                            c.POINTER(u64)]
    lib.hydra_phsp_server_counters_get.argtypes = [vp, c.POINTER(ServerCounters)]
    lib.hydra_phsp_server_counters_get.restype = c.c_int
    lib.hydra_phsp_server_destroy.argtypes = [vp]
    for name in ("create", "submit", "step", "completed", "poll", "release", "drain", "replay", "stats",
                 "destroy"):
        getattr(lib, f"hydra_phsp_server_{name}").restype = i


def request(parent_mass: float, masses: Sequence[float], nevents: int, *, seed: int = 42,
            stream_id: int = 0, integrate_only: bool = False) -> RequestDesc:
    r = RequestDesc()
    r.parent_mass = float(parent_mass)
    for k, mk in enumerate(masses):
        r.masses[k] = float(mk)
    r.n_daughters = len(masses)
    r.integrate_only = 1 if integrate_only else 0
    r.nevents = nevents
    r.seed = seed
    r.stream_id = stream_id
    return r


class Server:
    """Continuous-batching request server (device memory bounded by ``budget_bytes``)."""

    def __init__(self, budget_bytes: int, max_events_per_tick: int = 0, max_active: int = 0):
        h = ctypes.c_void_p()
        _check(lib().hydra_phsp_server_create(budget_bytes, max_events_per_tick, max_active,
                                              ctypes.byref(h)))
        self._h = h

    def submit(self, req: RequestDesc) -> int:
        rid = ctypes.c_uint64()
        _check(lib().hydra_phsp_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        return rid.value

    def submit_status(self, req: RequestDesc) -> int:
        rid = ctypes.c_uint64()
        return lib().hydra_phsp_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid))

    def step(self) -> int:
        n = lib().hydra_phsp_server_step(self._h)
        if n < 0:
            _check(n)
        return n

    def completed(self, max_ids: int = 1024):
        ids = (ctypes.c_uint64 * max_ids)()
        n = lib().hydra_phsp_server_completed(self._h, ids, max_ids)
        if n < 0:
            _check(n)
        return [ids[i] for i in range(n)]

    def poll(self, rid: int):
        """ResultDesc when finished, else None."""
        res = ResultDesc()
        st = lib().hydra_phsp_server_poll(self._h, rid, ctypes.byref(res))
        if st == EAGAIN:
            return None
        _check(st)
        return res

    def release(self, rid: int):
        _check(lib().hydra_phsp_server_release(self._h, rid))

    def drain(self):
        _check(lib().hydra_phsp_server_drain(self._h))

    def replay(self, reqs, arrivals):
        """Native real-time replay; returns (latencies [s], wall seconds, peak arena bytes)."""
        n = len(reqs)
        arr = (RequestDesc * n)(*reqs)
        at = (ctypes.c_double * n)(*arrivals)
        lat = (ctypes.c_double * n)()
        wall = ctypes.c_double()
        peak = ctypes.c_uint64()
        _check(lib().hydra_phsp_server_replay(self._h, arr, at, n, lat, ctypes.byref(wall),
                                              ctypes.byref(peak)))
        return [lat[i] for i in range(n)], wall.value, peak.value

    def counters(self):
        """Admission counters: bytes in use / peak, ticks, finished requests, steps
        that left the queue's head waiting for budget or for an active slot, and
        the longest and summed submit-to-admit waits (seconds)."""
        c = ServerCounters()
        _check(lib().hydra_phsp_server_counters_get(self._h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in ServerCounters._fields_}

    def stats(self):
        a, b, c, d = (ctypes.c_uint64() for _ in range(4))
        _check(lib().hydra_phsp_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                             ctypes.byref(d)))
        return {"bytes_in_use": a.value, "peak_bytes": b.value, "ticks": c.value, "finished": d.value}

    def destroy(self):
        if self._h:
            _check(lib().hydra_phsp_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def device_view(ptr: int, shape, dtype=None) -> torch.Tensor:
    """Copy server-owned device memory into a new torch tensor (before release)."""
    import numpy as _np
    dtype = dtype or torch.float64
    n = int(_np.prod(shape))
    out = torch.empty(n, dtype=dtype, device="cuda")
    nbytes = n * out.element_size()
    if n:
        import ctypes as _c
        hip = _hip_runtime()
        st = hip.hipMemcpy(_c.c_void_p(out.data_ptr()), _c.c_void_p(ptr), _c.c_size_t(nbytes), 3)
        if st != 0:
            raise RuntimeError(f"hipMemcpy failed: {st}")
    return out.reshape(shape)


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip
