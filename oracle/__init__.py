"""CPU oracle for N-body phase-space generation and integration (test infrastructure).

This package is the plain, slow, single-threaded FP64 implementation that the HIP
library is checked against (arXiv:1711.05683 sec. 4.2, Raubold-Lynch method; the
conventions are documented at the top of ``phsp_oracle.c``).  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code with the product library: the C source is compiled here with gcc
(``-O2 -ffp-contract=off``, no fast-math) into ``_liboracle.so`` and called via ctypes.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests against
rocRAND's Philox4x32-10 (independent implementation), closed-form and quadrature
phase-space volumes, exact two-body kinematics, per-event conservation laws and
Dalitz-plot flatness.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phsp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]

NMAX = 10
OK, EINVAL, EKINEMATICS = 0, -1, -2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``_liboracle.so`` (always, when force)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dp = ctypes.c_void_p
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_uniforms_per_event.argtypes = [ctypes.c_int]
    lib.oracle_uniforms_per_event.restype = ctypes.c_int
    lib.oracle_event_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_int, dp]
    lib.oracle_event_uniforms.restype = None
    lib.oracle_weight_constant.argtypes = [ctypes.c_double, dp, ctypes.c_int]
    lib.oracle_weight_constant.restype = ctypes.c_double
    lib.oracle_generate.argtypes = [ctypes.c_double, dp, ctypes.c_int, dp, dp, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint64, dp, ctypes.c_uint64, dp]
    lib.oracle_generate.restype = ctypes.c_int
    lib.oracle_integrate.argtypes = [ctypes.c_double, dp, ctypes.c_int, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.oracle_integrate.restype = ctypes.c_int
    lib.oracle_calls_per_event.argtypes = [ctypes.c_int]
    lib.oracle_calls_per_event.restype = ctypes.c_int
    lib.oracle_accept_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int]
    lib.oracle_accept_uniform.restype = ctypes.c_double
    lib.oracle_unweight.argtypes = [ctypes.c_double, dp, ctypes.c_int, dp, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, dp, ctypes.c_uint64,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.oracle_unweight.restype = ctypes.c_int
    lib.oracle_model_integrate.argtypes = [ctypes.c_double, dp, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp,
                                           ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, dp,
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.oracle_model_integrate.restype = ctypes.c_int
    lib.oracle_unweight_model.argtypes = [ctypes.c_double, dp, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp,
                                          ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_double, dp, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double)]
    lib.oracle_unweight_model.restype = ctypes.c_int
    lib.oracle_vegas_iteration.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_uint64,
                                           ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), dp, dp]
    lib.oracle_vegas_iteration.restype = ctypes.c_int
    lib.oracle_vegas_refine.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double]
    lib.oracle_vegas_refine.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _masses(masses):
    m = np.ascontiguousarray(np.asarray(masses, dtype=np.float64))
    return m


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: four 32-bit words for a 4-word counter and 2-word key."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def uniforms_per_event(n: int) -> int:
    return _load().oracle_uniforms_per_event(n)


def event_uniforms(seed: int, stream_id: int, g: int, n: int) -> np.ndarray:
    """The 3N-4 uniforms of global event g, in consumption order."""
    u = np.zeros(3 * n - 4, dtype=np.float64)
    _load().oracle_event_uniforms(seed, stream_id, g, n, _ptr(u))
    return u


def weight_constant(parent_mass: float, masses) -> float:
    m = _masses(masses)
    return _load().oracle_weight_constant(parent_mass, _ptr(m), len(m))


def generate(parent_mass, masses, nevents, seed=42, stream_id=0, event_offset=0,
             parent_p4=None, parent_soa=None, want_momenta=True):
    """Return (p4, weights): p4 has shape [N, 4, nevents] (SoA), weights [nevents]."""
    lib = _load()
    m = _masses(masses)
    n = len(m)
    out = np.zeros((n, 4, nevents), dtype=np.float64) if want_momenta else None
    w = np.zeros(nevents, dtype=np.float64)
    pp = None if parent_p4 is None else np.ascontiguousarray(parent_p4, dtype=np.float64)
    ps = None if parent_soa is None else np.ascontiguousarray(parent_soa, dtype=np.float64)
    ldp = 0 if ps is None else ps.shape[1]
    st = lib.oracle_generate(parent_mass, _ptr(m), n, _ptr(pp), _ptr(ps), ldp, nevents, seed,
                             stream_id, event_offset, _ptr(out), nevents, _ptr(w))
    if st != OK:
        raise OracleError(st)
    return out, w


def generate_status(parent_mass, masses, nevents=1):
    """Status code of a generate call (argument and kinematic validation only)."""
    lib = _load()
    m = _masses(masses)
    w = np.zeros(max(nevents, 1), dtype=np.float64)
    return lib.oracle_generate(parent_mass, _ptr(m), len(m), None, None, 0, nevents, 1, 0, 0,
                               None, 0, _ptr(w))


def integrate(parent_mass, masses, nevents, seed=42, stream_id=0, event_offset=0):
    """Return (mean, sigma): Monte Carlo estimate of the N-body volume and its error."""
    lib = _load()
    m = _masses(masses)
    mean = ctypes.c_double()
    sigma = ctypes.c_double()
    st = lib.oracle_integrate(parent_mass, _ptr(m), len(m), nevents, seed, stream_id,
                              event_offset, ctypes.byref(mean), ctypes.byref(sigma))
    if st != OK:
        raise OracleError(st)
    return mean.value, sigma.value


def calls_per_event(n: int) -> int:
    """Philox calls one event's own uniforms use."""
    return _load().oracle_calls_per_event(n)


def accept_uniform(seed: int, stream_id: int, g: int, n: int) -> float:
    """The hit-or-miss acceptance uniform of global event g."""
    return _load().oracle_accept_uniform(seed, stream_id, g, n)


def unweight(parent_mass, masses, ntrials, seed=42, stream_id=0, event_offset=0, w_max=0.0,
             parent_p4=None, capacity=None, want_momenta=True):
    """Hit-or-miss unweighting of ntrials weighted events (trial e kept when
    v_e * w_max < w_e; w_max = 0: the largest trial weight).

    Returns (p4, index, kept, over, w_max_used): p4 [N, 4, min(kept, capacity)] of the
    kept events in trial order, index their global event indices, kept the number
    kept, over the number of trials with w > w_max."""
    lib = _load()
    m = _masses(masses)
    n = len(m)
    cap = ntrials if capacity is None else capacity
    out = np.zeros((n, 4, max(cap, 1)), dtype=np.float64) if want_momenta else None
    idx = np.zeros(max(cap, 1), dtype=np.uint64)
    counts = np.zeros(2, dtype=np.uint64)
    used = ctypes.c_double()
    pp = None if parent_p4 is None else np.ascontiguousarray(parent_p4, dtype=np.float64)
    st = lib.oracle_unweight(parent_mass, _ptr(m), n, _ptr(pp), ntrials, seed, stream_id, event_offset,
                             float(w_max), _ptr(out), max(cap, 1) if want_momenta else cap, _ptr(idx),
                             _ptr(counts), ctypes.byref(used))
    if st != OK:
        raise OracleError(st)
    kept, over = int(counts[0]), int(counts[1])
    k = min(kept, cap)
    p4 = None if out is None else out[:, :, :k]
    return p4, idx[:k], kept, over, used.value


def unweight_model(parent_mass, masses, ntrials, resonances=(), seed=42, stream_id=0, event_offset=0, w_max=0.0,
                   capacity=None, want_momenta=True):
    """Hit-or-miss unweighting of ntrials events of a model (parent at rest): trial
    e is kept when v_e * w_max < w_e |A_e|^2, |A|^2 the Breit-Wigner product of
    model_integrate; w_max = 0: the largest trial value.  Returns (p4, index, kept,
    over, w_max_used) as unweight."""
    lib = _load()
    m = _masses(masses)
    n = len(m)
    k = len(resonances)
    pi = np.array([r[0] for r in resonances] + [0], dtype=np.int32)
    pj = np.array([r[1] for r in resonances] + [0], dtype=np.int32)
    rm = np.array([r[2] for r in resonances] + [0.0], dtype=np.float64)
    rg = np.array([r[3] for r in resonances] + [0.0], dtype=np.float64)
    cap = ntrials if capacity is None else capacity
    out = np.zeros((n, 4, max(cap, 1)), dtype=np.float64) if want_momenta else None
    idx = np.zeros(max(cap, 1), dtype=np.uint64)
    counts = np.zeros(2, dtype=np.uint64)
    used = ctypes.c_double()
    st = lib.oracle_unweight_model(parent_mass, _ptr(m), n, k, _ptr(pi), _ptr(pj), _ptr(rm), _ptr(rg), ntrials,
                                   seed, stream_id, event_offset, float(w_max), _ptr(out),
                                   max(cap, 1) if want_momenta else cap, _ptr(idx), _ptr(counts),
                                   ctypes.byref(used))
    if st != OK:
        raise OracleError(st)
    kept, over = int(counts[0]), int(counts[1])
    kk = min(kept, cap)
    p4 = None if out is None else out[:, :, :kk]
    return p4, idx[:kk], kept, over, used.value


def model_integrate(parent_mass, masses, nevents, resonances=(), seed=42, stream_id=0, event_offset=0,
                    want_values=False):
    """Integral of |A|^2 over phase space (parent at rest), |A|^2 the product of
    relativistic Breit-Wigner intensities 1/((M^2 - s_ij)^2 + M^2 G^2) given as
    (i, j, M, G) tuples.  Returns (mean, sigma, values or None)."""
    lib = _load()
    m = _masses(masses)
    k = len(resonances)
    pi = np.array([r[0] for r in resonances] + [0], dtype=np.int32)
    pj = np.array([r[1] for r in resonances] + [0], dtype=np.int32)
    rm = np.array([r[2] for r in resonances] + [0.0], dtype=np.float64)
    rg = np.array([r[3] for r in resonances] + [0.0], dtype=np.float64)
    vals = np.zeros(nevents, dtype=np.float64) if want_values else None
    mean = ctypes.c_double()
    sigma = ctypes.c_double()
    st = lib.oracle_model_integrate(parent_mass, _ptr(m), len(m), k, _ptr(pi), _ptr(pj), _ptr(rm), _ptr(rg),
                                    nevents, seed, stream_id, event_offset, _ptr(vals), ctypes.byref(mean),
                                    ctypes.byref(sigma))
    if st != OK:
        raise OracleError(st)
    return mean.value, sigma.value, vals


def gaussian_integral(lo, hi, mu, sigma) -> float:
    """Closed form of the product-of-Gaussians integrand over the box (erf)."""
    import math
    r = 1.0
    for a, b, m, s in zip(lo, hi, mu, sigma):
        r *= 0.5 * (math.erf((b - m) / (s * math.sqrt(2.0))) - math.erf((a - m) / (s * math.sqrt(2.0))))
    return r


def uniform_grid(dim: int, bins: int) -> np.ndarray:
    return np.tile(np.arange(bins + 1, dtype=np.float64) / bins, (dim, 1))


def vegas_iteration(lo, hi, mu, sigma, grid, calls, seed=42, iteration=0, want_hist=True, want_values=False):
    """One VEGAS iteration: (mean, sigma, histogram [dim, bins] or None), plus the
    per-sample values as a fourth item when want_values."""
    lib = _load()
    lo, hi, mu, sg = (np.ascontiguousarray(a, dtype=np.float64) for a in (lo, hi, mu, sigma))
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    dim, bins = grid.shape[0], grid.shape[1] - 1
    hist = np.zeros((dim, bins), dtype=np.float64) if want_hist else None
    vals = np.zeros(calls, dtype=np.float64) if want_values else None
    mean = ctypes.c_double()
    sig = ctypes.c_double()
    st = lib.oracle_vegas_iteration(dim, bins, _ptr(lo), _ptr(hi), _ptr(mu), _ptr(sg), _ptr(grid), calls, seed,
                                    iteration, ctypes.byref(mean), ctypes.byref(sig), _ptr(hist), _ptr(vals))
    if st != OK:
        raise OracleError(st)
    if want_values:
        return mean.value, sig.value, hist, vals
    return mean.value, sig.value, hist


def vegas_refine(grid, hist, alpha=1.5):
    """Refined copy of the grid."""
    lib = _load()
    g = np.array(grid, dtype=np.float64, copy=True)
    h = np.ascontiguousarray(hist, dtype=np.float64)
    st = lib.oracle_vegas_refine(g.shape[0], g.shape[1] - 1, _ptr(g), _ptr(h), float(alpha))
    if st != OK:
        raise OracleError(st)
    return g


def vegas(lo, hi, mu, sigma, calls, iterations, warmup=0, bins=50, alpha=1.5, seed=42):
    """VEGAS: `warmup` iterations that only adapt the grid, then `iterations`
    that also estimate; each ends with a refinement.  Returns (result, error,
    chi2/dof, per-iteration (mean, sigma) of the estimating iterations, final
    grid); the result is their inverse-variance weighted mean.  Iteration t uses
    counter word 3 = t (independent samples)."""
    grid = uniform_grid(len(lo), bins)
    its = []
    for t in range(warmup + iterations):
        m, s, h = vegas_iteration(lo, hi, mu, sigma, grid, calls, seed=seed, iteration=t)
        if t >= warmup:
            its.append((m, s))
        grid = vegas_refine(grid, h, alpha)
    w = np.array([1.0 / (s * s) for _, s in its])
    v = np.array([m for m, _ in its])
    res = float((w * v).sum() / w.sum())
    err = float(1.0 / math.sqrt(w.sum()))
    chi2 = float((w * (v - res) ** 2).sum() / max(len(its) - 1, 1))
    return res, err, chi2, its, grid
