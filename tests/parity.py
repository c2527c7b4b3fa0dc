"""Comparison helpers shared by the GPU parity tests.

Tolerance reading (FP64 path): every momentum component c of daughter d must
satisfy |c_gpu - c_oracle| <= tol * E_d,oracle (components near zero are measured
against the daughter's energy, the natural scale of its four-vector), weights
|w_gpu - w_oracle| <= tol * w_oracle, integrals relative to the oracle's value.
"""
from __future__ import annotations

import numpy as np

FP64_TOL = 1e-11
MIXED_TOL = 1e-5
MIXED_INTEGRAL_TOL = 1e-6


def event_errors(p4_gpu: np.ndarray, p4_ora: np.ndarray):
    """Max over events and components of |dc| / E_d (per daughter), shape [N]."""
    scale = np.abs(p4_ora[:, 0:1, :])  # E_d, broadcast over components
    err = np.abs(p4_gpu.astype(np.float64) - p4_ora) / scale
    return err.max(axis=(1, 2))


def assert_events_close(p4_gpu, w_gpu, p4_ora, w_ora, tol=FP64_TOL, wtol=FP64_TOL):
    assert p4_gpu.shape == p4_ora.shape, (p4_gpu.shape, p4_ora.shape)
    assert np.all(np.isfinite(p4_gpu))
    err = event_errors(p4_gpu, p4_ora)
    assert np.all(err <= tol), f"max |dc|/E per daughter {err} > {tol}"
    werr = np.abs(w_gpu - w_ora)
    assert np.all(werr <= wtol * np.abs(w_ora) + 1e-300), f"max weight error {np.max(werr / np.abs(w_ora))}"
    return err


def mixed_error_report(p4_gpu, p4_ora, parent_mass):
    """FP32-kinematics error summary: |dc|/E_d (max, 1-1e-6 quantile, fraction of
    components above 1e-5) and max |dc|/M."""
    d = np.abs(p4_gpu.astype(np.float64) - p4_ora)
    r = d / np.abs(p4_ora[:, 0:1, :])
    return {"max_rel_E": float(r.max()), "q999999_rel_E": float(np.quantile(r, 1 - 1e-6)),
            "frac_above_1e-5": float((r > MIXED_TOL).mean()), "max_rel_M": float(d.max() / parent_mass)}


def rel(a, b):
    return abs(a - b) / abs(b)
