"""Independent phase-space volumes used to pin the oracle (tests only).

Nothing here calls the oracle or the HIP library.  The measure is
prod_i d^3p_i / (2 E_i) delta^4(P - sum p_i) with no factors of 2*pi, in which the
two-body volume is R_2(M; a, b) = pi p*(M; a, b) / M.

* ``massless_volume``: closed form for N massless bodies (Kleiss, Stirling, Ellis,
  "A new Monte Carlo treatment of multiparticle phase space at high energies",
  Comput. Phys. Commun. 40 (1986) 359): R_N = (pi/2)^{N-1} M^{2N-4} / ((N-1)! (N-2)!).
* ``two_body_momentum``: the textbook Kallen-function form
  p* = sqrt((M^2 - (a+b)^2) (M^2 - (a-b)^2)) / (2M).
* ``recursive_volume``: nested Gauss-Legendre quadrature of the recursion
  R_N(M) = int d(s^2) R_2(M; s, m_{N-1}) R_{N-1}(s; m_0..m_{N-2}),
  with the substitution s = lo + (hi-lo) sin^2(t) to remove the square-root
  end-point behaviour.
* ``dalitz_area``: area of the allowed region of the three-body Dalitz plot in
  (m01^2, m12^2), from the m12^2 limits at fixed m01^2.
"""
from __future__ import annotations

import math

import numpy as np


def massless_volume(n: int, M: float) -> float:
    return (math.pi / 2.0) ** (n - 1) * M ** (2 * n - 4) / (math.factorial(n - 1) * math.factorial(n - 2))


def kallen(x, y, z):
    return x * x + y * y + z * z - 2.0 * x * y - 2.0 * x * z - 2.0 * y * z


def two_body_momentum(M, a, b):
    M = np.asarray(M, dtype=np.float64)
    lam = (M * M - (a + b) ** 2) * (M * M - (a - b) ** 2)
    return np.sqrt(np.maximum(lam, 0.0)) / (2.0 * M)


def _gauss_legendre(k: int):
    x, w = np.polynomial.legendre.leggauss(k)
    return x, w


def recursive_volume(M, masses, k: int = 48):
    """R_N(M; masses) by nested quadrature; M may be an array (vectorised)."""
    masses = [float(m) for m in masses]
    M = np.atleast_1d(np.asarray(M, dtype=np.float64))
    n = len(masses)
    if n == 2:
        return np.pi * two_body_momentum(M, masses[0], masses[1]) / M
    lo = sum(masses[:-1])
    x, w = _gauss_legendre(k)
    # t in [0, pi/2]; s = lo + (hi - lo) sin^2 t;  ds = (hi - lo) sin(2t) dt
    t = (x + 1.0) * (np.pi / 4.0)
    wt = w * (np.pi / 4.0)
    hi = M - masses[-1]
    span = (hi - lo)[:, None]
    s = lo + span * np.sin(t)[None, :] ** 2
    ds = span * np.sin(2.0 * t)[None, :] * wt[None, :]
    inner = recursive_volume(s.reshape(-1), masses[:-1], k).reshape(s.shape)
    r2 = np.pi * two_body_momentum(M[:, None], s, masses[-1]) / M[:, None]
    return np.sum(2.0 * s * r2 * inner * ds, axis=1)


def dalitz_area(M: float, m0: float, m1: float, m2: float, k: int = 200) -> float:
    """Area of the three-body Dalitz region in (m01^2, m12^2)."""
    lo, hi = (m0 + m1) ** 2, (M - m2) ** 2
    x, w = _gauss_legendre(k)
    t = (x + 1.0) * (np.pi / 4.0)
    s = lo + (hi - lo) * np.sin(t) ** 2
    ds = (hi - lo) * np.sin(2.0 * t) * w * (np.pi / 4.0)
    return float(np.sum(dalitz_m12sq_width(M, m0, m1, m2, s) * ds))


def dalitz_m12sq_limits(M, m0, m1, m2, s01):
    """(min, max) of m12^2 at fixed m01^2 = s01 (energies in the {0,1} rest frame)."""
    rs = np.sqrt(s01)
    e1 = (s01 - m0 * m0 + m1 * m1) / (2.0 * rs)
    e2 = (M * M - s01 - m2 * m2) / (2.0 * rs)
    q1 = np.sqrt(np.maximum(e1 * e1 - m1 * m1, 0.0))
    q2 = np.sqrt(np.maximum(e2 * e2 - m2 * m2, 0.0))
    return (e1 + e2) ** 2 - (q1 + q2) ** 2, (e1 + e2) ** 2 - (q1 - q2) ** 2


def dalitz_m12sq_width(M, m0, m1, m2, s01):
    lo, hi = dalitz_m12sq_limits(M, m0, m1, m2, s01)
    return hi - lo


def three_body_volume_1d(M: float, m0: float, m1: float, m2: float, k: int = 200) -> float:
    """R_3 = (2 pi^2 / M) int p*(s; m0, m1) p*(M; s, m2) ds over s in [m0+m1, M-m2]."""
    lo, hi = m0 + m1, M - m2
    x, w = _gauss_legendre(k)
    t = (x + 1.0) * (np.pi / 4.0)
    s = lo + (hi - lo) * np.sin(t) ** 2
    ds = (hi - lo) * np.sin(2.0 * t) * w * (np.pi / 4.0)
    f = two_body_momentum(s, m0, m1) * two_body_momentum(M, s, m2)
    return float(2.0 * np.pi ** 2 / M * np.sum(f * ds))


def bw_dalitz_integral_one(M, m0, m1, m2, mr, gr, k: int = 4000) -> float:
    """Integral over three-body phase space of one relativistic Breit-Wigner
    intensity 1/((mr^2 - s12)^2 + (mr gr)^2) in the (1,2) pair mass.

    The Dalitz density is uniform, pi^2/(4 M^2) per unit (s01, s12), so the
    integral is pi^2/(4M^2) int ds12 W01(s12) |BW(s12)|^2 with W01 the width of
    the s01 range at fixed s12; s12 = mr^2 + mr gr tan(theta) flattens the peak."""
    lo, hi = (m1 + m2) ** 2, (M - m0) ** 2
    g = mr * gr
    a, b = np.arctan((lo - mr * mr) / g), np.arctan((hi - mr * mr) / g)
    x, w = _gauss_legendre(k)
    th = 0.5 * (b - a) * x + 0.5 * (a + b)
    s = mr * mr + g * np.tan(th)
    s = np.clip(s, lo, hi)
    l01, h01 = dalitz_m12sq_limits(M, m2, m1, m0, s)  # range of s01 at fixed s12 (relabelled)
    f = (h01 - l01) / g  # |BW|^2 ds = dtheta / g
    return float(np.pi ** 2 / (4.0 * M * M) * 0.5 * (b - a) * np.sum(w * f))


def bw_dalitz_integral_two(M, m0, m1, m2, r01, r12, k: int = 4000) -> float:
    """Two Breit-Wigner intensities, in s01 (r01 = (mass, width)) and in s12
    (r12).  The s12 integral of the second at fixed s01 is an arctangent
    difference, leaving one dimension: s01 = m^2 + m g tan(theta)."""
    (ma, ga), (mb, gb) = r01, r12
    lo, hi = (m0 + m1) ** 2, (M - m2) ** 2
    g = ma * ga
    gb2 = mb * gb
    a, b = np.arctan((lo - ma * ma) / g), np.arctan((hi - ma * ma) / g)
    x, w = _gauss_legendre(k)
    th = 0.5 * (b - a) * x + 0.5 * (a + b)
    s = np.clip(ma * ma + g * np.tan(th), lo, hi)
    l12, h12 = dalitz_m12sq_limits(M, m0, m1, m2, s)
    inner = (np.arctan((h12 - mb * mb) / gb2) - np.arctan((l12 - mb * mb) / gb2)) / gb2
    return float(np.pi ** 2 / (4.0 * M * M) * 0.5 * (b - a) * np.sum(w * inner / g))
