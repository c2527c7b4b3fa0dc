"""Pins of the CPU oracle against facts fixed outside it (no GPU needed).

Each test checks the oracle against something it does not compute itself: an
independent Philox4x32-10 implementation (rocRAND), closed-form or quadrature
phase-space volumes, exact two-body kinematics, conservation laws and Lorentz
invariants evaluated from the outputs, and the flatness of the three-body Dalitz
plot (arXiv:1711.05683 sec. 4.2: kinematics of a particle of given four-momentum
decaying to n bodies without resonances, Raubold-Lynch weighted events).
"""
from __future__ import annotations

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import volumes as V

CFG0_M = 5.279
CFG0_MASSES = [3.097, 0.4937, 0.13957]


# ---------------------------------------------------------------- Philox ----

@pytest.fixture(scope="session")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND known-answer harness")
    src = os.path.join(os.path.dirname(__file__), "kat", "rocrand_philox_kat.cpp")
    exe = str(tmp_path_factory.mktemp("kat") / "rocrand_philox_kat")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)

    def run(seed, subsequence, offset, nblocks):
        out = subprocess.run([exe, str(seed), str(subsequence), str(offset), str(nblocks)],
                             check=True, capture_output=True, text=True).stdout
        return [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    return run


KAT_CASES = [
    # (seed, stream_id, g, j)
    (0, 0, 0, 0),
    (42, 0, 0, 0),
    (42, 0, 12345, 2),
    (42, 7, 99999, 1),
    (0x0123456789ABCDEF, 3, (1 << 32) + 17, 5),
    (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF, (1 << 61) + 3, 12),  # 4 g must fit in 64 bits
    (43, 1, 100_000_000 - 1, 0),
]


@pytest.mark.parametrize("seed,stream,g,j", KAT_CASES)
def test_philox_words_match_rocrand(oracle_lib, rocrand_kat, seed, stream, g, j):
    # rocRAND's state maps (seed, subsequence, offset) to key (seed lo, seed hi) and
    # counter (offset/4 as 64 bits, subsequence as 64 bits); the oracle's counter is
    # (g lo, g hi, j, stream), i.e. subsequence = stream<<32 | j, offset = 4 g.
    blocks = rocrand_kat(seed, (stream << 32) | j, 4 * g, 3)
    for b in range(3):
        gg = g + b
        want = oracle_lib.philox4x32_10([gg & 0xFFFFFFFF, gg >> 32, j, stream],
                                        [seed & 0xFFFFFFFF, seed >> 32])
        assert blocks[b] == want, (seed, stream, gg, j)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 10])
def test_event_uniforms_from_rocrand_words(oracle_lib, rocrand_kat, n):
    seed, stream, g = 42, 5, 777
    nu = 3 * n - 4
    assert oracle_lib.uniforms_per_event(n) == nu
    ncalls = (2 * nu + 3) // 4
    words = []
    for j in range(ncalls):
        words += rocrand_kat(seed, (stream << 32) | j, 4 * g, 1)[0]
    u = oracle_lib.event_uniforms(seed, stream, g, n)
    for k in range(nu):
        bits = (words[2 * k + 1] << 32) | words[2 * k]
        x = bits >> 12
        assert u[k] == (2 * x + 1) / 2.0 ** 53
        assert 0.0 < u[k] < 1.0


def test_uniform_grid_is_exact_and_open(oracle_lib):
    for g in range(200):
        u = oracle_lib.event_uniforms(42, 0, g, 10)
        scaled = u * 2.0 ** 53
        assert np.all(scaled == np.floor(scaled))
        assert np.all(np.mod(scaled, 2.0) == 1.0)
        assert np.all(u >= 2.0 ** -53) and np.all(u <= 1.0 - 2.0 ** -53)


# ------------------------------------------------------ volumes (integral) ----

def _assert_within(mean, sigma, exact, nsig=4.0):
    assert sigma > 0.0
    assert abs(mean - exact) < nsig * sigma, (mean, sigma, exact, (mean - exact) / sigma)


@pytest.mark.parametrize("n,M,nev", [(3, 1.0, 100_000), (4, 3.0, 100_000), (5, 7.0, 60_000),
                                     (6, 10.0, 60_000), (10, 10.0, 40_000)])
def test_massless_volume_closed_form(oracle_lib, n, M, nev):
    mean, sigma = oracle_lib.integrate(M, [0.0] * n, nev, seed=42)
    _assert_within(mean, sigma, V.massless_volume(n, M))
    # The estimate must also be sharp enough to reject a factor-of-2 normalisation error.
    assert sigma < 0.1 * V.massless_volume(n, M)


def test_massless_three_body_weight_per_event(oracle_lib):
    # Massless N=3 at mass M: sigma_1 = M R, p_0 = M R / 2, p_1 = M (1 - R^2)/2, so
    # w = (pi^2 / 2) M^2 R (1 - R^2) with R the event's single mass uniform.
    M = 2.5
    _, w = oracle_lib.generate(M, [0.0, 0.0, 0.0], 2000, seed=42, want_momenta=False)
    for e in range(2000):
        r = oracle_lib.event_uniforms(42, 0, e, 3)[0]
        want = 0.5 * math.pi ** 2 * M * M * r * ((1.0 - r) * (1.0 + r))
        assert abs(w[e] - want) <= 4e-15 * want
    # per-event spread: sigma_w = pi^2 M^2 sqrt(23/6720)
    _, w = oracle_lib.generate(1.0, [0.0] * 3, 200_000, seed=7, want_momenta=False)
    sd = float(np.std(w, ddof=1))
    assert abs(sd - math.pi ** 2 * math.sqrt(23.0 / 6720.0)) < 0.01 * sd


def test_two_body_is_exact(oracle_lib):
    M, a, b = CFG0_M, 3.097, 0.4937
    pstar = float(V.two_body_momentum(M, a, b))
    p4, w = oracle_lib.generate(M, [a, b], 5000, seed=42)
    want_w = math.pi * pstar / M
    assert np.all(np.abs(w - want_w) <= 2e-15 * want_w)
    for d, m in ((0, a), (1, b)):
        pmag = np.sqrt(p4[d, 1] ** 2 + p4[d, 2] ** 2 + p4[d, 3] ** 2)
        assert np.all(np.abs(pmag - pstar) <= 1e-14 * M)
        assert np.all(np.abs(p4[d, 0] - math.sqrt(pstar ** 2 + m * m)) <= 1e-14 * M)
    mean, sigma = oracle_lib.integrate(M, [a, b], 5000, seed=42)
    assert abs(mean - want_w) <= 2e-15 * want_w
    assert sigma <= 1e-15 * want_w


def test_massive_three_body_volume_config0(oracle_lib):
    exact = V.three_body_volume_1d(CFG0_M, *CFG0_MASSES)
    # two routes to the same number: 1-D recursion integral and the Dalitz area
    area = V.dalitz_area(CFG0_M, *CFG0_MASSES)
    assert abs(exact - math.pi ** 2 / (4 * CFG0_M ** 2) * area) < 1e-12 * exact
    assert abs(exact - float(V.recursive_volume(CFG0_M, CFG0_MASSES)[0])) < 1e-12 * exact
    mean, sigma = oracle_lib.integrate(CFG0_M, CFG0_MASSES, 200_000, seed=42)
    _assert_within(mean, sigma, exact)
    assert sigma < 2e-3 * exact


def test_six_pion_volume(oracle_lib):
    masses = [0.13957] * 6
    exact = float(V.recursive_volume(10.0, masses, k=40)[0])
    # the same quadrature reproduces the massless closed form
    ml = float(V.recursive_volume(10.0, [0.0] * 6, k=40)[0])
    assert abs(ml - V.massless_volume(6, 10.0)) < 1e-12 * ml
    mean, sigma = oracle_lib.integrate(10.0, masses, 60_000, seed=42)
    _assert_within(mean, sigma, exact)


@pytest.mark.parametrize("masses,M", [([0.5, 1.0, 0.2, 0.3], 4.0), ([0.1, 0.2, 0.3, 0.4, 0.5], 3.0)])
def test_massive_volume_quadrature(oracle_lib, masses, M):
    exact = float(V.recursive_volume(M, masses, k=40)[0])
    mean, sigma = oracle_lib.integrate(M, masses, 80_000, seed=11)
    _assert_within(mean, sigma, exact)


def test_integral_is_mean_and_standard_error(oracle_lib):
    _, w = oracle_lib.generate(CFG0_M, CFG0_MASSES, 3000, seed=42, event_offset=500,
                               want_momenta=False)
    mean, sigma = oracle_lib.integrate(CFG0_M, CFG0_MASSES, 3000, seed=42, event_offset=500)
    exact_mean = math.fsum(w) / len(w)
    var = math.fsum((x - exact_mean) ** 2 for x in w) / (len(w) - 1)
    assert abs(mean - exact_mean) <= 1e-15 * exact_mean
    assert abs(sigma - math.sqrt(var / len(w))) <= 1e-14 * sigma


# ---------------------------------------------------- per-event kinematics ----

def _minkowski_sq(v):
    return v[0] ** 2 - v[1] ** 2 - v[2] ** 2 - v[3] ** 2


def _check_event_physics(oracle_lib, M, masses, parent, p4, w, seed, stream, offset):
    n = len(masses)
    nev = p4.shape[2]
    total = p4.sum(axis=0)
    P = np.array([M, 0.0, 0.0, 0.0]) if parent is None else parent
    P = P.reshape(4, -1) if P.ndim == 2 else P[:, None]
    scale = max(M, float(np.max(np.abs(P))))
    assert np.all(np.abs(total - P) <= 1e-12 * scale)
    for d in range(n):
        E = p4[d, 0]
        m2 = _minkowski_sq(p4[d])
        assert np.all(np.abs(m2 - masses[d] ** 2) <= 1e-12 * E * E + 1e-300)
        assert np.all(E >= masses[d] * (1 - 1e-15))
    s = np.cumsum(masses)
    T = M - s[-1]
    for e in range(nev):
        u = oracle_lib.event_uniforms(seed, stream, offset + e, n)
        R = np.concatenate([[0.0], np.sort(u[: n - 2]), [1.0]])
        sig = [masses[0]] + [s[i] + T * R[i] for i in range(1, n - 1)] + [M]
        acc = p4[0, :, e].copy()
        for i in range(1, n):
            k = p4[i, :, e]
            acc_prev = acc.copy()
            acc = acc + k
            # invariant mass of {0..i} equals sigma_i
            mi = math.sqrt(max(_minkowski_sq(acc), 0.0))
            assert abs(mi - sig[i]) <= 1e-11 * M, (e, i, mi, sig[i])
            # breakup momentum of daughter i in the rest frame of {0..i}
            Pk = acc[0] * k[0] - acc[1] * k[1] - acc[2] * k[2] - acc[3] * k[3]
            estar = Pk / mi
            pstar = math.sqrt(max(estar * estar - masses[i] ** 2, 0.0))
            want = float(V.two_body_momentum(sig[i], sig[i - 1], masses[i]))
            assert abs(pstar - want) <= 1e-9 * M, (e, i, pstar, want)
            del acc_prev
        assert w[e] >= 0.0 and np.isfinite(w[e])


def test_event_physics_config0_at_rest(oracle_lib):
    p4, w = oracle_lib.generate(CFG0_M, CFG0_MASSES, 400, seed=42)
    _check_event_physics(oracle_lib, CFG0_M, CFG0_MASSES, None, p4, w, 42, 0, 0)


@pytest.mark.parametrize("n", [2, 4, 7, 10])
def test_event_physics_various_n(oracle_lib, n):
    rng = np.random.default_rng(100 + n)
    M = 5.0
    masses = list(rng.uniform(0.0, 0.4 * M / n, size=n))
    p4, w = oracle_lib.generate(M, masses, 150, seed=9, stream_id=3, event_offset=1000)
    _check_event_physics(oracle_lib, M, masses, None, p4, w, 9, 3, 1000)


def test_event_physics_moving_parent(oracle_lib):
    M = CFG0_M
    parent = np.array([math.sqrt(M * M + 1.0 + 4.0 + 9.0), 1.0, -2.0, 3.0])
    p4, w = oracle_lib.generate(M, CFG0_MASSES, 300, seed=42, parent_p4=parent)
    _check_event_physics(oracle_lib, M, CFG0_MASSES, parent, p4, w, 42, 0, 0)
    # Lorentz invariance: identical weights and pair masses as at rest
    p4r, wr = oracle_lib.generate(M, CFG0_MASSES, 300, seed=42)
    assert np.array_equal(w, wr)
    for a, b in ((0, 1), (1, 2), (0, 2)):
        m_mov = np.sqrt(_minkowski_sq(p4[a] + p4[b]))
        m_rest = np.sqrt(_minkowski_sq(p4r[a] + p4r[b]))
        assert np.all(np.abs(m_mov - m_rest) <= 1e-12 * M)


def test_event_physics_per_event_parents(oracle_lib):
    M = CFG0_M
    nev = 200
    rng = np.random.default_rng(5)
    pz = rng.uniform(0.0, 20.0, nev)
    soa = np.stack([np.sqrt(M * M + pz * pz), np.zeros(nev), np.zeros(nev), pz])
    p4, w = oracle_lib.generate(M, CFG0_MASSES, nev, seed=42, parent_soa=soa)
    _check_event_physics(oracle_lib, M, CFG0_MASSES, soa, p4, w, 42, 0, 0)


def test_sequential_decay_chain(oracle_lib):
    """Sequential decays: daughter 0 of a first generation is the per-event parent
    of a second (another stream, so the uniforms are independent).  The chain
    conserves four-momentum, the second stage's weights do not depend on the
    parent's motion, and the mean of the product of the two weights is the product
    of the two volumes (the intermediate has a fixed mass)."""
    M, m = CFG0_M, CFG0_MASSES
    n = 100_000
    p4, w1 = oracle_lib.generate(M, m, n, seed=42, stream_id=0)
    mid = m[0]
    soa = np.ascontiguousarray(p4[0])  # [4][n]: the J/psi-like daughter of each event
    q4, w2 = oracle_lib.generate(mid, [0.0, 0.0, 0.0], n, seed=42, stream_id=1, parent_soa=soa)
    assert np.all(np.abs(q4.sum(axis=0) - soa) <= 1e-12 * np.abs(soa).max())
    _check_event_physics(oracle_lib, mid, [0.0, 0.0, 0.0], soa[:, :300], q4[:, :, :300], w2[:300], 42, 1, 0)
    _, w2_rest = oracle_lib.generate(mid, [0.0, 0.0, 0.0], n, seed=42, stream_id=1, want_momenta=False)
    assert np.array_equal(w2, w2_rest)
    ww = w1 * w2
    want = V.three_body_volume_1d(M, *m) * V.massless_volume(3, mid)
    _assert_within(float(ww.mean()), float(ww.std(ddof=1)) / math.sqrt(n), want)


def _direction(u, v):
    ct = 2.0 * u - 1.0
    st = math.sqrt(max(0.0, 1.0 - ct * ct))
    return np.array([st * math.cos(2 * math.pi * v), st * math.sin(2 * math.pi * v), ct])


@pytest.mark.parametrize("n", [2, 3, 5, 10])
def test_last_daughter_direction(oracle_lib, n):
    # The last daughter is emitted in the parent rest frame and never boosted
    # again: its direction is the last (theta, phi) pair of uniforms.
    masses = [0.1 * (i + 1) for i in range(n)]
    M = sum(masses) + 2.0
    p4, _ = oracle_lib.generate(M, masses, 200, seed=3)
    for e in range(200):
        u = oracle_lib.event_uniforms(3, 0, e, n)
        want = _direction(u[3 * n - 6], u[3 * n - 5])
        p = p4[n - 1, 1:, e]
        assert np.allclose(p / np.linalg.norm(p), want, rtol=0, atol=1e-12)


def test_level0_direction_three_body(oracle_lib):
    # Undo the single pure boost of {0,1} and recover the level-0 direction.
    p4, _ = oracle_lib.generate(CFG0_M, CFG0_MASSES, 200, seed=42)
    for e in range(200):
        u = oracle_lib.event_uniforms(42, 0, e, 3)
        P = p4[0, :, e] + p4[1, :, e]
        sig = math.sqrt(_minkowski_sq(P))
        eta = -P[1:] / sig
        gam = P[0] / sig
        k = p4[1, :, e]
        ep = float(eta @ k[1:])
        kp = k[1:] + (ep / (gam + 1.0) + k[0]) * eta
        want = _direction(u[1], u[2])
        assert np.allclose(kp / np.linalg.norm(kp), want, rtol=0, atol=1e-10)


@pytest.mark.parametrize("n,moving", [(4, False), (6, False), (10, False), (6, True)])
def test_every_level_direction(oracle_lib, n, moving):
    # Top-down levels: daughter i+1, taken into the rest frame of {0..i+1} by the
    # pure boost of that subsystem's four-momentum (summed from the outputs, in
    # the parent's rest frame), points along the direction of level i's
    # (theta, phi) uniforms.  (Boosting the inner daughters level by level
    # instead would rotate these frames, and the directions of all but the top
    # level would differ.)
    masses = [0.05 * (i + 1) for i in range(n)]
    M = sum(masses) + 3.0
    parent = np.array([math.sqrt(M * M + 1.0 + 0.25 + 4.0), 1.0, 0.5, -2.0]) if moving else None
    p4, _ = oracle_lib.generate(M, masses, 60, seed=11, stream_id=2, parent_p4=parent)
    if moving:  # back into the parent's rest frame first
        eta, gam = -parent[1:] / M, parent[0] / M
        for d in range(n):
            ep = np.einsum("k,ke->e", eta, p4[d, 1:])
            f = ep / (gam + 1.0) + p4[d, 0]
            p4[d, 0] = gam * p4[d, 0] + ep
            p4[d, 1:] = p4[d, 1:] + f[None, :] * eta[:, None]
    for e in range(60):
        u = oracle_lib.event_uniforms(11, 2, e, n)
        for i in range(n - 1):
            P = p4[: i + 2, :, e].sum(axis=0)
            sig = math.sqrt(_minkowski_sq(P))
            eta, gam = -P[1:] / sig, P[0] / sig
            k = p4[i + 1, :, e]
            ep = float(eta @ k[1:])
            kp = k[1:] + (ep / (gam + 1.0) + k[0]) * eta
            want = _direction(u[n - 2 + 2 * i], u[n - 1 + 2 * i])
            assert np.allclose(kp / np.linalg.norm(kp), want, rtol=0, atol=1e-9), (e, i)


# --------------------------------------------------- distributions ----

def test_dalitz_plot_is_flat(oracle_lib):
    M, m = CFG0_M, CFG0_MASSES
    nev = 400_000
    p4, w = oracle_lib.generate(M, m, nev, seed=42)
    s01 = _minkowski_sq(p4[0] + p4[1])
    s12 = _minkowski_sq(p4[1] + p4[2])
    lo01, hi01 = (m[0] + m[1]) ** 2, (M - m[2]) ** 2
    edges01 = np.linspace(lo01, hi01, 13)
    lo12, hi12 = (m[1] + m[2]) ** 2, (M - m[0]) ** 2
    edges12 = np.linspace(lo12, hi12, 13)
    H, _, _ = np.histogram2d(s01, s12, bins=[edges01, edges12], weights=w)
    H2, _, _ = np.histogram2d(s01, s12, bins=[edges01, edges12], weights=w * w)
    density = math.pi ** 2 / (4.0 * M * M)
    chi2, ndf = 0.0, 0
    for i in range(12):
        for j in range(12):
            # bin fully inside the kinematic boundary: check its four corners
            inside = True
            for s in (edges01[i], edges01[i + 1]):
                a, b = V.dalitz_m12sq_limits(M, *m, s)
                if not (a <= edges12[j] and edges12[j + 1] <= b):
                    inside = False
            if not inside:
                continue
            area = (edges01[i + 1] - edges01[i]) * (edges12[j + 1] - edges12[j])
            want = density * area
            var = H2[i, j] / nev ** 2 - (H[i, j] / nev) ** 2 / nev
            chi2 += (H[i, j] / nev - want) ** 2 / var
            ndf += 1
    assert ndf >= 20
    # chi^2 with ndf degrees of freedom: mean ndf, sd sqrt(2 ndf)
    assert chi2 < ndf + 5.0 * math.sqrt(2.0 * ndf), (chi2, ndf)


def test_isotropy(oracle_lib):
    masses = [0.2, 0.3, 0.1, 0.4]
    p4, w = oracle_lib.generate(3.0, masses, 100_000, seed=21)
    W = w.sum()
    for d in range(4):
        p = p4[d, 1:]
        nhat = p / np.linalg.norm(p, axis=0)
        for k in range(3):
            mu = float((w * nhat[k]).sum() / W)
            sd = math.sqrt(float((w * w * nhat[k] ** 2).sum())) / W
            assert abs(mu) < 5 * sd
        c2 = float((w * nhat[2] ** 2).sum() / W)
        assert abs(c2 - 1.0 / 3.0) < 0.01


# --------------------------------------------------- unweighted samples ----
# Hit-or-miss unweighting keeps trial e when v_e * w_max < w_e.  The kept events
# must be distributed as phase space itself (unit weight): the pins below check
# the accepted fraction against E[w]/w_max, the kept-event densities against
# closed forms, and that the kept events are the weighted events of the same
# index.

def test_accept_uniform_uses_the_first_unused_call(oracle_lib):
    for n in range(2, 11):
        words = 2 * (3 * n - 4)  # words the event's own uniforms consume
        j = oracle_lib.calls_per_event(n)
        assert 4 * (j - 1) < words <= 4 * j
        # words 0 and 1 of call j, converted like every other uniform
        w = oracle_lib.philox4x32_10([77, 5, j, 3], [11, 0])
        x = ((w[1] << 32) | w[0]) >> 12
        assert oracle_lib.accept_uniform(11, 3, (5 << 32) | 77, n) == (2 * x + 1) * 2.0 ** -53


def test_unweight_two_body_keeps_every_trial(oracle_lib):
    M, m = 5.279, [3.097, 0.4937]
    p4, idx, kept, over, used = oracle_lib.unweight(M, m, 3000, seed=9, event_offset=100)
    assert kept == 3000 and over == 0 and np.array_equal(idx, np.arange(100, 3100, dtype=np.uint64))
    q4, w = oracle_lib.generate(M, m, 3000, seed=9, event_offset=100)
    assert used == w[0] and np.array_equal(p4, q4)


def test_unweight_massless_three_body_acceptance(oracle_lib):
    # w = (pi^2/2) M^2 R (1 - R^2) with R uniform: w_max = pi^2 M^2 / (3 sqrt 3), and
    # the kept fraction is E[w] / w_max = (pi^2 M^2 / 8) / w_max = 3 sqrt(3) / 8.
    M, n = 1.0, 200_000
    wmax = math.pi ** 2 * M * M / (3.0 * math.sqrt(3.0)) * (1.0 + 1e-12)
    p4, idx, kept, over, used = oracle_lib.unweight(M, [0.0, 0.0, 0.0], n, seed=5, w_max=wmax)
    assert over == 0 and used == wmax
    p = 3.0 * math.sqrt(3.0) / 8.0
    assert abs(kept / n - p) < 5.0 * math.sqrt(p * (1.0 - p) / n), (kept / n, p)
    # kept R = m01 / M has density 4 R (1 - R^2): CDF 2R^2 - R^4
    r = np.sqrt(np.maximum(_minkowski_sq(p4[0] + p4[1]), 0.0)) / M
    edges = np.linspace(0.0, 1.0, 21)
    cnt, _ = np.histogram(r, bins=edges)
    cdf = 2.0 * edges ** 2 - edges ** 4
    want = kept * np.diff(cdf)
    chi2 = float(((cnt - want) ** 2 / want).sum())
    assert chi2 < 19 + 5.0 * math.sqrt(2.0 * 19), chi2


def test_unweighted_dalitz_plot_is_flat(oracle_lib):
    M, m = CFG0_M, CFG0_MASSES
    p4, idx, kept, over, used = oracle_lib.unweight(M, m, 300_000, seed=42)
    s01 = _minkowski_sq(p4[0] + p4[1])
    s12 = _minkowski_sq(p4[1] + p4[2])
    lo01, hi01 = (m[0] + m[1]) ** 2, (M - m[2]) ** 2
    lo12, hi12 = (m[1] + m[2]) ** 2, (M - m[0]) ** 2
    edges01, edges12 = np.linspace(lo01, hi01, 11), np.linspace(lo12, hi12, 11)
    H, _, _ = np.histogram2d(s01, s12, bins=[edges01, edges12])
    area_total = V.dalitz_area(M, *m)
    chi2, ndf = 0.0, 0
    for i in range(10):
        for j in range(10):
            inside = True
            for sv in (edges01[i], edges01[i + 1]):
                a, b = V.dalitz_m12sq_limits(M, *m, sv)
                if not (a <= edges12[j] and edges12[j + 1] <= b):
                    inside = False
            if not inside:
                continue
            want = kept * (edges01[i + 1] - edges01[i]) * (edges12[j + 1] - edges12[j]) / area_total
            chi2 += (H[i, j] - want) ** 2 / want
            ndf += 1
    assert ndf >= 15
    assert chi2 < ndf + 5.0 * math.sqrt(2.0 * ndf), (chi2, ndf)


def test_unweighted_isotropy(oracle_lib):
    masses = [0.2, 0.3, 0.1, 0.4]
    p4, idx, kept, over, used = oracle_lib.unweight(3.0, masses, 200_000, seed=21)
    assert kept > 20_000
    for d in range(4):
        p = p4[d, 1:]
        nhat = p / np.linalg.norm(p, axis=0)
        for k in range(3):
            assert abs(float(nhat[k].mean())) < 5.0 / math.sqrt(3.0 * kept)
        assert abs(float((nhat[2] ** 2).mean()) - 1.0 / 3.0) < 5.0 * math.sqrt(4.0 / 45.0 / kept)


def test_kept_events_are_the_weighted_events(oracle_lib):
    M, m, off, n = 4.0, [0.5, 1.0, 0.2, 0.3], 7, 20_000
    q4, w = oracle_lib.generate(M, m, n, seed=3, stream_id=2, event_offset=off)
    p4, idx, kept, over, used = oracle_lib.unweight(M, m, n, seed=3, stream_id=2, event_offset=off)
    assert used == float(w.max()) and over == 0
    v = np.array([oracle_lib.accept_uniform(3, 2, off + e, len(m)) for e in range(n)])
    want = np.nonzero(v * used < w)[0]
    assert kept == len(want) and np.array_equal(idx, (want + off).astype(np.uint64))
    assert np.array_equal(p4, q4[:, :, want])
    # a smaller w_max: the trials above it are counted and always kept
    wm = float(np.median(w))
    _, idx2, kept2, over2, _ = oracle_lib.unweight(M, m, n, seed=3, stream_id=2, event_offset=off, w_max=wm)
    assert over2 == int((w > wm).sum())
    assert np.array_equal(idx2, (np.nonzero(v * wm < w)[0] + off).astype(np.uint64))
    # capacity smaller than the kept count: the first kept events, full count
    p4c, idxc, keptc, _, _ = oracle_lib.unweight(M, m, n, seed=3, stream_id=2, event_offset=off, capacity=100)
    assert keptc == kept and np.array_equal(idxc, idx[:100]) and np.array_equal(p4c, p4[:, :, :100])


# --------------------------------------------------- model evaluation ----
# The integral of a product of relativistic Breit-Wigner intensities in pair
# masses over three-body phase space, against one-dimensional quadratures of the
# uniform Dalitz density (the second intensity integrated in closed form).

KSTAR = (0.8955, 0.0473)   # a K pi resonance in the (1, 2) pair of config 0
PSI2S = (3.686, 0.3)       # a broad resonance in the (0, 1) pair of config 0


def test_model_constant_is_the_plain_integral(oracle_lib):
    a = oracle_lib.model_integrate(CFG0_M, CFG0_MASSES, 50_000, seed=3)
    b = oracle_lib.integrate(CFG0_M, CFG0_MASSES, 50_000, seed=3)
    assert a[:2] == b


def test_model_one_breit_wigner(oracle_lib):
    M, m = CFG0_M, CFG0_MASSES
    mean, sigma, _ = oracle_lib.model_integrate(M, m, 400_000, resonances=[(1, 2, *KSTAR)], seed=11)
    want = V.bw_dalitz_integral_one(M, *m, *KSTAR)
    _assert_within(mean, sigma, want)
    # a quadrature-independent cross-check of the quadrature: narrow-width limit
    # pi/(mr gr) W01(mr^2) pi^2/(4M^2), to a few percent for this width
    l01, h01 = V.dalitz_m12sq_limits(M, m[2], m[1], m[0], KSTAR[0] ** 2)
    narrow = math.pi / (KSTAR[0] * KSTAR[1]) * (h01 - l01) * math.pi ** 2 / (4 * M * M)
    assert abs(want / narrow - 1.0) < 0.05


def test_model_two_breit_wigners(oracle_lib):
    M, m = CFG0_M, CFG0_MASSES
    res = [(0, 1, *PSI2S), (1, 2, *KSTAR)]
    mean, sigma, _ = oracle_lib.model_integrate(M, m, 400_000, resonances=res, seed=12)
    want = V.bw_dalitz_integral_two(M, *m, PSI2S, KSTAR)
    _assert_within(mean, sigma, want)


def test_model_values_are_weight_times_intensity(oracle_lib):
    M, m = 4.0, [0.5, 1.0, 0.2, 0.3]
    res = [(0, 3, 1.2, 0.1), (1, 2, 1.5, 0.2)]
    _, _, v = oracle_lib.model_integrate(M, m, 2000, resonances=res, seed=5, want_values=True)
    p4, w = oracle_lib.generate(M, m, 2000, seed=5)
    a2 = np.ones(2000)
    for i, j, mr, gr in res:
        s = _minkowski_sq(p4[i] + p4[j])
        a2 = a2 / ((mr * mr - s) ** 2 + (mr * gr) ** 2)
    assert np.allclose(v, w * a2, rtol=1e-12, atol=0.0)


def test_model_validation(oracle_lib):
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.model_integrate(CFG0_M, CFG0_MASSES, 100, resonances=[(1, 1, 1.0, 0.1)])
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.model_integrate(CFG0_M, CFG0_MASSES, 100, resonances=[(0, 3, 1.0, 0.1)])
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.model_integrate(CFG0_M, CFG0_MASSES, 100, resonances=[(0, 1, 1.0, 0.0)])
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.model_integrate(CFG0_M, CFG0_MASSES, 100, resonances=[(0, 1, 1.0, 0.1)] * 5)


# ----------------------------------------- unweighted samples of a model ----
# Hit-or-miss against w |A|^2: the kept events follow the model's density over
# phase space, for config 0 with one Breit-Wigner in the (1, 2) pair mass the
# density in s12 is W01(s12) |BW(s12)|^2 (the Dalitz density is uniform).

def _bw_bin_integrals(M, m, mr, gr, edges, k=400):
    """int over each [edges[b], edges[b+1]] of W01(s12) |BW(s12)|^2 ds12, with the
    same arctangent substitution as volumes.bw_dalitz_integral_one, per bin."""
    g = mr * gr
    x, w = np.polynomial.legendre.leggauss(k)
    out = []
    for a_s, b_s in zip(edges[:-1], edges[1:]):
        a, b = np.arctan((a_s - mr * mr) / g), np.arctan((b_s - mr * mr) / g)
        th = 0.5 * (b - a) * x + 0.5 * (a + b)
        s12 = mr * mr + g * np.tan(th)
        l01, h01 = V.dalitz_m12sq_limits(M, m[2], m[1], m[0], s12)
        out.append(0.5 * (b - a) * np.sum(w * (h01 - l01) / g))
    return np.array(out)


def test_unweight_model_without_factor_is_unweight(oracle_lib):
    a = oracle_lib.unweight(CFG0_M, CFG0_MASSES, 30_000, seed=8, event_offset=5)
    b = oracle_lib.unweight_model(CFG0_M, CFG0_MASSES, 30_000, [], seed=8, event_offset=5)
    assert a[2:] == b[2:] and np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])


def test_unweight_model_acceptance(oracle_lib):
    """Under a bound B above every value, a trial is kept with probability
    w |A|^2 / B: the kept fraction is the model's integral (1-D quadrature) over B."""
    M, m = CFG0_M, CFG0_MASSES
    n, bound = 400_000, 4000.0
    _, _, kept, over, used = oracle_lib.unweight_model(M, m, n, [(1, 2, *KSTAR)], seed=12, w_max=bound,
                                                       want_momenta=False)
    assert over == 0 and used == bound
    p = V.bw_dalitz_integral_one(M, *m, *KSTAR) / bound
    assert abs(kept / n - p) < 5.0 * math.sqrt(p * (1.0 - p) / n), (kept / n, p)


def test_unweight_model_pair_mass_distribution(oracle_lib):
    """The kept events' s12 follows W01(s12) |BW(s12)|^2 (chi^2 over bins that
    span the peak and both tails)."""
    M, m = CFG0_M, CFG0_MASSES
    p4, idx, kept, over, used = oracle_lib.unweight_model(M, m, 600_000, [(1, 2, *KSTAR)], seed=13)
    assert over == 0 and kept > 5000
    s12 = _minkowski_sq(p4[1] + p4[2])
    lo, hi = (m[1] + m[2]) ** 2, (M - m[0]) ** 2
    mr, gr = KSTAR
    inner = np.linspace(mr * mr - 4 * mr * gr, mr * mr + 4 * mr * gr, 17)
    edges = np.concatenate([[lo], inner, [hi]])
    cnt, _ = np.histogram(s12, bins=edges)
    per_bin = _bw_bin_integrals(M, m, mr, gr, edges)
    # the bins cover the whole s12 range: with the Dalitz density pi^2/(4 M^2)
    # they add up to the model's integral
    assert abs(per_bin.sum() * math.pi ** 2 / (4 * M * M) / V.bw_dalitz_integral_one(M, *m, mr, gr) - 1) < 1e-8
    want = kept * per_bin / per_bin.sum()
    chi2 = float(((cnt - want) ** 2 / want).sum())
    ndf = len(cnt) - 1
    assert chi2 < ndf + 5.0 * math.sqrt(2.0 * ndf), (chi2, cnt, want)


def test_unweight_model_validation(oracle_lib):
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.unweight_model(CFG0_M, CFG0_MASSES, 100, [(1, 1, 1.0, 0.1)])
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.unweight_model(CFG0_M, CFG0_MASSES, 100, [(0, 1, 1.0, 0.1)], w_max=-1.0)


# --------------------------------------------------- VEGAS / plain MC ----
# Integrand: a product of Gaussians over a box, whose integral is a product of
# error-function differences.

def test_plain_mc_gaussian_closed_form(oracle_lib):
    lo, hi, mu, sg = [0.0, -1.0, 0.5], [1.0, 2.0, 1.5], [0.4, 0.3, 1.0], [0.5, 0.8, 0.6]
    m, s, _ = oracle_lib.vegas_iteration(lo, hi, mu, sg, oracle_lib.uniform_grid(3, 50), 200_000, seed=7)
    _assert_within(m, s, oracle_lib.gaussian_integral(lo, hi, mu, sg))


def test_vegas_ten_dimensional_gaussian(oracle_lib):
    # the integrand of the paper's VEGAS benchmark: a 10-dimensional Gaussian
    D = 10
    lo, hi, mu, sg = [0.0] * D, [1.0] * D, [0.5] * D, [0.1] * D
    exact = oracle_lib.gaussian_integral(lo, hi, mu, sg)
    res, err, chi2, its, grid = oracle_lib.vegas(lo, hi, mu, sg, 50_000, 5, warmup=5, seed=11)
    _assert_within(res, err, exact)
    assert chi2 < 5.0
    # adaptation: the same calls on the uniform grid give a far larger error
    _, s_plain, _ = oracle_lib.vegas_iteration(lo, hi, mu, sg, oracle_lib.uniform_grid(D, 50), 50_000, seed=11)
    assert its[-1][1] < 0.05 * s_plain


def test_vegas_refinement_invariants(oracle_lib):
    rng = np.random.default_rng(3)
    g = oracle_lib.uniform_grid(4, 50)
    h = rng.exponential(size=(4, 50))
    g2 = oracle_lib.vegas_refine(g, h)
    assert np.all(g2[:, 0] == 0.0) and np.all(g2[:, -1] == 1.0) and np.all(np.diff(g2, axis=1) > 0.0)
    # a flat histogram keeps the grid
    g3 = oracle_lib.vegas_refine(g, np.ones((4, 50)))
    assert np.allclose(g3, g, rtol=0.0, atol=1e-12)
    # a histogram peaked in the middle draws bins towards it
    k = np.arange(50)
    peak = np.exp(-0.5 * ((k - 24.5) / 5.0) ** 2)[None, :]
    g4 = oracle_lib.vegas_refine(oracle_lib.uniform_grid(1, 50), peak)[0]
    w = np.diff(g4)
    assert w[24] < 0.5 * w[0] and w[25] < 0.5 * w[-1]


def test_vegas_refinement_single_spike_by_hand(oracle_lib):
    """Worked examples of one refinement step (Lepage's smoothing, damping and
    equal-importance re-cut), derived by hand from a single-spike histogram on a
    uniform grid; they fail if the neighbour smoothing is dropped or its end-bin
    divisor changed."""
    # K = 6, all of value^2 in bin 2, alpha = 0 (every bin with smoothed content
    # gets importance 1): smoothing spreads the spike to bins 1, 2, 3, i.e.
    # [1/6, 2/3], which the six new bins share equally (1/12 each), the first new
    # bin also taking the empty bin 0
    g = oracle_lib.uniform_grid(1, 6)
    h = np.array([[0.0, 0.0, 1.0, 0.0, 0.0, 0.0]])
    want = np.array([0.0, 1 / 4, 1 / 3, 5 / 12, 1 / 2, 7 / 12, 1.0])
    assert np.allclose(oracle_lib.vegas_refine(g, h, alpha=0.0)[0], want, rtol=0.0, atol=1e-15)
    # K = 3, spike in bin 0, alpha = 1: smoothed (1/2, 1/3, 0), total 5/6, so
    # R = 5/3 and 5/2 and importances r0 = (2/5)/ln(5/3), r1 = (3/5)/ln(5/2);
    # each new bin holds (r0 + r1)/3: edge 1 lies in old bin 0 at that share of
    # r0, edge 2 in old bin 1 at (2(r0 + r1)/3 - r0)/r1
    r0, r1 = 0.4 / math.log(5 / 3), 0.6 / math.log(2.5)
    per = (r0 + r1) / 3
    want = np.array([0.0, per / r0 / 3, 1 / 3 + (2 * per - r0) / r1 / 3, 1.0])
    got = oracle_lib.vegas_refine(oracle_lib.uniform_grid(1, 3), np.array([[1.0, 0.0, 0.0]]), alpha=1.0)[0]
    assert np.allclose(got, want, rtol=0.0, atol=1e-14), (got, want)


def test_vegas_grid_converges_to_the_integrand(oracle_lib):
    # one dimension: the adapted density is close to |f| normalised, so the
    # grid's edges sit near the quantiles of the (truncated) Gaussian
    lo, hi, mu, sg = [0.0], [1.0], [0.3], [0.08]
    *_, grid = oracle_lib.vegas(lo, hi, mu, sg, 20_000, 10, seed=5)
    g = grid[0]
    for q, z in ((0.25, -0.6745), (0.5, 0.0), (0.75, 0.6745)):
        assert abs(g[int(50 * q)] - (mu[0] + z * sg[0])) < 0.02, (q, g[int(50 * q)])


def test_vegas_sampling_is_deterministic_per_iteration(oracle_lib):
    args = ([0.0] * 4, [1.0] * 4, [0.5] * 4, [0.2] * 4, oracle_lib.uniform_grid(4, 50), 5000)
    a = oracle_lib.vegas_iteration(*args, seed=1, iteration=2)
    b = oracle_lib.vegas_iteration(*args, seed=1, iteration=2)
    c = oracle_lib.vegas_iteration(*args, seed=1, iteration=3)
    assert a[0] == b[0] and np.array_equal(a[2], b[2]) and a[0] != c[0]


# --------------------------------------------------- determinism / validation ----

def test_chunking_is_bit_identical(oracle_lib):
    p4, w = oracle_lib.generate(CFG0_M, CFG0_MASSES, 1000, seed=42, event_offset=0)
    pa, wa = oracle_lib.generate(CFG0_M, CFG0_MASSES, 333, seed=42, event_offset=0)
    pb, wb = oracle_lib.generate(CFG0_M, CFG0_MASSES, 667, seed=42, event_offset=333)
    assert np.array_equal(np.concatenate([pa, pb], axis=2), p4)
    assert np.array_equal(np.concatenate([wa, wb]), w)


def test_streams_and_seeds_differ(oracle_lib):
    _, w0 = oracle_lib.generate(CFG0_M, CFG0_MASSES, 100, seed=42, stream_id=0, want_momenta=False)
    _, w1 = oracle_lib.generate(CFG0_M, CFG0_MASSES, 100, seed=42, stream_id=1, want_momenta=False)
    _, w2 = oracle_lib.generate(CFG0_M, CFG0_MASSES, 100, seed=43, stream_id=0, want_momenta=False)
    assert not np.array_equal(w0, w1) and not np.array_equal(w0, w2)


def test_validation(oracle_lib):
    o = oracle_lib
    assert o.generate_status(5.0, [1.0]) == o.EINVAL
    assert o.generate_status(50.0, [0.1] * 11) == o.EINVAL
    assert o.generate_status(5.0, [1.0, -0.1]) == o.EINVAL
    assert o.generate_status(5.0, [1.0, float("nan")]) == o.EINVAL
    assert o.generate_status(5.0, [3.0, 2.0]) == o.EKINEMATICS
    assert o.generate_status(5.0, [3.0, 2.5]) == o.EKINEMATICS
    assert o.generate_status(5.0, [0.0, 0.0]) == o.OK


# --------------------------------------------------- property tests ----

from hypothesis import given, settings, strategies as st  # noqa: E402


@settings(max_examples=60, deadline=None)
@given(n=st.integers(2, 10), M=st.floats(0.5, 50.0), frac=st.floats(0.0, 0.95),
       seed=st.integers(0, 2 ** 64 - 1), stream=st.integers(0, 2 ** 32 - 1),
       offset=st.integers(0, 2 ** 50), moving=st.booleans(), mseed=st.integers(0, 10 ** 6))
def test_property_conservation_and_ordering(oracle_lib, n, M, frac, seed, stream, offset, moving, mseed):
    rng = np.random.default_rng(mseed)
    raw = rng.uniform(0.0, 1.0, size=n)
    masses = list(raw / raw.sum() * frac * M)  # sum of masses = frac * M < M
    parent = None
    if moving:
        p = rng.normal(size=3) * M
        parent = np.array([math.sqrt(M * M + float(p @ p)), *p])
    p4, w = oracle_lib.generate(M, masses, 16, seed=seed, stream_id=stream, event_offset=offset,
                                parent_p4=parent)
    assert np.all(np.isfinite(p4)) and np.all(w >= 0.0) and np.all(np.isfinite(w))
    P = np.array([M, 0.0, 0.0, 0.0]) if parent is None else parent
    scale = float(np.max(np.abs(P)))
    assert np.all(np.abs(p4.sum(axis=0) - P[:, None]) <= 1e-11 * scale)
    for d in range(n):
        m2 = _minkowski_sq(p4[d])
        assert np.all(np.abs(m2 - masses[d] ** 2) <= 1e-10 * p4[d, 0] ** 2 + 1e-300)
    # invariant masses of the nested subsystems never decrease
    acc = p4[0].copy()
    prev = np.full(16, masses[0])
    for i in range(1, n):
        acc = acc + p4[i]
        mi = np.sqrt(np.maximum(_minkowski_sq(acc), 0.0))
        assert np.all(mi >= prev + masses[i] - 1e-9 * M)
        prev = mi
