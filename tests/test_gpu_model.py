"""GPU parity of model evaluation over phase space (Breit-Wigner intensities)
against the CPU oracle.

Tolerance: the events agree to 1e-11 of each daughter's energy, so a pair mass
squared s moves by at most ~4e-11 M^2, and a factor 1/((m^2 - s)^2 + (m g)^2)
by at most that over m g relative; a value therefore carries
1e-11 + sum_k 4e-11 M^2 / (m_k g_k) relative (stated per case below)."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle
import volumes as V
from parity import FP64_TOL, rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CFG0 = (5.279, [3.097, 0.4937, 0.13957])
KSTAR = (0.8955, 0.0473)
PSI2S = (3.686, 0.3)


def _say(*args):
    print("[model]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()
    oracle.build(force=False)
    return P


def _tol(M, res):
    return FP64_TOL + sum(4e-11 * M * M / (r[2] * r[3]) for r in res)


CASES = [
    ("cfg0 K*", CFG0[0], CFG0[1], [(1, 2, *KSTAR)]),
    ("cfg0 psi' x K*", CFG0[0], CFG0[1], [(0, 1, *PSI2S), (1, 2, *KSTAR)]),
    ("four-body two factors", 4.0, [0.5, 1.0, 0.2, 0.3], [(0, 3, 1.2, 0.1), (1, 2, 1.5, 0.2)]),
    ("six pions four factors", 10.0, [0.13957] * 6,
     [(0, 1, 0.775, 0.149), (2, 3, 0.775, 0.149), (4, 5, 0.775, 0.149), (1, 4, 1.27, 0.185)]),
    ("ten bodies one factor", 10.0, [0.13957] * 10, [(3, 9, 0.98, 0.05)]),
    ("no factor", 4.0, [0.5, 1.0, 0.2, 0.3], []),
]


@pytest.mark.parametrize("name,M,m,res", CASES, ids=[c[0] for c in CASES])
def test_model_matches_oracle(P, name, M, m, res):
    _say(name)
    nev = 20_011
    stats, vals = P.integrate_model(M, m, nev, res, seed=9, stream_id=2, event_offset=12345, want_values=True)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    v = vals[:nev].cpu().numpy()
    mo, so, vo = oracle.model_integrate(M, m, nev, res, seed=9, stream_id=2, event_offset=12345, want_values=True)
    tol = _tol(M, res)
    assert np.all(np.abs(v - vo) <= tol * np.abs(vo)), float(np.max(np.abs(v - vo) / np.abs(vo)))
    assert st[0] == nev and rel(st[1], mo) <= tol and rel(st[3], so) <= tol


def test_model_without_factors_is_the_integral(P):
    _say("no factor == integrate")
    M, m = CFG0
    stats, _ = P.integrate_model(M, m, 100_003, [], seed=4)
    st2 = P.integrate_async(M, m, 100_003, seed=4)  # four events per thread, the model kernel's shape
    torch.cuda.synchronize()
    assert torch.equal(stats, st2)


@pytest.mark.parametrize("nev", [0, 1, 2, 1023, 1025])
def test_model_edge_sizes(P, nev):
    _say(f"edge {nev}")
    M, m = CFG0
    res = [(1, 2, *KSTAR)]
    stats, vals = P.integrate_model(M, m, nev, res, seed=4, want_values=True)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    assert st[0] == nev
    if nev == 0:
        assert st[1] == 0.0 and st[3] == 0.0
        return
    _, _, vo = oracle.model_integrate(M, m, max(nev, 2), res, seed=4, want_values=True)
    v = vals[:nev].cpu().numpy()
    assert np.all(np.abs(v - vo[:nev]) <= _tol(M, res) * np.abs(vo[:nev]))
    assert rel(st[1], float(np.mean(vo[:nev]))) <= _tol(M, res)


def test_model_full_size_config1(P):
    """1e8 events of the throughput workload with the K* intensity: the integral
    against the Dalitz quadrature, and sampled per-event values against the
    oracle."""
    _say("full size 1e8")
    M, m = CFG0
    n = 100_000_000
    res = [(1, 2, *KSTAR)]
    stats, vals = P.integrate_model(M, m, n, res, seed=42, want_values=True)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    want = V.bw_dalitz_integral_one(M, *m, *KSTAR)
    assert abs(st[1] - want) < 5.0 * st[3], (st[1], st[3], want)
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 200)]))
    g = vals[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    for j, e in enumerate(idx):
        _, _, vo = oracle.model_integrate(M, m, 2, res, seed=42, event_offset=int(e), want_values=True)
        assert abs(g[j] - vo[0]) <= _tol(M, res) * abs(vo[0])
    del vals


# --------------------------------------------------------------------------
# User intensities compiled at run time

# The built-in Breit-Wigner product written as user code: the same expression
# in the same order (pair components summed first, s = e^2 - x^2 - y^2 - z^2,
# each factor divided into the running product), for up to four factors given
# as par = (i, j, mass, width) per factor; a factor with mass 0 is unused.
USER_BW = """
__device__ double hydra_phsp_user_intensity(const double* e, const double* px, const double* py,
                                            const double* pz, const double* par) {
    double a2 = 1.0;
    for (int k = 0; k < 4; ++k) {
        if (par[4 * k + 2] > 0.0) {
            const int i = (int)par[4 * k], j = (int)par[4 * k + 1];
            const double se = e[i] + e[j], sx = px[i] + px[j], sy = py[i] + py[j], sz = pz[i] + pz[j];
            const double s = se * se - sx * sx - sy * sy - sz * sz;
            const double d = par[4 * k + 2] * par[4 * k + 2] - s;
            const double mg = par[4 * k + 2] * par[4 * k + 3];
            a2 = a2 / (d * d + mg * mg);
        }
    }
    return a2;
}
"""

# A kinematic intensity of all daughters (for any N): sum_d (E_d - par0)^2 +
# par1 pz_0^2 + par2 |p_{N-1}|.
USER_KIN = """
__device__ double hydra_phsp_user_intensity(const double* e, const double* px, const double* py,
                                            const double* pz, const double* par) {
    double f = par[1] * pz[0] * pz[0] + par[2] * sqrt(px[HYDRA_PHSP_N - 1] * px[HYDRA_PHSP_N - 1] +
               py[HYDRA_PHSP_N - 1] * py[HYDRA_PHSP_N - 1] + pz[HYDRA_PHSP_N - 1] * pz[HYDRA_PHSP_N - 1]);
    for (int d = 0; d < HYDRA_PHSP_N; ++d) f += (e[d] - par[0]) * (e[d] - par[0]);
    return f;
}
"""


def _bw_params(res):
    par = [0.0] * 16
    for k, (i, j, mass, width) in enumerate(res):
        par[4 * k:4 * k + 4] = [float(i), float(j), mass, width]
    return par


@pytest.mark.parametrize("name,M,m,res", CASES, ids=[c[0] for c in CASES])
def test_user_model_matches_builtin(P, name, M, m, res):
    """The Breit-Wigner product as user code, compiled at run time, gives the
    built-in model's per-event values and integral bit for bit (same events,
    same expression, same compiler flags)."""
    _say(f"user model = built-in: {name}")
    n = 50_021
    model = P.UserModel(USER_BW, len(m))
    try:
        st_u, v_u = model.integrate(M, m, n, _bw_params(res), seed=13, event_offset=5, want_values=True)
        st_b, v_b = P.integrate_model(M, m, n, res, seed=13, event_offset=5, want_values=True)
        torch.cuda.synchronize()
        assert torch.equal(v_u[:n], v_b[:n]), name
        assert torch.equal(st_u, st_b), (st_u.cpu().tolist(), st_b.cpu().tolist())
    finally:
        model.destroy()


@pytest.mark.parametrize("M,m", [CFG0, (10.0, [0.13957] * 6), (10.0, [0.0] * 10), (5.0, [1.0, 2.0])])
def test_user_model_against_oracle(P, M, m):
    """A kinematic intensity of every daughter: per-event values against the
    intensity evaluated (in numpy) on the oracle's events times the oracle's
    weights, and the integral against the mean of those values."""
    N = len(m)
    _say(f"user kinematic model vs oracle, N={N}")
    n = 20_011
    par = [0.3 * M, 2.0, 0.7]
    model = P.UserModel(USER_KIN, N)
    try:
        st, v = model.integrate(M, m, n, par, seed=77, stream_id=2, event_offset=1 << 33, want_values=True)
        torch.cuda.synchronize()
        g = v[:n].cpu().numpy()
        s = st.cpu().numpy()
    finally:
        model.destroy()
    p4, w = oracle.generate(M, m, n, seed=77, stream_id=2, event_offset=1 << 33)
    E, X, Y, Z = p4[:, 0, :], p4[:, 1, :], p4[:, 2, :], p4[:, 3, :]
    f = par[1] * Z[0] ** 2 + par[2] * np.sqrt(X[N - 1] ** 2 + Y[N - 1] ** 2 + Z[N - 1] ** 2) + \
        ((E - par[0]) ** 2).sum(axis=0)
    ref = w * f
    # momenta agree to 1e-11 E_d: f moves by about 2 sum_d |E_d - par0| 1e-11 E_d + ... <= 1e-10 of its scale
    scale = w * (par[1] * M * M + par[2] * M + ((np.abs(E) + abs(par[0])) ** 2).sum(axis=0))
    assert np.max(np.abs(g - ref) / scale) <= 1e-10
    mean = math.fsum(ref) / n
    # the mean inherits the per-event bound (plus the rounding of the two sums)
    assert s[0] == n and abs(s[1] - mean) <= 1e-10 * math.fsum(scale) / n + FP64_TOL * abs(mean)


def test_user_model_constant_is_the_volume(P):
    """|A|^2 = par[0] = 1: the stats are those of the plain integral at four
    events per thread (the integrate-only default)."""
    _say("user model constant = volume")
    src = ("__device__ double hydra_phsp_user_intensity(const double* e, const double* px, const double* py, "
           "const double* pz, const double* par) { return par[0]; }")
    model = P.UserModel(src, 3)
    try:
        st, _ = model.integrate(*CFG0, 100_003, [1.0], seed=4)
        ref = P.integrate_async(*CFG0, 100_003, seed=4)
        torch.cuda.synchronize()
        assert torch.equal(st, ref), (st.cpu().tolist(), ref.cpu().tolist())
    finally:
        model.destroy()


def test_user_model_two_models_and_reuse(P):
    """Two models live at once and each keeps its own code; a model is reused
    across calls (its code object is loaded once per device)."""
    _say("two user models")
    a = P.UserModel(USER_BW, 3)
    b = P.UserModel(USER_KIN, 3)
    try:
        for _ in range(2):
            sa, _ = a.integrate(*CFG0, 30_000, _bw_params([(1, 2, *KSTAR)]), seed=9)
            sb, _ = b.integrate(*CFG0, 30_000, [1.0, 2.0, 0.7], seed=9)
            ra, _ = P.integrate_model(*CFG0, 30_000, [(1, 2, *KSTAR)], seed=9)
            torch.cuda.synchronize()
            assert torch.equal(sa, ra)
            assert not torch.equal(sa, sb)
    finally:
        a.destroy()
        b.destroy()
