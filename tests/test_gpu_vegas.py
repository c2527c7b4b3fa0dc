"""GPU parity of VEGAS / plain Monte Carlo against the CPU oracle.

A sample's value is a product of D Gaussian factors and D Jacobian factors; the
two sides differ only in the last bit of exp, so values agree to ~4D ulp and
the tests allow 1e-13 D relative.  Sums (estimate, histogram) differ in their
order; 1e-11 relative covers that.  Refined grids then agree to ~1e-13, and
later iterations stay within the same tolerances."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from parity import rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[vegas]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()
    oracle.build(force=False)
    return P


CASES = [
    ("1-D", [0.0], [1.0], [0.3], [0.08], 50),
    ("3-D broad", [0.0, -1.0, 0.5], [1.0, 2.0, 1.5], [0.4, 0.3, 1.0], [0.5, 0.8, 0.6], 50),
    ("10-D paper integrand", [0.0] * 10, [1.0] * 10, [0.5] * 10, [0.1] * 10, 50),
    ("16-D, 128 bins", [0.0] * 16, [1.0] * 16, [0.5] * 16, [0.3] * 16, 128),
]


@pytest.mark.parametrize("name,lo,hi,mu,sg,bins", CASES, ids=[c[0] for c in CASES])
def test_vegas_iterations_match_oracle(P, name, lo, hi, mu, sg, bins):
    _say(name)
    D = len(lo)
    f = P.gauss_box(lo, hi, mu, sg)
    calls = 20_011
    grid_g = oracle.uniform_grid(D, bins)
    grid_o = grid_g.copy()
    for t in range(3):
        g_dev = torch.as_tensor(grid_g, device="cuda")
        st, h, v = P.vegas_iteration(f, g_dev, calls, seed=5, iteration=t, want_values=(t == 0))
        torch.cuda.synchronize()
        st, h = st.cpu().numpy(), h.cpu().numpy()
        mo, so, ho, vo = oracle.vegas_iteration(lo, hi, mu, sg, grid_o, calls, seed=5, iteration=t, want_values=True)
        tol = 1e-11 if t == 0 else 1e-9
        assert st[0] == calls and rel(st[1], mo) <= tol and rel(st[3], so) <= tol, (t, st, mo, so)
        assert np.allclose(h, ho, rtol=tol, atol=0.0), (t, float(np.max(np.abs(h - ho) / np.maximum(ho, 1e-300))))
        if t == 0:
            # per-sample values on the same grid
            vals = v[:calls].cpu().numpy()
            assert np.allclose(vals, vo, rtol=1e-13 * D, atol=0.0)
        grid_g = P.vegas_refine(grid_g, h, 1.5)
        grid_o = oracle.vegas_refine(grid_o, ho, 1.5)
        assert np.allclose(grid_g, grid_o, rtol=0.0, atol=1e-9)


def test_vegas_is_deterministic(P):
    _say("determinism")
    f = P.gauss_box([0.0] * 10, [1.0] * 10, [0.5] * 10, [0.1] * 10)
    g = torch.as_tensor(oracle.uniform_grid(10, 50), device="cuda")
    a = P.vegas_iteration(f, g, 1_000_003, seed=9, iteration=1)
    b = P.vegas_iteration(f, g, 1_000_003, seed=9, iteration=1)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_vegas_driver_matches_oracle_driver(P):
    _say("driver")
    lo, hi, mu, sg = [0.0] * 10, [1.0] * 10, [0.5] * 10, [0.1] * 10
    f = P.gauss_box(lo, hi, mu, sg)
    r, e, c, g = P.vegas(f, 50_000, 4, warmup=3, seed=11)
    ro, eo, co, _, go = oracle.vegas(lo, hi, mu, sg, 50_000, 4, warmup=3, seed=11)
    assert rel(r, ro) <= 1e-8 and rel(e, eo) <= 1e-8 and abs(c - co) <= 1e-6 * max(1.0, co)
    assert np.allclose(g, go, rtol=0.0, atol=1e-8)


def test_vegas_full_size_ten_dimensions(P):
    """The paper's benchmark integrand at 1e7 calls per iteration: the result
    against the erf closed form."""
    _say("10-D, 1e7 calls x (5 + 5) iterations")
    lo, hi, mu, sg = [0.0] * 10, [1.0] * 10, [0.5] * 10, [0.1] * 10
    f = P.gauss_box(lo, hi, mu, sg)
    r, e, c, _ = P.vegas(f, 10_000_000, 5, warmup=5, seed=42)
    exact = oracle.gaussian_integral(lo, hi, mu, sg)
    assert abs(r - exact) < 4.0 * e, (r, e, exact)
    assert e < 3e-4 * exact and c < 5.0


def test_plain_mc_full_size(P):
    """Plain Monte Carlo (uniform grid, one iteration) at 1e8 samples of a broad
    3-D Gaussian against the closed form."""
    _say("plain MC 1e8")
    lo, hi, mu, sg = [0.0, -1.0, 0.5], [1.0, 2.0, 1.5], [0.4, 0.3, 1.0], [0.5, 0.8, 0.6]
    f = P.gauss_box(lo, hi, mu, sg)
    g = torch.as_tensor(oracle.uniform_grid(3, 50), device="cuda")
    st, _, _ = P.vegas_iteration(f, g, 100_000_000, seed=3, want_hist=False)
    st = st.cpu().numpy()
    exact = oracle.gaussian_integral(lo, hi, mu, sg)
    assert abs(st[1] - exact) < 4.0 * st[3], (st, exact)


# --------------------------------------------------------------------------
# User integrands compiled at run time

# The product of Gaussians as user code, with per-dimension (mean, sigma) in
# par[2d], par[2d + 1] (up to eight dimensions).
USER_GAUSS = """
__device__ double hydra_phsp_user_integrand(const double* x, const double* par) {
    double v = 1.0;
    for (int d = 0; d < HYDRA_PHSP_DIM; ++d) {
        const double t = (x[d] - par[2 * d]) / par[2 * d + 1];
        v = v * (exp(-0.5 * t * t) / (par[2 * d + 1] * 2.5066282746310002));
    }
    return v;
}
"""

# A non-separable integrand with a closed form over [0,1]^3 x [-1,1]:
# x0 x1^2 e^{x2} (1 + par0 x3) integrates to (e - 1) / 3 for any par0.
USER_POLY = """
__device__ double hydra_phsp_user_integrand(const double* x, const double* par) {
    return x[0] * x[1] * x[1] * exp(x[2]) * (1.0 + par[0] * x[3]);
}
"""


@pytest.mark.parametrize("lo,hi,mu,sg,bins", [
    ([0.0, -1.0, 0.5], [1.0, 2.0, 1.5], [0.4, 0.3, 1.0], [0.5, 0.8, 0.6], 50),
    ([0.0] * 8, [1.0] * 8, [0.5] * 8, [0.12] * 8, 37),
])
def test_user_integrand_matches_oracle(P, lo, hi, mu, sg, bins):
    """The Gaussian product as a user integrand: per-sample values, estimate and
    histogram against the oracle's iteration on the same counters, over three
    refined grids."""
    D = len(lo)
    _say(f"user integrand, {D}-D Gaussian vs oracle")
    par = [v for pair in zip(mu, sg) for v in pair]
    f = P.UserIntegrand(USER_GAUSS, D)
    calls = 30_011
    grid = oracle.uniform_grid(D, bins)
    try:
        for t in range(3):
            st, h, v = f.iteration(lo, hi, torch.as_tensor(grid, device="cuda"), calls, par, seed=6, iteration=t,
                                   want_values=True)
            torch.cuda.synchronize()
            st, h, vals = st.cpu().numpy(), h.cpu().numpy(), v[:calls].cpu().numpy()
            mo, so, ho, vo = oracle.vegas_iteration(lo, hi, mu, sg, grid, calls, seed=6, iteration=t,
                                                    want_values=True)
            # the user code divides on the device where the oracle multiplies by
            # host reciprocals, and multiplies the Jacobians last: a few more ulp
            assert np.allclose(vals, vo, rtol=4e-13 * D, atol=0.0), float(np.max(np.abs(vals - vo) / vo))
            assert st[0] == calls and rel(st[1], mo) <= 1e-11 and rel(st[3], so) <= 1e-11, (t, st, mo, so)
            assert np.allclose(h, ho, rtol=1e-11, atol=0.0)
            grid = oracle.vegas_refine(grid, ho, 1.5)
    finally:
        f.destroy()


def test_user_integrand_vegas_closed_form(P):
    """VEGAS (5 adapting + 5 estimating iterations) and plain MC on a
    non-separable integrand against its closed form; VEGAS beats plain MC's
    error at equal calls."""
    _say("user integrand, closed form")
    lo, hi = [0.0, 0.0, 0.0, -1.0], [1.0, 1.0, 1.0, 1.0]
    exact = (np.e - 1.0) / 3.0
    f = P.UserIntegrand(USER_POLY, 4)
    try:
        r, e, c, g = f.vegas(lo, hi, 1_000_000, 5, [0.7], warmup=5, seed=21)
        assert abs(r - exact) < 4.0 * e and c < 5.0, (r, e, c, exact)
        st, _, _ = f.iteration(lo, hi, torch.as_tensor(oracle.uniform_grid(4, 50), device="cuda"), 1_000_000,
                               [0.7], seed=22, want_hist=False)
        st = st.cpu().numpy()
        assert abs(st[1] - exact) < 4.0 * st[3], (st, exact)
        assert e * np.sqrt(5.0) < st[3]  # per-iteration VEGAS error below plain MC's
        assert g.shape == (4, 51) and np.all(np.diff(g, axis=1) > 0)
    finally:
        f.destroy()
