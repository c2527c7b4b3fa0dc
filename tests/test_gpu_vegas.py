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
