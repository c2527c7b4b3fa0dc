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
