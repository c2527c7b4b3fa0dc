"""GPU parity of unweighted samples of a model (built-in Breit-Wigner product or
a user intensity compiled at run time) against the CPU oracle.

Trial g is kept when v_g * w_max < w_g |A|^2(g).  The kept set is an integer
result decided in FP64 on both sides from values that agree to the model
tolerance (the Breit-Wigner factors amplify the momenta's 1e-11 by about
M^2 / (mass width)); a trial may be kept on one side only when its acceptance
test is that close to the boundary, which the tests check explicitly."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle
from parity import FP64_TOL, assert_events_close, rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CFG0 = (5.279, [3.097, 0.4937, 0.13957])
KSTAR = (0.8955, 0.0473)
PSI2S = (3.686, 0.3)

CASES = [
    ("cfg0 K*", CFG0[0], CFG0[1], [(1, 2, *KSTAR)]),
    ("cfg0 psi' x K*", CFG0[0], CFG0[1], [(0, 1, *PSI2S), (1, 2, *KSTAR)]),
    ("four-body two factors", 4.0, [0.5, 1.0, 0.2, 0.3], [(0, 3, 1.2, 0.1), (1, 2, 1.5, 0.2)]),
    ("six pions four factors", 10.0, [0.13957] * 6,
     [(0, 1, 0.775, 0.149), (2, 3, 0.775, 0.149), (4, 5, 0.775, 0.149), (1, 4, 1.27, 0.185)]),
    ("ten bodies one factor", 10.0, [0.13957] * 10, [(3, 9, 0.98, 0.05)]),
]


def _say(*args):
    print("[unweight model]", *args, flush=True)
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


def _host(out, idx, counts, wm):
    torch.cuda.synchronize()
    kept, over = (int(x) for x in counts.cpu().tolist())
    k = min(kept, idx.shape[0])
    p4 = None if out is None else out[:, :, :k].cpu().numpy()
    return p4, idx[:k].cpu().numpy().astype(np.uint64), kept, over, float(wm.item())


def _gpu(P, M, m, ntrials, res, **kw):
    return _host(*P.generate_unweighted_model(M, m, ntrials, res, want_index=True, **kw))


def _clear_bound(values, q, tol):
    """A bound near the q quantile of the values, in a gap between two of them
    wider than the two sides' disagreement (so both count the same trials above
    it)."""
    v = np.sort(values)
    k = int(q * (len(v) - 1))
    for j in range(k, len(v) - 1):
        if v[j + 1] - v[j] > 20.0 * tol * v[j + 1]:
            return float(0.5 * (v[j] + v[j + 1]))
    raise AssertionError("no gap in the values")


def _compare(gp4, gidx, gkept, okept, oidx, op4, borderline):
    a, b = set(gidx.tolist()), set(oidx.tolist())
    for g in a ^ b:
        assert borderline(g), f"trial {g} kept on one side only"
    assert abs(gkept - okept) == len(a ^ b)
    common = sorted(a & b)
    if gp4 is not None and len(common):
        ig = np.searchsorted(gidx, common)
        io = np.searchsorted(oidx, common)
        wdummy = np.ones(len(common))
        assert_events_close(gp4[:, :, ig], wdummy, op4[:, :, io], wdummy)


@pytest.mark.parametrize("mode", ["sample_max", "given_bound"])
@pytest.mark.parametrize("name,M,m,res", CASES, ids=[c[0] for c in CASES])
def test_unweighted_model_matches_oracle(P, name, M, m, res, mode):
    _say(name, mode)
    ntrials, seed, sid, off = 20_011, 31, 2, 7_000_000_001
    tol = _tol(M, res)
    _, _, vals = oracle.model_integrate(M, m, ntrials, res, seed=seed, stream_id=sid, event_offset=off,
                                        want_values=True)
    w_max = 0.0 if mode == "sample_max" else _clear_bound(vals, 0.9, tol)
    gp4, gidx, gkept, gover, gwm = _gpu(P, M, m, ntrials, res, seed=seed, stream_id=sid, event_offset=off,
                                        w_max=w_max)
    op4, oidx, okept, oover, owm = oracle.unweight_model(M, m, ntrials, res, seed=seed, stream_id=sid,
                                                         event_offset=off, w_max=w_max)
    if w_max == 0.0:
        assert rel(gwm, owm) <= tol and owm == float(np.max(vals)) and gover == oover == 0
    else:
        assert gwm == w_max and owm == w_max and gover == oover > 0
    assert np.all(np.diff(gidx.astype(np.int64)) > 0)
    assert 0 < okept < ntrials

    def borderline(g):
        v = oracle.accept_uniform(seed, sid, int(g), len(m))
        val = vals[int(g) - off]
        return abs(v * owm - val) <= 4.0 * tol * val

    _compare(gp4, gidx, gkept, okept, oidx, op4, borderline)


def test_unweighted_model_without_factors_is_weight_only(P):
    """No factor: |A|^2 = 1 and the sample is the weight-only one, bit for bit."""
    _say("no factor")
    M, m = 4.0, [0.5, 1.0, 0.2, 0.3]
    a = _gpu(P, M, m, 100_003, [], seed=6, event_offset=9)
    out, idx, counts, wm = P.generate_unweighted(M, m, 100_003, seed=6, event_offset=9, want_index=True)
    b = _host(out, idx, counts, wm)
    assert a[2:] == b[2:] and np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])


@pytest.mark.parametrize("ntrials", [0, 1, 1023, 1025, 65_537])
def test_unweighted_model_edge_sizes(P, ntrials):
    _say(f"edge {ntrials}")
    M, m = CFG0
    res = [(1, 2, *KSTAR)]
    tol = _tol(M, res)
    gp4, gidx, gkept, gover, gwm = _gpu(P, M, m, ntrials, res, seed=4, event_offset=77)
    op4, oidx, okept, oover, owm = oracle.unweight_model(M, m, ntrials, res, seed=4, event_offset=77)
    if ntrials == 0:
        assert gkept == 0 and gover == 0 and gwm == 0.0
        return
    assert rel(gwm, owm) <= tol and gover == 0
    if ntrials == 1:
        assert gkept == okept == 1  # the one trial is the bound: v < 1 keeps it
    # the integral needs two events; the per-event values depend only on the index
    _, _, vals = oracle.model_integrate(M, m, max(ntrials, 2), res, seed=4, event_offset=77, want_values=True)

    def borderline(g):
        v = oracle.accept_uniform(4, 0, int(g), 3)
        return abs(v * owm - vals[int(g) - 77]) <= 4.0 * tol * vals[int(g) - 77]

    _compare(gp4, gidx, gkept, okept, oidx, op4, borderline)


def test_unweighted_model_capacity_and_count_only(P):
    _say("capacity / count only")
    M, m = CFG0
    res = [(0, 1, *PSI2S), (1, 2, *KSTAR)]
    full = _gpu(P, M, m, 200_003, res, seed=8)
    cap = 1000
    assert full[2] > cap
    part = _gpu(P, M, m, 200_003, res, seed=8, capacity=cap)
    assert part[2] == full[2] and np.array_equal(part[1], full[1][:cap])
    assert np.array_equal(part[0], full[0][:, :, :cap])
    _, _, counts, wm = P.generate_unweighted_model(M, m, 200_003, res, seed=8, want_events=False)
    torch.cuda.synchronize()
    assert int(counts[0].item()) == full[2] and float(wm.item()) == full[4]


def test_unweighted_model_full_size(P):
    """1e8 trials of the three-body channel with the K*(892) factor: the kept
    fraction against the model integral over the same trials, increasing
    indices, and sampled kept and rejected trials against the oracle's events,
    values and decisions."""
    _say("full size 1e8 trials, K* model")
    M, m = CFG0
    res = [(1, 2, *KSTAR)]
    tol = _tol(M, res)
    n = 100_000_000
    out, idx, counts, wm = P.generate_unweighted_model(M, m, n, res, seed=42, want_index=True)
    stats, _ = P.integrate_model(M, m, n, res, seed=42)
    torch.cuda.synchronize()
    kept, over = (int(x) for x in counts.cpu().tolist())
    w_max = float(wm.item())
    p = float(stats[1].item()) / w_max
    assert over == 0 and abs(kept / n - p) < 6.0 * math.sqrt(p * (1 - p) / n), (kept, p)
    gidx = idx[:kept]
    assert bool((gidx[1:] > gidx[:-1]).all().item())

    def one(e):
        op4, _ = oracle.generate(M, m, 1, seed=42, event_offset=int(e))
        _, _, v = oracle.model_integrate(M, m, 2, res, seed=42, event_offset=int(e), want_values=True)
        return op4, float(v[0]), oracle.accept_uniform(42, 0, int(e), 3)

    rng = np.random.default_rng(1)
    pos = np.unique(np.concatenate([[0, kept - 1], rng.integers(0, kept, 200)]))
    tpos = torch.as_tensor(pos, device="cuda")
    g = gidx[tpos].cpu().numpy()
    gp4 = out[:, :, tpos].cpu().numpy()
    for j, e in enumerate(g):
        op4, val, v = one(e)
        assert_events_close(gp4[:, :, j:j + 1], np.ones(1), op4, np.ones(1))
        assert v * w_max < val or abs(v * w_max - val) <= 4.0 * tol * val
    trials = rng.integers(0, n, 200)
    kept_set = torch.isin(torch.as_tensor(trials, device="cuda"), gidx).cpu().numpy()
    for t, k in zip(trials, kept_set):
        _, val, v = one(t)
        assert (v * w_max < val) == bool(k) or abs(v * w_max - val) <= 4.0 * tol * val
    del out, idx


# --------------------------------------------------------------------------
# User intensities compiled at run time

# The built-in Breit-Wigner product written as user code (same expression in
# the same order); par = (i, j, mass, width) per factor, mass 0 unused.
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

# sum_d (E_d - par0)^2 + par1 pz_0^2 + par2 |p_{N-1}|
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


@pytest.mark.parametrize("name,M,m,res", [CASES[1], CASES[3]], ids=[CASES[1][0], CASES[3][0]])
def test_unweighted_user_model_matches_builtin(P, name, M, m, res):
    """The Breit-Wigner product as user code keeps the same trials with the
    same events, bound and counts as the built-in model, bit for bit."""
    _say(f"user = built-in: {name}")
    model = P.UserModel(USER_BW, len(m))
    try:
        sampled = _gpu(P, M, m, 300_007, res, seed=3, event_offset=11)
        for w_max in (0.0, 0.5 * sampled[4]):  # the sampled bound, then half of it (some trials above)
            b = _gpu(P, M, m, 300_007, res, seed=3, event_offset=11, w_max=w_max)
            u = _host(*model.generate_unweighted(M, m, 300_007, _bw_params(res), seed=3, event_offset=11,
                                                 w_max=w_max, want_index=True))
            assert u[2:] == b[2:], (u[2:], b[2:])
            assert np.array_equal(u[1], b[1]) and np.array_equal(u[0], b[0])
    finally:
        model.destroy()


@pytest.mark.parametrize("M,m", [CFG0, (10.0, [0.13957] * 6), (10.0, [0.0] * 10), (5.0, [1.0, 2.0])])
def test_unweighted_user_model_against_oracle(P, M, m):
    """A kinematic intensity of every daughter: the kept set against the
    hit-or-miss test applied (in numpy) to the oracle's events, weights and
    acceptance uniforms, and the kept events against the oracle's."""
    N = len(m)
    _say(f"user kinematic model unweighted vs oracle, N={N}")
    n, seed, sid, off = 20_011, 77, 2, 1 << 33
    par = [0.3 * M, 2.0, 0.7]
    model = P.UserModel(USER_KIN, N)
    try:
        gp4, gidx, gkept, gover, gwm = _host(*model.generate_unweighted(M, m, n, par, seed=seed, stream_id=sid,
                                                                        event_offset=off, want_index=True))
    finally:
        model.destroy()
    p4, w = oracle.generate(M, m, n, seed=seed, stream_id=sid, event_offset=off)
    E, X, Y, Z = p4[:, 0, :], p4[:, 1, :], p4[:, 2, :], p4[:, 3, :]
    f = par[1] * Z[0] ** 2 + par[2] * np.sqrt(X[N - 1] ** 2 + Y[N - 1] ** 2 + Z[N - 1] ** 2) + \
        ((E - par[0]) ** 2).sum(axis=0)
    ref = w * f
    # the two sides' values agree to 1e-10 of this scale (see the model evaluation tests)
    scale = w * (par[1] * M * M + par[2] * M + ((np.abs(E) + abs(par[0])) ** 2).sum(axis=0))
    k_max = int(np.argmax(ref))
    assert gover == 0 and abs(gwm - ref[k_max]) <= 1e-10 * scale[k_max]
    v = np.array([oracle.accept_uniform(seed, sid, off + t, N) for t in range(n)])
    okept = np.nonzero(v * ref[k_max] < ref)[0]
    oidx = (okept + off).astype(np.uint64)

    def borderline(g):
        t = int(g) - off
        return abs(v[t] * ref[k_max] - ref[t]) <= 4e-10 * max(scale[t], scale[k_max])

    _compare(gp4, gidx, gkept, len(okept), oidx, p4[:, :, okept], borderline)
    assert 0 < gkept < n


@pytest.mark.parametrize("w_max_mode", ["sample_max", "given_bound"])
def test_unweighted_model_chunked(P, w_max_mode):
    """The Breit-Wigner model through the fused write-and-count launches (chunked
    on request): every chunk count keeps the same trials with the same events,
    counts and bound, bit for bit, and they match the oracle."""
    _say(f"model chunked {w_max_mode}")
    M, m = CFG0
    res = [(0, 1, *PSI2S), (1, 2, *KSTAR)]
    n = 2_600_003
    tol = _tol(M, res)
    w_max = 0.0
    if w_max_mode == "given_bound":
        _, _, vals = oracle.model_integrate(M, m, 20_000, res, seed=6, event_offset=5, want_values=True)
        w_max = _clear_bound(vals, 0.95, tol)
    runs = {}
    try:
        for chunks in (1, 3, 16):
            P.set_unweight_chunks(chunks)
            runs[chunks] = _gpu(P, M, m, n, res, seed=6, event_offset=5, w_max=w_max)
    finally:
        P.set_unweight_chunks(0)
    ref = runs[1]
    for chunks, r in runs.items():
        assert r[2:] == ref[2:], (chunks, r[2:], ref[2:])
        assert np.array_equal(r[1], ref[1]) and np.array_equal(r[0], ref[0]), chunks
    gp4, gidx, gkept, gover, gwm = ref
    op4, oidx, okept, oover, owm = oracle.unweight_model(M, m, n, res, seed=6, event_offset=5, w_max=w_max)
    assert rel(gwm, owm) <= tol and gover == oover
    _, _, vals = oracle.model_integrate(M, m, n, res, seed=6, event_offset=5, want_values=True)

    def borderline(g):
        v = oracle.accept_uniform(6, 0, int(g), 3)
        return abs(v * owm - vals[int(g) - 5]) <= 4.0 * tol * vals[int(g) - 5]

    _compare(gp4, gidx, gkept, okept, oidx, op4, borderline)


@pytest.mark.parametrize("name,M,m,res", [CASES[0], CASES[3], CASES[4]], ids=[CASES[0][0], CASES[3][0], CASES[4][0]])
def test_unweighted_model_stored_values_match_recomputed(P, name, M, m, res):
    """With no bound given, the max pass keeps every trial's value for the count
    pass; with that same bound given, the count pass computes the values itself.
    Both keep the same trials with the same events and counts, bit for bit, for
    the built-in model and the same intensity as user code; twice in a row, the
    second call smaller (the stored values of the first are not reused)."""
    _say(f"stored vs recomputed values: {name}")
    model = P.UserModel(USER_BW, len(m))
    try:
        for n in (400_009, 150_001):
            sampled = _gpu(P, M, m, n, res, seed=13, event_offset=3)
            given = _gpu(P, M, m, n, res, seed=13, event_offset=3, w_max=sampled[4])
            assert sampled[2:] == given[2:], (sampled[2:], given[2:])
            assert np.array_equal(sampled[1], given[1]) and np.array_equal(sampled[0], given[0])
            u = _host(*model.generate_unweighted(M, m, n, _bw_params(res), seed=13, event_offset=3,
                                                 want_index=True))
            assert u[2:] == sampled[2:] and np.array_equal(u[1], sampled[1]) and np.array_equal(u[0], sampled[0])
    finally:
        model.destroy()


@pytest.mark.parametrize("w_max_mode", ["sample_max", "given_bound"])
@pytest.mark.parametrize("name,M,m,res", CASES[2:], ids=[c[0] for c in CASES[2:]])
def test_unweighted_model_chunked_every_n(P, name, M, m, res, w_max_mode):
    """The Breit-Wigner fused store-and-count launch for four, six and ten
    daughters: five chunks give the one-chunk result bit for bit (values stored
    by the max pass or recomputed), and it matches the oracle."""
    _say(f"model chunked {name} {w_max_mode}")
    n = 1_300_007
    tol = _tol(M, res)
    w_max = 0.0
    if w_max_mode == "given_bound":
        _, _, vals = oracle.model_integrate(M, m, 20_000, res, seed=8, event_offset=2, want_values=True)
        w_max = _clear_bound(vals, 0.9, tol)
    runs = {}
    try:
        for chunks in (1, 5):
            P.set_unweight_chunks(chunks)
            runs[chunks] = _gpu(P, M, m, n, res, seed=8, event_offset=2, w_max=w_max)
    finally:
        P.set_unweight_chunks(0)
    a, b = runs[1], runs[5]
    assert a[2:] == b[2:] and np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])
    gp4, gidx, gkept, gover, gwm = b
    op4, oidx, okept, oover, owm = oracle.unweight_model(M, m, n, res, seed=8, event_offset=2, w_max=w_max)
    assert rel(gwm, owm) <= tol and gover == oover
    _, _, vals = oracle.model_integrate(M, m, n, res, seed=8, event_offset=2, want_values=True)

    def borderline(g):
        v = oracle.accept_uniform(8, 0, int(g), len(m))
        return abs(v * owm - vals[int(g) - 2]) <= 4.0 * tol * vals[int(g) - 2]

    _compare(gp4, gidx, gkept, okept, oidx, op4, borderline)
