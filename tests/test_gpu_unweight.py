"""GPU parity of the unweighted (hit-or-miss) path against the CPU oracle.

The kept set is an integer result decided in FP64 on both sides from weights
that agree to 1e-11; a trial may only be kept on one side when its acceptance
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


def _say(*args):
    print("[unweight]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()
    oracle.build(force=False)
    return P


def _random_masses(n, seed):
    rng = np.random.default_rng(seed)
    M = float(rng.uniform(2.0, 12.0))
    return M, [float(x) for x in rng.uniform(0.0, 0.4 * M / n, size=n)]


def _gpu(P, M, m, ntrials, **kw):
    out, idx, counts, wm = P.generate_unweighted(M, m, ntrials, want_index=True, **kw)
    torch.cuda.synchronize()
    kept, over = (int(x) for x in counts.cpu().tolist())
    k = min(kept, idx.shape[0])
    p4 = None if out is None else out[:, :, :k].cpu().numpy()
    return p4, idx[:k].cpu().numpy().astype(np.uint64), kept, over, float(wm.item())


def _borderline(M, m, g, w_max, seed, stream_id, parent_p4=None):
    """|v w_max - w| within 1e-10 w for global event g (oracle values)."""
    _, w = oracle.generate(M, m, 1, seed=seed, stream_id=stream_id, event_offset=int(g), parent_p4=parent_p4,
                           want_momenta=False)
    v = oracle.accept_uniform(seed, stream_id, int(g), len(m))
    return abs(v * w_max - w[0]) <= 1e-10 * w[0]


def _compare(M, m, gp4, gidx, gkept, okept, oidx, op4, w_max, seed, sid, parent_p4=None):
    a, b = set(gidx.tolist()), set(oidx.tolist())
    for g in a ^ b:
        assert _borderline(M, m, g, w_max, seed, sid, parent_p4), f"trial {g} kept on one side only"
    assert abs(gkept - okept) == len(a ^ b)
    common = sorted(a & b)
    ig = np.searchsorted(gidx, common)
    io = np.searchsorted(oidx, common)
    if gp4 is not None and len(common):
        wdummy = np.ones(len(common))
        assert_events_close(gp4[:, :, ig], wdummy, op4[:, :, io], wdummy)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 10])
@pytest.mark.parametrize("mode", ["rest_sample_max", "broadcast_given_bound"])
def test_unweighted_matches_oracle(P, n, mode):
    _say(f"N={n} {mode}")
    M, m = _random_masses(n, 4000 + n)
    ntrials, seed, sid, off = 20_011, 17 + n, 3, 5_000_000_123
    parent = None
    w_max = 0.0
    if mode == "broadcast_given_bound":
        p = np.array([1.5, -0.7, 3.0])
        parent = [math.sqrt(M * M + float(p @ p)), *p]
        _, w = oracle.generate(M, m, 2000, seed=seed, stream_id=sid, event_offset=off, want_momenta=False)
        # a bound some trials exceed, kept clear of every weight by more than the
        # 1e-11 the two sides may differ by (two-body weights are all equal)
        w_max = float(np.quantile(w, 0.9)) * (1.0 + 1e-9)
    gp4, gidx, gkept, gover, gwm = _gpu(P, M, m, ntrials, seed=seed, stream_id=sid, event_offset=off,
                                        w_max=w_max, parent_p4=parent)
    op4, oidx, okept, oover, owm = oracle.unweight(M, m, ntrials, seed=seed, stream_id=sid, event_offset=off,
                                                   w_max=w_max, parent_p4=parent)
    if w_max == 0.0:
        assert rel(gwm, owm) <= FP64_TOL
    else:
        assert gwm == w_max and owm == w_max
    assert np.all(np.diff(gidx.astype(np.int64)) > 0)
    assert gover == oover
    _compare(M, m, gp4, gidx, gkept, okept, oidx, op4, owm, seed, sid, parent)
    if n == 2 and mode == "rest_sample_max":
        assert gkept == ntrials  # equal weights, bound = that weight: every trial is kept


def test_unweighted_capacity_and_count_only(P):
    _say("capacity / count only")
    M, m = CFG0
    full = _gpu(P, M, m, 50_000, seed=8)
    cap = 1000
    part = _gpu(P, M, m, 50_000, seed=8, capacity=cap)
    assert part[2] == full[2] and np.array_equal(part[1], full[1][:cap])
    assert np.array_equal(part[0], full[0][:, :, :cap])
    _, _, counts, wm = P.generate_unweighted(M, m, 50_000, seed=8, want_events=False)
    torch.cuda.synchronize()
    assert int(counts[0].item()) == full[2] and float(wm.item()) == full[4]


def test_unweighted_repeat_and_low_acceptance(P):
    """A large call repeated, then a smaller one on the same (grown) workspace,
    must give identical results and the kept trials of the small call must be the
    prefix of the large call's; a bound far above every weight keeps few trials
    (most blocks store nothing or a few partial lines)."""
    _say("repeat / low acceptance")
    M, m = CFG0
    a = _gpu(P, M, m, 3_000_017, seed=21, w_max=4.8)
    b = _gpu(P, M, m, 3_000_017, seed=21, w_max=4.8)
    assert a[2] == b[2] and a[2] < 2**63 and np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])
    small = _gpu(P, M, m, 100_003, seed=21, w_max=4.8)
    k = int(np.searchsorted(a[1], 100_003))
    assert small[2] == k and np.array_equal(small[1], a[1][:k]) and np.array_equal(small[0], a[0][:, :, :k])
    gp4, gidx, gkept, gover, _ = _gpu(P, M, m, 200_003, seed=5, w_max=480.0)
    op4, oidx, okept, oover, owm = oracle.unweight(M, m, 200_003, seed=5, w_max=480.0)
    assert gover == oover == 0 and 0 < okept < 5000
    _compare(M, m, gp4, gidx, gkept, okept, oidx, op4, owm, 5, 0)


@pytest.mark.parametrize("ntrials", [0, 1, 1023, 1024, 1025])
def test_unweighted_edge_sizes(P, ntrials):
    _say(f"edge {ntrials}")
    M, m = CFG0
    gp4, gidx, gkept, gover, gwm = _gpu(P, M, m, ntrials, seed=4, event_offset=77)
    op4, oidx, okept, oover, owm = oracle.unweight(M, m, ntrials, seed=4, event_offset=77)
    if ntrials == 0:
        assert gkept == 0 and gover == 0 and gwm == 0.0
        return
    assert rel(gwm, owm) <= FP64_TOL and gover == 0
    _compare(M, m, gp4, gidx, gkept, okept, oidx, op4, owm, 4, 0)


def test_unweighted_full_size_config1(P):
    """1e8 trials of the throughput workload: the kept fraction against the
    integral, increasing indices, and sampled kept and rejected trials against
    the oracle's events and decisions."""
    _say("full size 1e8 trials")
    M, m = CFG0
    n = 100_000_000
    out, idx, counts, wm = P.generate_unweighted(M, m, n, seed=42, want_index=True)
    mean, _ = P.integrate(M, m, n, seed=42)
    torch.cuda.synchronize()
    kept, over = (int(x) for x in counts.cpu().tolist())
    w_max = float(wm.item())
    p = mean / w_max
    assert over == 0 and abs(kept / n - p) < 6.0 * math.sqrt(p * (1 - p) / n), (kept, p)
    gidx = idx[:kept]
    assert bool((gidx[1:] > gidx[:-1]).all().item())
    rng = np.random.default_rng(0)
    pos = np.unique(np.concatenate([[0, kept - 1], rng.integers(0, kept, 300)]))
    tpos = torch.as_tensor(pos, device="cuda")
    g = gidx[tpos].cpu().numpy()
    gp4 = out[:, :, tpos].cpu().numpy()
    for j, e in enumerate(g):
        op4, ow = oracle.generate(M, m, 1, seed=42, event_offset=int(e))
        assert_events_close(gp4[:, :, j:j + 1], np.ones(1), op4, np.ones(1))
        v = oracle.accept_uniform(42, 0, int(e), 3)
        assert v * w_max < ow[0] or _borderline(M, m, e, w_max, 42, 0)
    # sampled trials: kept exactly when the oracle's test says so
    trials = rng.integers(0, n, 300)
    kept_set = torch.isin(torch.as_tensor(trials, device="cuda"), gidx).cpu().numpy()
    for t, k in zip(trials, kept_set):
        _, ow = oracle.generate(M, m, 1, seed=42, event_offset=int(t), want_momenta=False)
        v = oracle.accept_uniform(42, 0, int(t), 3)
        assert (v * w_max < ow[0]) == bool(k) or _borderline(M, m, t, w_max, 42, 0)
    del out, idx


def test_unweighted_sparse_span_beyond_32_bits(P):
    """A bound far above every weight over 2.2e9 trials keeps a few hundred: the
    write pass's one output range then spans more than 2^31 trials, so its list
    of trials is stored and restarted from a new base.  The result must be the
    same, bit for bit, as the same trials taken in three calls of fewer than
    2^31 trials each (event_offset continues the counter), and every kept event
    must be the oracle's."""
    M, m = CFG0
    n, w_max = 2_200_000_000, 1.0e7
    _say(f"sparse wide span: {n} trials, w_max {w_max}")
    big = _gpu(P, M, m, n, seed=12, w_max=w_max, capacity=4096)
    chunks = [(0, 1_000_000_000), (1_000_000_000, 1_000_000_000), (2_000_000_000, 200_000_000)]
    parts = [_gpu(P, M, m, c, seed=12, w_max=w_max, capacity=4096, event_offset=o) for o, c in chunks]
    assert big[3] == 0 and sum(p[3] for p in parts) == 0
    assert big[2] == sum(p[2] for p in parts) and 0 < big[2] < 4096
    assert np.array_equal(big[1], np.concatenate([p[1] for p in parts]))
    assert np.array_equal(big[0], np.concatenate([p[0] for p in parts], axis=2))
    assert big[1][-1] - big[1][0] > 2**31  # the kept trials do span beyond 32 bits of offset
    for j in range(0, big[2], max(big[2] // 40, 1)):
        e = int(big[1][j])
        op4, ow = oracle.generate(M, m, 1, seed=12, event_offset=e)
        assert_events_close(big[0][:, :, j:j + 1], np.ones(1), op4, np.ones(1))
        v = oracle.accept_uniform(12, 0, e, 3)
        assert v * w_max < ow[0]


@pytest.mark.parametrize("w_max,capacity", [(0.0, None), (0.0, 1_234_567), (480.0, None)],
                         ids=["sample_max", "capacity_mid_chunk", "few_kept"])
def test_unweighted_chunked_pipeline(P, w_max, capacity):
    """The write pass of chunk k and the count of chunk k+1 share one launch:
    for every chunk count the kept set, order, events, counts and
    bound are bit-identical to the unchunked sequence, and they match the
    oracle.  2.6e6 trials are ten scan groups, so up to ten chunks, the last one
    ragged; the capacity case ends the output inside a chunk, the few-kept case
    carries one partial output range through many chunks."""
    _say(f"chunked pipeline w_max={w_max} capacity={capacity}")
    M, m = CFG0
    n = 2_600_003
    runs = {}
    try:
        for chunks in (1, 2, 3, 4, 16):
            P.set_unweight_chunks(chunks)
            runs[chunks] = _gpu(P, M, m, n, seed=31, event_offset=9, w_max=w_max, capacity=capacity)
    finally:
        P.set_unweight_chunks(0)
    ref = runs[1]
    for chunks, r in runs.items():
        assert r[2:] == ref[2:], (chunks, r[2:], ref[2:])
        assert np.array_equal(r[1], ref[1]) and np.array_equal(r[0], ref[0]), chunks
    if capacity is not None:
        # the capacity truncates the full output: its prefix, bit for bit
        P.set_unweight_chunks(1)
        try:
            full = _gpu(P, M, m, n, seed=31, event_offset=9, w_max=w_max)
        finally:
            P.set_unweight_chunks(0)
        k = min(capacity, full[2])
        assert ref[2:] == full[2:] and ref[1].shape[0] == k
        assert np.array_equal(ref[1], full[1][:k]) and np.array_equal(ref[0], full[0][:, :, :k])
        ref = full
    op4, oidx, okept, oover, owm = oracle.unweight(M, m, n, seed=31, event_offset=9, w_max=w_max)
    assert ref[3] == oover and (w_max > 0.0 or rel(ref[4], owm) <= FP64_TOL)
    _compare(M, m, ref[0], ref[1], ref[2], okept, oidx, op4, owm, 31, 0)


def test_unweighted_chunked_on_a_side_stream(P):
    """On a caller's stream other than the null stream, work queued after the
    call on that stream sees every chunk's stores."""
    _say("chunked pipeline on a side stream")
    M, m = CFG0
    n = 2_600_003
    P.set_unweight_chunks(8)
    try:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            out, idx, counts, wm = P.generate_unweighted(M, m, n, seed=3, want_index=True, stream=s)
            snap = (out.clone(), idx.clone(), counts.clone())
        s.synchronize()
    finally:
        P.set_unweight_chunks(0)
    torch.cuda.synchronize()
    assert torch.equal(snap[2], counts)
    k = int(counts[0].item())
    assert torch.equal(snap[1][:k], idx[:k]) and torch.equal(snap[0][:, :, :k], out[:, :, :k])
    P.set_unweight_chunks(1)
    try:
        ref = _gpu(P, M, m, n, seed=3)
    finally:
        P.set_unweight_chunks(0)
    assert ref[2] == k and np.array_equal(ref[1], snap[1][:k].cpu().numpy().astype(np.uint64))
    assert np.array_equal(ref[0], snap[0][:, :, :k].cpu().numpy())


@pytest.mark.parametrize("n", [2, 4, 6, 10])
@pytest.mark.parametrize("mode", ["rest", "broadcast"])
def test_unweighted_chunked_every_n(P, n, mode):
    """The fused store-and-count launch for other daughter counts and for a
    moving parent: five chunks give the one-chunk result bit for bit, and that
    matches the oracle."""
    _say(f"chunked N={n} {mode}")
    M, m = _random_masses(n, 7000 + n)
    ntrials, seed, sid, off = 1_300_007, 29 + n, 5, 77_000_000_001
    parent = None
    if mode == "broadcast":
        p = np.array([-0.4, 2.5, 1.1])
        parent = [math.sqrt(M * M + float(p @ p)), *p]
    runs = {}
    try:
        for chunks in (1, 5):
            P.set_unweight_chunks(chunks)
            runs[chunks] = _gpu(P, M, m, ntrials, seed=seed, stream_id=sid, event_offset=off, parent_p4=parent)
    finally:
        P.set_unweight_chunks(0)
    a, b = runs[1], runs[5]
    assert a[2:] == b[2:] and np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])
    op4, oidx, okept, oover, owm = oracle.unweight(M, m, ntrials, seed=seed, stream_id=sid, event_offset=off,
                                                   parent_p4=parent)
    assert rel(b[4], owm) <= FP64_TOL and b[3] == oover
    _compare(M, m, b[0], b[1], b[2], okept, oidx, op4, owm, seed, sid, parent)
