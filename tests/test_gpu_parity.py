"""GPU parity: the HIP library (called through its C ABI) against the CPU oracle.

Every case runs the same seeded inputs through both sides and compares event by
event (FP64: |dc| <= 1e-11 E_d, weights and integrals <= 1e-11 relative), over
sizes that span many blocks with ragged tails; the full-size configurations are
checked on sampled events that the oracle computes one by one, plus properties
that hold at any size.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle
from parity import (FP64_TOL, MIXED_INTEGRAL_TOL, MIXED_TOL,
                    assert_events_close, event_errors, mixed_error_report, rel)

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[parity]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()  # raises if the HIP library is missing: no fallback
    oracle.build(force=False)
    return P


def _run(P, M, masses, nevents, seed=42, stream_id=0, offset=0, parent_p4=None, parent_dev=None,
         mixed=False, ld=None):
    n = len(masses)
    dtype = torch.float32 if mixed else torch.float64
    out = torch.empty((n, 4, ld or max(nevents, 1)), dtype=dtype, device="cuda")
    w = torch.empty(max(nevents, 1), dtype=torch.float64, device="cuda")
    _, _, stats = P.generate(M, masses, nevents, seed=seed, stream_id=stream_id, event_offset=offset,
                             parent_p4=parent_p4, parent_dev=parent_dev, out=out, weights=w,
                             mixed=mixed)
    torch.cuda.synchronize()
    return out[:, :, :nevents].cpu().numpy(), w[:nevents].cpu().numpy(), stats.cpu().numpy()


CFG0 = (5.279, [3.097, 0.4937, 0.13957])


def test_config0_full_event_by_event(P):
    _say("config0 1e5 N=3")
    M, m = CFG0
    p4, w, st = _run(P, M, m, 100_000)
    p4o, wo = oracle.generate(M, m, 100_000, seed=42)
    assert_events_close(p4, w, p4o, wo)
    mo, so = oracle.integrate(M, m, 100_000, seed=42)
    assert st[0] == 100_000
    assert rel(st[1], mo) <= FP64_TOL and rel(st[3], so) <= FP64_TOL


def test_config0_massless(P):
    _say("config0 massless M=1")
    p4, w, st = _run(P, 1.0, [0.0, 0.0, 0.0], 100_000)
    p4o, wo = oracle.generate(1.0, [0.0] * 3, 100_000, seed=42)
    assert_events_close(p4, w, p4o, wo)
    mo, so = oracle.integrate(1.0, [0.0] * 3, 100_000, seed=42)
    assert rel(st[1], mo) <= FP64_TOL and rel(st[3], so) <= FP64_TOL
    assert abs(st[1] - math.pi ** 2 / 8) < 4 * st[3]


def _random_masses(n, seed):
    rng = np.random.default_rng(seed)
    M = float(rng.uniform(2.0, 12.0))
    return M, [float(x) for x in rng.uniform(0.0, 0.4 * M / n, size=n)]


@pytest.mark.parametrize("n", list(range(2, 11)))
@pytest.mark.parametrize("pmode", ["rest", "broadcast", "per_event"])
def test_n_sweep(P, n, pmode):
    _say(f"n_sweep N={n} parent={pmode}")
    M, m = _random_masses(n, 1000 + n)
    nev = 10_007
    parent_p4 = None
    parent_dev = None
    parent_soa = None
    if pmode == "broadcast":
        p = np.array([0.3, -1.1, 2.5])
        parent_p4 = [math.sqrt(M * M + float(p @ p)), *p]
    elif pmode == "per_event":
        from paper_1711_05683_amd.workloads import per_event_parents
        parent_dev = per_event_parents(M, nev)
        parent_soa = parent_dev.cpu().numpy()
    p4, w, st = _run(P, M, m, nev, seed=7 + n, stream_id=n, offset=123_456_789, parent_p4=parent_p4,
                     parent_dev=parent_dev)
    p4o, wo = oracle.generate(M, m, nev, seed=7 + n, stream_id=n, event_offset=123_456_789,
                              parent_p4=parent_p4, parent_soa=parent_soa)
    assert_events_close(p4, w, p4o, wo)
    mo, so = oracle.integrate(M, m, nev, seed=7 + n, stream_id=n, event_offset=123_456_789)
    assert rel(st[1], mo) <= FP64_TOL
    if n > 2:
        assert rel(st[3], so) <= FP64_TOL


@pytest.mark.parametrize("n", [2, 3, 6, 10])
def test_integrate_matches_oracle(P, n):
    _say(f"integrate N={n}")
    M, m = _random_masses(n, 2000 + n)
    for nev in (2, 3, 255, 256, 257, 100_003):
        mean, sigma = P.integrate(M, m, nev, seed=5, stream_id=1, event_offset=99)
        mo, so = oracle.integrate(M, m, nev, seed=5, stream_id=1, event_offset=99)
        assert rel(mean, mo) <= FP64_TOL, (nev, mean, mo)
        # sigma of identical (two-body) weights is 0 up to the rounding of the
        # oracle's compensated mean, so an absolute floor of 1e-15 mean applies
        assert abs(sigma - so) <= FP64_TOL * so + 1e-15 * mo, (nev, sigma, so)


@pytest.mark.parametrize("n", [3, 6])
def test_counter_high_words(P, n):
    """Events whose global index crosses 2^32 (counter word 1 changes), a seed
    with both key words non-zero and a large stream id."""
    _say(f"counter high words N={n}")
    M, m = _random_masses(n, 3000 + n)
    seed, sid, off, nev = 0xDEADBEEF12345678, 0x80000005, (1 << 32) - 1000, 5000
    p4, w, st = _run(P, M, m, nev, seed=seed, stream_id=sid, offset=off)
    p4o, wo = oracle.generate(M, m, nev, seed=seed, stream_id=sid, event_offset=off)
    assert_events_close(p4, w, p4o, wo)
    mo, so = oracle.integrate(M, m, nev, seed=seed, stream_id=sid, event_offset=off)
    assert rel(st[1], mo) <= FP64_TOL and rel(st[3], so) <= FP64_TOL
    # chunked across the boundary: the same events
    p4a, wa, _ = _run(P, M, m, 1000, seed=seed, stream_id=sid, offset=off)
    p4b, wb, _ = _run(P, M, m, nev - 1000, seed=seed, stream_id=sid, offset=1 << 32)
    assert np.array_equal(np.concatenate([p4a, p4b], axis=2), p4) and np.array_equal(np.concatenate([wa, wb]), w)


def test_binding_allocates_line_aligned_columns(P):
    _say("binding output layout")
    M, m = CFG0
    nev = 1001
    out, w, _ = P.generate(M, m, nev)
    assert tuple(out.shape) == (3, 4, nev) and out.stride(1) == P.aligned_ld(nev) and out.stride(1) % 32 == 0
    assert out.data_ptr() % 128 == 0
    torch.cuda.synchronize()
    p4o, wo = oracle.generate(M, m, nev, seed=42)
    assert_events_close(out.cpu().numpy(), w.cpu().numpy(), p4o, wo)


def test_sequential_decay_chain(P):
    """Daughter 0 of a first generation as the per-event parent of a second one
    (its four rows of the first output, read in place): element-wise parity of
    both stages with the oracle chain, and four-momentum conservation."""
    _say("sequential decays")
    M, m = CFG0
    nev = 20_011
    ld = P.aligned_ld(nev)
    out1 = torch.empty((3, 4, ld), dtype=torch.float64, device="cuda")
    w1 = torch.empty(nev, dtype=torch.float64, device="cuda")
    P.generate(M, m, nev, seed=42, out=out1, weights=w1)
    out2, w2, st2 = P.generate(m[0], [0.0, 0.0, 0.0], nev, seed=42, stream_id=1, parent_dev=out1[0])
    torch.cuda.synchronize()
    p1 = out1[:, :, :nev].cpu().numpy()
    p2 = out2.cpu().numpy()
    q1, v1 = oracle.generate(M, m, nev, seed=42)
    assert_events_close(p1, w1.cpu().numpy(), q1, v1)
    q2, v2 = oracle.generate(m[0], [0.0, 0.0, 0.0], nev, seed=42, stream_id=1, parent_soa=np.ascontiguousarray(q1[0]))
    assert_events_close(p2, w2.cpu().numpy(), q2, v2)
    assert np.all(np.abs(p2.sum(axis=0) - p1[0]) <= 1e-12 * np.abs(p1[0]).max())


CHAIN_CASES = [  # (M, first-stage masses, chained daughter, second-stage masses)
    (5.279, [3.097, 0.4937, 0.13957], 0, [0.1056583755, 0.1056583755]),
    (5.279, [3.097, 0.4937, 0.13957], 0, [0.13957, 0.13957, 0.13957]),
    (5.279, [3.097, 0.4937, 0.13957], 1, [0.13957, 0.13957]),
    (10.0, [0.13957, 1.5, 0.13957, 0.13957, 0.13957, 0.13957], 1, [0.13957, 0.13957, 0.13957, 0.13957]),
    (10.0, [0.0] * 9 + [2.0], 9, [0.0, 0.0, 0.0]),
    (4.0, [1.0, 2.0], 1, [0.5, 0.6, 0.1, 0.2]),
]


def _chain_reference(P, M, m, d, m2, nev, seed, off):
    """The two single-channel calls the fused launch is defined by."""
    ld = P.aligned_ld(nev)
    o1 = torch.empty((len(m), 4, ld), dtype=torch.float64, device="cuda")
    w1 = torch.empty(nev, dtype=torch.float64, device="cuda")
    _, _, s1 = P.generate(M, m, nev, seed=seed, stream_id=3, event_offset=off, out=o1, weights=w1)
    o2, w2, s2 = P.generate(m[d], m2, nev, seed=seed, stream_id=8, event_offset=off, parent_dev=o1[d])
    torch.cuda.synchronize()
    return (o1[:, :, :nev].cpu().numpy(), w1.cpu().numpy(), s1.cpu().numpy(), o2.cpu().numpy(),
            w2.cpu().numpy(), s2.cpu().numpy())


@pytest.mark.parametrize("case", range(len(CHAIN_CASES)))
def test_chain_in_one_launch_equals_two_calls(P, case):
    """The fused two-stage launch against the two calls it is defined by: both
    stages' events and weights bit for bit, the integrals bit for bit when the
    calls run one event per thread (as the fused launch does) and to rounding at
    their defaults; the second stage against the oracle's chain."""
    M, m, d, m2 = CHAIN_CASES[case]
    _say(f"chain case {case}: N1={len(m)} chained {d} N2={len(m2)}")
    nev, seed, off = 100_003, 17 + case, 5_000_000_007
    r = P.generate_chain(M, m, d, m2, nev, seed=seed, stream_id=3, stream_id2=8, event_offset=off)
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in r]
    P.set_events_per_thread(1, 1)
    try:
        ref1 = _chain_reference(P, M, m, d, m2, nev, seed, off)
    finally:
        P.set_events_per_thread(1, 0)
    for g, e in zip(got, ref1):
        assert np.array_equal(g[..., :nev] if g.ndim == 3 else g, e)
    ref = _chain_reference(P, M, m, d, m2, nev, seed, off)
    for k in (0, 1, 3, 4):
        assert np.array_equal(got[k], ref[k])
    for k in (2, 5):
        assert got[k][0] == ref[k][0] and rel(got[k][1], ref[k][1]) <= 1e-13
        assert abs(got[k][3] - ref[k][3]) <= 1e-12 * ref[k][3] + 1e-15 * ref[k][1]  # two-body: sigma = 0
    q1, v1 = oracle.generate(M, m, nev, seed=seed, stream_id=3, event_offset=off)
    q2, v2 = oracle.generate(m[d], m2, nev, seed=seed, stream_id=8, event_offset=off,
                             parent_soa=np.ascontiguousarray(q1[d]))
    assert_events_close(got[0], got[1], q1, v1)
    assert_events_close(got[3], got[4], q2, v2)


@pytest.mark.parametrize("nev", [0, 1, 255, 257, 70_001])
def test_chain_edge_sizes(P, nev):
    """Empty, single-event and ragged launches of the one-launch chain: the
    two calls' events, weights and integrals bit for bit (one event per
    thread), and nothing written past nevents."""
    _say(f"chain edge size {nev}")
    M, m, d, m2 = CHAIN_CASES[1]
    ld = P.aligned_ld(nev)
    o1 = torch.full((3, 4, ld), float("nan"), dtype=torch.float64, device="cuda")
    o2 = torch.full((3, 4, ld), float("nan"), dtype=torch.float64, device="cuda")
    w1 = torch.full((ld,), float("nan"), dtype=torch.float64, device="cuda")
    w2 = torch.full((ld,), float("nan"), dtype=torch.float64, device="cuda")
    s1 = torch.empty(4, dtype=torch.float64, device="cuda")
    s2 = torch.empty(4, dtype=torch.float64, device="cuda")
    P.generate_chain(M, m, d, m2, nev, seed=9, stream_id=3, stream_id2=8, event_offset=123, out=o1, weights=w1,
                     stats=s1, out2=o2, weights2=w2, stats2=s2)
    torch.cuda.synchronize()
    assert int(s1[0].item()) == nev and int(s2[0].item()) == nev
    assert bool(torch.isnan(o1[:, :, nev:]).all()) and bool(torch.isnan(o2[:, :, nev:]).all())
    assert bool(torch.isnan(w1[nev:]).all()) and bool(torch.isnan(w2[nev:]).all())
    if nev == 0:
        return
    P.set_events_per_thread(1, 1)
    try:
        ref = _chain_reference(P, M, m, d, m2, nev, 9, 123)
    finally:
        P.set_events_per_thread(1, 0)
    got = [o1[:, :, :nev], w1[:nev], s1, o2[:, :, :nev], w2[:nev], s2]
    for g, e in zip(got, ref):
        assert np.array_equal(g.cpu().numpy(), e)


def test_chain_off_the_line_grid_runs_the_two_calls(P):
    """Columns that start mid-line (ld = n + 1): the library runs the two calls
    (staged kernels); the result is theirs, bit for bit."""
    _say("chain off the line grid")
    M, m, d, m2 = CHAIN_CASES[0]
    nev = 50_001
    o1 = torch.empty((3, 4, nev + 1), dtype=torch.float64, device="cuda")
    o2 = torch.empty((2, 4, nev + 1), dtype=torch.float64, device="cuda")
    r = P.generate_chain(M, m, d, m2, nev, seed=5, stream_id=3, stream_id2=8, out=o1, out2=o2)
    r1 = torch.empty_like(o1)
    r2 = torch.empty_like(o2)
    _, w1, s1 = P.generate(M, m, nev, seed=5, stream_id=3, out=r1)
    _, w2, s2 = P.generate(m[d], m2, nev, seed=5, stream_id=8, parent_dev=r1[d], out=r2)
    torch.cuda.synchronize()
    for g, e in zip([r[0][:, :, :nev], r[1], r[2], r[3][:, :, :nev], r[4], r[5]],
                    [r1[:, :, :nev], w1, s1, r2[:, :, :nev], w2, s2]):
        assert torch.equal(g, e)


@pytest.mark.parametrize("n", [2, 3, 6, 10])
@pytest.mark.parametrize("mixed", [False, True])
def test_line_aligned_and_staged_layouts_agree(P, n, mixed):
    """Outputs whose columns start mid-line take the staged kernel (whole-line
    writes through LDS): events, weights and stats must be bit-identical to the
    direct-store kernel on a line-aligned layout, for every events-per-thread
    setting, and nothing outside the events may be written."""
    _say(f"staged vs direct N={n} mixed={mixed}")
    M, m = _random_masses(n, 5000 + n)
    dtype = torch.float32 if mixed else torch.float64
    nev = 9_999
    ld_al = P.aligned_ld(nev)
    path = 2 if mixed else 1
    for ept in (1, 2, 4):
        P.set_events_per_thread(path, ept)
        try:
            a = torch.full((n, 4, ld_al), float("nan"), dtype=dtype, device="cuda")
            wa = torch.full((ld_al,), float("nan"), dtype=torch.float64, device="cuda")
            _, _, sa = P.generate(M, m, nev, seed=3, event_offset=77, out=a, weights=wa, mixed=mixed)
            # columns off the line grid: ld = nev + 3 and both buffers shifted by one element
            ld = nev + 3
            rawb = torch.full((n * 4 * ld + 1,), float("nan"), dtype=dtype, device="cuda")
            rawwb = torch.full((nev + 2,), float("nan"), dtype=torch.float64, device="cuda")
            b = rawb[1:].view(n, 4, ld)
            wb = rawwb[1:nev + 1]
            _, _, sb = P.generate(M, m, nev, seed=3, event_offset=77, out=b, weights=wb, mixed=mixed)
            torch.cuda.synchronize()
        finally:
            P.set_events_per_thread(path, 0)
        assert torch.equal(a[:, :, :nev], b[:, :, :nev]) and torch.equal(wa[:nev], wb), ept
        assert torch.equal(sa, sb), ept
        assert bool(torch.isnan(b[:, :, nev:]).all()) and bool(torch.isnan(rawb[:1]).all())
        assert bool(torch.isnan(rawwb[:1]).all()) and bool(torch.isnan(rawwb[nev + 1:]).all())


def test_two_body_sigma_is_exactly_zero(P):
    _say("two-body sigma")
    p4, w, st = _run(P, 5.279, [3.097, 0.4937], 70_001)
    assert np.all(w == w[0])
    assert st[2] == 0.0 and st[3] == 0.0 and st[1] == w[0]
    mean, sigma = P.integrate(5.279, [3.097, 0.4937], 70_001)
    assert sigma == 0.0 and mean == w[0]
    wo = oracle.generate(5.279, [3.097, 0.4937], 10, seed=42, want_momenta=False)[1]
    assert rel(w[0], wo[0]) <= FP64_TOL


@pytest.mark.parametrize("nev", [0, 1, 2, 63, 64, 65, 255, 256, 257, 511, 513, 1023, 1025])
def test_edge_sizes(P, nev):
    _say(f"edge size {nev}")
    M, m = CFG0
    p4, w, st = _run(P, M, m, nev, offset=31)
    assert st[0] == nev
    if nev == 0:
        assert st[1] == 0.0 and st[3] == 0.0
        return
    p4o, wo = oracle.generate(M, m, nev, seed=42, event_offset=31)
    assert_events_close(p4, w, p4o, wo)
    assert rel(st[1], float(np.mean(wo))) <= 1e-13
    if nev >= 2:
        mo, so = oracle.integrate(M, m, nev, seed=42, event_offset=31)
        assert rel(st[1], mo) <= FP64_TOL and rel(st[3], so) <= FP64_TOL
    else:
        assert st[3] == 0.0 and st[1] == w[0]


def test_padding_beyond_nevents_untouched(P):
    _say("ld padding")
    M, m = CFG0
    nev, ld = 1000, 1536
    out = torch.full((3, 4, ld), float("nan"), dtype=torch.float64, device="cuda")
    wt = torch.full((ld,), float("nan"), dtype=torch.float64, device="cuda")
    P.generate(M, m, nev, out=out, weights=wt)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(np.isfinite(o[:, :, :nev])) and np.all(np.isnan(o[:, :, nev:]))
    ww = wt.cpu().numpy()
    assert np.all(np.isfinite(ww[:nev])) and np.all(np.isnan(ww[nev:]))


def test_determinism_and_chunking(P):
    _say("determinism")
    M, m = CFG0
    p4a, wa, sa = _run(P, M, m, 300_000)
    p4b, wb, sb = _run(P, M, m, 300_000)
    assert np.array_equal(p4a, p4b) and np.array_equal(wa, wb) and np.array_equal(sa, sb)
    p41, w1, _ = _run(P, M, m, 123_457, offset=0)
    p42, w2, _ = _run(P, M, m, 300_000 - 123_457, offset=123_457)
    assert np.array_equal(np.concatenate([p41, p42], axis=2), p4a)
    assert np.array_equal(np.concatenate([w1, w2]), wa)


def test_integral_resumed_in_pieces(P):
    """A job integrated in pieces (event_offset ranges of one seed and stream,
    as a resumed job or shards on several devices would take them), its
    statistics merged left to right with hydra_phsp_stats_merge: the same n,
    the mean and sigma of the single call up to rounding, and both within the
    FP64 tolerance of the oracle."""
    _say("integral resumed in pieces")
    M, m = CFG0
    n = 3_000_017
    cuts = [0, 1_000_000, 1_000_001, 2_345_678, n]
    whole = P.integrate_async(M, m, n, seed=19, stream_id=4).cpu().tolist()
    acc = [0.0, 0.0, 0.0, 0.0]
    for a, b in zip(cuts[:-1], cuts[1:]):
        acc = P.stats_merge(acc, P.integrate_async(M, m, b - a, seed=19, stream_id=4, event_offset=a))
    assert acc[0] == whole[0] == n
    assert rel(acc[1], whole[1]) <= 1e-13 and rel(acc[3], whole[3]) <= 1e-12
    mo, so = oracle.integrate(M, m, n, seed=19, stream_id=4)
    assert rel(acc[1], mo) <= FP64_TOL and rel(acc[3], so) <= FP64_TOL


def test_near_threshold(P):
    _say("near threshold")
    m = [0.13957, 0.13957, 0.13957, 0.4937]
    M = sum(m) * (1.0 + 1e-7)
    p4, w, st = _run(P, M, m, 20_000)
    p4o, wo = oracle.generate(M, m, 20_000, seed=42)
    assert_events_close(p4, w, p4o, wo)


def test_non_default_stream(P):
    _say("side stream")
    M, m = CFG0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out, w, st = P.generate(M, m, 5000, seed=3)
    s.synchronize()
    p4o, wo = oracle.generate(M, m, 5000, seed=3)
    assert_events_close(out.cpu().numpy(), w.cpu().numpy(), p4o, wo)


MIXED_CASES = [(3, 5.279, [3.097, 0.4937, 0.13957]), (6, 10.0, [0.13957] * 6),
               (10, 10.0, [0.13957] * 10), (6, 10.0, [0.0] * 6), (3, 1.0, [0.0] * 3)]


@pytest.mark.parametrize("n,M,masses", MIXED_CASES)
def test_mixed_precision(P, n, M, masses):
    _say(f"mixed N={n} m={masses[0]}")
    nev = 200_000
    p4, w, st = _run(P, M, masses, nev, mixed=True)
    # FP64 prologue: weights are bit-identical to the FP64 path, and so is the
    # integral when both run the same launch shape (the reduction tree follows
    # the block partials)
    P.set_events_per_thread(1, 4)
    P.set_events_per_thread(2, 4)
    try:
        _, wm4, sm4 = _run(P, M, masses, nev, mixed=True)
        p4d, wd, sd = _run(P, M, masses, nev)
    finally:
        P.set_events_per_thread(1, 0)
        P.set_events_per_thread(2, 0)
    assert np.array_equal(w, wd) and np.array_equal(wm4, wd) and np.array_equal(sm4, sd)
    assert rel(st[1], sd[1]) <= 1e-13
    # the FP32 momenta are the FP64 path's momenta rounded once
    assert np.array_equal(p4, p4d.astype(np.float32))
    p4o, wo = oracle.generate(M, masses, nev, seed=42)
    rep = mixed_error_report(p4, p4o, M)
    _say(f"mixed N={n} m={masses[0]}: {rep}")
    assert rep["max_rel_E"] <= MIXED_TOL, rep
    mo, so = oracle.integrate(M, masses, nev, seed=42)
    assert rel(st[1], mo) <= MIXED_INTEGRAL_TOL


# ------------------------------------------------------------ full sizes ----

def _sample_indices(nev, k=1500, seed=0):
    rng = np.random.default_rng(seed)
    idx = np.concatenate([np.arange(min(500, nev)), np.arange(max(nev - 500, 0), nev),
                          rng.integers(0, nev, size=k)])
    return np.unique(idx)


def _check_samples(P, out, w, M, m, idx, seed=42, parent_soa=None, tol=FP64_TOL):
    n = len(m)
    ti = torch.as_tensor(idx, device="cuda")
    g = out[:, :, ti].cpu().numpy()
    gw = w[ti].cpu().numpy()
    worst = np.zeros(n)
    for j, e in enumerate(idx):
        ps = None if parent_soa is None else parent_soa[:, j:j + 1]
        p4o, wo = oracle.generate(M, m, 1, seed=seed, event_offset=int(e), parent_soa=ps)
        err = event_errors(g[:, :, j:j + 1], p4o)
        worst = np.maximum(worst, err)
        assert abs(gw[j] - wo[0]) <= FP64_TOL * wo[0], (e, gw[j], wo[0])
    assert np.all(worst <= tol), worst
    return worst


def test_full_size_config1_at_rest(P):
    _say("config1 1e8 at rest")
    M, m = CFG0
    nev = 100_000_000
    out, w, st = P.generate(M, m, nev)
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    assert s[0] == nev
    _check_samples(P, out, w, M, m, _sample_indices(nev))
    # the full integral against the quadrature volume, and against a chunked run
    import volumes
    exact = volumes.three_body_volume_1d(M, *m)
    assert abs(s[1] - exact) < 4 * s[3], (s, exact)
    wsum = torch.sum(w).item()
    assert rel(s[1], wsum / nev) <= 1e-12
    del out
    # integrate-only at 1e7 against the oracle's compensated two-pass integral
    mean, sigma = P.integrate(M, m, 10_000_000)
    mo, so = oracle.integrate(M, m, 10_000_000, seed=42)
    assert rel(mean, mo) <= FP64_TOL and rel(sigma, so) <= FP64_TOL


def test_integral_at_full_size_against_oracle(P):
    """The fused reduction's merge tree (per-lane Welford, wave and block trees,
    two-stage merge of the block partials) against the oracle's compensated
    two-pass integral over the same 1e8 weights: mean and sigma within 1e-11
    relative (pairwise merging keeps the rounding error near log2(n) ulp).  The
    mixed path's weights and integral are the FP64 path's bit for bit (checked
    in test_full_size_config2), so this covers both."""
    M, m = CFG0
    nev = 100_000_000
    _say("integral of 1e8 events: generate (stats), integrate-only, oracle")
    w = torch.empty(nev, dtype=torch.float64, device="cuda")
    out = torch.empty((3, 4, P.aligned_ld(nev)), dtype=torch.float64, device="cuda")
    _, _, st = P.generate(M, m, nev, out=out, weights=w)
    torch.cuda.synchronize()
    del out, w
    s = st.cpu().numpy()
    mean_i, sigma_i = P.integrate(M, m, nev)
    mo, so = oracle.integrate(M, m, nev, seed=42)
    _say(f"1e8 integral: generate mean rel err {rel(s[1], mo):.3e}, sigma {rel(s[3], so):.3e}; "
         f"integrate-only mean {rel(mean_i, mo):.3e}, sigma {rel(sigma_i, so):.3e}")
    assert s[0] == nev
    assert rel(s[1], mo) <= FP64_TOL and rel(s[3], so) <= FP64_TOL
    assert rel(mean_i, mo) <= FP64_TOL and rel(sigma_i, so) <= FP64_TOL


def test_integrate_largest_single_launch(P):
    """The largest count one integrate launch takes ((2^32 - 1) / 256 blocks of
    1024 events, 1.7e10 events): every block counted, the volume within 5 sigma
    of the quadrature; one more event is refused."""
    import volumes
    M, m = CFG0
    nmax = (0xFFFFFFFF // 256) * 1024
    _say(f"integrate {nmax} events in one launch")
    assert P.events_per_thread(0, 3) == 4
    st = P.integrate_async(M, m, nmax, seed=7)
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    assert s[0] == nmax
    exact = volumes.three_body_volume_1d(M, *m)
    assert abs(s[1] - exact) < 5 * s[3] and 0 < s[3] < 1e-5 * exact, (s, exact)
    with pytest.raises(P.PhspError):
        P.integrate_async(M, m, nmax + 1, seed=7)


def test_full_size_config1_per_event_parent(P):
    _say("config1 1e8 per-event parents")
    from paper_1711_05683_amd.workloads import per_event_parents
    M, m = CFG0
    nev = 100_000_000
    parents = per_event_parents(M, nev)
    out, w, st = P.generate(M, m, nev, parent_dev=parents)
    torch.cuda.synchronize()
    idx = _sample_indices(nev, seed=1)
    soa = parents[:, torch.as_tensor(idx, device="cuda")].cpu().numpy()
    _check_samples(P, out, w, M, m, idx, parent_soa=soa)
    # weights do not depend on the parent's motion
    w_rest = torch.empty(nev, dtype=torch.float64, device="cuda")
    o2 = torch.empty((3, 4, nev), dtype=torch.float64, device="cuda")
    del out
    P.generate(M, m, nev, out=o2, weights=w_rest)
    torch.cuda.synchronize()
    assert torch.equal(w, w_rest)


@pytest.mark.parametrize("masses", [[0.13957] * 6, [0.0] * 6])
def test_full_size_config2(P, masses):
    _say(f"config2 5e7 N=6 masses={masses[0]}")
    M = 10.0
    nev = 50_000_000
    out, w, st = P.generate(M, masses, nev)
    torch.cuda.synchronize()
    idx = _sample_indices(nev, k=800, seed=2)
    _check_samples(P, out, w, M, masses, idx)
    ti = torch.as_tensor(idx, device="cuda")
    g64 = out[:, :, ti].cpu().numpy()
    del out
    outm, wm, stm = P.generate(M, masses, nev, mixed=True)
    torch.cuda.synchronize()
    assert torch.equal(w, wm) and torch.equal(st, stm)
    g = outm[:, :, ti].cpu().numpy()
    assert np.array_equal(g, g64.astype(np.float32))
    ora = np.concatenate([oracle.generate(M, masses, 1, seed=42, event_offset=int(e))[0] for e in idx],
                         axis=2)
    rep = mixed_error_report(g, ora, M)
    _say(f"config2 mixed sampled errors: {rep}")
    assert rep["max_rel_E"] <= MIXED_TOL, rep


@pytest.mark.parametrize("mixed", [False, True])
def test_events_per_thread_variants_are_bit_identical(P, mixed):
    _say(f"ept variants mixed={mixed}")
    M, m = 10.0, [0.13957] * 5
    nev = 77_777
    ref = None
    path = 2 if mixed else 1
    try:
        for ept in (1, 2, 4):
            P.set_events_per_thread(path, ept)
            P.set_events_per_thread(0, ept)
            p4, w, st = _run(P, M, m, nev, offset=5, mixed=mixed)
            mean, sigma = P.integrate(M, m, nev, event_offset=5)
            if ref is None:
                ref = (p4, w, st, mean, sigma)
                continue
            assert np.array_equal(p4, ref[0]) and np.array_equal(w, ref[1])
            assert rel(st[1], ref[2][1]) <= 1e-14 and rel(st[3], ref[2][3]) <= 1e-13
            assert rel(mean, ref[3]) <= 1e-14 and rel(sigma, ref[4]) <= 1e-13
    finally:
        P.set_events_per_thread(path, 0)
        P.set_events_per_thread(0, 0)


def test_threads_on_separate_streams(P):
    """Six host threads, each on its own stream, call generate, integrate,
    unweighted generation and model evaluation at once (the calls release the
    interpreter lock): every result equals the same call made alone."""
    import threading
    _say("six threads, six streams")
    M, m = CFG0
    res = [(1, 2, 0.8955, 0.0473)]

    def calls(i, stream):
        out, w, st = P.generate(M, m, 200_003 + 17 * i, seed=100 + i, stream=stream)
        st2 = P.integrate_async(M, m, 300_007 + i, seed=200 + i, stream=stream)
        p4u, idx, cnt, _ = P.generate_unweighted(M, m, 100_003, seed=300 + i, want_index=True, stream=stream)
        stm, vals = P.integrate_model(M, m, 150_001, res, seed=400 + i, want_values=True, stream=stream)
        return out, w, st, st2, p4u, idx, cnt, stm, vals

    def host(r):
        return [t.cpu() for t in r]

    results, errors = [None] * 6, []

    def work(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                r = calls(i, s)
            s.synchronize()
            results[i] = host(r)
        except Exception as e:  # reported by the main thread
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(6)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    assert all(not t.is_alive() for t in threads)
    for i in range(6):
        want = host(calls(i, None))
        got = results[i]
        k = int(want[6][0])  # kept events: the unweighted outputs beyond them are unset
        assert torch.equal(got[6], want[6]), i
        got[4], want[4] = got[4][:, :, :k], want[4][:, :, :k]
        got[5], want[5] = got[5][:k], want[5][:k]
        for j, (a, b) in enumerate(zip(got, want)):
            assert torch.equal(a, b), (i, j)


def test_binding_rejects_host_short_and_foreign_buffers(P):
    """With a GPU present the binding still refuses buffers the kernels could not
    use: host memory, too few elements, another device than the launch one."""
    _say("binding buffer checks")
    M, m = 5.279, [3.097, 0.4937, 0.13957]
    dev = torch.device("cuda", torch.cuda.current_device())
    with pytest.raises(ValueError, match="CUDA"):
        P.generate(M, m, 100, weights=torch.zeros(100, dtype=torch.float64))
    with pytest.raises(ValueError, match="weights"):
        P.generate(M, m, 100, weights=torch.zeros(99, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError, match="stats"):
        P.integrate_async(M, m, 100, stats=torch.zeros(3, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError, match="counts"):
        P.generate_unweighted(M, m, 100, counts=torch.zeros(1, dtype=torch.int64, device=dev))
    with pytest.raises(ValueError, match="device"):
        P.generate(M, m, 100, device=f"cuda:{dev.index + 1}")
    out, w, st = P.generate(M, m, 100, device=dev)  # the current device is accepted
    torch.cuda.synchronize()
    assert out.shape == (3, 4, 100) and torch.isfinite(w).all()
