"""GPU tests of the continuous-batching server: each request's result is the same
alone and in a mix of concurrently running requests, the HBM budget bounds the
memory held and forces queuing, invalid requests fail alone, and the native
arrival replay reports sane latencies."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from parity import FP64_TOL, assert_events_close, rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[serve]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()
    oracle.build(force=False)
    return P


def _requests(n=40, seed=5683, log_events=(3.0, 5.0)):
    from paper_1711_05683_amd.workloads import serving_requests
    reqs = serving_requests(rate_hz=2000.0, duration_s=1.0, seed=seed, log_events=log_events)[:n]
    return reqs


def _desc(P, r):
    return P.request(r.parent_mass, r.masses, r.nevents, seed=r.seed, stream_id=r.stream_id,
                     integrate_only=r.integrate_only)


def _collect(P, srv, rid, r):
    res = srv.poll(rid)
    assert res is not None and res.status == 0
    out = w = None
    if not r.integrate_only:
        n = len(r.masses)
        out = P.device_view(res.p4_dev, (n, 4, r.nevents)).cpu()
        w = P.device_view(res.weights_dev, (r.nevents,)).cpu()
    return out, w, res.mean, res.sigma


def test_results_identical_alone_and_in_mix(P):
    reqs = _requests()
    _say(f"{len(reqs)} requests, {sum(r.nevents for r in reqs)} events")
    srv = P.Server(8 << 30, max_events_per_tick=1 << 18)
    ids = []
    # arrivals interleaved with scheduling steps: later requests join running ticks
    for k, r in enumerate(reqs):
        ids.append(srv.submit(_desc(P, r)))
        if k % 3 == 0:
            srv.step()
    srv.drain()
    mixed = [_collect(P, srv, rid, r) for rid, r in zip(ids, reqs)]
    st = srv.stats()
    _say(f"mix: {st}")
    assert st["ticks"] > 1
    for rid in ids:
        srv.release(rid)
    assert srv.stats()["bytes_in_use"] == 0
    srv.destroy()
    for k, r in enumerate(reqs):
        alone = P.Server(1 << 30)
        rid = alone.submit(_desc(P, r))
        alone.drain()
        a = _collect(P, alone, rid, r)
        alone.release(rid)
        alone.destroy()
        m = mixed[k]
        if not r.integrate_only:
            assert torch.equal(a[0], m[0]) and torch.equal(a[1], m[1]), k
        assert a[2] == m[2] and a[3] == m[3], (k, a[2:], m[2:])


def test_server_matches_single_channel_and_oracle(P):
    reqs = _requests(n=12, seed=7)
    srv = P.Server(4 << 30)
    ids = [srv.submit(_desc(P, r)) for r in reqs]
    srv.drain()
    P.set_events_per_thread(0, 1)  # the server's tiles are 256 events
    P.set_events_per_thread(1, 1)
    try:
        for rid, r in zip(ids, reqs):
            out, w, mean, sigma = _collect(P, srv, rid, r)
            if r.integrate_only:
                s = P.integrate_async(r.parent_mass, r.masses, r.nevents, seed=r.seed,
                                      stream_id=r.stream_id).cpu().numpy()
            else:
                so, sw, s = P.generate(r.parent_mass, r.masses, r.nevents, seed=r.seed, stream_id=r.stream_id)
                torch.cuda.synchronize()
                assert torch.equal(so.cpu(), out) and torch.equal(sw.cpu(), w)
                s = s.cpu().numpy()
                k = min(r.nevents, 2000)
                p4o, wo = oracle.generate(r.parent_mass, r.masses, k, seed=r.seed, stream_id=r.stream_id)
                assert_events_close(out[:, :, :k].numpy(), w[:k].numpy(), p4o, wo)
            assert mean == s[1] and sigma == s[3]
            if r.nevents >= 2:
                mo, so_ = oracle.integrate(r.parent_mass, r.masses, r.nevents, seed=r.seed,
                                           stream_id=r.stream_id)
                assert rel(mean, mo) <= FP64_TOL
            srv.release(rid)
    finally:
        P.set_events_per_thread(0, 0)
        P.set_events_per_thread(1, 0)
    srv.destroy()


def test_tiny_budget_forces_queuing(P):
    reqs = [r for r in _requests(n=30, seed=11) if not r.integrate_only][:12]
    biggest = max(r.nevents * (4 * len(r.masses) + 1) * 8 + 24 * (r.nevents // 256 + 1) for r in reqs)
    budget = max(int(biggest * 1.6), 1 << 20)
    _say(f"budget {budget} bytes for {len(reqs)} requests")
    srv = P.Server(budget)
    ids = [srv.submit(_desc(P, r)) for r in reqs]
    done = {}
    while len(done) < len(ids):
        srv.step()
        for rid in srv.completed():
            done[rid] = True
            res = srv.poll(rid)
            assert res.status == 0
            srv.release(rid)
        assert srv.stats()["bytes_in_use"] <= budget
    st = srv.stats()
    assert st["peak_bytes"] <= budget and st["finished"] == len(ids)
    c = srv.counters()
    assert c["finished"] == len(ids) and c["ticks"] == st["ticks"] and c["peak_bytes"] == st["peak_bytes"]
    assert c["budget_stalls"] > 0 and c["active_stalls"] == 0  # requests waited for memory, never for a slot
    assert c["queue_wait_max_s"] > 0.0 and c["queue_wait_max_s"] * len(ids) >= c["queue_wait_sum_s"] >= 0.0
    srv.destroy()
    # one active slot: every request but the first waits for it
    srv = P.Server(8 << 30, max_active=1)
    ids = [srv.submit(_desc(P, r)) for r in reqs[:4]]
    srv.drain()
    c = srv.counters()
    assert c["finished"] == 4 and c["active_stalls"] > 0 and c["budget_stalls"] == 0
    srv.destroy()


def test_invalid_requests_fail_alone(P):
    srv = P.Server(1 << 30)
    good = P.request(5.279, [3.097, 0.4937, 0.13957], 5000, seed=1)
    rid = srv.submit(good)
    assert srv.submit_status(P.request(5.0, [3.0, 3.0], 100)) == P.EKINEMATICS
    assert srv.submit_status(P.request(5.0, [1.0], 100)) == P.EINVAL
    assert srv.submit_status(P.request(5.0, [1.0, 1.0], 0)) == P.EINVAL
    assert srv.submit_status(P.request(5.0, [1.0, 1.0], 10 ** 9)) == P.ENOMEM  # cannot fit the budget
    rid2 = srv.submit(good)
    srv.drain()
    a, b = srv.poll(rid), srv.poll(rid2)
    assert a.status == 0 and b.status == 0 and a.mean == b.mean and a.sigma == b.sigma
    with pytest.raises(P.PhspError):
        srv.poll(987654)
    srv.release(rid)
    srv.release(rid2)
    with pytest.raises(P.PhspError):
        srv.release(rid)
    srv.destroy()


def test_replay_short_trace(P):
    from paper_1711_05683_amd.workloads import serving_requests
    reqs = serving_requests(rate_hz=2000.0, duration_s=0.5, seed=5683)
    descs = [_desc(P, r) for r in reqs]
    arrivals = [r.arrival_s for r in reqs]
    srv = P.Server(16 << 30)
    lat, wall, peak = srv.replay(descs, arrivals)
    lat = np.array(lat)
    _say(f"replay {len(reqs)} requests: wall {wall:.3f} s, p50 {np.median(lat) * 1e3:.3f} ms, "
         f"p99 {np.quantile(lat, 0.99) * 1e3:.3f} ms, peak {peak} B")
    assert np.all(lat >= 0) and wall >= arrivals[-1]
    assert srv.stats()["bytes_in_use"] == 0
    srv.destroy()
