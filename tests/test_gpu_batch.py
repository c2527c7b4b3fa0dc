"""GPU tests of the batched persistent kernel: every channel of a batch must be
bit-identical to a single-channel call (events, weights, and -- with the same
events per thread -- the integral), graph replays must reproduce the eager
result, and sampled events must match the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from parity import FP64_TOL, assert_events_close, rel

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[batch]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()
    oracle.build(force=False)
    return P


def _channels(P, n_channels=24, seed=1711, log_events=(2.0, 4.5), integrate_every=5, nmax=8):
    from paper_1711_05683_amd.workloads import batched_channels
    specs = batched_channels(n_channels, seed=seed, nmax=nmax, log_events=log_events)
    # edge channels: empty, single event, ragged, two-body
    specs[0].nevents = 0
    specs[1].nevents = 1
    specs[2].nevents = 257
    specs[3].masses = specs[3].masses[:2]
    bufs, descs = [], []
    for i, c in enumerate(specs):
        integ = integrate_every and i % integrate_every == integrate_every - 1
        st = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        if integ:
            out = w = None
        else:
            out = torch.full((c.n, 4, max(c.nevents, 1)), float("nan"), dtype=torch.float64, device="cuda")
            w = torch.full((max(c.nevents, 1),), float("nan"), dtype=torch.float64, device="cuda")
        bufs.append((out, w, st))
        descs.append(P.channel(c.parent_mass, c.masses, c.nevents, seed=c.seed + i, stream_id=c.stream_id,
                               event_offset=1000 * i, out=out, weights=w, stats=st))
    return specs, bufs, descs


def _aligned_channels(P, n_channels, seed, nmax=10, integrate_every=4):
    """Channels whose columns start on 128-byte lines (ld = aligned_ld(n))."""
    from paper_1711_05683_amd.workloads import batched_channels
    specs = batched_channels(n_channels, seed=seed, nmax=nmax, log_events=(2.0, 4.5))
    specs[0].nevents = 0
    specs[1].nevents = 1
    specs[2].nevents = 257
    bufs, descs = [], []
    for i, c in enumerate(specs):
        integ = integrate_every and i % integrate_every == integrate_every - 1
        st = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        if integ:
            out = w = None
        else:
            out = torch.full((c.n, 4, P.aligned_ld(c.nevents)), float("nan"), dtype=torch.float64, device="cuda")
            w = torch.full((P.aligned_ld(c.nevents),), float("nan"), dtype=torch.float64, device="cuda")
        bufs.append((out, w, st))
        descs.append(P.channel(c.parent_mass, c.masses, c.nevents, seed=c.seed + i, stream_id=c.stream_id,
                               event_offset=1000 * i, out=out, weights=w, stats=st))
    return specs, bufs, descs


def _single(P, c, i, integ, ept=1, aligned=False):
    if integ:
        P.set_events_per_thread(0, ept)
        try:
            st = P.integrate_async(c.parent_mass, c.masses, c.nevents, seed=c.seed + i,
                                   stream_id=c.stream_id, event_offset=1000 * i)
        finally:
            P.set_events_per_thread(0, 0)
        return None, None, st
    P.set_events_per_thread(1, ept)
    try:
        # the batch channel's layout (ld = nevents, or aligned_ld), so that default
        # settings pick the same kernel
        ld = P.aligned_ld(c.nevents) if aligned else max(c.nevents, 1)
        out = torch.empty((len(c.masses), 4, ld), dtype=torch.float64, device="cuda")
        w = torch.empty(ld, dtype=torch.float64, device="cuda")
        out, w, st = P.generate(c.parent_mass, c.masses, c.nevents, seed=c.seed + i, stream_id=c.stream_id,
                                event_offset=1000 * i, out=out, weights=w)
    finally:
        P.set_events_per_thread(1, 0)
    return out, w, st


def _compare_with_single(P, specs, bufs, ept, exact_stats=True, aligned=False):
    for i, c in enumerate(specs):
        out, w, st = bufs[i]
        so, sw, sst = _single(P, c, i, out is None, ept, aligned)
        torch.cuda.synchronize()
        if out is not None and c.nevents > 0:
            assert torch.equal(out[:, :, :c.nevents], so[:, :, :c.nevents]), f"channel {i} momenta"
            assert torch.equal(w[:c.nevents], sw[:c.nevents]), f"channel {i} weights"
        a, b = st.cpu().numpy(), sst.cpu().numpy()
        if exact_stats:
            assert np.array_equal(a, b), (i, a, b)
        else:
            assert a[0] == b[0]
            assert rel(a[1], b[1]) <= 1e-14 if b[1] != 0 else a[1] == 0
            assert abs(a[3] - b[3]) <= 1e-13 * b[3] + 1e-15 * abs(b[1])


def test_batch_matches_single_channel(P):
    _say("batch vs single channel, ept 1")
    specs, bufs, descs = _channels(P)
    P.batch_run(descs, ept=1)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 1)


@pytest.mark.parametrize("ept,gpc,sched", [(2, 1, 0), (4, 16, 0), (1, 2, 0), (4, 8, 1), (1, 1, 1), (2, 16, 1),
                                            (1, 0, 2), (2, 0, 2), (4, 0, 2)])
def test_batch_tuning_variants(P, ept, gpc, sched):
    _say(f"batch variant ept={ept} grid/cu={gpc} schedule={sched}")
    specs, bufs, descs = _channels(P, n_channels=16, seed=7)
    P.batch_run(descs, ept=ept, grid_per_cu=gpc, schedule=sched)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, ept)


@pytest.mark.parametrize("streams,sched", [(2, 2), (3, 2), (4, 2), (4, 0), (3, 1)])
def test_batch_class_streams(P, streams, sched):
    """Class kernels spread over several streams: the same events, weights and
    integrals as single-channel calls (every class of N up to 10, both modes)."""
    _say(f"batch classes over {streams} streams, schedule={sched}")
    specs, bufs, descs = _channels(P, n_channels=24, seed=41 + streams, nmax=10, integrate_every=4)
    P.batch_run(descs, schedule=sched, grid_per_cu=0 if sched == 2 else 4, streams=streams)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 0)


def test_plan_graph_with_class_streams(P):
    """A plan whose class kernels sit on parallel graph branches replays to the
    eager one-stream result, with eager work between replays."""
    _say("graph replays, classes over 3 streams")
    specs, bufs, descs = _channels(P, n_channels=16, seed=13, nmax=10)
    P.batch_run(descs, streams=1)
    torch.cuda.synchronize()
    ref = [(None if o is None else o.clone(), None if w is None else w.clone(), s.clone()) for o, w, s in bufs]
    plan = P.Plan(descs, streams=3)
    for rep in range(3):
        for o, w, s in bufs:
            if o is not None:
                o.fill_(float("nan"))
                w.fill_(float("nan"))
            s.fill_(float("nan"))
        P.integrate_async(5.279, [3.097, 0.4937, 0.13957], 100_000, seed=rep)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for i, (o, w, s) in enumerate(bufs):
            ro, rw, rs = ref[i]
            n = specs[i].nevents
            if o is not None:
                assert torch.equal(o[:, :, :n], ro[:, :, :n]) and torch.equal(w[:n], rw[:n]), (rep, i)
            assert torch.equal(s, rs), (rep, i)
    plan.destroy()


def test_batch_single_launch(P):
    """Schedule 3: every tile of every channel (N up to 10, generate and
    integrate-only) in one launch, one block per tile -- the events, weights and
    integrals of single-channel calls with default settings (ept 0) or at one
    event per thread (ept 1)."""
    _say("batch single launch, N up to 10")
    specs, bufs, descs = _aligned_channels(P, 24, seed=57)
    P.batch_run(descs, schedule=3)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 0, aligned=True)
    specs, bufs, descs = _aligned_channels(P, 12, seed=58, nmax=8, integrate_every=3)
    P.batch_run(descs, schedule=3, ept=1)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 1)


def test_plan_graph_single_launch(P):
    """A single-launch plan replays to its eager result with other work between."""
    _say("graph replays, single launch")
    specs, bufs, descs = _aligned_channels(P, 16, seed=59)
    P.batch_run(descs, schedule=3)
    torch.cuda.synchronize()
    ref = [(None if o is None else o.clone(), None if w is None else w.clone(), s.clone()) for o, w, s in bufs]
    plan = P.Plan(descs, schedule=3)
    ntiles, grid = plan.info()
    assert grid == ntiles > 0
    for rep in range(3):
        for o, w, s in bufs:
            if o is not None:
                o.fill_(float("nan"))
                w.fill_(float("nan"))
            s.fill_(float("nan"))
        P.integrate_async(5.279, [3.097, 0.4937, 0.13957], 100_000, seed=rep)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for i, (o, w, s) in enumerate(bufs):
            ro, rw, rs = ref[i]
            n = specs[i].nevents
            if o is not None:
                assert torch.equal(o[:, :, :n], ro[:, :, :n]) and torch.equal(w[:n], rw[:n]), (rep, i)
            assert torch.equal(s, rs), (rep, i)
    plan.destroy()


@pytest.mark.parametrize("sched,gpc", [(4, 1), (4, 4), (5, 1), (5, 4)])
def test_batch_single_persistent_launch(P, sched, gpc):
    """Schedules 4 and 5: one persistent launch over every tile (N up to 10,
    then up to 8; generate and integrate-only), blocks taking tiles with a
    static stride or claiming them from a counter -- events, weights and
    integrals bit-identical to single-channel calls with default settings on
    the same layout, or at one event per thread."""
    _say(f"batch single persistent launch, schedule {sched}, {gpc} block(s) per CU, N up to 10")
    specs, bufs, descs = _aligned_channels(P, 24, seed=61)
    P.batch_run(descs, schedule=sched, grid_per_cu=gpc)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 0, aligned=True)
    _say(f"batch single persistent launch, schedule {sched}, {gpc} block(s) per CU, N up to 8, ept 1")
    specs, bufs, descs = _aligned_channels(P, 12, seed=62, nmax=8, integrate_every=3)
    P.batch_run(descs, schedule=sched, grid_per_cu=gpc, ept=1)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 1)


def test_batch_single_persistent_launch_ignores_ept_override(P):
    """The single launches run their compiled per-N defaults even while the
    host's events-per-thread setting is overridden."""
    _say("batch single persistent launch under an events-per-thread override")
    specs, bufs, descs = _aligned_channels(P, 12, seed=63, nmax=8, integrate_every=3)
    for sched in (3, 4, 5):
        P.set_events_per_thread(0, 1)
        P.set_events_per_thread(1, 1)
        try:
            P.batch_run(descs, schedule=sched)
            torch.cuda.synchronize()
        finally:
            P.set_events_per_thread(0, 0)
            P.set_events_per_thread(1, 0)
        _compare_with_single(P, specs, bufs, 0, aligned=True)


@pytest.mark.parametrize("sched", [4, 5])
def test_plan_graph_single_persistent_launch(P, sched):
    """A persistent single-launch plan (schedule 5: its tile counter reset by a
    kernel in the graph) replays to its eager result with other work between
    replays."""
    _say(f"graph replays, single persistent launch, schedule {sched}")
    specs, bufs, descs = _aligned_channels(P, 16, seed=64)
    P.batch_run(descs, schedule=sched, grid_per_cu=2)
    torch.cuda.synchronize()
    ref = [(None if o is None else o.clone(), None if w is None else w.clone(), s.clone()) for o, w, s in bufs]
    plan = P.Plan(descs, schedule=sched, grid_per_cu=2)
    ntiles, grid = plan.info()
    assert 0 < grid <= ntiles
    for rep in range(4):
        for o, w, s in bufs:
            if o is not None:
                o.fill_(float("nan"))
                w.fill_(float("nan"))
            s.fill_(float("nan"))
        P.integrate_async(5.279, [3.097, 0.4937, 0.13957], 100_000, seed=rep)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for i, (o, w, s) in enumerate(bufs):
            ro, rw, rs = ref[i]
            n = specs[i].nevents
            if o is not None:
                assert torch.equal(o[:, :, :n], ro[:, :, :n]) and torch.equal(w[:n], rw[:n]), (rep, i)
            assert torch.equal(s, rs), (rep, i)
    plan.destroy()


def test_batch_default_shape_matches_single_channel_defaults(P):
    _say("batch ept 0 (per class) vs single-channel defaults, N up to 10, both modes")
    specs, bufs, descs = _channels(P, n_channels=24, seed=31, nmax=10, integrate_every=4)
    P.batch_run(descs)  # ept 0: every class takes its single-channel setting
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 0)


def test_batch_with_ten_body_channels(P):
    _say("batch with N up to 10")
    specs, bufs, descs = _channels(P, n_channels=12, seed=99, nmax=10)
    P.batch_run(descs, ept=1)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, 1)


def test_batch_against_oracle(P):
    _say("batch vs oracle")
    specs, bufs, descs = _channels(P, n_channels=10, seed=3, integrate_every=0)
    P.batch_run(descs)
    torch.cuda.synchronize()
    for i, c in enumerate(specs):
        if c.nevents == 0:
            continue
        out, w, st = bufs[i]
        k = min(c.nevents, 3000)
        p4o, wo = oracle.generate(c.parent_mass, c.masses, k, seed=c.seed + i, stream_id=c.stream_id,
                                  event_offset=1000 * i)
        assert_events_close(out[:, :, :k].cpu().numpy(), w[:k].cpu().numpy(), p4o, wo)
        if c.nevents >= 2:
            mo, so = oracle.integrate(c.parent_mass, c.masses, c.nevents, seed=c.seed + i,
                                      stream_id=c.stream_id, event_offset=1000 * i)
            s = st.cpu().numpy()
            assert rel(s[1], mo) <= FP64_TOL and abs(s[3] - so) <= FP64_TOL * so + 1e-15 * mo


def test_plan_graph_replays(P):
    _say("graph replays")
    specs, bufs, descs = _channels(P, n_channels=12, seed=11)
    P.batch_run(descs, ept=1)
    torch.cuda.synchronize()
    ref = [(None if o is None else o.clone(), None if w is None else w.clone(), s.clone()) for o, w, s in bufs]
    plan = P.Plan(descs, ept=1)
    ntiles, grid = plan.info()
    assert ntiles > 0 and grid > 0
    other = torch.empty((3, 4, 5000), dtype=torch.float64, device="cuda")
    for rep in range(4):
        # eager work between replays: clobber every output, run unrelated kernels
        for o, w, s in bufs:
            if o is not None:
                o.fill_(float("nan"))
                w.fill_(float("nan"))
            s.fill_(float("nan"))
        P.generate(5.279, [3.097, 0.4937, 0.13957], 5000, out=other, seed=rep)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for i, (o, w, s) in enumerate(bufs):
            ro, rw, rs = ref[i]
            n = specs[i].nevents
            if o is not None:
                assert torch.equal(o[:, :, :n], ro[:, :, :n]) and torch.equal(w[:n], rw[:n]), (rep, i)
            assert torch.equal(s, rs), (rep, i)
    plan.destroy()


def test_autotune(P):
    _say("autotune")
    specs, bufs, descs = _channels(P, n_channels=16, seed=5, log_events=(3.0, 5.0))
    ept, gpc, sched, nstr, ms = P.autotune(descs)
    assert ept in (0, 1, 2, 4) and sched in (0, 1, 2) and nstr in (0, 1, 2, 3, 4) and ms > 0
    assert (gpc == 0) if sched == 2 else (1 <= gpc <= 16)
    # cached: same answer
    assert P.autotune(descs) == (ept, gpc, sched, nstr, ms)
    # the tuned shape still gives the single-channel events
    P.batch_run(descs, ept=ept, grid_per_cu=gpc, schedule=sched, streams=nstr)
    torch.cuda.synchronize()
    _compare_with_single(P, specs, bufs, ept)


def test_autotune_file_cache(P, tmp_path, monkeypatch):
    """HYDRA_PHSP_TUNE_CACHE: a sweep's answer is appended to the file, and a
    line written for another shape class is returned without a sweep."""
    import math
    _say("autotune file cache")
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("HYDRA_PHSP_TUNE_CACHE", str(path))
    _, _, descs = _channels(P, n_channels=7, seed=77, log_events=(3.0, 4.0))
    ept, gpc, sched, nstr, ms = P.autotune(descs)
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert f[:2] == ["hydra_phsp_tune", "1"] and f[3] == "7"
    assert [int(x) for x in f[8:12]] == [ept, gpc, sched, nstr] and abs(float(f[12]) - ms) <= 1e-8 * ms
    # another shape class (nine channels): its key, as the library forms it
    _, _, descs2 = _channels(P, n_channels=9, seed=78, log_events=(3.0, 4.0))
    nmax = max(d.n_daughters for d in descs2)
    integ = sum(1 for d in descs2 if not d.p4_out_dev)
    staged = sum(1 for d in descs2 if d.p4_out_dev and not (d.p4_out_dev % 128 == 0 and (d.ld * 8) % 128 == 0
                                                          and d.weights_dev % 128 == 0))
    bucket = math.floor(4.0 * math.log2(sum(d.nevents for d in descs2) + 1.0) + 0.5)
    with open(path, "a") as fh:
        fh.write(f"hydra_phsp_tune 1 {f[2]} 9 {nmax} {integ} {staged} {bucket} 2 3 1 2 0.123\n")
    assert P.autotune(descs2) == (2, 3, 1, 2, 0.123)
    assert len(path.read_text().splitlines()) == 2  # nothing appended: no sweep ran


def test_config3_full_batch(P):
    _say("config3: 64 channels, one persistent launch")
    from paper_1711_05683_amd.workloads import batched_channels
    specs = batched_channels()
    total = sum(c.nevents for c in specs)
    _say(f"config3 total events {total}")
    bufs, descs = [], []
    for c in specs:
        out = torch.empty((c.n, 4, c.nevents), dtype=torch.float64, device="cuda")
        w = torch.empty(c.nevents, dtype=torch.float64, device="cuda")
        st = torch.empty(4, dtype=torch.float64, device="cuda")
        bufs.append((out, w, st))
        descs.append(P.channel(c.parent_mass, c.masses, c.nevents, seed=c.seed, stream_id=c.stream_id,
                               out=out, weights=w, stats=st))
    plan = P.Plan(descs)  # default shape: each class as its single-channel launch
    plan.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for i in rng.choice(len(specs), size=6, replace=False):
        c = specs[i]
        out, w, st = bufs[i]
        idx = np.unique(np.concatenate([[0, c.nevents - 1], rng.integers(0, c.nevents, 200)]))
        ti = torch.as_tensor(idx, device="cuda")
        g = out[:, :, ti].cpu().numpy()
        gw = w[ti].cpu().numpy()
        for j, e in enumerate(idx):
            p4o, wo = oracle.generate(c.parent_mass, c.masses, 1, seed=c.seed, stream_id=c.stream_id,
                                      event_offset=int(e))
            assert_events_close(g[:, :, j:j + 1], gw[j:j + 1], p4o, wo)
        # a single-channel call on the same layout (ld = nevents) takes the same kernel and shape
        so = torch.empty_like(out)
        sw = torch.empty_like(w)
        so, sw, sst = P.generate(c.parent_mass, c.masses, c.nevents, seed=c.seed, stream_id=c.stream_id,
                                 out=so, weights=sw)
        torch.cuda.synchronize()
        assert torch.equal(so, out) and torch.equal(sw, w) and torch.equal(sst, st), i
        del so, sw
    plan.destroy()


def test_config3_single_persistent_launch(P):
    """The 64-channel workload on line-aligned columns as one launch (schedules
    3, 4 and 5 at their defaults): every channel's integral bit-identical to the
    per-class launches at default settings, sampled events against the oracle."""
    _say("config3: 64 channels, single persistent launch")
    from paper_1711_05683_amd.workloads import batched_channels
    specs = batched_channels()
    bufs, descs = [], []
    for c in specs:
        ld = P.aligned_ld(c.nevents)
        out = torch.empty((c.n, 4, ld), dtype=torch.float64, device="cuda")
        w = torch.empty(ld, dtype=torch.float64, device="cuda")
        st = torch.empty(4, dtype=torch.float64, device="cuda")
        bufs.append((out, w, st))
        descs.append(P.channel(c.parent_mass, c.masses, c.nevents, seed=c.seed, stream_id=c.stream_id,
                               out=out, weights=w, stats=st))
    rng = np.random.default_rng(1)
    pick = rng.choice(len(specs), size=6, replace=False)
    P.batch_run(descs)  # per-class launches, each class at its single-channel default
    torch.cuda.synchronize()
    ref_stats = torch.stack([st for _, _, st in bufs]).clone()
    ref_w = {int(i): bufs[i][1][:specs[i].nevents].clone() for i in pick}
    for sched in (3, 4, 5):
        _say(f"config3 single launch, schedule {sched}")
        for _, w, st in bufs:
            w.fill_(float("nan"))
            st.fill_(float("nan"))
        plan = P.Plan(descs, schedule=sched)
        plan.launch()
        torch.cuda.synchronize()
        plan.destroy()
        assert torch.equal(torch.stack([st for _, _, st in bufs]), ref_stats), sched
        for i in pick:
            assert torch.equal(bufs[i][1][:specs[i].nevents], ref_w[int(i)]), (sched, i)
    for i in pick:
        c = specs[i]
        out, w, st = bufs[i]
        idx = np.unique(np.concatenate([[0, c.nevents - 1], rng.integers(0, c.nevents, 100)]))
        ti = torch.as_tensor(idx, device="cuda")
        g = out[:, :, ti].cpu().numpy()
        gw = w[ti].cpu().numpy()
        for j, e in enumerate(idx):
            p4o, wo = oracle.generate(c.parent_mass, c.masses, 1, seed=c.seed, stream_id=c.stream_id,
                                      event_offset=int(e))
            assert_events_close(g[:, :, j:j + 1], gw[j:j + 1], p4o, wo)
