#!/usr/bin/env python3
"""Benchmark: phase-space events/s on one MI355X and the HBM-write roofline.

Workload (the throughput configuration): a parent of mass 5.279 GeV at rest
decays to (3.097, 0.4937, 0.13957) GeV; 1e8 events per step, FP64, Philox seed
42; each step writes the SoA four-momenta (3 x 4 doubles) and the weight of every
event (104 B/event, 10.4 GB) and the fused integral (mean, sigma).  One step is
one ``hydra_phsp_generate`` call: the main kernel plus the finalize kernel.

Prints ONE JSON line.  ``roofline`` uses the main kernel's average duration,
measured with HIP events recorded by the library on the launch stream over the
timed region; ``cpu_baseline`` times the CPU oracle on a bounded sample of the
same workload on this host.  ``ceilings`` measures the two rates that bound
the main kernel with the library's probes: its stores alone (constant data, same
buffers and launch shape) and its Philox calls alone.  ``extras`` reports the other configurations
(per-event parents, six-body FP64 vs mixed, integrate-only, batched) when
their code paths exist.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "phase-space events/s (N=3, FP64) and % HBM roofline; mixed vs plain at tol"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, AMD public specification
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_phsp_n3_1e8_traffic.txt")
COPY_BYTES = 1 << 30  # calibration copy: reads and writes exactly this many bytes


def kernel_source_hash() -> str:
    """Hash of the sources the main kernel is built from (invalidates stale counters)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1711_05683_amd", "csrc")
    for name in ("phsp_device.hpp", "phsp_sortnet.hpp", "phsp_reduce.hpp", "phsp_kernels.hpp",
                 "phsp_inst.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str = "", algorithmic_bytes: float = 0.0):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when missing, taken on a different kernel source, on another instantiation
    than `kernel` (e.g. another events-per-thread setting), or on a launch of
    another size than `algorithmic_bytes` (when given)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_hash") != kernel_source_hash():
        return None
    if kernel and kernel not in fields.get("kernel", ""):
        return None
    try:
        if algorithmic_bytes and abs(float(fields["algorithmic_bytes_per_launch"]) - algorithmic_bytes) > \
                1e-6 * algorithmic_bytes:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


_T0 = time.perf_counter()


def progress(msg: str) -> None:
    """One line on stderr when a part of the run ends (the JSON line stays alone on stdout)."""
    print(f"bench: {msg} ({time.perf_counter() - _T0:.1f} s)", file=sys.stderr, flush=True)


def cpu_all_cores(workers: int, per_worker: int = 10_000_000, chunk: int = 1_000_000):
    """The same plain oracle on `workers` host threads, each on its own event
    ranges (partitioned by event_offset, so together they produce exactly the
    events of one run; ctypes releases the interpreter lock around each oracle
    call, and the oracle keeps no global state): whole-job events/s over the
    wall time of the parallel section."""
    import threading
    import oracle
    M, m = 5.279, [3.097, 0.4937, 0.13957]
    oracle.generate(M, m, 1000, seed=42)  # load the library, untimed
    nchunks = workers * (per_worker // chunk)
    lock = threading.Lock()
    nxt = [0]

    def worker():
        while True:
            with lock:
                k = nxt[0]
                nxt[0] += 1
            if k >= nchunks:
                return
            oracle.generate(M, m, chunk, seed=42, event_offset=k * chunk)

    threads = [threading.Thread(target=worker) for _ in range(workers)]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    dt = time.perf_counter() - t0
    return nchunks * chunk / dt, dt, nchunks * chunk


def cpu_baseline(target_s: float = 10.0, chunk: int = 1_000_000, max_events: int = 100_000_000):
    """The CPU oracle (single thread) on a bounded sample of the same workload,
    then the same code on all the cores this process may use."""
    import oracle
    oracle.build(force=False)
    M, m = 5.279, [3.097, 0.4937, 0.13957]
    done = 0
    t0 = time.perf_counter()
    while done < max_events:
        oracle.generate(M, m, chunk, seed=42, event_offset=done)
        done += chunk
        if time.perf_counter() - t0 >= target_s:
            break
    dt = time.perf_counter() - t0
    # the other configurations' generators, a short sample each (same thread)
    others = {}
    for name, Mo, mo, n in (("config0_3body_1e5", 5.279, [3.097, 0.4937, 0.13957], 100_000),
                            ("config2_six_pions", 10.0, [0.13957] * 6, 500_000),
                            ("config2_six_massless", 10.0, [0.0] * 6, 500_000)):
        t1 = time.perf_counter()
        oracle.generate(Mo, mo, n, seed=42)
        others[name] = {"events": n, "events_per_s": n / (time.perf_counter() - t1)}
    nproc = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = nproc
    # the GPU machine grants one GPU's share of the host (16 threads), whatever the
    # machine's core count; OMP_NUM_THREADS states that share
    share = int(os.environ.get("OMP_NUM_THREADS", usable) or usable)
    workers = max(1, min(usable, share))
    rate_all, dt_all, n_all = cpu_all_cores(workers)
    return {"value": done / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} events of the 1e8-event workload (momenta + weights), "
                      f"{chunk}-event chunks, single thread, {dt:.1f} s",
            "cpu_model": _cpu_model(), "nproc": nproc, "usable_cpus": usable,
            "all_cores_events_per_s": rate_all, "all_cores_threads": workers,
            "all_cores_sample": f"events [0, {n_all}) of the same workload on {workers} threads, "
                                f"1e6-event ranges by event_offset, {dt_all:.1f} s wall",
            "other_configs": others}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def warm_clocks(fn, torch, seconds):
    """Run the step back to back, untimed, for at least `seconds` of wall time,
    so the timed region starts at steady clocks (the first launches of a
    process run slower while the GPU's clocks ramp up).  Returns (seconds, steps)."""
    t0 = time.perf_counter()
    n = 0
    while True:
        for _ in range(8):
            fn()
        n += 8
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if dt >= seconds:
            return dt, n


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    import paper_1711_05683_amd as P
    P.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = P.timing_read()
    P.timing_enable(False)
    return (t1 - t0) * 1e3 / steps, (kms / launches if launches else float("nan"))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nevents", type=int, default=100_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--clock-warm-s", type=float, default=2.0,
                    help="seconds of untimed back-to-back steps after the warm-up steps, so the timed "
                         "steps run at steady clocks")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson serving trace replayed in the extras (60 = the full trace)")
    ap.add_argument("--serve-tight-budget-mib", type=int, default=384,
                    help="HBM budget of the second serving replay, small enough that admission binds "
                         "(0 = skip it)")
    ap.add_argument("--counters", nargs="?", const="headline", default=None, choices=sorted(COUNTER_RUNS),
                    help="short run for rocprofv3 --pmc, prints no JSON: 'headline' (default) runs a 1 GiB "
                         "torch copy (the calibration kernel of known traffic) x3, then the main step x3; "
                         "the other names run one configuration's launch x3 after two warm-up launches")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 64-channel batched configuration and print its figures")
    ap.add_argument("--only", choices=["unweighted", "model", "sequential", "vegas", "by_n"],
                    help="run only this extra on the 1e8-event workload and print its figures")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(events shard across GPUs by event_offset; this benchmark measures one GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1711_05683_amd as P

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    P.lib()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if args.batched_only:
        print(json.dumps(batched_extra(P, torch, dev, args.steps)), flush=True)
        return
    if args.only == "vegas":
        print(json.dumps(vegas_extra(P, torch, dev)), flush=True)
        return
    if args.only == "by_n":
        print(json.dumps(by_n_extra(P, torch, dev, args.steps)), flush=True)
        return
    if args.only:
        M, m = 5.279, [3.097, 0.4937, 0.13957]
        n = args.nevents
        out = torch.empty((3, 4, n), dtype=torch.float64, device=dev)
        w = torch.empty(n, dtype=torch.float64, device=dev)
        st = torch.empty(4, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            P.generate(M, m, n, out=out, weights=w, stats=st)
        if args.only == "unweighted":
            r = unweighted_extra(P, torch, dev, M, m, n, out, args.steps)
        elif args.only == "model":
            r = model_extra(P, torch, dev, M, m, n, w, st, args.steps)
        else:
            r = sequential_extra(P, torch, dev, M, m, n, out, w, st, args.steps)
        print(json.dumps(r), flush=True)
        return

    M, m = 5.279, [3.097, 0.4937, 0.13957]
    n_ev = args.nevents
    out = torch.empty((3, 4, n_ev), dtype=torch.float64, device=dev)
    w = torch.empty(n_ev, dtype=torch.float64, device=dev)
    st = torch.empty(4, dtype=torch.float64, device=dev)

    def step():
        P.generate(M, m, n_ev, seed=42, out=out, weights=w, stats=st)

    if args.counters and args.counters != "headline":
        counter_run(P, torch, dev, args.counters)
        return
    if args.counters:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        print(f"counter run done: copy {COPY_BYTES} B x3, {n_ev} events x3", flush=True)
        return

    for _ in range(args.warmup):
        step()
    warm_s, warm_steps = warm_clocks(step, torch, args.clock_warm_s)
    ms_step, ms_kernel = time_steps(step, args.steps, 0, torch)
    bytes_per_event = 8 * (4 * 3 + 1)
    achieved = bytes_per_event * n_ev / (ms_kernel * 1e-3) / 1e9
    stats = st.cpu().tolist()
    ept = P.events_per_thread(1, 3)
    main_kernel = f"k_phsp<3, 0, 1, {ept}>"
    traffic = read_traffic(main_kernel, float(bytes_per_event * n_ev))

    result = {
        "metric": METRIC,
        "value": n_ev / (ms_step * 1e-3),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-body decay at rest, M=5.279 -> (3.097, 0.4937, 0.13957) GeV, "
                               f"{n_ev:.0e} events/step, FP64, Philox4x32-10 seed 42, SoA momenta "
                               "+ weights + fused integral",
                   "n_daughters": 3, "nevents": n_ev, "bytes_per_event": bytes_per_event},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": f"{main_kernel} (N=3, at rest, FP64, {ept} event(s) per thread)",
                     "kernel_ms": ms_kernel},
        "clock_warm": {"seconds": warm_s, "steps": warm_steps,
                       "note": "untimed steps after the warm-up steps, before the timed region"},
        "integral": {"mean": stats[1], "sigma": stats[3], "n": stats[0]},
        "ceilings": ceilings(P, torch, out, w, n_ev, ept, ms_kernel, bytes_per_event, args),
    }
    del out
    progress("headline timed")

    if not args.no_extras:
        result["extras"] = extras(P, torch, dev, args)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline()
        progress("CPU oracle timed")
    print(json.dumps(result), flush=True)


# Short programs profiled by counter passes: name -> (parent mass, masses, events, mixed)
COUNTER_RUNS = {"headline": None,
                "six_pion_fp64": (10.0, [0.13957] * 6, 50_000_000, False),
                "six_pion_mixed": (10.0, [0.13957] * 6, 50_000_000, True),
                "six_massless_mixed": (10.0, [0.0] * 6, 50_000_000, True),
                "ten_pion_fp64": (10.0, [0.13957] * 10, 31_700_000, False),
                "unweighted": (5.279, [3.097, 0.4937, 0.13957], 100_000_000, False),
                "unweighted_pipeline": (5.279, [3.097, 0.4937, 0.13957], 100_000_000, False),
                "chain": (5.279, [3.097, 0.4937, 0.13957], 100_000_000, False),
                "integrate": (5.279, [3.097, 0.4937, 0.13957], 100_000_000, False),
                "model": (5.279, [3.097, 0.4937, 0.13957], 100_000_000, False),
                "vegas": None}


def counter_run(P, torch, dev, name):
    """Two warm-up launches and three profiled launches of one configuration."""
    if name == "vegas":
        # one iteration of 1e8 calls on the 10-D Gaussian of the VEGAS extra (uniform grid)
        import numpy as np
        D, bins = 10, 50
        f = P.gauss_box([0.0] * D, [1.0] * D, [0.5] * D, [0.1] * D)
        g = torch.as_tensor(np.tile(np.linspace(0.0, 1.0, bins + 1), (D, 1)), dtype=torch.float64, device=dev)
        for _ in range(5):
            P.vegas_iteration(f, g, 100_000_000, seed=7, iteration=100)
        torch.cuda.synchronize()
        print(f"counter run {name}: 1e8 calls x5 done", flush=True)
        return
    M, m, n, mixed = COUNTER_RUNS[name]
    dtype = torch.float32 if mixed else torch.float64
    w = torch.empty(n, dtype=torch.float64, device=dev)
    st = torch.empty(4, dtype=torch.float64, device=dev)
    if name == "integrate":
        fn = lambda: P.integrate_async(M, m, n, stats=st)  # noqa: E731
    elif name == "model":
        one = [(1, 2, 0.8955, 0.0473)]  # the model extra's one-factor model: per-event values and integral
        fn = lambda: P.integrate_model(M, m, n, one, values=w, stats=st)  # noqa: E731
    elif name == "chain":
        # the sequential-decay extra in one launch: daughter 0 -> mu mu
        out = torch.empty((len(m), 4, P.aligned_ld(n)), dtype=dtype, device=dev)
        out2 = torch.empty((2, 4, P.aligned_ld(n)), dtype=dtype, device=dev)
        w2 = torch.empty(n, dtype=torch.float64, device=dev)
        st2 = torch.empty(4, dtype=torch.float64, device=dev)
        fn = lambda: P.generate_chain(M, m, 0, [0.1056583755] * 2, n, out=out, weights=w, stats=st,  # noqa: E731
                                      out2=out2, weights2=w2, stats2=st2)
    else:
        out = torch.empty((len(m), 4, P.aligned_ld(n)), dtype=dtype, device=dev)
        if name.startswith("unweighted"):
            # 'unweighted': the passes one after the other (one chunk); 'unweighted_pipeline': the
            # default four chunks, each store launch also counting the next chunk
            P.set_unweight_chunks(1 if name == "unweighted" else 0)
            cnt = torch.empty(2, dtype=torch.int64, device=dev)
            wmo = torch.empty(1, dtype=torch.float64, device=dev)
            P.generate_unweighted(M, m, n, out=out, counts=cnt, w_max_out=wmo)
            torch.cuda.synchronize()
            bound = float(wmo.item())
            fn = lambda: P.generate_unweighted(M, m, n, w_max=bound, out=out, counts=cnt,  # noqa: E731
                                               w_max_out=wmo)
        else:
            fn = lambda: P.generate(M, m, n, out=out, weights=w, stats=st, mixed=mixed)  # noqa: E731
    for _ in range(5):
        fn()
    torch.cuda.synchronize()
    print(f"counter run {name}: {n} events x5 done", flush=True)


def time_launches(fn, steps, warmup, torch):
    """Mean duration of one launch of ``fn``: a pair of events on the current
    stream (the stream the probes launch on) around each launch."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    pairs = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in pairs) / steps


def ceilings(P, torch, out, w, n, ept, ms_kernel, bytes_per_event, args):
    """The two rates that bound the generator, measured with the library's
    probes on the headline workload: the same stores with constant data (same
    buffers, launch shape and events per thread), and the same Philox calls
    with nothing else."""
    cols = out.shape[0] * out.shape[1]
    flat = out.view(cols, out.shape[2])
    warm = max(10, args.warmup // 2)
    ms_w = time_launches(lambda: P.probe_write(flat, w, n, events_per_thread=ept), args.steps, warm, torch)
    calls = (3 * 3 - 4 + 1) // 2
    fold = torch.empty((n + P.PROBE_SPAN - 1) // P.PROBE_SPAN, dtype=torch.int32, device=out.device)
    ms_p = time_launches(lambda: P.probe_philox(n, calls, fold=fold), args.steps, warm, torch)
    gbs = bytes_per_event * n / (ms_w * 1e-3) / 1e9
    return {
        "write": {"kernel": f"k_write_bw<{cols}, {ept}>", "ms": ms_w, "GB/s": gbs, "frac": gbs / PEAK_HBM_GBS,
                  "generator_over_ceiling": ms_w / ms_kernel},
        "philox": {"kernel": "k_philox_only", "ms": ms_p, "calls_per_s": n * calls / (ms_p * 1e-3),
                   "calls_per_event": calls, "events_per_s": n / (ms_p * 1e-3)},
    }


def extras(P, torch, dev, args):
    """Other configurations at their own sizes, each timed like the main step."""
    from paper_1711_05683_amd.workloads import per_event_parents
    ex = {}
    steps = max(3, args.steps // 2)
    M, m = 5.279, [3.097, 0.4937, 0.13957]
    n1 = args.nevents
    # config 1b: per-event parents (reads 32 B/event more)
    parents = per_event_parents(M, n1)
    out = torch.empty((3, 4, n1), dtype=torch.float64, device=dev)
    w = torch.empty(n1, dtype=torch.float64, device=dev)
    st = torch.empty(4, dtype=torch.float64, device=dev)
    ms, kms = time_steps(lambda: P.generate(M, m, n1, out=out, weights=w, stats=st, parent_dev=parents),
                         steps, 1, torch)
    progress("per-event parents timed")
    ex["cfg1_per_event_parent"] = {"events_per_s": n1 / (ms * 1e-3), "kernel_ms": kms,
                                   "write_GBs": 104 * n1 / (kms * 1e-3) / 1e9,
                                   "total_GBs": 136 * n1 / (kms * 1e-3) / 1e9}
    del parents
    # integrate-only (no stores): the arithmetic ceiling of the same events
    ms, kms = time_steps(lambda: P.integrate_async(M, m, n1, stats=st), steps, 1, torch)
    ex["cfg1_integrate_only"] = {"events_per_s": n1 / (ms * 1e-3), "kernel_ms": kms}
    # the same events into columns off the 128-byte line grid (ld = n + 1): the staged kernel
    del out
    raw = torch.empty((3 * 4 * (n1 + 1),), dtype=torch.float64, device=dev)
    ms, kms = time_steps(lambda: P.generate(M, m, n1, out=raw.view(3, 4, n1 + 1), weights=w, stats=st), steps, 1,
                         torch)
    ex["cfg1_ld_off_line_grid"] = {"ld": n1 + 1, "kernel_ms": kms, "events_per_s": n1 / (ms * 1e-3),
                                   "write_GBs": 104 * n1 / (kms * 1e-3) / 1e9}
    del raw
    out = torch.empty((3, 4, n1), dtype=torch.float64, device=dev)
    P.generate(M, m, n1, out=out, weights=w, stats=st)
    ex["cfg1_unweighted"] = unweighted_extra(P, torch, dev, M, m, n1, out, steps)
    progress("unweighted timed")
    ex["cfg1_sequential"] = sequential_extra(P, torch, dev, M, m, n1, out, w, st, steps)
    ex["cfg1_model"] = model_extra(P, torch, dev, M, m, n1, w, st, steps)
    progress("sequential and model timed")
    del out, w
    # config 2: six pions at M=10, 5e7 events, FP64 vs mixed
    n2 = max(n1 // 2, 1)
    six = [0.13957] * 6
    out = torch.empty((6, 4, n2), dtype=torch.float64, device=dev)
    w = torch.empty(n2, dtype=torch.float64, device=dev)
    ms, kms = time_steps(lambda: P.generate(10.0, six, n2, out=out, weights=w, stats=st), steps, 1, torch)
    ex["cfg2_six_pion_fp64"] = {"events_per_s": n2 / (ms * 1e-3), "kernel_ms": kms,
                                "write_GBs": 200 * n2 / (kms * 1e-3) / 1e9}
    del out
    outm = torch.empty((6, 4, n2), dtype=torch.float32, device=dev)
    ms, kms = time_steps(lambda: P.generate(10.0, six, n2, out=outm, weights=w, stats=st, mixed=True),
                         steps, 1, torch)
    ex["cfg2_six_pion_mixed"] = {"events_per_s": n2 / (ms * 1e-3), "kernel_ms": kms,
                                 "write_GBs": 104 * n2 / (kms * 1e-3) / 1e9}
    del outm, w
    progress("six-pion FP64 and mixed timed")
    ex["cfg3_batched_64_channels"] = batched_extra(P, torch, dev, steps)
    progress("64-channel batch timed")
    ex["vegas_10d_gaussian"] = vegas_extra(P, torch, dev)
    progress("VEGAS timed")
    if args.serve_seconds > 0:
        ex["cfg4_serving"] = serving_extra(P, args.serve_seconds, 32 << 30)
        progress("serving replay done")
        if args.serve_tight_budget_mib > 0:
            ex["cfg4_serving_tight_budget"] = serving_extra(P, args.serve_seconds,
                                                             args.serve_tight_budget_mib << 20)
            progress("tight-budget serving replay done")
    return ex


def by_n_extra(P, torch, dev, steps):
    """Single channel by daughter count: N pions from M = 10 GeV, FP64 at rest,
    about 10.4 GB of output per launch on line-aligned columns, default events
    per thread; each N's generator against the write probe with the same
    stores, and its integrate-only time."""
    r = {}
    for n in range(2, 11):
        m = [0.13957] * n
        nev = int(10.4e9 // (8 * (4 * n + 1)))
        nev -= nev % 1024
        out = torch.empty((n, 4, P.aligned_ld(nev)), dtype=torch.float64, device=dev)
        w = torch.empty(nev, dtype=torch.float64, device=dev)
        st = torch.empty(4, dtype=torch.float64, device=dev)
        ept = P.events_per_thread(1, n)
        _, k = time_steps(lambda: P.generate(10.0, m, nev, out=out, weights=w, stats=st), steps, 15, torch)
        kw = time_launches(lambda: P.probe_write(out.view(4 * n, out.shape[2]), w, nev, events_per_thread=ept),
                           steps, 10, torch)
        _, ki = time_steps(lambda: P.integrate_async(10.0, m, nev, stats=st), steps, 10, torch)
        b = 8 * (4 * n + 1) * nev
        r[str(n)] = {"nevents": nev, "ept": ept, "kernel": f"k_phsp<{n}, 0, 1, {ept}>", "kernel_ms": k,
                     "write_GBs": b / (k * 1e-3) / 1e9, "probe_kernel": f"k_write_bw<{4 * n}, {ept}>",
                     "probe_ms": kw, "probe_GBs": b / (kw * 1e-3) / 1e9, "kernel_over_probe_rate": kw / k,
                     "integrate_ms": ki}
        del out, w
        torch.cuda.empty_cache()
    return r


def vegas_extra(P, torch, dev):
    """VEGAS on the integrand of the paper's VEGAS benchmark, a 10-dimensional
    Gaussian (here mean 0.5, sigma 0.1 per dimension over the unit cube, 50
    bins): 5 adapting + 5 estimating iterations of 1e7 calls, and single
    iterations of 1e7 / 1e8 calls timed on the adapted grid."""
    import numpy as np
    D = 10
    lo, hi, mu, sg = [0.0] * D, [1.0] * D, [0.5] * D, [0.1] * D
    exact = 1.0
    for a, b, m, s in zip(lo, hi, mu, sg):
        exact *= 0.5 * (math.erf((b - m) / (s * math.sqrt(2.0))) - math.erf((a - m) / (s * math.sqrt(2.0))))
    f = P.gauss_box(lo, hi, mu, sg)
    walls = []
    for _ in range(2):  # the first run also loads the kernels and allocates the workspace
        t0 = time.perf_counter()
        res, err, chi2, grid = P.vegas(f, 10_000_000, 5, warmup=5, seed=42)
        walls.append(time.perf_counter() - t0)
    g = torch.as_tensor(np.ascontiguousarray(grid), device=dev)
    r = {"integrand": "10-D Gaussian, mean 0.5, sigma 0.1, unit cube, 50 bins", "exact": exact,
         "result": res, "error": err, "chi2_dof": chi2, "pull": (res - exact) / err,
         "driver_s_10_iterations_1e7_calls_first": walls[0],
         "driver_s_10_iterations_1e7_calls": walls[1]}
    for calls in (10_000_000, 100_000_000):
        ms, k = time_steps(lambda: P.vegas_iteration(f, g, calls, seed=7, iteration=100), 5, 1, torch)
        r[f"iteration_{calls:.0e}_calls"] = {"kernel_ms": k, "ms": ms, "samples_per_s": calls / (k * 1e-3)}
    # the same integrand as a user function compiled at run time (hiprtc)
    src = """
__device__ double hydra_phsp_user_integrand(const double* x, const double* par) {
    double v = 1.0;
    for (int d = 0; d < HYDRA_PHSP_DIM; ++d) {
        const double t = (x[d] - par[0]) * par[1];
        v = v * (exp(-0.5 * t * t) * par[2]);
    }
    return v;
}
"""
    t0 = time.perf_counter()
    u = P.UserIntegrand(src, D)
    compile_s = time.perf_counter() - t0
    par = [0.5, 1.0 / 0.1, 1.0 / (0.1 * math.sqrt(2.0 * math.pi))]
    ms, k = time_steps(lambda: u.iteration(lo, hi, g, 100_000_000, par, seed=7, iteration=100), 5, 1, torch)
    ru, eu, cu, _ = u.vegas(lo, hi, 10_000_000, 5, par, warmup=5, seed=42)
    u.destroy()
    r["user_integrand"] = {"iteration_1e+08_calls_kernel_ms": k, "samples_per_s": 1e8 / (k * 1e-3),
                           "compile_s": compile_s, "result": ru, "error": eu, "chi2_dof": cu,
                           "pull": (ru - exact) / eu}
    return r


# One relativistic Breit-Wigner intensity in the (1, 2) pair mass as a user
# intensity compiled at run time: par = (mass, width).
USER_KSTAR = """
__device__ double hydra_phsp_user_intensity(const double* e, const double* px, const double* py,
                                            const double* pz, const double* par) {
    const double se = e[1] + e[2], sx = px[1] + px[2], sy = py[1] + py[2], sz = pz[1] + pz[2];
    const double s = se * se - sx * sx - sy * sy - sz * sz;
    const double d = par[0] * par[0] - s;
    const double mg = par[0] * par[1];
    return 1.0 / (d * d + mg * mg);
}
"""


def model_extra(P, torch, dev, M, m, n, w, st, steps):
    """Model evaluation over the 1e8 events: one Breit-Wigner intensity (a K pi
    resonance) and two (plus a broad one in the other pair); the per-event values
    w |A|^2 are written (8 B/event) and integrated."""
    one = [(1, 2, 0.8955, 0.0473)]
    two = [(0, 1, 3.686, 0.3), (1, 2, 0.8955, 0.0473)]
    r = {}
    for name, res in (("one_factor", one), ("two_factors", two)):
        ms, k = time_steps(lambda: P.integrate_model(M, m, n, res, values=w, stats=st), steps, 1, torch)
        r[name] = {"kernel_ms": k, "events_per_s": n / (ms * 1e-3), "integral": float(st[1].item()),
                   "sigma": float(st[3].item())}
    # the one-factor model as a user intensity compiled at run time (hiprtc)
    t0 = time.perf_counter()
    model = P.UserModel(USER_KSTAR, len(m))
    compile_s = time.perf_counter() - t0
    ms, k = time_steps(lambda: model.integrate(M, m, n, one[0][2:], values=w, stats=st), steps, 1, torch)
    integral = float(st[1].item())
    model.destroy()
    r["user_one_factor"] = {"kernel_ms": k, "events_per_s": n / (ms * 1e-3), "integral": integral,
                            "same_integral_as_built_in": integral == r["one_factor"]["integral"],
                            "compile_s": compile_s}
    return r


def sequential_extra(P, torch, dev, M, m, n, out, w, st, steps):
    """Sequential decays: each event's daughter 0 (mass 3.097, read in place from
    the first output) decays to mu+ mu- in a second call on another stream id.
    Stage 2 reads 32 B and writes 72 B per event."""
    mmu = 0.1056583755
    out2 = torch.empty((2, 4, n), dtype=torch.float64, device=dev)
    w2 = torch.empty(n, dtype=torch.float64, device=dev)
    st2 = torch.empty(4, dtype=torch.float64, device=dev)

    def stage2():
        P.generate(m[0], [mmu, mmu], n, seed=42, stream_id=1, parent_dev=out[0], out=out2, weights=w2, stats=st2)

    def chain():
        P.generate(M, m, n, seed=42, out=out, weights=w, stats=st)
        stage2()

    def fused():
        P.generate_chain(M, m, 0, [mmu, mmu], n, seed=42, stream_id=0, stream_id2=1, out=out, weights=w, stats=st,
                         out2=out2, weights2=w2, stats2=st2)

    chain()
    ms2, k2 = time_steps(stage2, steps, 1, torch)
    msc, _ = time_steps(chain, steps, 1, torch)
    fused()
    msf, kf = time_steps(fused, steps, 1, torch)
    del out2, w2
    # the fused launch writes both stages (104 + 72 B per event) and reads nothing
    return {"decay": "5.279 -> (3.097 -> mu mu, 0.4937, 0.13957)", "stage2_kernel_ms": k2,
            "stage2_total_GBs": 104 * n / (k2 * 1e-3) / 1e9, "chain_ms_per_step": msc,
            "chain_events_per_s": n / (msc * 1e-3), "fused_chain_ms_per_step": msf, "fused_chain_kernel_ms": kf,
            "fused_chain_events_per_s": n / (msf * 1e-3),
            "fused_chain_write_GBs": 176 * n / (kf * 1e-3) / 1e9}


def unweighted_extra(P, torch, dev, M, m, n, out, steps):
    """Hit-or-miss unweighted sample of the 1e8 trials: with the sample maximum as
    the bound (max, count, scan and write passes) and with that bound given
    (count, scan, write).  Kernel time = the whole launch sequence."""
    cnt = torch.empty(2, dtype=torch.int64, device=dev)
    wmo = torch.empty(1, dtype=torch.float64, device=dev)
    ms0, k0 = time_steps(lambda: P.generate_unweighted(M, m, n, out=out, counts=cnt, w_max_out=wmo), steps, 1,
                         torch)
    kept, over = (int(x) for x in cnt.cpu().tolist())
    w_max = float(wmo.item())
    ms1, k1 = time_steps(lambda: P.generate_unweighted(M, m, n, w_max=w_max, out=out, counts=cnt, w_max_out=wmo),
                         steps, 1, torch)
    bytes_kept = kept * 8 * 4 * len(m)
    # the same sequence with its passes one after the other (one chunk: count,
    # scan, then write) instead of the default four-chunk pipeline
    P.set_unweight_chunks(1)
    try:
        _, k1_serial = time_steps(lambda: P.generate_unweighted(M, m, n, w_max=w_max, out=out, counts=cnt,
                                                                w_max_out=wmo), steps, 1, torch)
    finally:
        P.set_unweight_chunks(0)
    r = {"trials": n, "kept": kept, "kept_fraction": kept / n, "w_max": w_max, "over_bound": over,
         "ms_sample_max": k0, "ms_given_bound": k1, "trials_per_s_given_bound": n / (k1 * 1e-3),
         "kept_per_s_given_bound": kept / (k1 * 1e-3), "kept_per_s_sample_max": kept / (k0 * 1e-3),
         "write_GBs_given_bound": bytes_kept / (k1 * 1e-3) / 1e9, "frac_of_8TBs_given_bound":
         bytes_kept / (k1 * 1e-3) / 8e12, "chunks": 4, "ms_given_bound_one_chunk": k1_serial}
    # samples of the one-factor K pi model (kept events follow w |A|^2), built in
    # and as the same intensity compiled at run time
    one = [(1, 2, 0.8955, 0.0473)]
    model = P.UserModel(USER_KSTAR, len(m))
    runs = {"model_one_factor": lambda wm: P.generate_unweighted_model(M, m, n, one, w_max=wm, out=out,
                                                                       counts=cnt, w_max_out=wmo),
            "user_model_one_factor": lambda wm: model.generate_unweighted(M, m, n, one[0][2:], w_max=wm, out=out,
                                                                          counts=cnt, w_max_out=wmo)}
    for name, run in runs.items():
        ms0, k0 = time_steps(lambda: run(0.0), steps, 1, torch)
        kept = int(cnt[0].item())
        w_max = float(wmo.item())
        ms1, k1 = time_steps(lambda: run(w_max), steps, 1, torch)
        r[name] = {"kept": kept, "kept_fraction": kept / n, "w_max": w_max, "ms_sample_max": k0,
                   "ms_given_bound": k1, "trials_per_s_given_bound": n / (k1 * 1e-3),
                   "kept_per_s_sample_max": kept / (k0 * 1e-3)}
    model.destroy()
    r["user_model_one_factor"]["same_sample_as_built_in"] = \
        r["user_model_one_factor"]["kept"] == r["model_one_factor"]["kept"] and \
        r["user_model_one_factor"]["w_max"] == r["model_one_factor"]["w_max"]
    return r


def serving_extra(P, seconds, budget):
    """Poisson arrivals at 2000 req/s replayed in real time by the native loop,
    with an HBM budget of `budget` bytes for the server's arena."""
    import numpy as np
    from paper_1711_05683_amd.workloads import serving_requests
    reqs = serving_requests(rate_hz=2000.0, duration_s=seconds)
    descs = [P.request(r.parent_mass, r.masses, r.nevents, seed=r.seed, stream_id=r.stream_id,
                       integrate_only=r.integrate_only) for r in reqs]
    srv = P.Server(budget, max_events_per_tick=1 << 22)
    lat, wall, peak = srv.replay(descs, [r.arrival_s for r in reqs])
    st = srv.stats()
    cnt = srv.counters()
    srv.destroy()
    lat = np.array(lat)
    ok = lat >= 0
    events = sum(r.nevents for r in reqs)
    return {"requests": len(reqs), "trace_s": seconds, "wall_s": wall, "events": events,
            "events_per_s": events / wall, "p50_ms": float(np.median(lat[ok]) * 1e3),
            "p99_ms": float(np.quantile(lat[ok], 0.99) * 1e3), "max_ms": float(lat[ok].max() * 1e3),
            "failed": int((~ok).sum()), "ticks": st["ticks"], "peak_arena_bytes": peak,
            "budget_bytes": budget, "admission_budget_stalls": cnt["budget_stalls"],
            "admission_active_stalls": cnt["active_stalls"],
            "queue_wait_mean_ms": cnt["queue_wait_sum_s"] / max(cnt["finished"], 1) * 1e3,
            "queue_wait_max_ms": cnt["queue_wait_max_s"] * 1e3}


def batched_extra(P, torch, dev, steps):
    """64 channels of uneven N and size in one persistent launch (autotuned shape,
    HIP-graph replay); kernel time from a direct launch of the same shape."""
    from paper_1711_05683_amd.workloads import batched_channels
    specs = batched_channels()
    total_events = sum(c.nevents for c in specs)
    total_bytes = sum(c.nevents * (4 * c.n + 1) * 8 for c in specs)
    keep, descs = [], []
    for c in specs:
        # columns on 128-byte lines (the layout the library recommends)
        out = torch.empty((c.n, 4, P.aligned_ld(c.nevents)), dtype=torch.float64, device=dev)
        w = torch.empty(c.nevents, dtype=torch.float64, device=dev)
        st = torch.empty(4, dtype=torch.float64, device=dev)
        keep.append((out, w, st))
        descs.append(P.channel(c.parent_mass, c.masses, c.nevents, seed=c.seed, stream_id=c.stream_id,
                               out=out, weights=w, stats=st))
    t0 = time.perf_counter()
    ept, gpc, sched, nstr, tuned_ms = P.autotune(descs)
    tune_s = time.perf_counter() - t0
    plan = P.Plan(descs, ept=ept, grid_per_cu=gpc, schedule=sched, streams=nstr)
    ms_graph, _ = time_steps(plan.launch, steps, 1, torch)
    ms_direct, kms = time_steps(lambda: P.batch_run(descs, ept=ept, grid_per_cu=gpc, schedule=sched, streams=nstr),
                                steps, 1, torch)
    # the same shape with the class kernels one after another on one stream
    ms_direct1, kms1 = time_steps(lambda: P.batch_run(descs, ept=ept, grid_per_cu=gpc, schedule=sched, streams=1),
                                  steps, 1, torch)
    ntiles, grid = plan.info()
    plan.destroy()
    # the same batch as one launch over every tile, heaviest tiles first, for
    # comparison with the per-class launches: one block per tile (schedule 3),
    # a persistent grid with a static stride (4) or dynamic claims (5); every N
    # at its single-channel default (ept 0) or at one event per thread (ept 1)
    single = {}
    for sc, name in ((3, "one block per tile"), (4, "persistent, static stride"),
                     (5, "persistent, dynamic claims")):
        for e in (0, 1):
            for g in ((0,) if sc == 3 else (1, 2, 4)):
                plan1 = P.Plan(descs, schedule=sc, ept=e, grid_per_cu=g)
                ms_graph1, _ = time_steps(plan1.launch, steps, 1, torch)
                ntiles1, grid1 = plan1.info()
                plan1.destroy()
                _, kms1s = time_steps(lambda: P.batch_run(descs, schedule=sc, ept=e, grid_per_cu=g), steps, 1,
                                      torch)
                single[f"schedule {sc} ept {e}" + (f" grid_per_cu {g}" if g else "")] = {
                    "kernel": f"k_phsp_batched_mixed<8, {e}>, {name}", "kernel_ms": kms1s,
                    "kernel_write_GBs": total_bytes / (kms1s * 1e-3) / 1e9,
                    "kernel_frac_of_8TBs": total_bytes / (kms1s * 1e-3) / 1e9 / PEAK_HBM_GBS,
                    "ms_per_step_graph": ms_graph1, "tiles": ntiles1, "grid": grid1}
    best_single = min(single, key=lambda k: single[k]["kernel_ms"])
    P.release()
    del keep, descs
    # the same batch with ld = nevents (columns start mid-line): partial-line stores
    keep, descs = [], []
    for c in specs:
        out = torch.empty((c.n, 4, c.nevents), dtype=torch.float64, device=dev)
        w = torch.empty(c.nevents, dtype=torch.float64, device=dev)
        st = torch.empty(4, dtype=torch.float64, device=dev)
        keep.append((out, w, st))
        descs.append(P.channel(c.parent_mass, c.masses, c.nevents, seed=c.seed, stream_id=c.stream_id,
                               out=out, weights=w, stats=st))
    ept_u, gpc_u, sched_u, nstr_u, _ = P.autotune(descs)  # off the line grid: its own classes and shape
    _, kms_unaligned = time_steps(lambda: P.batch_run(descs, ept=ept_u, grid_per_cu=gpc_u, schedule=sched_u,
                                                      streams=nstr_u), steps, 1, torch)
    P.release()
    del keep, descs
    sched_names = ["static", "dynamic", "one block per tile", "single launch, one block per tile",
                   "single persistent launch, static stride", "single persistent launch, dynamic claims"]
    return {"channels": len(specs), "events": total_events, "bytes": total_bytes,
            "tuning": {"ept": ept, "grid_per_cu": gpc, "schedule": sched_names[sched],
                       "streams": max(nstr, 1), "autotune_s": tune_s, "tiles": ntiles,
                       "grid": grid},
            "kernel_ms_one_stream": kms1, "ms_per_step_direct_one_stream": ms_direct1,
            "events_per_s_graph": total_events / (ms_graph * 1e-3), "ms_per_step_graph": ms_graph,
            "kernel_ms": kms, "kernel_write_GBs": total_bytes / (kms * 1e-3) / 1e9,
            "kernel_frac_of_8TBs": total_bytes / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "ms_per_step_direct": ms_direct, "ld": "aligned_ld(nevents)",
            "kernel_ms_ld_eq_nevents": kms_unaligned,
            "single_launch": {"best": best_single, **single[best_single], "by_shape": single},
            "tuning_ld_eq_nevents": {"ept": ept_u, "grid_per_cu": gpc_u,
                                     "schedule": sched_names[sched_u],
                                     "streams": max(nstr_u, 1)},
            "kernel_write_GBs_ld_eq_nevents": total_bytes / (kms_unaligned * 1e-3) / 1e9}


if __name__ == "__main__":
    main()
