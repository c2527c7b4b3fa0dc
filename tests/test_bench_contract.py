"""The benchmark's command-line contract: one GPU only, one JSON line with the
required fields, counter traffic reported only for the launch it was taken on."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_profiled_launch():
    want = 8.0 * 13 * 1e8
    t = bench.read_traffic("k_phsp<3, 0, 1, 1>", want)
    if t is None:
        pytest.skip("counter summary missing or taken on other kernel sources")
    assert 0.99 * want <= t <= 1.05 * want
    assert bench.read_traffic("k_phsp<3, 0, 1, 1>", want / 50) is None   # another size
    assert bench.read_traffic("k_phsp<3, 0, 1, 4>", want) is None        # another instantiation


@pytest.mark.gpu
def test_bench_json_line_small():
    pytest.importorskip("torch")
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    print("[bench] small run: 2e6 events, 3 steps", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--nevents", "2000000", "--steps", "3",
                        "--warmup", "2", "--no-extras", "--no-cpu-baseline"], capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    j = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "ceilings"):
        assert k in j, k
    assert j["n_gpus"] == 1 and j["steps"] == 3 and j["dtype"] == "f64" and "workload" in j["config"]
    rf = j["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12 and rf["traffic"] is None  # not the profiled size
    assert j["value"] > 0 and rf["achieved"] > 0
    assert j["ceilings"]["write"]["ms"] > 0 and j["ceilings"]["philox"]["calls_per_s"] > 0
