"""The C ABI used from plain C: tests/c_client/phsp_client.c is built with gcc
against include/ and the library (no Python, no torch in the client); on a GPU
its output is compared with the oracle."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1711_05683_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build_client(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.exists(os.path.join(PKG, "libhydra_phsp.so")):
        pytest.skip("gcc or the built library is missing")
    exe = str(tmp_path / "phsp_client")
    subprocess.run([gcc, "-std=c99", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    f"-I{ROCM}/include", f"-I{ROOT}/include", "-o", exe,
                    os.path.join(ROOT, "tests", "c_client", "phsp_client.c"),
                    f"-L{PKG}", "-lhydra_phsp", f"-L{ROCM}/lib", "-lamdhip64",
                    f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib"], check=True, capture_output=True, text=True)
    return exe


def test_c_client_builds_against_the_headers(tmp_path):
    exe = _build_client(tmp_path)
    assert os.path.exists(exe)


@pytest.mark.gpu
def test_c_client_matches_oracle(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import oracle
    from parity import FP64_TOL, rel
    exe = _build_client(tmp_path)
    n, seed = 100_003, 42
    print(f"[c-client] {n} events, seed {seed}", flush=True)
    r = subprocess.run([exe, str(n), str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    rows = {}
    events, chain = [], []
    for line in r.stdout.splitlines():
        f = line.split()
        if f[0] in ("event", "chain"):
            (events if f[0] == "event" else chain).append((int(f[1]), float(f[2]),
                                                            np.array([float(x) for x in f[3:]])))
        else:
            rows[f[0]] = [float(x) for x in f[1:]]
    assert rows["status"] == [0.0, 0.0] and rows["status2"] == [0.0, 0.0, 0.0, 0.0]
    M, m = 5.279, [3.097, 0.4937, 0.13957]
    oracle.build(force=False)
    mo, so = oracle.integrate(M, m, n, seed=seed)
    st = rows["stats"]
    assert st[0] == n and rel(st[1], mo) <= FP64_TOL and rel(st[3], so) <= FP64_TOL
    assert rel(rows["integral"][0], mo) <= FP64_TOL and rel(rows["integral"][1], so) <= FP64_TOL
    for g, w, p in events:
        p4o, wo = oracle.generate(M, m, 1, seed=seed, event_offset=g)
        assert rel(w, wo[0]) <= FP64_TOL
        po = p4o[:, :, 0]  # [3][4]
        for d in range(3):
            assert np.all(np.abs(p[4 * d:4 * d + 4] - po[d]) <= FP64_TOL * po[d][0]), (g, d)
    # the integral merged from two pieces, and the second stage of the one-launch chain
    mg = rows["merged"]
    assert mg[0] == n and rel(mg[1], mo) <= FP64_TOL and rel(mg[3], so) <= FP64_TOL
    mmu = 0.1056583755
    for g, w, p in chain:
        p4o, _ = oracle.generate(M, m, 1, seed=seed, event_offset=g)
        q4o, wo = oracle.generate(m[0], [mmu, mmu], 1, seed=seed, stream_id=1, event_offset=g,
                                  parent_soa=np.ascontiguousarray(p4o[0]))
        assert rel(w, wo[0]) <= FP64_TOL
        for d in range(2):
            assert np.all(np.abs(p[4 * d:4 * d + 4] - q4o[d, :, 0]) <= FP64_TOL * q4o[d, 0, 0]), (g, d)
    sys.stdout.flush()
