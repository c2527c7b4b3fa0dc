"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid arguments before touching the device."""
from __future__ import annotations

import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1711_05683_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1711_05683_amd import build
        build.build()
    return P


def _declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(hydra_phsp_[a-z0-9_]+)\s*\(", text):
            names.append(m.group(1))
    return sorted(set(names))


def test_every_declared_symbol_is_exported(P):
    names = _declared_functions()
    assert "hydra_phsp_generate" in names and "hydra_phsp_integrate" in names
    lib = P.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_and_sortnet(P):
    assert P.lib().hydra_phsp_abi_version() == 1
    assert P.selftest_sortnet()


def test_strerror(P):
    for code in (P.OK, P.EINVAL, P.EKINEMATICS, P.ENOMEM, P.EDEVICE, P.EAGAIN, P.ENOTFOUND):
        assert P.lib().hydra_phsp_strerror(code)


def _gen_status(P, M, masses, nevents=10, ld=None, out=8, w=8, parent_host=None, parent_dev=None,
                ldp=0):
    m, n = P._masses(masses)
    ph = None if parent_host is None else (ctypes.c_double * 4)(*parent_host)
    return P.lib().hydra_phsp_generate(M, m, n, ph, parent_dev, ldp, nevents, 1, 0, 0,
                                       ctypes.c_void_p(out) if out else None,
                                       nevents if ld is None else ld,
                                       ctypes.c_void_p(w) if w else None, None, None)


def test_validation_before_any_device_work(P):
    # Fake non-NULL pointers: every case must fail in validation, before launch.
    assert _gen_status(P, 5.0, [1.0]) == P.EINVAL
    assert _gen_status(P, 50.0, [0.1] * 11) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, -0.1]) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, float("nan")]) == P.EINVAL
    assert _gen_status(P, float("inf"), [1.0, 1.0]) == P.EINVAL
    assert _gen_status(P, -5.0, [1.0, 1.0]) == P.EINVAL
    assert _gen_status(P, 5.0, [3.0, 2.0]) == P.EKINEMATICS
    assert _gen_status(P, 5.0, [3.0, 2.5]) == P.EKINEMATICS
    assert _gen_status(P, 5.0, [1.0, 1.0], ld=5) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, 1.0], out=0) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, 1.0], w=0) == P.EINVAL
    # parent four-vector whose mass is not M
    assert _gen_status(P, 5.0, [1.0, 1.0], parent_host=[5.0, 1.0, 0.0, 0.0]) == P.EINVAL
    # both parent forms at once
    assert _gen_status(P, 5.0, [1.0, 1.0], parent_host=[5.0, 0.0, 0.0, 0.0],
                       parent_dev=ctypes.c_void_p(8), ldp=10) == P.EINVAL
    # per-event parents with a too-short leading dimension
    assert _gen_status(P, 5.0, [1.0, 1.0], parent_dev=ctypes.c_void_p(8), ldp=3) == P.EINVAL
    assert "ld_parent" in P.lib().hydra_phsp_last_error().decode()
    # device pointers not aligned to their element size
    assert _gen_status(P, 5.0, [1.0, 1.0], out=12) == P.EINVAL
    assert "aligned" in P.lib().hydra_phsp_last_error().decode()
    assert _gen_status(P, 5.0, [1.0, 1.0], w=4) == P.EINVAL
    assert _gen_status(P, 5.0, [1.0, 1.0], parent_dev=ctypes.c_void_p(12), ldp=10) == P.EINVAL


def test_unweight_chunks_setting(P):
    for c in (0, 1, 4, 16):
        assert P.lib().hydra_phsp_set_unweight_chunks(c) == P.OK
    assert P.lib().hydra_phsp_set_unweight_chunks(-1) == P.EINVAL
    assert P.lib().hydra_phsp_set_unweight_chunks(17) == P.EINVAL
    assert "chunks" in P.lib().hydra_phsp_last_error().decode()
    P.set_unweight_chunks(0)


def test_events_per_thread_query(P):
    for path in (0, 1, 2):
        for n in range(2, 11):
            for pe in (0, 1):
                assert P.events_per_thread(path, n, bool(pe)) in (1, 2, 4)
    assert P.events_per_thread(0, 3) == 4
    P.set_events_per_thread(1, 2)
    try:
        assert P.events_per_thread(1, 3) == 2 and P.events_per_thread(1, 10, True) == 2
    finally:
        P.set_events_per_thread(1, 0)
    assert P.lib().hydra_phsp_events_per_thread(3, 3, 0) == P.EINVAL
    assert P.lib().hydra_phsp_events_per_thread(1, 11, 0) == P.EINVAL
    assert P.lib().hydra_phsp_events_per_thread(1, 3, 4) == P.EINVAL  # unknown flag
    # columns off the line grid (staged kernel) have their own defaults
    staged_fp64 = [2, 4, 2, 1, 1, 1, 1, 1, 1]
    staged_mixed = [4, 4, 2, 1, 1, 1, 1, 1, 1]
    aligned_fp64 = [2, 1, 2, 2, 4, 4, 4, 4, 4]
    aligned_mixed = [2, 4, 4, 4, 4, 4, 4, 4, 4]
    for n in range(2, 11):
        assert P.events_per_thread(1, n, off_line_grid=True) == staged_fp64[n - 2]
        assert P.events_per_thread(1, n, True, True) == staged_fp64[n - 2]
        assert P.events_per_thread(2, n, off_line_grid=True) == staged_mixed[n - 2]
        assert P.events_per_thread(1, n) == aligned_fp64[n - 2]
        assert P.events_per_thread(2, n) == aligned_mixed[n - 2]
        assert P.events_per_thread(0, n, off_line_grid=True) == 4  # integrate-only has no layout
    assert P.events_per_thread(1, 3) == 1 and P.events_per_thread(1, 3, True) == 1
    assert P.lib().hydra_phsp_events_per_thread(1, 1, 0) == P.EINVAL


def test_integrate_validation(P):
    m, n = P._masses([1.0, 1.0])
    mean, sigma = ctypes.c_double(), ctypes.c_double()
    assert P.lib().hydra_phsp_integrate(5.0, m, n, 1, 1, 0, 0, ctypes.byref(mean),
                                        ctypes.byref(sigma), None) == P.EINVAL
    assert P.lib().hydra_phsp_integrate(5.0, m, n, 10, 1, 0, 0, None, ctypes.byref(sigma),
                                        None) == P.EINVAL
    assert P.lib().hydra_phsp_integrate_async(5.0, m, n, 10, 1, 0, 0, None, None) == P.EINVAL
    m3, n3 = P._masses([3.0, 3.0])
    assert P.lib().hydra_phsp_integrate_async(5.0, m3, n3, 10, 1, 0, 0, ctypes.c_void_p(8),
                                              None) == P.EKINEMATICS


def test_product_path_does_not_import_oracle():
    # The product package must never route through the CPU oracle.
    pkg = os.path.join(ROOT, "paper_1711_05683_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if path.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
            text = open(path).read()
            assert "import oracle" not in text and "from oracle" not in text, path
            assert "phsp_oracle" not in text and "_liboracle" not in text, path


def test_struct_layouts_match_headers(P, tmp_path):
    # Compile a probe against the public header and compare with the binding.
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "hydra_phsp_batch.h"
#include "hydra_phsp_serve.h"
#include "hydra_phsp_model.h"
#include "hydra_phsp_serve.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu %zu ", sizeof(hydra_phsp_channel),
           offsetof(hydra_phsp_channel, n_daughters), offsetof(hydra_phsp_channel, nevents),
           offsetof(hydra_phsp_channel, p4_out_dev), offsetof(hydra_phsp_channel, stats_dev),
           sizeof(hydra_phsp_tuning), offsetof(hydra_phsp_tuning, grid_per_cu));
    printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(hydra_phsp_request),
           offsetof(hydra_phsp_request, integrate_only), offsetof(hydra_phsp_request, stream_id),
           sizeof(hydra_phsp_result), offsetof(hydra_phsp_result, mean),
           offsetof(hydra_phsp_result, weights_dev), offsetof(hydra_phsp_result, done_s));
    printf("%zu %zu %zu ", sizeof(hydra_phsp_breit_wigner), offsetof(hydra_phsp_breit_wigner, mass),
           offsetof(hydra_phsp_breit_wigner, width));
    printf("%zu %zu %zu\n", sizeof(hydra_phsp_server_counters), offsetof(hydra_phsp_server_counters, budget_stalls),
           offsetof(hydra_phsp_server_counters, queue_wait_sum_s));
    return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    C, T, Q, R = P.ChannelDesc, P.Tuning, P.RequestDesc, P.ResultDesc
    want = [ctypes.sizeof(C), C.n_daughters.offset, C.nevents.offset, C.p4_out_dev.offset,
            C.stats_dev.offset, ctypes.sizeof(T), T.grid_per_cu.offset,
            ctypes.sizeof(Q), Q.integrate_only.offset, Q.stream_id.offset,
            ctypes.sizeof(R), R.mean.offset, R.weights_dev.offset, R.done_s.offset,
            ctypes.sizeof(P.BreitWigner), P.BreitWigner.mass.offset, P.BreitWigner.width.offset,
            ctypes.sizeof(P.ServerCounters), P.ServerCounters.budget_stalls.offset,
            P.ServerCounters.queue_wait_sum_s.offset]
    assert got == want


def test_batch_tuning_validation(P):
    good = P.channel(5.0, [1.0, 1.0], 10, stats=None)
    good.stats_dev = 8  # fake device pointer: validation happens before any device work
    arr = P._channel_array([good])
    for kw in ({"streams": 5}, {"streams": -1}, {"schedule": 6}, {"ept": 3}, {"grid_per_cu": 65}):
        t = P._tuning(**kw)
        assert P.lib().hydra_phsp_batch_run(arr, 1, ctypes.byref(t), None, None) == P.EINVAL, kw


def test_batch_validation_names_bad_channel(P):
    good = P.channel(5.0, [1.0, 1.0], 10, stats=None)
    good.stats_dev = 8  # fake device pointer: validation happens before any device work
    bad = P.channel(5.0, [3.0, 3.0], 10)
    bad.stats_dev = 8
    arr = P._channel_array([good, good, bad])
    idx = ctypes.c_int(-1)
    st = P.lib().hydra_phsp_batch_run(arr, 3, None, None, ctypes.byref(idx))
    assert st == P.EKINEMATICS and idx.value == 2
    half = P.channel(5.0, [1.0, 1.0], 10)
    half.stats_dev = 8
    half.p4_out_dev = 16  # outputs without weights
    half.ld = 10
    arr = P._channel_array([half])
    assert P.lib().hydra_phsp_batch_run(arr, 1, None, None, ctypes.byref(idx)) == P.EINVAL
    assert idx.value == 0
    t = P._tuning(ept=3)
    arr = P._channel_array([good])
    assert P.lib().hydra_phsp_batch_run(arr, 1, ctypes.byref(t), None, ctypes.byref(idx)) == P.EINVAL
    assert P.lib().hydra_phsp_batch_run(arr, 0, None, None, ctypes.byref(idx)) == P.EINVAL
    for bad_t in (P._tuning(schedule=6), P._tuning(schedule=-1), P._tuning(grid_per_cu=65)):
        assert P.lib().hydra_phsp_batch_run(arr, 1, ctypes.byref(bad_t), None, ctypes.byref(idx)) == P.EINVAL


def test_batch_single_launch_needs_line_aligned_columns(P):
    """Schedules 3, 4 and 5 (one launch over every tile) run the direct-store
    kernel only: a generating channel off the 128-byte line grid, or an
    events-per-thread setting other than 0 or 1, is rejected before any device
    work."""
    aligned = P.channel(5.0, [1.0, 1.0], 100, stats=None)
    aligned.stats_dev, aligned.p4_out_dev, aligned.weights_dev, aligned.ld = 8, 1 << 20, 1 << 21, 128
    off = P.channel(5.0, [1.0, 1.0], 100, stats=None)
    off.stats_dev, off.p4_out_dev, off.weights_dev, off.ld = 8, 1 << 20, 1 << 21, 100
    idx = ctypes.c_int(-1)
    arr = P._channel_array([aligned, off])
    for sched in (3, 4, 5):
        arr = P._channel_array([aligned, off])
        t = P._tuning(schedule=sched)
        assert P.lib().hydra_phsp_batch_run(arr, 2, ctypes.byref(t), None, ctypes.byref(idx)) == P.EINVAL
        assert idx.value == 1 and "line grid" in P.lib().hydra_phsp_last_error().decode()
        arr = P._channel_array([aligned])
        for ept in (2, 4):
            t = P._tuning(schedule=sched, ept=ept)
            assert P.lib().hydra_phsp_batch_run(arr, 1, ctypes.byref(t), None, ctypes.byref(idx)) == P.EINVAL
            assert "ept 0" in P.lib().hydra_phsp_last_error().decode()
        t = P._tuning(schedule=sched, grid_per_cu=65)
        assert P.lib().hydra_phsp_batch_run(arr, 1, ctypes.byref(t), None, ctypes.byref(idx)) == P.EINVAL
    t = P._tuning(schedule=6)
    assert P.lib().hydra_phsp_batch_run(arr, 1, ctypes.byref(t), None, ctypes.byref(idx)) == P.EINVAL


def test_unweighted_validation(P):
    m, n = P._masses([1.0, 1.0, 0.5])
    f = P.lib().hydra_phsp_generate_unweighted
    cnt, out, idx = ctypes.c_void_p(64), ctypes.c_void_p(128), ctypes.c_void_p(256)

    def call(M=5.0, w_max=0.0, out=out, ld=10, idx=None, counts=cnt, parent=None, ntrials=100, mm=m, nn=n):
        ph = None if parent is None else (ctypes.c_double * 4)(*parent)
        return f(M, mm, nn, ph, ntrials, 1, 0, 0, w_max, out, ld, idx, counts, None, None)

    assert call(w_max=-1.0) == P.EINVAL
    assert call(w_max=float("nan")) == P.EINVAL
    assert call(w_max=float("inf")) == P.EINVAL
    assert call(counts=None) == P.EINVAL
    assert "counts_dev" in P.lib().hydra_phsp_last_error().decode()
    assert call(ld=0) == P.EINVAL
    assert call(out=None, idx=idx, ld=0) == P.EINVAL
    assert call(out=ctypes.c_void_p(132)) == P.EINVAL
    assert call(counts=ctypes.c_void_p(68)) == P.EINVAL
    assert call(M=2.0) == P.EKINEMATICS
    assert call(parent=[5.0, 1.0, 0.0, 0.0]) == P.EINVAL  # parent mass is not M
    m1, n1 = P._masses([1.0])
    assert call(mm=m1, nn=n1) == P.EINVAL


def test_model_validation(P):
    m, n = P._masses([3.097, 0.4937, 0.13957])
    f = P.lib().hydra_phsp_integrate_model

    def call(res, st=ctypes.c_void_p(64), vals=None, k=None, M=5.279):
        arr = (P.BreitWigner * max(len(res), 1))(*[P.BreitWigner(*r) for r in res])
        return f(M, m, n, ctypes.cast(arr, ctypes.c_void_p), len(res) if k is None else k, 100, 1, 0, 0, vals, st,
                 None)

    assert call([(0, 1, 1.0, 0.1)], st=None) == P.EINVAL
    assert call([(1, 1, 1.0, 0.1)]) == P.EINVAL
    assert call([(1, 0, 1.0, 0.1)]) == P.EINVAL
    assert call([(0, 3, 1.0, 0.1)]) == P.EINVAL
    assert call([(0, 1, 0.0, 0.1)]) == P.EINVAL
    assert call([(0, 1, 1.0, -0.1)]) == P.EINVAL
    assert call([(0, 1, float("inf"), 0.1)]) == P.EINVAL
    assert call([(0, 1, 1.0, 0.1)] * 5) == P.EINVAL
    assert call([(0, 1, 1.0, 0.1)], k=-1) == P.EINVAL
    assert call([(0, 1, 1.0, 0.1)], vals=ctypes.c_void_p(12)) == P.EINVAL
    assert call([(0, 1, 1.0, 0.1)], M=3.5) == P.EKINEMATICS


def test_unweighted_model_validation(P):
    m, n = P._masses([3.097, 0.4937, 0.13957])
    f = P.lib().hydra_phsp_generate_unweighted_model
    out, cnt = ctypes.c_void_p(1024), ctypes.c_void_p(256)

    def call(res=((1, 2, 0.8955, 0.0473),), k=None, M=5.279, w_max=0.0, o=out, ld=128, counts=cnt):
        arr = (P.BreitWigner * max(len(res), 1))(*[P.BreitWigner(*r) for r in res])
        return f(M, m, n, ctypes.cast(arr, ctypes.c_void_p), len(res) if k is None else k, 100, 1, 0, 0, w_max, o,
                 ld, None, counts, None, None)

    assert call([(1, 1, 1.0, 0.1)]) == P.EINVAL
    assert call([(0, 3, 1.0, 0.1)]) == P.EINVAL
    assert call([(0, 1, 1.0, 0.0)]) == P.EINVAL
    assert call([(0, 1, float("nan"), 0.1)]) == P.EINVAL
    assert call([(0, 1, 1.0, 0.1)] * 5) == P.EINVAL
    assert call(k=-1) == P.EINVAL
    assert call(counts=None) == P.EINVAL
    assert call(w_max=-2.0) == P.EINVAL
    assert call(w_max=float("inf")) == P.EINVAL
    assert call(ld=0) == P.EINVAL
    assert call(counts=ctypes.c_void_p(260)) == P.EINVAL
    assert call(M=3.5) == P.EKINEMATICS
    assert f(5.279, None, 3, None, 0, 100, 1, 0, 0, 0.0, out, 128, None, cnt, None, None) == P.EINVAL


def test_vegas_validation_and_host_refinement(P):
    import numpy as np
    import oracle
    f = P.gauss_box([0.0] * 3, [1.0] * 3, [0.5] * 3, [0.2] * 3)
    st = ctypes.c_void_p(64)
    g = ctypes.c_void_p(128)
    call = P.lib().hydra_phsp_vegas_iteration
    assert call(ctypes.byref(f), 1, g, 100, 1, 0, st, None, None, None) == P.EINVAL      # bins < 2
    assert call(ctypes.byref(f), 129, g, 100, 1, 0, st, None, None, None) == P.EINVAL    # bins > 128
    assert call(ctypes.byref(f), 50, None, 100, 1, 0, st, None, None, None) == P.EINVAL  # no grid
    assert call(ctypes.byref(f), 50, g, 100, 1, 0, None, None, None, None) == P.EINVAL   # no stats
    assert call(ctypes.byref(f), 50, g, 1, 1, 0, st, None, None, None) == P.EINVAL       # one call: no error
    assert call(ctypes.byref(f), 50, g, 0, 1, 0, st, None, None, None) == P.EINVAL       # no calls
    bad = P.gauss_box([0.0] * 3, [1.0, 0.0, 1.0], [0.5] * 3, [0.2] * 3)
    assert call(ctypes.byref(bad), 50, g, 100, 1, 0, st, None, None, None) == P.EINVAL   # hi <= lo
    bad = P.gauss_box([0.0] * 3, [1.0] * 3, [0.5] * 3, [0.2, 0.0, 0.2])
    assert call(ctypes.byref(bad), 50, g, 100, 1, 0, st, None, None, None) == P.EINVAL   # sigma <= 0
    bad.dim = 17
    assert call(ctypes.byref(bad), 50, g, 100, 1, 0, st, None, None, None) == P.EINVAL
    # the library's host refinement against the oracle's (independent code, same rule)
    oracle.build(force=False)
    rng = np.random.default_rng(4)
    for dim, bins in ((1, 2), (3, 50), (10, 50), (2, 128)):
        grid = oracle.uniform_grid(dim, bins)
        for _ in range(4):
            h = rng.exponential(size=(dim, bins)) * np.exp(-0.5 * ((np.arange(bins) - bins / 3) / (bins / 8)) ** 2)
            h[:, rng.integers(0, bins)] = 0.0
            a = P.vegas_refine(grid, h, 1.5)
            b = oracle.vegas_refine(grid, h, 1.5)
            assert np.allclose(a, b, rtol=0.0, atol=1e-13), float(np.abs(a - b).max())
            grid = a


def test_probe_validation(P):
    w = P.lib().hydra_phsp_probe_write
    o, wt = ctypes.c_void_p(256), ctypes.c_void_p(512)
    assert w(None, 100, 12, wt, 100, 1, None) == P.EINVAL                     # no output
    assert w(o, 100, 12, None, 100, 1, None) == P.EINVAL                      # no weights
    assert w(ctypes.c_void_p(260), 100, 12, wt, 100, 1, None) == P.EINVAL     # misaligned
    assert w(o, 100, 0, wt, 100, 1, None) == P.EINVAL                         # no column
    assert w(o, 100, 41, wt, 100, 1, None) == P.EINVAL                        # more than 4 NMAX
    assert w(o, 100, 12, wt, 100, 3, None) == P.EINVAL                        # events per thread
    assert w(o, 99, 12, wt, 100, 1, None) == P.EINVAL                         # ld < nevents
    assert w(o, 100, 12, wt, 0, 1, None) == P.OK                              # nothing to enqueue
    ph = P.lib().hydra_phsp_probe_philox
    f = ctypes.c_void_p(64)
    assert ph(100, 3, 1, 0, None, None) == P.EINVAL
    assert ph(100, 3, 1, 0, ctypes.c_void_p(66), None) == P.EINVAL
    assert ph(100, 0, 1, 0, f, None) == P.EINVAL
    assert ph(100, 17, 1, 0, f, None) == P.EINVAL
    assert ph(0, 3, 1, 0, f, None) == P.OK


def test_event_counts_beyond_one_launch_are_rejected(P):
    """Counts whose grid would pass 2^32 - 1 threads (up to 2^64 - 1, where a
    naive ceil(n / span) wraps) fail in validation on every entry point."""
    L = P.lib()
    m, n = P._masses([1.0, 1.0, 0.5])
    big = (1 << 64) - 1
    fake = ctypes.c_void_p(256)
    # generate / mixed (FP64 at rest: 2 events per thread for N = 2, 1 for N = 3 -> 4294967040 events max)
    for cnt in (big, 1 << 40, (0xFFFFFFFF // 256) * 256 + 1):
        # columns on the line grid (one event per thread for N = 3); ld rounded up without wrapping
        ld = cnt if cnt > (1 << 63) else (cnt + 15) // 16 * 16
        assert _gen_status(P, 5.0, [1.0, 1.0, 0.5], nevents=cnt, ld=ld, out=256, w=256) == P.EINVAL, cnt
        assert "too large" in L.hydra_phsp_last_error().decode()
        if cnt > (0xFFFFFFFF // 256) * 1024:  # the mixed path runs 4 events per thread
            assert L.hydra_phsp_generate_mixed(5.0, m, n, None, None, 0, cnt, 1, 0, 0, fake, cnt, fake, None,
                                               None) == P.EINVAL
    for cnt in (big, (0xFFFFFFFF // 256) * 1024 + 1):   # integrate: 4 events per thread
        assert L.hydra_phsp_integrate_async(5.0, m, n, cnt, 1, 0, 0, fake, None) == P.EINVAL, cnt
        assert L.hydra_phsp_integrate_model(5.0, m, n, None, 0, cnt, 1, 0, 0, None, fake, None) == P.EINVAL
        assert L.hydra_phsp_generate_unweighted(5.0, m, n, None, cnt, 1, 0, 0, 1.0, None, 0, None, fake, None,
                                                None) == P.EINVAL
        assert L.hydra_phsp_probe_philox(cnt, 3, 1, 0, fake, None) == P.EINVAL
    assert L.hydra_phsp_probe_write(fake, big, 12, fake, big, 4, None) == P.EINVAL
    f = P.gauss_box([0.0] * 3, [1.0] * 3, [0.5] * 3, [0.2] * 3)
    assert L.hydra_phsp_vegas_iteration(ctypes.byref(f), 50, fake, big, 1, 0, fake, None, None, None) == P.EINVAL
    # the batch: one channel too large for its class launch
    c = P.channel(5.0, [1.0, 1.0], 10, stats=None)
    c.stats_dev = 8
    c.nevents = big
    assert L.hydra_phsp_batch_run(P._channel_array([c]), 1, None, None, None) == P.EINVAL


def test_binding_rejects_bad_buffers_before_any_launch(P):
    """The C ABI cannot see buffer sizes or residency, so the binding rejects
    short, mistyped and host buffers before any device query or launch (this
    runs on a machine without a GPU: every case must raise ValueError first)."""
    import torch
    M, m = 5.279, [3.097, 0.4937, 0.13957]
    f64, f32, i64, i32 = torch.float64, torch.float32, torch.int64, torch.int32
    host = lambda n, dt=f64: torch.zeros(n, dtype=dt)  # noqa: E731
    cases = [
        ("weights", lambda: P.generate(M, m, 100, weights=host(99))),
        ("stats", lambda: P.generate(M, m, 100, stats=host(3))),
        ("weights", lambda: P.generate(M, m, 100, weights=host(100, f32))),
        ("out", lambda: P.generate(M, m, 100, out=torch.zeros(3, 4, 100, dtype=f32))),
        ("out", lambda: P.generate(M, m, 100, out=torch.zeros(2, 4, 100, dtype=f64))),
        ("out", lambda: P.generate(M, m, 100, out=torch.zeros(3, 4, 100, dtype=f64).transpose(0, 1))),
        ("parent_dev", lambda: P.generate(M, m, 100, parent_dev=torch.zeros(4, 99, dtype=f64))),
        ("parent_dev", lambda: P.generate(M, m, 100, parent_dev=torch.zeros(3, 100, dtype=f64))),
        ("CUDA", lambda: P.generate(M, m, 100, weights=host(100))),
        ("CUDA", lambda: P.generate(M, m, 100, out=torch.zeros(3, 4, 128, dtype=f64))),
        ("CUDA", lambda: P.generate(M, m, 100, parent_dev=torch.zeros(4, 100, dtype=f64))),
        ("counts", lambda: P.generate_unweighted(M, m, 100, counts=host(1, i64))),
        ("counts", lambda: P.generate_unweighted(M, m, 100, counts=host(2, i32))),
        ("w_max_out", lambda: P.generate_unweighted(M, m, 100, w_max_out=host(0))),
        ("index", lambda: P.generate_unweighted(M, m, 100, index=torch.zeros(2, 64, dtype=i64))),
        ("index", lambda: P.generate_unweighted(M, m, 100, out=torch.zeros(3, 4, 128, dtype=f64),
                                                index=host(64, i64))),
        ("CUDA", lambda: P.generate_unweighted(M, m, 100, counts=host(2, i64))),
        ("values", lambda: P.integrate_model(M, m, 100, values=host(99))),
        ("stats", lambda: P.integrate_model(M, m, 100, stats=host(2))),
        ("CUDA", lambda: P.integrate_model(M, m, 100, stats=host(4))),
        ("stats", lambda: P.integrate_async(M, m, 100, stats=host(3))),
        ("CUDA", lambda: P.integrate_async(M, m, 100, stats=host(4))),
        ("weights", lambda: P.probe_write(torch.zeros(12, 128, dtype=f64), host(99), 100)),
        ("CUDA", lambda: P.probe_write(torch.zeros(12, 128, dtype=f64), host(100), 100)),
        ("fold", lambda: P.probe_philox(5000, 3, fold=host(4, i32))),
        ("CUDA", lambda: P.probe_philox(5000, 3, fold=host(5, i32))),
        ("grid", lambda: P.vegas_iteration(P.gauss_box([0.0], [1.0], [0.5], [0.1]),
                                           torch.zeros(2, 51, dtype=f64), 100)),
        ("CUDA", lambda: P.vegas_iteration(P.gauss_box([0.0], [1.0], [0.5], [0.1]),
                                           torch.zeros(1, 51, dtype=f64), 100)),
        ("weights", lambda: P.channel(M, m, 100, out=torch.zeros(3, 4, 128, dtype=f64), weights=host(50),
                                      stats=host(4))),
        ("ld", lambda: P.channel(M, m, 100, out=torch.zeros(3, 4, 64, dtype=f64), weights=host(100))),
        ("stats", lambda: P.channel(M, m, 100, stats=host(2))),
        ("CUDA", lambda: P.channel(M, m, 100, stats=host(4))),
    ]
    for what, fn in cases:
        with pytest.raises(ValueError) as e:
            fn()
        assert what in str(e.value), (what, str(e.value))


def test_noalloc_rejects_counts_beyond_its_scratch_before_device_work(P):
    """hydra_phsp_generate_noalloc keeps its block partials in a fixed array of
    2^20 entries: a count that needs more blocks fails with EINVAL, before any
    device call (fake pointers, no GPU needed)."""
    f = P.lib().hydra_phsp_generate_noalloc
    m, n = P._masses([3.097, 0.4937, 0.13957])
    ept = P.events_per_thread(1, 3)
    fits = (1 << 20) * 256 * ept
    out, w, st = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), ctypes.c_void_p(1 << 22)
    # ld a multiple of 16 doubles keeps the columns on the line grid, the layout
    # whose events per thread the query above reports
    r = f(5.279, m, n, None, None, 0, fits + 1, 42, 0, 0, out, fits + 32, w, st, None)
    assert r == P.EINVAL and "noalloc" in P.lib().hydra_phsp_last_error().decode()
    m6, n6 = P._masses([0.13957] * 6)
    ept6 = P.events_per_thread(1, 6)
    r = f(10.0, m6, n6, None, None, 0, (1 << 20) * 256 * ept6 + 1, 42, 0, 0, out, 1 << 40, w, st, None)
    assert r == P.EINVAL and "noalloc" in P.lib().hydra_phsp_last_error().decode()
    # the ordinary argument checks come first, as for hydra_phsp_generate
    assert f(5.279, m, n, None, None, 0, 10, 42, 0, 0, None, 10, w, st, None) == P.EINVAL
    assert f(1.0, m, n, None, None, 0, 10, 42, 0, 0, out, 10, w, st, None) == P.EKINEMATICS


def test_stats_merge_is_the_statistics_of_the_union(P):
    """Merging the (n, mean, M2) of disjoint pieces, left to right, gives the
    statistics numpy computes over the union (two-pass, in extended precision);
    an empty piece is neutral; sigma is the standard error of the mean."""
    rng = np.random.default_rng(11)
    w = rng.lognormal(0.0, 1.5, size=100_003) * 3.0
    cuts = [0, 1, 2, 17, 50_000, 99_999, 100_003]

    def stats(x):
        x = np.asarray(x, dtype=np.longdouble)
        if len(x) == 0:
            return [0.0, 0.0, 0.0, 0.0]
        mu = x.mean()
        return [float(len(x)), float(mu), float(((x - mu) ** 2).sum()), 0.0]

    acc = [0.0, 0.0, 0.0, 0.0]
    for a, b in zip(cuts[:-1], cuts[1:]):
        acc = P.stats_merge(acc, stats(w[a:b]))
    ref = stats(w)
    n = ref[0]
    assert acc[0] == n
    assert abs(acc[1] - ref[1]) <= 1e-14 * ref[1]
    assert abs(acc[2] - ref[2]) <= 1e-12 * ref[2]
    assert abs(acc[3] - math.sqrt(ref[2] / ((n - 1) * n))) <= 1e-12 * acc[3]
    assert P.stats_merge(stats(w), [0.0, 0.0, 0.0, 0.0])[:3] == stats(w)[:3]
    assert P.stats_merge([1.0, 2.5, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]) == [1.0, 2.5, 0.0, 0.0]


@pytest.mark.parametrize("bad", [[-1.0, 1.0, 0.0], [1.5, 1.0, 0.0], [float("nan"), 1.0, 0.0],
                                 [2.0, float("inf"), 0.0], [2.0, 1.0, -1.0]])
def test_stats_merge_rejects_bad_records(P, bad):
    good = [2.0, 1.0, 0.5, 0.0]
    with pytest.raises(P.PhspError):
        P.stats_merge(bad, good)
    with pytest.raises(P.PhspError):
        P.stats_merge(good, bad)
    assert P.lib().hydra_phsp_stats_merge(None, None, None) == P.EINVAL


def test_chain_validation_before_device_work(P):
    """The two-stage entry point rejects bad arguments on the host."""
    lib = P.lib()
    m = (ctypes.c_double * 3)(3.097, 0.4937, 0.13957)
    m2 = (ctypes.c_double * 2)(0.1056583755, 0.1056583755)
    heavy = (ctypes.c_double * 2)(2.0, 1.5)
    five = (ctypes.c_double * 5)(0.1, 0.1, 0.1, 0.1, 0.1)
    fake = ctypes.c_void_p(0x10000)

    def call(chained=0, masses2=m2, n2=2, out=fake, out2=fake, ld=10, ld2=10, nev=10):
        return lib.hydra_phsp_generate_chain(5.279, m, 3, chained, masses2, n2, nev, 1, 0, 1, 0, out, ld, fake, None,
                                             out2, ld2, fake, None, None)

    assert call(chained=3) == P.EINVAL and "chained" in lib.hydra_phsp_last_error().decode()
    assert call(chained=-1) == P.EINVAL
    assert call(masses2=five, n2=5) == P.EINVAL and "n2" in lib.hydra_phsp_last_error().decode()
    assert call(masses2=heavy) == P.EKINEMATICS
    assert call(out2=None) == P.EINVAL
    assert call(ld2=5) == P.EINVAL
    assert call(out=ctypes.c_void_p(0x10004)) == P.EINVAL
