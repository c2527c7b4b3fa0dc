"""The allocation-free entry point hydra_phsp_generate_noalloc against
hydra_phsp_generate: two calls in a row through the C ABI (the second smaller),
each compared element by element with the ordinary entry point on the same
inputs (the rejection of counts beyond its fixed scratch array is checked on
the CPU, where it happens before any device work)."""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from parity import FP64_TOL, rel  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()
    return P


def _call(P, fn, M, masses, nev, out, w, st, offset=0):
    m, n = P._masses(masses)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return fn(M, m, n, None, None, 0, nev, 42, 0, offset, ctypes.c_void_p(out.data_ptr()), out.shape[2],
              ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(st.data_ptr()), s)


@pytest.mark.parametrize("masses,nevs", [([3.097, 0.4937, 0.13957], (3_000_017, 70_001)),
                                         ([0.13957] * 6, (1_000_003, 4_099))])
def test_noalloc_matches_generate_twice(P, masses, nevs):
    M = 5.279 if len(masses) == 3 else 10.0
    L = P.lib()
    n = len(masses)
    big = nevs[0]
    out = torch.empty((n, 4, P.aligned_ld(big)), dtype=torch.float64, device="cuda")
    w = torch.empty(big, dtype=torch.float64, device="cuda")
    st = torch.empty(4, dtype=torch.float64, device="cuda")
    for k, nev in enumerate(nevs):
        print(f"[noalloc] N={n} call {k}: {nev} events", flush=True)
        out.fill_(-7.0)
        w.fill_(-7.0)
        assert _call(P, L.hydra_phsp_generate_noalloc, M, masses, nev, out, w, st, offset=k) == P.OK, \
            L.hydra_phsp_last_error()
        torch.cuda.synchronize()
        p4a, wa, sa = out[:, :, :nev].cpu().numpy(), w[:nev].cpu().numpy(), st.cpu().numpy()
        # the rest of the buffers is untouched
        assert bool((out[:, :, nev:] == -7.0).all()) and bool((w[nev:] == -7.0).all())
        assert _call(P, L.hydra_phsp_generate, M, masses, nev, out, w, st, offset=k) == P.OK
        torch.cuda.synchronize()
        p4b, wb, sb = out[:, :, :nev].cpu().numpy(), w[:nev].cpu().numpy(), st.cpu().numpy()
        # same kernels, same merge tree: element-wise equal; the bar is the FP64 tolerance
        scale = np.abs(p4b[:, 0:1, :])
        assert np.max(np.abs(p4a - p4b) / scale) <= FP64_TOL
        assert np.max(np.abs(wa - wb) / wb) <= FP64_TOL
        assert sa[0] == nev == sb[0]
        assert rel(sa[1], sb[1]) <= FP64_TOL and rel(sa[3], sb[3]) <= FP64_TOL
        assert np.array_equal(p4a, p4b) and np.array_equal(wa, wb) and np.array_equal(sa, sb)


def test_noalloc_setup_call_with_no_events(P):
    """nevents = 0 performs the one-time set-up and writes empty stats."""
    L = P.lib()
    out = torch.empty((3, 4, 64), dtype=torch.float64, device="cuda")
    w = torch.empty(64, dtype=torch.float64, device="cuda")
    st = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    assert _call(P, L.hydra_phsp_generate_noalloc, 5.279, [3.097, 0.4937, 0.13957], 0, out, w, st) == P.OK
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0.0, 0.0, 0.0, 0.0]
