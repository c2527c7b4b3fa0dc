"""GPU checks of the measurement probes: the write probe stores exactly the
generator's columns and nothing past the last event; the Philox probe folds the
same words as the oracle's Philox4x32-10 (bit-exact)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[probe]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1711_05683_amd as P
    P.lib()
    oracle.build(force=False)
    return P


@pytest.mark.parametrize("cols", [12, 24, 40, 7])
@pytest.mark.parametrize("ept", [1, 2, 4])
def test_write_probe_columns(P, cols, ept):
    _say(f"write cols={cols} ept={ept}")
    n = 3 * 1024 + 77
    ld = P.aligned_ld(n) + 32
    out = torch.full((cols, ld), float("nan"), dtype=torch.float64, device="cuda")
    w = torch.full((ld,), float("nan"), dtype=torch.float64, device="cuda")
    P.probe_write(out, w, n, events_per_thread=ept)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.array_equal(o[:, :n], np.broadcast_to(np.arange(cols, dtype=np.float64)[:, None], (cols, n)))
    assert np.all(np.isnan(o[:, n:]))
    wv = w.cpu().numpy()
    assert np.all(wv[:n] == -1.0) and np.all(np.isnan(wv[n:]))


@pytest.mark.parametrize("calls", [1, 3, 13])
def test_philox_probe_matches_oracle(P, calls):
    _say(f"philox calls={calls}")
    n = 2 * 1024 + 333
    seed, sid = 0x1234_5678_9ABC_DEF1, 7
    fold = P.probe_philox(n, calls, seed=seed, stream_id=sid)
    torch.cuda.synchronize()
    got = fold.cpu().numpy().view(np.uint32)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    want = []
    for b in range((n + P.PROBE_SPAN - 1) // P.PROBE_SPAN):
        x = 0
        for e in range(b * P.PROBE_SPAN, min(n, (b + 1) * P.PROBE_SPAN)):
            for j in range(calls):
                for word in oracle.philox4x32_10((e & 0xFFFFFFFF, e >> 32, j, sid), key):
                    x ^= word
        want.append(x)
    assert got.tolist() == want
