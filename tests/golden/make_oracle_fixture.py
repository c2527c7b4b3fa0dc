"""Writes tests/golden/oracle_events.txt: output of the CPU oracle (and nothing
else) for a few fixed cases, so that any later change to the oracle's
arithmetic shows up as a changed fixture.  These values pin the oracle to its
own past, not to the paper: the paper prints no worked phase-space example.

Run from the repository root: python tests/golden/make_oracle_fixture.py
"""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

CASES = [
    # name, parent mass, daughter masses, seed, stream id, event offset, events
    ("config0", 5.279, [3.097, 0.4937, 0.13957], 42, 0, 0, 4),
    ("config0_high_counter", 5.279, [3.097, 0.4937, 0.13957], 42, 0, (1 << 32) - 2, 4),
    ("six_pions", 10.0, [0.13957] * 6, 42, 3, 1000, 3),
    ("two_body", 5.0, [1.0, 2.0], 7, 1, 0, 2),
    ("ten_massless", 10.0, [0.0] * 10, 11, 0, 5, 2),
]
INTEGRALS = [
    ("config0", 5.279, [3.097, 0.4937, 0.13957], 42, 0, 0, 100_000),
    ("six_pions", 10.0, [0.13957] * 6, 42, 0, 0, 50_000),
]


def lines():
    out = []
    for name, M, m, seed, sid, off, n in CASES:
        p4, w = oracle.generate(M, m, n, seed=seed, stream_id=sid, event_offset=off)
        for e in range(n):
            comps = " ".join(repr(float(p4[d, c, e])) for d in range(len(m)) for c in range(4))
            out.append(f"event {name} {off + e} {repr(float(w[e]))} {comps}")
    for name, M, m, seed, sid, off, n in INTEGRALS:
        mean, sigma = oracle.integrate(M, m, n, seed=seed, stream_id=sid, event_offset=off)
        out.append(f"integral {name} {n} {repr(float(mean))} {repr(float(sigma))}")
    return out


HEADER = [
    "# CPU oracle output for fixed cases (written by tests/golden/make_oracle_fixture.py, which calls only oracle/).",
    "# A regression fixture of the oracle itself, not a pin from the paper (sec. 4.2 prints no worked example).",
    "# event <case> <global index> <weight> <E px py pz of daughter 0> ... ; integral <case> <events> <mean> <sigma>",
]

if __name__ == "__main__":
    oracle.build(force=False)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_events.txt")
    with open(path, "w") as f:
        f.write("\n".join(HEADER + lines()) + "\n")
    print(f"wrote {path}")
