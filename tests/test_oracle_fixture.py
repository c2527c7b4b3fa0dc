"""The oracle against its own frozen output (tests/golden/oracle_events.txt):
a change to its arithmetic must show up here and be justified by the passage
of the paper, or the reading of it, that requires it."""
from __future__ import annotations

import importlib.util
import os

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _maker():
    spec = importlib.util.spec_from_file_location("make_oracle_fixture",
                                                  os.path.join(HERE, "golden", "make_oracle_fixture.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_matches_its_frozen_output():
    oracle.build(force=False)
    want = [ln for ln in open(os.path.join(HERE, "golden", "oracle_events.txt")).read().splitlines()
            if not ln.startswith("#")]
    got = _maker().lines()
    assert len(got) == len(want)
    for a, b in zip(got, want):
        assert a == b, (a[:120], b[:120])
