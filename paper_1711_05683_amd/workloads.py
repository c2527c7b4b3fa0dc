"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

The paper's phase-space experiment (arXiv:1711.05683 sec. 4.2, figure
"fig:phsp") times three-body decays against sample size without publishing the
masses, sizes or precision, so these synthetic configurations stand in for it.
Both the HIP path and the CPU oracle take their inputs from here.

* ``CFG0`` -- B -> J/psi K pi-like three-body decay at rest, 1e5 events (the
  parity configuration) and its massless counterpart at M = 1;
* ``CFG1`` -- the same topology at 1e8 events (the throughput configuration),
  parent at rest or one parent per event with pz ~ U[0, 20] GeV;
* ``CFG2`` -- six pions (and six massless bodies) from M = 10 GeV, 5e7 events;
* ``batched_channels`` -- 64 channels: N ~ U{2..8}, M ~ U(2, 12) GeV, masses
  ~ U(0, 0.4 M / N), events ~ log-U(1e3, 1e7);
* ``serving_requests`` -- Poisson arrivals at 2000 req/s over 60 s; N ~
  U{2..10}, masses as above, events ~ log-U(1e3, 1e6), 30% integrate-only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass(frozen=True)
class Decay:
    parent_mass: float
    masses: tuple
    nevents: int
    seed: int = 42
    stream_id: int = 0

    @property
    def n(self) -> int:
        return len(self.masses)


CFG0 = Decay(5.279, (3.097, 0.4937, 0.13957), 100_000)
CFG0_MASSLESS = Decay(1.0, (0.0, 0.0, 0.0), 100_000)
CFG1 = Decay(5.279, (3.097, 0.4937, 0.13957), 100_000_000)
CFG2_PIONS = Decay(10.0, (0.13957,) * 6, 50_000_000)
CFG2_MASSLESS = Decay(10.0, (0.0,) * 6, 50_000_000)

PARENT_PZ_MAX = 20.0
PARENT_SEED = 43


def per_event_parents(parent_mass: float, nevents: int, device="cuda", seed: int = PARENT_SEED):
    """[4, nevents] float64 tensor of parents (E, 0, 0, pz), pz ~ U[0, 20) GeV.

    Drawn with torch's seeded generator on ``device``; E = sqrt(M^2 + pz^2) so
    every parent has invariant mass M."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    pz = torch.rand(nevents, generator=gen, dtype=torch.float64, device=device) * PARENT_PZ_MAX
    out = torch.zeros((4, nevents), dtype=torch.float64, device=device)
    out[3] = pz
    out[0] = torch.sqrt(parent_mass * parent_mass + pz * pz)
    return out


@dataclass
class Channel:
    parent_mass: float
    masses: List[float]
    nevents: int
    seed: int
    stream_id: int

    @property
    def n(self) -> int:
        return len(self.masses)


def _random_decay(rng, nmin, nmax):
    n = int(rng.integers(nmin, nmax + 1))
    M = float(rng.uniform(2.0, 12.0))
    masses = [float(x) for x in rng.uniform(0.0, 0.4 * M / n, size=n)]
    return M, masses


def batched_channels(n_channels: int = 64, seed: int = 1711, nmin: int = 2, nmax: int = 8,
                     log_events=(3.0, 7.0), event_seed: int = 42) -> List[Channel]:
    """Decay channels of the batched configuration (stream id = channel index)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_channels):
        M, masses = _random_decay(rng, nmin, nmax)
        nev = int(round(10.0 ** rng.uniform(*log_events)))
        out.append(Channel(M, masses, nev, event_seed, c))
    return out


@dataclass
class Request:
    arrival_s: float
    parent_mass: float
    masses: List[float]
    nevents: int
    seed: int
    stream_id: int
    integrate_only: bool


def serving_requests(rate_hz: float = 2000.0, duration_s: float = 60.0, seed: int = 5683,
                     nmin: int = 2, nmax: int = 10, log_events=(3.0, 6.0),
                     integrate_fraction: float = 0.3) -> List[Request]:
    """Poisson request stream of the serving configuration."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        M, masses = _random_decay(rng, nmin, nmax)
        nev = int(round(10.0 ** rng.uniform(*log_events)))
        req_seed = int(rng.integers(0, 2 ** 63 - 1))
        integ = bool(rng.uniform() < integrate_fraction)
        reqs.append(Request(t, M, masses, nev, req_seed, 0, integ))
    return reqs


def output_bytes(n: int, nevents: int, mixed: bool = False) -> int:
    """Bytes one event set occupies in HBM: 4N momentum components + a weight."""
    comp = 4 if mixed else 8
    return nevents * (4 * n * comp + 8)
