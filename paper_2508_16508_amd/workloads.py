"""Seeded synthetic workloads (host numpy arrays).

These generators hold none of the method's arithmetic: they only draw the
inputs a caller hands to the library (masks, update records, initial
attributes, model sizes, request traces) from numpy's PCG64 generator, with
the shapes and distributions of the workloads:

* select_update microbenchmark: n = 2^24 slots x 8 int32 attributes, a
  Bernoulli(p) slot mask with p in {0.001, 0.05, 0.5}, k = popcount(mask)
  uniform int32 update records; add_agents uses the same mask as the free-slot
  pattern (alive = 1 - mask) and the same k records as newborns; remove_agents
  kills with the same mask over an all-live population.
* batched predation: 4096 models, grid side uniform in [32, 256], initial
  sheep = cells / 10 and wolves = cells / 40, capacities 4x the initial counts,
  model m seeded base + m.
* served predation: Poisson arrivals at 200 req/s over 60 s, grid side
  log-uniform in [32, 1024], step count log-uniform in [100, 5000], per-request
  seed.

The predation model's own random draws are not generated here: both the
library and the oracle compute them from the (seed, step, agent, purpose)
counter-based generator.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_SLOTS = 1 << 24
N_ATTRS = 8
DENSITIES = (0.001, 0.05, 0.5)


def _gen(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(list(key)))


def bernoulli_mask(seed: int, p: float, n: int = N_SLOTS, stream: int = 0) -> np.ndarray:
    """uint8[n], each byte 1 with probability p."""
    g = _gen(1, seed, int(round(p * 1e6)), stream)
    return (g.random(n, dtype=np.float32) < np.float32(p)).astype(np.uint8)


def int32_rows(seed: int, rows: int, cols: int, stream: int = 0) -> np.ndarray:
    """int32[rows, cols], uniform over the whole int32 range."""
    g = _gen(2, seed, rows, stream)
    return g.integers(-(2 ** 31), 2 ** 31, size=(rows, cols), dtype=np.int32)


@dataclass
class SelectUpdateCase:
    p: float
    mask: np.ndarray      # uint8[n]
    records: np.ndarray   # int32[A, k], k = popcount(mask)
    attrs: np.ndarray     # int32[A, n] initial attributes

    @property
    def k(self) -> int:
        return self.records.shape[1]


def select_update_case(seed: int, p: float, n: int = N_SLOTS, A: int = N_ATTRS,
                       with_attrs: bool = True) -> SelectUpdateCase:
    mask = bernoulli_mask(seed, p, n)
    k = int(np.count_nonzero(mask))
    recs = int32_rows(seed * 7 + 1, A, k, stream=int(round(p * 1e6)))
    attrs = int32_rows(seed * 7 + 2, A, n) if with_attrs else np.empty((A, 0), np.int32)
    return SelectUpdateCase(p, mask, recs, attrs)


@dataclass
class ModelSpec:
    side: int
    n_s0: int
    n_w0: int
    cap_s: int
    cap_w: int
    seed: int


def batched_models(base_seed: int = 0, n_models: int = 4096, lo: int = 32,
                   hi: int = 256) -> list:
    g = _gen(3, base_seed)
    sides = g.integers(lo, hi + 1, size=n_models)
    out = []
    for m, L in enumerate(sides):
        cells = int(L) * int(L)
        ns, nw = cells // 10, cells // 40
        out.append(ModelSpec(int(L), ns, nw, max(1, 4 * ns), max(1, 4 * nw), base_seed + m))
    return out


@dataclass
class Request:
    arrival_s: float
    side: int
    steps: int
    seed: int


def served_trace(seed: int = 0, rate: float = 200.0, duration_s: float = 60.0,
                 side_lo: int = 32, side_hi: int = 1024, steps_lo: int = 100,
                 steps_hi: int = 5000) -> list:
    g = _gen(4, seed)
    t, out = 0.0, []
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= duration_s:
            break
        side = int(round(np.exp(g.uniform(np.log(side_lo), np.log(side_hi)))))
        steps = int(round(np.exp(g.uniform(np.log(steps_lo), np.log(steps_hi)))))
        out.append(Request(t, side, steps, int(g.integers(0, 2 ** 32))))
    return out
