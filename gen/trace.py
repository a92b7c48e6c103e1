"""Seeded request traces for the served form.

Each request is an independent graph embedding job: a Chung-Lu graph
(exponent 2.1) with N log-uniform in [100, 200k] and mean degree uniform in
[5, 30], arriving as a Poisson process at a fixed rate.  The graph itself is
generated on demand from the request's own seed.
"""

from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from .graphs import BASE_SEED, Graph, chung_lu_small, log_uniform_int


@dataclasses.dataclass
class Request:
    index: int
    arrival_s: float
    n: int
    mean_degree: float
    seed: int

    def graph(self) -> Graph:
        return chung_lu_small(self.n, self.mean_degree, self.seed)


def served_trace(n_requests: int, rate_per_s: float, seed: int = BASE_SEED + 4,
                 n_lo: int = 100, n_hi: int = 200_000,
                 deg_lo: float = 5.0, deg_hi: float = 30.0) -> List[Request]:
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        n = log_uniform_int(rng, n_lo, n_hi)
        c = float(rng.uniform(deg_lo, deg_hi))
        out.append(Request(i, float(arrivals[i]), n, c, seed * 1_000_003 + i))
    return out


def _make(req: Request) -> Graph:
    return req.graph()


def materialize(requests: List[Request], workers: int = 0) -> List[Graph]:
    """Generate every request's graph (in worker processes when workers > 1)."""
    if workers <= 1 or len(requests) < 8:
        return [r.graph() for r in requests]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        return pool.map(_make, requests, chunksize=max(1, len(requests) // (4 * workers)))
