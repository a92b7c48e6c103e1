"""Seeded synthetic graphs shaped like the paper's workloads.

The paper evaluates on public social / road / follower graphs (its dataset
table in Section 5) that are not shipped here.  These generators stand in for
them with the same kind of structure:

* Erdos-Renyi G(n, m): uniform degrees, the small correctness workload.
* Chung-Lu with a power-law weight sequence: heavy-tailed degrees like the
  social and follower graphs, with hub rows of hundreds of thousands of
  neighbours.
* A weighted user-item bipartite graph with Zipf item popularity and
  log-normal interaction weights, the interaction-network case the paper's
  transition-matrix definition (Section 3.2) is written for: repeated events
  between the same pair are kept as separate edges so that the CSR build has
  to sum them.

Node ids are shuffled with a seeded permutation, so hubs are not clustered at
low ids (the paper hashes entity ids, Section 4.3).  Every generator is a
pure function of its arguments and seed; the arithmetic of the embedding
method does not appear here.
"""

from __future__ import annotations

import dataclasses
import math
import os
import time
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, Optional

import numpy as np

# print one line per drawing round (for long generations)
PROGRESS = False

BASE_SEED = 2102

# threads for the inverse-CDF lookups of large draws (the machine's CPU share)
THREADS = min(16, os.cpu_count() or 1)


def _inverse_cdf(cdf: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Index of the first CDF entry above each uniform draw, capped at the
    last index.  Large draws are looked up in parallel slices (numpy
    releases the GIL here); the result does not depend on the slicing."""
    n = cdf.size
    if u.size < (1 << 22) or THREADS < 2:
        return np.minimum(np.searchsorted(cdf, u, side="right"), n - 1)
    out = np.empty(u.size, np.int64)
    bounds = np.linspace(0, u.size, 4 * THREADS + 1).astype(np.int64)

    def look(i):
        a, b = bounds[i], bounds[i + 1]
        out[a:b] = np.minimum(np.searchsorted(cdf, u[a:b], side="right"), n - 1)

    with ThreadPoolExecutor(THREADS) as ex:
        list(ex.map(look, range(bounds.size - 1)))
    return out


@dataclasses.dataclass
class Graph:
    """An edge list.  ``src``/``dst`` are int32 node ids in [0, n);
    ``w`` is None (unweighted: every edge counts 1) or float32 > 0.
    Undirected graphs list each edge once; the CSR build stores both
    directions."""

    n: int
    src: np.ndarray
    dst: np.ndarray
    w: Optional[np.ndarray]
    directed: bool
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.size)

    def nnz_upper(self) -> int:
        """Upper bound on stored CSR entries before duplicate merging."""
        return self.m if self.directed else 2 * self.m


def _distinct_pairs(rng: np.random.Generator, n: int, m: int,
                    sampler: Callable[[int], np.ndarray],
                    max_rounds: int = 200) -> tuple[np.ndarray, np.ndarray]:
    """Draw endpoint pairs with ``sampler`` until at least ``m`` distinct
    unordered non-loop pairs are found, then drop a seeded uniform subset of
    the surplus so exactly ``m`` remain (no pair is favoured)."""
    if m > n * (n - 1) // 2:
        raise ValueError(f"m={m} exceeds the {n * (n - 1) // 2} possible pairs")
    kept = np.empty(0, np.int64)  # sorted, distinct keys lo * n + hi
    gain = 1.0  # distinct pairs gained per pair drawn, from the last round
    t0 = time.time()
    for rnd in range(max_rounds):
        deficit = m - kept.size
        if deficit <= 0:
            break
        k = int(deficit / max(gain, 1e-3) * 1.1) + 64
        a = sampler(k).astype(np.int64)
        b = sampler(k).astype(np.int64)
        ok = a != b
        a, b = a[ok], b[ok]
        if PROGRESS:
            print(f"[gen] n={n}: round {rnd}: sampled {k} pairs ({time.time() - t0:.1f}s)",
                  flush=True)
        new = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
        if kept.size:
            pos = np.searchsorted(kept, new)
            present = kept[np.minimum(pos, kept.size - 1)] == new
            new, pos = new[~present], pos[~present]
            kept = np.insert(kept, pos, new)
        else:
            kept = new
        gain = max(new.size / k, 1e-3)
        if PROGRESS:
            print(f"[gen] n={n}: round {rnd}: drew {k} pairs, {kept.size} of {m} distinct "
                  f"({time.time() - t0:.1f}s)", flush=True)
    else:
        raise RuntimeError(f"could not draw {m} distinct pairs on {n} nodes")
    if kept.size > m:
        drop = rng.choice(kept.size, kept.size - m, replace=False)
        kept = np.delete(kept, drop)
    kept = kept[rng.permutation(kept.size)]
    return kept // n, kept % n


def _relabel(rng: np.random.Generator, n: int, *arrays: np.ndarray):
    perm = rng.permutation(n).astype(np.int64)
    return [perm[a].astype(np.int32) for a in arrays]


def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """G(n, m): ``m`` distinct unordered non-loop pairs chosen uniformly."""
    rng = np.random.default_rng(seed)
    lo, hi = _distinct_pairs(rng, n, m, lambda k: rng.integers(0, n, k))
    src, dst = _relabel(rng, n, lo, hi)
    return Graph(n, src, dst, None, False, f"er_n{n}_m{m}")


def _power_law_cdf(n: int, exponent: float) -> np.ndarray:
    # Chung-Lu expected-degree sequence w_i proportional to (i+1)^(-1/(gamma-1)).
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (exponent - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def chung_lu(n: int, m: int, exponent: float, seed: int) -> Graph:
    """Chung-Lu graph: endpoints drawn i.i.d. proportional to a power-law
    weight sequence; loops and repeated pairs are rejected and the draw is
    topped up until ``m`` distinct undirected edges exist."""
    rng = np.random.default_rng(seed)
    cdf = _power_law_cdf(n, exponent)

    def sampler(k: int) -> np.ndarray:
        return _inverse_cdf(cdf, rng.random(k))

    lo, hi = _distinct_pairs(rng, n, m, sampler)
    src, dst = _relabel(rng, n, lo, hi)
    return Graph(n, src, dst, None, False, f"chunglu_g{exponent}_n{n}_m{m}")


def bipartite_zipf(n_users: int, n_items: int, n_events: int, zipf_a: float,
                   seed: int) -> Graph:
    """Weighted user-item interactions: users uniform, items Zipf(``zipf_a``)
    over popularity ranks (rank -> item id shuffled), weights log-normal(0, 1)
    rounded to float32.  Repeated (user, item) events stay separate edges."""
    rng = np.random.default_rng(seed)
    n = n_users + n_items
    users = rng.integers(0, n_users, n_events)
    rank_w = np.arange(1, n_items + 1, dtype=np.float64) ** (-zipf_a)
    cdf = np.cumsum(rank_w)
    cdf /= cdf[-1]
    ranks = _inverse_cdf(cdf, rng.random(n_events))
    item_of_rank = rng.permutation(n_items)
    items = n_users + item_of_rank[ranks]
    w = rng.lognormal(0.0, 1.0, n_events).astype(np.float32)
    # a float32 log-normal draw cannot round to zero or overflow, but keep
    # the contract (finite, > 0) explicit
    w = np.maximum(w, np.float32(np.finfo(np.float32).tiny))
    src, dst = _relabel(rng, n, users, items)
    return Graph(n, src, dst, w, False,
                 f"bipartite_u{n_users}_i{n_items}_e{n_events}")


def random_graph(n: int, m: int, seed: int, directed: bool = False,
                 weighted: bool = False, loops: bool = False,
                 multi: bool = False) -> Graph:
    """Small general-purpose test graph: ``m`` endpoint pairs drawn
    uniformly, optionally keeping loops and repeated pairs, optional
    log-normal weights."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, m)
    b = rng.integers(0, n, m)
    if not loops:
        ok = a != b
        a, b = a[ok], b[ok]
    if not multi:
        key = (a * n + b) if directed else (np.minimum(a, b) * n + np.maximum(a, b))
        _, idx = np.unique(key, return_index=True)
        idx.sort()
        a, b = a[idx], b[idx]
    w = rng.lognormal(0.0, 1.0, a.size).astype(np.float32) if weighted else None
    return Graph(n, a.astype(np.int32), b.astype(np.int32), w, directed,
                 f"random_n{n}_m{m}")


# Named workloads: (generator, d, k, dtype) with the shapes of the paper's
# dataset table (Section 5) scaled to the sizes used for measurement.
WORKLOADS = {
    "er10k": dict(make=lambda: erdos_renyi(10_000, 50_000, BASE_SEED + 0),
                  dim=128, k=4, dtype="f32",
                  desc="Erdos-Renyi N=10,000, 50,000 undirected edges, d=128, k=4"),
    "chunglu1m": dict(make=lambda: chung_lu(1_000_000, 20_000_000, 2.1, BASE_SEED + 1),
                      dim=256, k=4, dtype="f32",
                      desc="Chung-Lu gamma=2.1, N=1M, 20M undirected edges, d=256, k=4"),
    "chunglu10m": dict(make=lambda: chung_lu(10_000_000, 200_000_000, 2.2, BASE_SEED + 2),
                       dim=1024, k=5, dtype="f32",
                       desc="Chung-Lu gamma=2.2, N=10M, 200M undirected edges, d=1024, k=5"),
    "bipartite6m": dict(make=lambda: bipartite_zipf(5_000_000, 1_000_000, 100_000_000, 1.1,
                                                    BASE_SEED + 3),
                        dim=512, k=4, dtype="bf16",
                        desc="bipartite 5M users x 1M Zipf(1.1) items, 100M log-normal "
                             "weighted events, d=512, k=4"),
}


def workload(name: str) -> tuple[Graph, int, int, str]:
    spec = WORKLOADS[name]
    return spec["make"](), spec["dim"], spec["k"], spec["dtype"]


def chung_lu_small(n: int, mean_degree: float, seed: int, exponent: float = 2.1) -> Graph:
    """Chung-Lu graph with ``round(n * c / 2)`` edges, capped below the number
    of possible pairs (used for served requests)."""
    m = int(round(n * mean_degree / 2.0))
    m = max(1, min(m, (n * (n - 1) // 2) // 3))
    return chung_lu(n, m, exponent, seed)


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
