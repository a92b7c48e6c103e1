"""Seeded generators: determinism, counts, structure."""

import numpy as np

import gen


def _pairs(g):
    lo = np.minimum(g.src, g.dst).astype(np.int64)
    hi = np.maximum(g.src, g.dst).astype(np.int64)
    return lo * g.n + hi


def test_erdos_renyi_counts_and_determinism():
    a = gen.erdos_renyi(10_000, 50_000, 2102)
    b = gen.erdos_renyi(10_000, 50_000, 2102)
    assert a.m == 50_000 and a.src.dtype == np.int32
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
    assert np.unique(_pairs(a)).size == a.m
    assert not np.any(a.src == a.dst)
    deg = np.bincount(np.concatenate([a.src, a.dst]), minlength=a.n)
    assert abs(deg.mean() - 10.0) < 1e-9
    assert 9.0 < deg.var() < 11.0  # Poisson(10)-like


def test_chung_lu_heavy_tail():
    g = gen.chung_lu(50_000, 400_000, 2.1, 7)
    assert g.m == 400_000
    assert np.unique(_pairs(g)).size == g.m
    assert not np.any(g.src == g.dst)
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    assert deg.max() > 50 * deg.mean()      # hubs
    assert np.median(deg) < deg.mean()      # skewed
    # ids are shuffled: the hub is not node 0
    assert np.argmax(deg) != 0 or deg[1] > deg.mean()


def test_bipartite_structure():
    g = gen.bipartite_zipf(2000, 500, 20_000, 1.1, 3)
    assert g.w is not None and g.w.dtype == np.float32 and np.all(g.w > 0)
    assert g.m == 20_000
    # repeated events are kept, so some pairs occur more than once
    assert np.unique(_pairs(g)).size < g.m
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    assert deg.max() > 20 * deg.mean()


def test_trace_shape():
    tr = gen.served_trace(500, 100.0)
    n = np.array([r.n for r in tr])
    assert n.min() >= 100 and n.max() <= 200_000
    t = np.array([r.arrival_s for r in tr])
    assert np.all(np.diff(t) >= 0)
    assert 2.0 < t[-1] < 8.0  # ~500 / 100 per second
    g = tr[0].graph()
    assert g.n == tr[0].n and g.m >= 1
