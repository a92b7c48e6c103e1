"""The column-blocked scheme on the CPU: its passes (every block re-run from
T_0 with the row scalings known so far, squared norms summed over blocks)
written densely in numpy, against the oracle's plain recurrence.  This pins
the decomposition the GPU's column-blocked form relies on: columns interact
only through the row norms (Section 3.2), so T_t = diag(s_t) M T_{t-1} with
s_t = 1 / ||(M T_{t-1})_a|| per row (0 for a zero row)."""

import numpy as np
import pytest

import gen
import oracle


def dense_m(g, keep):
    adj = oracle.build_graph(g)
    n = g.n
    A = np.zeros((n, n))
    for a in range(n):
        for j in range(adj.row_ptr[a], adj.row_ptr[a + 1]):
            A[a, adj.col[j]] += adj.aval[j]
    deg = A.sum(1)
    M = np.zeros_like(A)
    M[deg > 0] = A[deg > 0] / deg[deg > 0, None]
    empty = np.where(deg == 0)[0]
    if keep:  # an empty row keeps its previous row (normalised below)
        M[empty, empty] = 1.0
    return M, len(empty)


def blocked_scheme(M, T0, k, block):
    n, d = T0.shape
    blocks = [(c0, min(block, d - c0)) for c0 in range(0, d, block)]
    scales = []
    for _ in range(k):
        ss = np.zeros(n)
        for c0, w in blocks:
            X = T0[:, c0:c0 + w]
            for s in scales:
                X = s[:, None] * (M @ X)
            U = M @ X
            ss += (U * U).sum(1)
        pos = ss > 0
        s = np.zeros(n)
        s[pos] = 1.0 / np.sqrt(ss[pos])
        scales.append(s)
    out = np.empty_like(T0)
    for c0, w in blocks:
        X = T0[:, c0:c0 + w]
        for s in scales:
            X = s[:, None] * (M @ X)
        out[:, c0:c0 + w] = X
    return out


@pytest.mark.parametrize("keep", [False, True])
@pytest.mark.parametrize("block", [1, 7, 16, 50, 64])
def test_blocked_scheme_equals_recurrence(keep, block):
    g = gen.random_graph(300, 700, 3, directed=True, weighted=True, loops=True, multi=True)
    d, k, seed = 50, 4, 5
    M, n_empty = dense_m(g, keep)
    assert n_empty > 0  # directed sinks: both empty-row rules are exercised
    got = blocked_scheme(M, oracle.init(seed, g.n, d), k, block)
    want = oracle.embed(g, d, k, seed, oracle.EMPTY_KEEP if keep else 0)
    assert np.abs(got - want).max() <= 1e-13


def test_blocked_scheme_k0_is_t0():
    g = gen.erdos_renyi(100, 300, 2)
    M, _ = dense_m(g, False)
    T0 = oracle.init(9, g.n, 20)
    assert np.array_equal(blocked_scheme(M, T0, 0, 6), T0)
