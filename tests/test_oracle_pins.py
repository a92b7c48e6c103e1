"""Pins for the FP64 oracle: checks against what the paper and the
mathematics fix, not against the oracle itself.

Each test names the passage it follows (arXiv 2102.02302).  Together they are
chosen so that a plausible slip in the oracle -- a dropped term, a transposed
M, a wrong normalisation axis, a missing merge of repeated edges, a wrong
generator constant -- fails at least one of them.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def dense_adjacency(n, src, dst, w, directed):
    """Brute-force e_ab (Section 3.2) as a dense matrix: one python loop over
    edges, no sorting, no CSR."""
    A = np.zeros((n, n))
    for e in range(len(src)):
        x = 1.0 if w is None else float(w[e])
        a, b = int(src[e]), int(dst[e])
        A[a, b] += x
        if not directed and a != b:
            A[b, a] += x
    return A


def normalise_rows(U):
    nrm = np.sqrt((U * U).sum(axis=1))
    out = np.zeros_like(U)
    nz = nrm > 0
    out[nz] = U[nz] / nrm[nz, None]
    return out


def dense_recurrence(A, T0, k, keep_empty=False, no_norm=False):
    """Algorithm 1 on dense matrices with numpy's matmul."""
    deg = A.sum(axis=1)
    M = np.zeros_like(A)
    nz = deg > 0
    M[nz] = A[nz] / deg[nz, None]
    T = T0.copy()
    for _ in range(k):
        U = M @ T
        if keep_empty:
            U[~nz] = T[~nz]
        T = U if no_norm else normalise_rows(U)
    return T


def run_oracle(n, src, dst, w, directed, T0, k, flags=0):
    adj = oracle.build_adjacency(n, np.asarray(src, np.int32), np.asarray(dst, np.int32),
                                 None if w is None else np.asarray(w, np.float32), directed)
    mval, _ = oracle.transition(adj)
    return oracle.propagate(adj, mval, T0, k, flags)


def _expr(s):
    return float(eval(s, {"sqrt": math.sqrt, "__builtins__": {}}))


# ----------------------------------------------------------- init (T_0)

def test_splitmix64_published_vectors():
    # Reference SplitMix64 generator seeded with 1234567: its first two
    # outputs are the output function applied to the seed and to the seed
    # plus the golden gamma (Steele, Lea, Flood 2014; published test values).
    assert oracle.splitmix64(1234567) == 6457827717110365317
    assert oracle.splitmix64(1234567 + 0x9E3779B97F4A7C15) == 3203168211198807973


def test_uniform_formula_and_range():
    # T_0 ~ U(-1, 1) (Section 3.2).  Reading: u = (x >> 40) / 2^23 - 1 with
    # x = splitmix64(seed ^ splitmix64(i*d + j)); exact in float32.
    seed, n, d = 99, 300, 37
    T = oracle.init(seed, n, d)
    x = oracle.splitmix64(seed ^ oracle.splitmix64(5 * d + 7))
    assert T[5, 7] == (x >> 40) / 2.0**23 - 1.0
    assert np.all(T >= -1.0) and np.all(T < 1.0)
    assert np.array_equal(T.astype(np.float32).astype(np.float64), T)
    # every value is a multiple of 2^-23
    assert np.array_equal(np.round(T * 2**23), T * 2**23)


def test_uniform_statistics():
    T = oracle.init(2102, 2000, 128).ravel()
    m = T.size
    # mean 0, variance 1/3 of U(-1,1): 6-sigma bands
    assert abs(T.mean()) < 6 * math.sqrt(1 / 3 / m)
    assert abs(T.var() - 1 / 3) < 6 * math.sqrt(4 / 45 / m)
    hist, _ = np.histogram(T, bins=16, range=(-1, 1))
    p = 1 / 16
    assert np.all(np.abs(hist - m * p) < 6 * math.sqrt(m * p * (1 - p)))


def test_init_row_offset_and_seed():
    a = oracle.init(5, 40, 16)
    b = oracle.init(5, 30, 16, row0=10)
    assert np.array_equal(a[10:], b)
    assert not np.array_equal(oracle.init(6, 40, 16), a)


# ------------------------------------------------------- adjacency / M

@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("weighted", [False, True])
def test_adjacency_matches_brute_force(directed, weighted):
    # e_ab = number of a->b edges or the sum of their weights (Section 3.2);
    # undirected edges stored both ways (Section 4.5); loops once.
    g = gen.random_graph(40, 300, seed=11, directed=directed, weighted=weighted,
                         loops=True, multi=True)
    adj = oracle.build_graph(g)
    A = dense_adjacency(g.n, g.src, g.dst, g.w, directed)
    D = np.zeros_like(A)
    for a in range(g.n):
        cols = adj.col[adj.row_ptr[a]:adj.row_ptr[a + 1]]
        assert np.all(np.diff(cols) > 0), "columns ascending, merged"
        D[a, cols] = adj.aval[adj.row_ptr[a]:adj.row_ptr[a + 1]]
    assert np.allclose(D, A, rtol=1e-15, atol=0)
    assert adj.nnz == np.count_nonzero(A)


def test_transition_row_stochastic():
    g = gen.random_graph(200, 1500, seed=3, directed=True, weighted=True, multi=True)
    adj = oracle.build_graph(g)
    mval, deg = oracle.transition(adj)
    A = dense_adjacency(g.n, g.src, g.dst, g.w, True)
    assert np.allclose(deg, A.sum(axis=1), rtol=1e-15)
    rows = np.repeat(np.arange(g.n), np.diff(adj.row_ptr))
    s = np.bincount(rows, weights=mval, minlength=g.n)
    assert np.all(np.abs(s[deg > 0] - 1.0) < 1e-14)   # M . 1 = 1
    assert np.all(s[deg == 0] == 0)


def test_invalid_inputs_rejected():
    with pytest.raises(ValueError):
        oracle.build_adjacency(3, np.array([0, 3]), np.array([1, 1]), None, False)
    with pytest.raises(ValueError):
        oracle.build_adjacency(3, np.array([0]), np.array([1]), np.array([0.0]), False)
    with pytest.raises(ValueError):
        oracle.build_adjacency(3, np.array([0]), np.array([1]), np.array([np.nan]), False)


# ------------------------------------------------------------ golden

@pytest.mark.parametrize("name", ["path3.json", "directed_weighted3.json"])
def test_golden_hand_derived(name):
    spec = json.load(open(os.path.join(GOLDEN, name)))
    g = spec["graph"]
    T0 = np.array([[_expr(x) for x in row] for row in spec["T0"]])
    for k, rows in spec["expected"].items():
        want = np.array([[_expr(x) for x in row] for row in rows])
        got = run_oracle(g["n"], g["src"], g["dst"], g["w"], g["directed"], T0, int(k))
        assert np.allclose(got, want, rtol=0, atol=1e-15), (name, k)


# ------------------------------------------------- brute force, dense

def test_all_simple_graphs_on_four_nodes():
    # Every one of the 2^6 simple undirected graphs on 4 nodes, k = 0..4,
    # against the dense recurrence (Algorithm 1).
    pairs = list(itertools.combinations(range(4), 2))
    T0 = oracle.init(17, 4, 5)
    for mask in range(64):
        e = [pairs[i] for i in range(6) if mask >> i & 1]
        src = [a for a, _ in e]
        dst = [b for _, b in e]
        A = dense_adjacency(4, src, dst, None, False)
        for k in range(5):
            got = run_oracle(4, src, dst, None, False, T0, k)
            want = dense_recurrence(A, T0, k)
            assert np.allclose(got, want, rtol=0, atol=1e-13), (mask, k)


@pytest.mark.parametrize("seed", range(6))
def test_random_weighted_directed_vs_dense(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 65))
    directed = bool(seed % 2)
    g = gen.random_graph(n, int(rng.integers(1, 4 * n)), seed=seed, directed=directed,
                         weighted=seed >= 2, loops=seed >= 4, multi=True)
    T0 = oracle.init(seed, n, 9)
    A = dense_adjacency(n, g.src, g.dst, g.w, directed)
    for flags, kw in [(0, {}), (oracle.EMPTY_KEEP, {"keep_empty": True}),
                      (oracle.NO_NORM, {"no_norm": True})]:
        got = oracle.propagate(*_adj_m(g), T0, 4, flags)
        want = dense_recurrence(A, T0, 4, **kw)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-13)


def _adj_m(g):
    adj = oracle.build_graph(g)
    return adj, oracle.transition(adj)[0]


# ------------------------------------------- closed forms, special cases

def test_k1_is_normalised_adjacency_product():
    # k = 1: T_1 = normalise(M T_0) = normalise(A T_0), since D^-1 is a
    # positive per-row factor (Section 3.2 definitions).
    g = gen.random_graph(50, 200, seed=5, weighted=True, multi=True)
    T0 = oracle.init(1, 50, 8)
    A = dense_adjacency(g.n, g.src, g.dst, g.w, False)
    got = oracle.propagate(*_adj_m(g), T0, 1)
    assert np.allclose(got, normalise_rows(np.matmul(A, T0)), atol=1e-14)


def test_no_norm_is_matrix_power():
    g = gen.random_graph(30, 90, seed=8, directed=True, weighted=True)
    T0 = oracle.init(2, 30, 6)
    A = dense_adjacency(g.n, g.src, g.dst, g.w, True)
    deg = A.sum(1)
    M = np.zeros_like(A)
    M[deg > 0] = A[deg > 0] / deg[deg > 0, None]
    got = oracle.propagate(*_adj_m(g), T0, 5, oracle.NO_NORM)
    assert np.allclose(got, np.linalg.matrix_power(M, 5) @ T0, atol=1e-13)


def test_normalised_iteration_is_not_a_matrix_power():
    # The row normalisation after every step (Algorithm 1) is not the same
    # as normalising once at the end.
    g = gen.random_graph(30, 90, seed=9)
    T0 = oracle.init(2, 30, 6)
    adj, mval = _adj_m(g)
    a = oracle.propagate(adj, mval, T0, 4)
    b = normalise_rows(oracle.propagate(adj, mval, T0, 4, oracle.NO_NORM))
    assert np.abs(a - b).max() > 1e-3


def test_degree_scaling_cancels():
    # Any positive factor per source row (here: all out-weights of row a
    # multiplied by s_a) leaves the output unchanged, and so does dropping
    # D^-1 (the unweighted and weighted-by-1 graphs agree).
    g = gen.random_graph(60, 400, seed=21, directed=True, weighted=True)
    s = np.exp(np.random.default_rng(0).normal(size=g.n)).astype(np.float32)
    g2 = gen.Graph(g.n, g.src, g.dst, (g.w * s[g.src]).astype(np.float32), True)
    T0 = oracle.init(4, g.n, 7)
    r1 = oracle.propagate(*_adj_m(g), T0, 3)
    r2 = oracle.propagate(*_adj_m(g2), T0, 3)
    assert np.allclose(r1, r2, atol=1e-6)  # float32 rounding of w * s
    ones = gen.Graph(g.n, g.src, g.dst, np.ones(g.m, np.float32), True)
    plain = gen.Graph(g.n, g.src, g.dst, None, True)
    assert np.allclose(oracle.propagate(*_adj_m(ones), T0, 3),
                       oracle.propagate(*_adj_m(plain), T0, 3), atol=1e-15)


def test_unit_rows_zero_rows_and_norm_bound():
    # Rows are normalised to unit L2 norm (Section 3.2); isolated nodes have
    # an all-zero row of M and stay zero; averaging cannot grow a norm, so
    # ||(M T_t)_a|| <= 1 for t >= 1.
    g = gen.random_graph(300, 500, seed=13)
    adj, mval = _adj_m(g)
    deg = np.diff(adj.row_ptr)
    assert (deg == 0).any()
    T = oracle.init(3, g.n, 16)
    for t in range(1, 5):
        T = oracle.propagate(adj, mval, T, 1)
        nrm = np.linalg.norm(T, axis=1)
        assert np.all(np.abs(nrm[deg > 0] - 1) < 1e-14)
        assert np.all(T[deg == 0] == 0)
        U = oracle.propagate(adj, mval, T, 1, oracle.NO_NORM)
        assert np.linalg.norm(U, axis=1).max() <= 1 + 1e-14


def test_empty_keep_reading():
    g = gen.random_graph(100, 80, seed=14)
    adj, mval = _adj_m(g)
    deg = np.diff(adj.row_ptr)
    T0 = oracle.init(3, g.n, 8)
    T = oracle.propagate(adj, mval, T0, 3, oracle.EMPTY_KEEP)
    iso = deg == 0
    assert np.allclose(T[iso], normalise_rows(T0[iso]), atol=1e-15)


def test_clique_with_loops_collapses_in_one_step():
    # Every row of M is 1/n: all rows of T_1 equal normalise(sum of T_0 rows).
    n = 7
    src = [a for a in range(n) for b in range(a, n)]
    dst = [b for a in range(n) for b in range(a, n)]
    T0 = oracle.init(8, n, 10)
    T1 = run_oracle(n, src, dst, None, False, T0, 1)
    want = T0.sum(0) / np.linalg.norm(T0.sum(0))
    assert np.allclose(T1, np.tile(want, (n, 1)), atol=1e-15)


def test_simple_clique_closed_form():
    # K_n without loops: row i of M T_0 is (S - T_0[i]) / (n-1).
    n = 6
    src = [a for a in range(n) for b in range(a + 1, n)]
    dst = [b for a in range(n) for b in range(a + 1, n)]
    T0 = oracle.init(9, n, 10)
    S = T0.sum(0)
    T1 = run_oracle(n, src, dst, None, False, T0, 1)
    assert np.allclose(T1, normalise_rows(S[None, :] - T0), atol=1e-15)


def test_star_closed_forms_and_leaf_property():
    # Star: hub 0, leaves 1..L.  The hub averages the leaves; a leaf has one
    # neighbour, so its row equals that neighbour's previous row (Section 6.2).
    L = 9
    src, dst = [0] * L, list(range(1, L + 1))
    T0 = oracle.init(10, L + 1, 12)
    T1 = run_oracle(L + 1, src, dst, None, False, T0, 1)
    hub = T0[1:].sum(0)
    assert np.allclose(T1[0], hub / np.linalg.norm(hub), atol=1e-15)
    assert np.allclose(T1[1:], np.tile(T0[0] / np.linalg.norm(T0[0]), (L, 1)), atol=1e-15)
    T_prev = T1
    for t in range(2, 6):
        T_t = run_oracle(L + 1, src, dst, None, False, T0, t)
        assert np.allclose(T_t[1:], np.tile(T_prev[0], (L, 1)), atol=1e-15)
        T_prev = T_t


def test_leaf_equals_neighbour_previous_row_general_graph():
    g = gen.random_graph(80, 120, seed=15)
    adj, mval = _adj_m(g)
    deg = np.diff(adj.row_ptr)
    leaves = np.nonzero(deg == 1)[0]
    assert leaves.size > 0
    T = oracle.init(4, g.n, 6)
    T1 = oracle.propagate(adj, mval, T, 1)
    T2 = oracle.propagate(adj, mval, T1, 1)
    nbr = adj.col[adj.row_ptr[leaves]]
    assert np.allclose(T2[leaves], T1[nbr], atol=1e-15)


# ---------------------------------------------------------- symmetries

def test_relabelling_equivariance():
    g = gen.random_graph(70, 300, seed=16, directed=True, weighted=True)
    perm = np.random.default_rng(1).permutation(g.n)
    T0 = oracle.init(5, g.n, 8)
    T0p = np.empty_like(T0)
    T0p[perm] = T0
    gp = gen.Graph(g.n, perm[g.src].astype(np.int32), perm[g.dst].astype(np.int32), g.w, True)
    r = oracle.propagate(*_adj_m(g), T0, 3)
    rp = oracle.propagate(*_adj_m(gp), T0p, 3)
    assert np.allclose(rp[perm], r, atol=1e-14)


def test_column_equivariances():
    # Dimensions are independent apart from the norm (Section 3.2): an
    # orthogonal map, a column permutation or sign flips of T_0 carry
    # through; a global positive scale of T_0 does not change T_k, k >= 1.
    g = gen.random_graph(60, 250, seed=17, weighted=True)
    adj, mval = _adj_m(g)
    T0 = oracle.init(6, g.n, 8)
    r = oracle.propagate(adj, mval, T0, 3)
    Q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(8, 8)))
    assert np.allclose(oracle.propagate(adj, mval, T0 @ Q, 3), r @ Q, atol=1e-13)
    p = np.random.default_rng(3).permutation(8)
    assert np.allclose(oracle.propagate(adj, mval, T0[:, p], 3), r[:, p], atol=1e-15)
    sgn = np.where(np.arange(8) % 3 == 0, -1.0, 1.0)
    assert np.allclose(oracle.propagate(adj, mval, T0 * sgn, 3), r * sgn, atol=1e-15)
    assert np.allclose(oracle.propagate(adj, mval, 3.5 * T0, 3), r, atol=1e-15)


# -------------------------------------------------------------- limits

def test_collapse_non_bipartite():
    # Many iterations make all embeddings identical on a connected graph
    # (Section 6.1); a triangle in the cycle breaks bipartiteness.
    n = 12
    src = list(range(n)) + [0]
    dst = [(i + 1) % n for i in range(n)] + [2]
    T0 = oracle.init(11, n, 6)
    T = run_oracle(n, src, dst, None, False, T0, 1500)
    assert np.abs(T - T[0]).max() < 1e-12


def test_collapse_bipartite_two_vectors():
    # On a connected bipartite graph the limit has one vector per side.
    n = 10  # even cycle
    src = list(range(n))
    dst = [(i + 1) % n for i in range(n)]
    T0 = oracle.init(12, n, 6)
    T = run_oracle(n, src, dst, None, False, T0, 400)
    assert np.abs(T[0::2] - T[0]).max() < 1e-12
    assert np.abs(T[1::2] - T[1]).max() < 1e-12
    assert np.abs(T[0] - T[1]).max() > 1e-3


# ------------------------------------------------------- sampled rows

def test_sampled_rows_match_dense_first_step():
    # T_1 for a subset of rows from the seed alone equals row-normalised
    # A T_0 of the dense brute-force build (Section 3.2, Algorithm 1, k = 1).
    g = gen.random_graph(120, 700, seed=31, directed=True, weighted=True, loops=True,
                         multi=True)
    rows = np.array([5, 0, 119, 37, 64, 2], np.int32)
    T0 = oracle.init(77, g.n, 12)
    A = dense_adjacency(g.n, g.src, g.dst, g.w, True)
    want = normalise_rows(np.matmul(A, T0))[rows]
    got = oracle.t1_rows(g, rows, 12, 77)
    assert np.allclose(got, want, atol=1e-14)
    sub = oracle.adjacency_rows(g, rows)
    for i, a in enumerate(rows):
        cols = sub.col[sub.row_ptr[i]:sub.row_ptr[i + 1]]
        assert np.array_equal(cols, np.nonzero(A[a])[0])
        assert np.allclose(sub.aval[sub.row_ptr[i]:sub.row_ptr[i + 1]], A[a, cols], rtol=1e-15)


def test_sampled_rows_undirected_and_empty_keep():
    g = gen.random_graph(200, 150, seed=32, loops=True)
    rows = np.arange(0, 200, 7, dtype=np.int32)
    for flags in (0, oracle.EMPTY_KEEP):
        full = oracle.embed(g, 9, 1, 5, flags)
        assert np.allclose(oracle.t1_rows(g, rows, 9, 5, flags), full[rows], atol=1e-15)


# --------------------------------------------- chunks (Algorithm 1 merge)

def test_chunked_single_chunk_is_plain():
    g = gen.random_graph(80, 300, seed=41, weighted=True, loops=True, multi=True)
    got = oracle.embed_chunked(g, [np.arange(g.m)], 8, 3, 7)
    want = oracle.embed(g, 8, 3, 7)
    deg = np.diff(oracle.build_graph(g).row_ptr)
    assert np.allclose(got[deg > 0], want[deg > 0], atol=1e-15)


def test_chunked_components_are_plain():
    # two disjoint graphs, one chunk each: every node sees its whole
    # neighbourhood in its chunk, and T_0 is keyed by global id
    a = gen.random_graph(50, 200, seed=42)
    b = gen.random_graph(40, 150, seed=43)
    g = gen.Graph(90, np.concatenate([a.src, b.src + 50]).astype(np.int32),
                  np.concatenate([a.dst, b.dst + 50]).astype(np.int32), None, False)
    chunks = [np.arange(a.m), a.m + np.arange(b.m)]
    assert np.allclose(oracle.embed_chunked(g, chunks, 6, 4, 3), oracle.embed(g, 6, 4, 3),
                       atol=1e-14)


def test_chunked_hand_example():
    # path 0-1-2 split into {0-1} and {1-2}, k = 1: node 1 occurs once in
    # each chunk, so it is the mean of normalise(T0[0]) and normalise(T0[2])
    g = gen.Graph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), None, False)
    T0 = oracle.init(5, 3, 4)
    nrm = lambda x: x / np.linalg.norm(x)  # noqa: E731
    got = oracle.embed_chunked(g, [np.array([0]), np.array([1])], 4, 1, 5)
    assert np.allclose(got[0], nrm(T0[1]), atol=1e-15)
    assert np.allclose(got[2], nrm(T0[1]), atol=1e-15)
    assert np.allclose(got[1], (nrm(T0[0]) + nrm(T0[2])) / 2, atol=1e-15)


def test_chunked_unequal_occurrence_weights():
    # node 1 has two edges in chunk A ({1,0}, {1,3}) and one in chunk B
    # ({1,2}); k = 1: T_A[1] = normalise(T0[0] + T0[3]), T_B[1] =
    # normalise(T0[2]), merged with weights 2/3 and 1/3 (Algorithm 1)
    g = gen.Graph(4, np.array([1, 1, 1], np.int32), np.array([0, 3, 2], np.int32), None, False)
    T0 = oracle.init(9, 4, 5)
    nrm = lambda x: x / np.linalg.norm(x)  # noqa: E731
    got = oracle.embed_chunked(g, [np.array([0, 1]), np.array([2])], 5, 1, 9)
    want1 = (2 * nrm(T0[0] + T0[3]) + nrm(T0[2])) / 3
    assert np.allclose(got[1], want1, atol=1e-15)
    assert np.allclose(got[0], nrm(T0[1]), atol=1e-15)   # one chunk only
    assert np.allclose(got[2], nrm(T0[1]), atol=1e-15)


def test_chunked_repeated_pair_counts_twice():
    # the pair {1,0} twice in chunk A: node 1 occurs twice there (entries
    # before merging), once in chunk B ({1,2})
    g = gen.Graph(3, np.array([1, 1, 1], np.int32), np.array([0, 0, 2], np.int32), None, False)
    T0 = oracle.init(10, 3, 6)
    nrm = lambda x: x / np.linalg.norm(x)  # noqa: E731
    got = oracle.embed_chunked(g, [np.array([0, 1]), np.array([2])], 6, 1, 10)
    assert np.allclose(got[1], (2 * nrm(T0[0]) + nrm(T0[2])) / 3, atol=1e-15)


# ------------------------------------------------- hypergraph expansion

def test_expansions_of_the_papers_example():
    # Section 3.1: customer c buys product p in store s -> hyperedge {c,p,s}
    c, p_, s_ = 0, 1, 2
    src, dst = oracle.expand_clique([0, 3], [c, p_, s_])
    assert sorted(zip(src.tolist(), dst.tolist())) == [(c, p_), (c, s_), (p_, s_)]
    src, dst = oracle.expand_star(3, [0, 3], [c, p_, s_])
    assert src.tolist() == [3, 3, 3] and dst.tolist() == [c, p_, s_]


def test_expansion_sizes():
    rng = np.random.default_rng(3)
    sizes = rng.integers(1, 12, 50)
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    members = rng.integers(0, 100, offsets[-1])
    src, _ = oracle.expand_clique(offsets, members)
    assert src.size == int((sizes * (sizes - 1) // 2).sum())
    src, _ = oracle.expand_star(100, offsets, members)
    assert src.size == offsets[-1]


def test_clique_expanded_hyperedge_embeds_like_simple_clique():
    # one hyperedge of 6 distinct members = K_6; k = 1 closed form
    src, dst = oracle.expand_clique([0, 6], np.arange(6))
    g = gen.Graph(6, src, dst, None, False)
    T0 = oracle.init(4, 6, 9)
    T1 = oracle.embed(g, 9, 1, 4)
    assert np.allclose(T1, normalise_rows(T0.sum(0)[None, :] - T0), atol=1e-15)
