"""New nodes after embedding (Section 3.2): one propagation step for the new
rows against the existing embedding, 1-hop and chained 2-hop."""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2102_02302_amd as cl
    cl.load()
    return cl


def rows_of(g, members):
    """Edges of the listed nodes as (position in `members`, neighbour)."""
    pos = -np.ones(g.n, np.int64)
    pos[members] = np.arange(members.size)
    r1 = pos[g.src] >= 0
    rows = [pos[g.src[r1]]]
    cols = [g.dst[r1]]
    ws = [g.w[r1]] if g.w is not None else []
    if not g.directed:
        r2 = (pos[g.dst] >= 0) & (g.src != g.dst)
        rows.append(pos[g.dst[r2]])
        cols.append(g.src[r2])
        if g.w is not None:
            ws.append(g.w[r2])
    w = np.concatenate(ws).astype(np.float32) if ws else None
    return np.concatenate(rows).astype(np.int32), np.concatenate(cols).astype(np.int32), w


@pytest.mark.parametrize("dtype,weighted", [("f32", False), ("f32", True), ("bf16", True)])
def test_known_node_reembedded_from_previous_iteration(cl, dtype, weighted):
    # A node's own edges averaged over T_{k-1} give exactly its row of T_k.
    if weighted:
        g = gen.bipartite_zipf(20_000, 2000, 150_000, 1.1, 51)
    else:
        g = gen.chung_lu(30_000, 200_000, 2.1, 50)
    dim, k, seed = 128, 4, 3
    members = np.random.default_rng(0).choice(g.n, 700, replace=False).astype(np.int32)
    # also a few of the largest rows (split into chunks on the GPU)
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    members = np.unique(np.concatenate([members, np.argsort(-deg)[:5].astype(np.int32)]))
    rows, cols, w = rows_of(g, members)
    with cl.Context(0) as base:
        base.build_graph(g).init(dim, dtype, seed).propagate(k)
        Tk = base.embedding().float().cpu().numpy()
        new = cl.embed_new_nodes(base, members.size, rows, cols, w=w, previous=True)
        new = new.float().cpu().numpy()
    assert np.array_equal(new, Tk[members])
    want = oracle.embed(g, dim, k, seed)[members]
    assert np.abs(new - want).max() <= (1e-5 if dtype == "f32" else 4e-3)


def test_two_hop_chain_matches_oracle(cl):
    # seen nodes embedded on their own graph; 1-hop nodes link to seen nodes;
    # 2-hop nodes link to 1-hop nodes (and some seen ones)
    rng = np.random.default_rng(5)
    dim, k, seed = 64, 3, 8
    seen = gen.chung_lu(5000, 30_000, 2.1, 52)
    n1, n2 = 400, 300
    r1 = rng.integers(0, n1, 3000).astype(np.int32)
    c1 = rng.integers(0, seen.n, 3000).astype(np.int32)
    r2 = rng.integers(0, n2, 2000).astype(np.int32)
    c2 = np.where(rng.random(2000) < 0.7, seen.n + rng.integers(0, n1, 2000),
                  rng.integers(0, seen.n, 2000)).astype(np.int32)
    with cl.Context(0) as base, cl.Context(0) as work:
        base.build_graph(seen).init(dim, "f32", seed).propagate(k)
        T = base.embedding()
        hop1 = work.propagate_rows(n1, seen.n, r1, c1, T, dim)
        hop2 = work.propagate_rows(n2, seen.n + n1, r2, c2, np.concatenate([
            T.cpu().numpy(), hop1.cpu().numpy()]), dim)
        hop1, hop2, T = hop1.cpu().numpy(), hop2.cpu().numpy(), T.cpu().numpy()
    To = oracle.embed(seen, dim, k, seed)

    def oracle_step(n_rows, n_cols, r, c, Tin):
        n = max(n_rows, n_cols)
        adj = oracle.build_adjacency(n, r, c, None, True)
        mval, _ = oracle.transition(adj)
        Tpad = np.zeros((n, dim))
        Tpad[:n_cols] = Tin
        out = np.zeros((n, dim))
        oracle.step_rows(adj, mval, Tpad, out, 0, n_rows)
        return out[:n_rows]

    o1 = oracle_step(n1, seen.n, r1, c1, To)
    o2 = oracle_step(n2, seen.n + n1, r2, c2, np.concatenate([To, o1]))
    assert np.abs(hop1 - o1).max() <= 1e-5
    assert np.abs(hop2 - o2).max() <= 1e-5


def test_propagate_rows_errors(cl):
    import torch
    from paper_2102_02302_amd import _lib
    T = torch.zeros((10, 16), device="cuda")
    with cl.Context(0) as work:
        with pytest.raises(cl.CleoraError) as e:
            work.propagate_rows(3, 10, [0, 1], [2, 10], T, 16)
        assert e.value.code == _lib.E_INPUT
        with pytest.raises(cl.CleoraError) as e:
            work.propagate_rows(3, 10, [0, 3], [2, 4], T, 16)
        assert e.value.code == _lib.E_INPUT
        out = work.propagate_rows(3, 10, [0, 1], [2, 4], T, 16)  # row 2: no edges
        assert torch.all(out[2] == 0)
    with cl.Context(0) as base:
        base.build_csr(4, [0, 1], [1, 2]).init(8, "f32", 1)
        with pytest.raises(cl.CleoraError) as e:
            base.embedding_ptr(previous=True)
        assert e.value.code == _lib.E_STATE
