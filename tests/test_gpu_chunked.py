"""Algorithm 1's chunks on the GPU: each chunk embedded on its own nodes
with T_0 keyed by global id, merged per node by occurrence weights."""

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


@pytest.mark.parametrize("q", [1, 3, 7])
def test_chunked_matches_oracle(cl, q):
    g = gen.chung_lu(20_000, 150_000, 2.1, 60)
    chunks = np.array_split(np.random.default_rng(q).permutation(g.m), q)
    got = cl.embed_chunked(g, list(chunks), 96, 4, 11).cpu().numpy()
    want = oracle.embed_chunked(g, list(chunks), 96, 4, 11)
    assert np.abs(got - want).max() <= 1e-5


def test_chunked_weighted_bf16(cl):
    g = gen.bipartite_zipf(8000, 1000, 80_000, 1.1, 61)
    got = cl.embed_chunked(g, 4, 64, 3, 2, dtype="bf16").float().cpu().numpy()
    want = oracle.embed_chunked(g, np.array_split(np.arange(g.m), 4), 64, 3, 2)
    assert np.abs(got - want).max() <= 4e-3


def test_chunk_nodes_and_occurrences(cl):
    import ctypes
    import torch
    from paper_2102_02302_amd import _lib
    g = gen.random_graph(1000, 3000, 62, loops=True, multi=True)
    idx = np.arange(0, g.m, 2)
    with cl.Context(0) as ctx:
        ctx.build_chunk(g.n, g.src[idx], g.dst[idx])
        n = ctypes.c_int64()
        _lib.check(ctx._lib.cleora_chunk_info(ctx.handle, ctypes.byref(n), None, None, None))
        ids = torch.empty(n.value, dtype=torch.int32, device="cuda")
        occ = torch.empty(n.value, dtype=torch.float32, device="cuda")
        _lib.check(ctx._lib.cleora_chunk_info(ctx.handle, None, ids.data_ptr(), occ.data_ptr(),
                                              None))
        ctx.sync()
    s, d = g.src[idx], g.dst[idx]
    nodes = np.unique(np.concatenate([s, d]))
    assert np.array_equal(ids.cpu().numpy(), nodes)
    want = np.bincount(s, minlength=g.n) + np.bincount(d[s != d], minlength=g.n)
    assert np.array_equal(occ.cpu().numpy(), want[nodes].astype(np.float32))
