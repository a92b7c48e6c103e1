"""Hypergraph clique/star expansion on the GPU vs plain loops."""

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


def hypergraph(seed, n_nodes=3000, n_hyper=800):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, 15, n_hyper)
    sizes[:3] = [300, 150, 65]  # a few wide hyperedges (several waves of pairs)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    members = rng.integers(0, n_nodes, offsets[-1]).astype(np.int32)
    return n_nodes, offsets, members


@pytest.mark.parametrize("mode", ["clique", "star"])
def test_expansion_is_exact_and_embeds(cl, mode):
    n, offsets, members = hypergraph(70)
    with cl.Context(0) as ctx:
        src, dst = ctx.expand(offsets, members, mode=mode, n_nodes=n)
        src, dst = src.cpu().numpy(), dst.cpu().numpy()
    if mode == "clique":
        ws, wd = oracle.expand_clique(offsets, members)
        n_total = n
    else:
        ws, wd = oracle.expand_star(n, offsets, members)
        n_total = n + offsets.size - 1
    assert np.array_equal(src, ws) and np.array_equal(dst, wd)
    g = gen.Graph(n_total, src, dst, None, False)
    got = cl.embed(g, 64, 3, 5).cpu().numpy()
    assert np.abs(got - oracle.embed(g, 64, 3, 5)).max() <= 1e-5


def test_expansion_errors_and_empty(cl):
    with cl.Context(0) as ctx:
        src, dst = ctx.expand(np.zeros(1, np.int64), np.zeros(0, np.int32), mode="clique")
        assert src.numel() == 0
        with pytest.raises(cl.CleoraError):
            ctx.expand([0, 2], [0, 1], mode="star", n_nodes=2**31 - 1)
