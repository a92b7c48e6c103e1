"""cleora_propagate_rows_noalloc (no device allocation, static scratch)
against cleora_propagate_rows on the same inputs, through the C ABI: the
same bits, on calls in a row whose later inputs are smaller (the scratch
keeps the previous call's contents), at the size limits, with split hub
rows, weights and BF16."""

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2102_02302_amd as cl
    cl.load()
    return cl


def case(n_rows, n_cols, m, seed, hub=0, weighted=False):
    """Edges rows -> cols: uniform, plus `hub` extra edges of row 0 (a row
    long enough to be split into pieces)."""
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n_rows, m - hub).astype(np.int32)
    c = rng.integers(0, n_cols, m - hub).astype(np.int32)
    if hub:
        r = np.concatenate([r, np.zeros(hub, np.int32)])
        c = np.concatenate([c, rng.integers(0, n_cols, hub).astype(np.int32)])
    w = rng.lognormal(0.0, 1.0, m).astype(np.float32) if weighted else None
    return r, c, w


def table(cl, n_cols, dim, dtype, seed):
    """A T_in of n_cols rows in the library's layout (unit rows, padded)."""
    import torch
    epv = 4 if dtype == "f32" else 8
    ld = (dim + epv - 1) // epv * epv
    g = torch.Generator().manual_seed(seed)
    t = torch.randn((n_cols, dim), generator=g)
    t = t / t.norm(dim=1, keepdim=True)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    out = torch.zeros((n_cols, ld), dtype=tdt)
    out[:, :dim] = t.to(tdt)
    return out.cuda()


def same(a, b):
    import torch
    if a.dtype == torch.bfloat16:
        a, b = a.view(torch.int16), b.view(torch.int16)
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("dtype,dim", [("f32", 128), ("bf16", 256), ("f32", 1000)])
def test_noalloc_equals_propagate_rows_twice(cl, dtype, dim):
    # first call larger, second smaller: stale scratch from the first must
    # not leak into the second
    calls = [(6000, 40_000, 300_000, 1, 5000, True), (700, 9_000, 20_000, 2, 900, False)]
    with cl.Context(0) as work:
        for n_rows, n_cols, m, seed, hub, weighted in calls:
            r, c, w = case(n_rows, n_cols, m, seed, hub, weighted)
            T = table(cl, n_cols, dim, dtype, seed)
            want = work.propagate_rows(n_rows, n_cols, r, c, T, dim, dtype, w=w)
            got = cl.propagate_rows_noalloc(n_rows, n_cols, r, c, T, dim, dtype, w=w)
            assert same(got, want), (dtype, dim, n_rows, m)
            # rows without edges are zero, the others unit vectors
            nrm = got.float().norm(dim=1).cpu().numpy()
            has = np.bincount(r, minlength=n_rows) > 0
            assert np.all(nrm[~has] == 0)
            tol = 1e-5 if dtype == "f32" else 1e-2
            assert np.abs(nrm[has] - 1).max() <= tol


def test_noalloc_at_the_limits(cl):
    import paper_2102_02302_amd as pkg
    n_rows, m = pkg._lib.NOALLOC_MAX_ROWS, pkg._lib.NOALLOC_MAX_EDGES
    dim = pkg._lib.NOALLOC_MAX_ROW_BYTES // 4
    r, c, w = case(n_rows, 200_000, m, 3, hub=20_000, weighted=True)
    T = table(cl, 200_000, dim, "f32", 3)
    with cl.Context(0) as work:
        want = work.propagate_rows(n_rows, 200_000, r, c, T, dim, "f32", w=w)
    got = cl.propagate_rows_noalloc(n_rows, 200_000, r, c, T, dim, "f32", w=w)
    assert same(got, want)
    # one more edge, row or column of width: refused, nothing written
    import torch
    out = torch.full((n_rows, dim), 7.0, device="cuda")
    r2, c2, _ = case(n_rows, 200_000, m + 1, 4)
    with pytest.raises(pkg.CleoraError, match="E_INVAL"):
        cl.propagate_rows_noalloc(n_rows, 200_000, r2, c2, T, dim, "f32", out=out)
    assert bool((out == 7.0).all())
