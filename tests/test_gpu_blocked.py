"""GPU parity of the column-blocked form (cleora_embed_blocked): the
embedding computed a block of columns at a time, against the FP64 oracle and
against the unblocked path, through the C ABI.

Bars: T_0 bit-exact for any block width (entries keyed by the full width);
float32 within max-abs 1e-5 of the oracle; bfloat16 storage within max-abs
4e-3 and minimum row cosine 0.9999; one block bit-identical to init +
propagate (the same arithmetic step for step); several blocks within 2e-6 of
the unblocked path (float32 summation order only).
"""

import ctypes

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_MAXABS = 4e-3
BF16_MINCOS = 0.9999


@pytest.fixture(scope="module")
def cl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2102_02302_amd as cl
    cl.load()  # raises if the HIP library is missing: no fallback
    return cl


def star(n_leaves):
    # the hub's row is longer than the 512-entry split size: chunks + combine
    return gen.Graph(n_leaves + 1, np.zeros(n_leaves, np.int32),
                     np.arange(1, n_leaves + 1, dtype=np.int32), None, False, f"star{n_leaves}")


def graphs():
    return [
        gen.chung_lu(20_000, 200_000, 2.1, 31),
        star(5000),
        gen.random_graph(700, 2000, 3, directed=True, weighted=True, loops=True, multi=True),
        gen.erdos_renyi(3000, 6000, 1),  # isolated nodes
    ]


def blocked(cl, g, dim, block, k, seed, dtype="f32", empty_keep=False):
    with cl.Context(0) as ctx:
        ctx.build_graph(g, empty_keep=empty_keep)
        return ctx.embed_blocked(dim, block, k, dtype, seed).float().cpu().numpy()


def unblocked(cl, g, dim, k, seed, dtype="f32", empty_keep=False):
    with cl.Context(0) as ctx:
        ctx.build_graph(g, empty_keep=empty_keep).init(dim, dtype, seed).propagate(k)
        return ctx.embedding().float().cpu().numpy()


def bf16_report(got, want):
    err = np.abs(got - want).max()
    nz = np.linalg.norm(want, axis=1) > 0
    cos = (got[nz] * want[nz]).sum(1) / (np.linalg.norm(got[nz], axis=1) *
                                         np.linalg.norm(want[nz], axis=1))
    return float(err), float(cos.min())


@pytest.mark.parametrize("dim,block,dtype", [(37, 8, "f32"), (100, 24, "f32"), (72, 32, "bf16"),
                                             (256, 64, "bf16")])
def test_t0_bitwise(cl, dim, block, dtype):
    import torch
    g = gen.erdos_renyi(900, 2000, 9)
    got = blocked(cl, g, dim, block, 0, 123, dtype)
    want = oracle.init(123, g.n, dim)
    if dtype == "bf16":
        want = torch.tensor(want, dtype=torch.float32).to(torch.bfloat16).float().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("gi", [0, 1, 2, 3])
@pytest.mark.parametrize("dim,block,k", [(64, 16, 4), (100, 24, 3), (256, 96, 1)])
def test_parity_f32(cl, gi, dim, block, k):
    g = graphs()[gi]
    got = blocked(cl, g, dim, block, k, 5)
    want = oracle.embed(g, dim, k, 5)
    err = np.abs(got - want).max()
    print(f"blocked f32 {g.name} d={dim} b={block} k={k}: max-abs {err:.3e}")
    assert err <= F32_TOL


@pytest.mark.parametrize("gi", [0, 1, 2])
def test_empty_keep_parity(cl, gi):
    g = graphs()[gi]
    got = blocked(cl, g, 48, 16, 4, 8, empty_keep=True)
    want = oracle.embed(g, 48, 4, 8, oracle.EMPTY_KEEP)
    assert np.abs(got - want).max() <= F32_TOL


@pytest.mark.parametrize("dim,block", [(128, 40), (200, 64)])
def test_bf16_bound(cl, dim, block):
    g = graphs()[0]
    got = blocked(cl, g, dim, block, 4, 6, "bf16")
    err, cmin = bf16_report(got, oracle.embed(g, dim, 4, 6))
    print(f"blocked bf16 d={dim} b={block}: max-abs {err:.3e} min-cos {cmin:.7f}")
    assert err <= BF16_MAXABS and cmin >= BF16_MINCOS


@pytest.mark.parametrize("dtype,dim", [("f32", 256), ("f32", 37), ("bf16", 200), ("bf16", 64)])
@pytest.mark.parametrize("gi,empty_keep", [(0, False), (1, False), (2, True)])
def test_single_block_bitwise(cl, dtype, dim, gi, empty_keep):
    g = graphs()[gi]
    want = unblocked(cl, g, dim, 3, 11, dtype, empty_keep)
    for block in (dim, dim + 5):  # block >= dim: one block
        got = blocked(cl, g, dim, block, 3, 11, dtype, empty_keep)
        assert np.array_equal(got, want), block


@pytest.mark.parametrize("gi", [0, 1, 2, 3])
def test_close_to_unblocked(cl, gi):
    g = graphs()[gi]
    want = unblocked(cl, g, 128, 4, 12)
    for block in (4, 32, 100):
        got = blocked(cl, g, 128, block, 4, 12)
        assert np.abs(got - want).max() <= 2e-6, block


def test_host_output_and_schedules(cl):
    # pinned and pageable host destinations, a wider row stride, and other
    # schedules (packing, persistent grid) give the same bits
    import torch
    g = graphs()[0]
    ref = torch.from_numpy(blocked(cl, g, 96, 40, 3, 4))
    with cl.Context(0) as ctx:
        ctx.build_graph(g)
        pinned = torch.empty((g.n, 96), dtype=torch.float32, pin_memory=True)
        ctx.embed_blocked(96, 40, 3, "f32", 4, out=pinned)
        assert torch.equal(pinned, ref)
        page = torch.empty((g.n, 96), dtype=torch.float32)
        ctx.embed_blocked(96, 40, 3, "f32", 4, out=page)
        assert torch.equal(page, ref)
        wide = torch.full((g.n, 130), 7.0, device="cuda")
        ctx.embed_blocked(96, 40, 3, "f32", 4, out=wide[:, :96])
        assert torch.equal(wide[:, :96].cpu(), ref)
        assert bool((wide[:, 96:] == 7.0).all())
    for pack, persistent in [(16, 1), (64, 2), (0, 0)]:
        with cl.Context(0) as ctx:
            ctx.set_schedule(pack, persistent)
            ctx.build_graph(g)
            got = ctx.embed_blocked(96, 40, 3, "f32", 4).cpu()
            assert torch.equal(got, ref), (pack, persistent)


def test_chunk_context(cl):
    # a chunk's T_0 rows are keyed by global node id, here too
    g = gen.random_graph(2000, 6000, 63, loops=True, multi=True)
    idx = np.arange(1, g.m, 3)
    with cl.Context(0) as ctx:
        ctx.build_chunk(g.n, g.src[idx], g.dst[idx])
        ctx.init(64, "f32", 3).propagate(2)
        want = ctx.embedding().cpu().numpy()
        assert np.array_equal(ctx.embed_blocked(64, 64, 2, "f32", 3).cpu().numpy(), want)
        assert np.abs(ctx.embed_blocked(64, 16, 2, "f32", 3).cpu().numpy() - want).max() <= 2e-6


def test_errors_and_state(cl):
    import torch
    from paper_2102_02302_amd import _lib
    g = graphs()[3]
    with cl.Context(0) as ctx:
        out = torch.empty((g.n, 32), device="cuda")
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

        def call(dim, block, k, ld, dtype=_lib.F32, ptr=out.data_ptr()):
            return ctx._lib.cleora_embed_blocked(ctx.handle, dim, block, dtype, 1, k, ptr, ld, s)

        assert call(32, 8, 2, 32) == _lib.E_STATE  # no graph yet
        ctx.build_graph(g)
        assert call(32, 0, 2, 32) == _lib.E_INVAL
        assert call(32, 8, -1, 32) == _lib.E_INVAL
        assert call(32, 8, 2, 31) == _lib.E_INVAL
        assert call(0, 8, 2, 32) == _lib.E_INVAL
        assert call(32, 8, 2, 32, dtype=7) == _lib.E_INVAL
        assert call(32, 8, 2, 32, ptr=None) == _lib.E_INVAL
        assert call(32, 8, 2, 32) == _lib.OK
        with pytest.raises(cl.CleoraError) as e:
            ctx.propagate(1)  # the blocked form leaves no embedding
        assert e.value.code == _lib.E_STATE
        ctx.init(32, "f32", 1).propagate(2)  # the graph is still there
        assert np.abs(ctx.embedding().cpu().numpy() - out.cpu().numpy()).max() <= 2e-6


def test_release_scratch(cl):
    # the build's temporaries, and the block buffers once no embedding is
    # held, go back to the device; the graph and a current embedding stay
    import torch
    from paper_2102_02302_amd import _lib
    g = gen.chung_lu(200_000, 2_000_000, 2.1, 64)
    free = lambda: torch.cuda.mem_get_info()[0]  # noqa: E731
    with cl.Context(0) as ctx:
        ctx.build_graph(g)
        torch.cuda.synchronize()
        f0 = free()
        ctx.release_scratch()
        f1 = free()
        assert f1 - f0 >= 100 << 20, (f0, f1)  # about 40 bytes per stored entry
        out = torch.empty((g.n, 96), device="cuda")
        ctx.embed_blocked(96, 40, 3, "f32", 4, out=out)
        f2 = free()
        ctx.release_scratch()
        assert free() - f2 >= 2 * g.n * 40 * 4, (f2, free())  # the two block buffers
        ctx.init(96, "f32", 4).propagate(2)
        ctx.release_scratch()  # keeps the embedding and its schedule
        ctx.propagate(1)
        ref = ctx.embedding()
        assert float((out - ref).abs().max()) <= 2e-6
        ctx.propagate(1)  # and it goes on propagating
        assert ctx.info()["iteration"] == 4
    assert _lib.load().cleora_release_scratch(None) == _lib.E_INVAL
