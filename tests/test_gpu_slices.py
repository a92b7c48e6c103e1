"""GPU parity of column-sliced iterations (cleora_set_slices): each
iteration gathered a slice of columns at a time, rows stored unscaled, one
row-scaling pass; through the C ABI, against the FP64 oracle and the
whole-row path.

Bars: float32 within max-abs 1e-5 of the oracle and 2e-6 of whole rows;
one slice (cols >= the padded width) bit-identical to whole rows;
resumption, graph replay, schedules and batch = solo bit-exact within the
sliced mode; BF16 contexts ignore the setting (bit-identical to whole rows).
"""

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5


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
        gen.chung_lu(20_000, 200_000, 2.1, 41),
        star(5000),
        gen.random_graph(700, 2000, 3, directed=True, weighted=True, loops=True, multi=True),
        gen.erdos_renyi(3000, 6000, 1),  # isolated nodes
    ]


def run(cl, g, dim, k, seed, cols=0, dtype="f32", empty_keep=False, steps=None):
    with cl.Context(0) as ctx:
        ctx.set_slices(cols)
        ctx.build_graph(g, empty_keep=empty_keep).init(dim, dtype, seed)
        for kk in (steps or [k]):
            ctx.propagate(kk)
        return ctx.embedding().float().cpu().numpy()


@pytest.mark.parametrize("gi", [0, 1, 2, 3])
@pytest.mark.parametrize("dim,cols", [(256, 64), (256, 100), (37, 8), (512, 128)])
def test_parity_f32(cl, gi, dim, cols):
    g = graphs()[gi]
    got = run(cl, g, dim, 4, 5, cols)
    want = oracle.embed(g, dim, 4, 5)
    err = np.abs(got - want).max()
    print(f"sliced {g.name} d={dim} cols={cols}: max-abs {err:.3e}")
    assert err <= F32_TOL
    assert np.abs(got - run(cl, g, dim, 4, 5)).max() <= 2e-6


@pytest.mark.parametrize("gi", [0, 1, 2])
def test_empty_keep_parity(cl, gi):
    g = graphs()[gi]
    got = run(cl, g, 64, 4, 8, 16, empty_keep=True)
    assert np.abs(got - oracle.embed(g, 64, 4, 8, oracle.EMPTY_KEEP)).max() <= F32_TOL


@pytest.mark.parametrize("gi,empty_keep", [(0, False), (1, False), (2, True)])
@pytest.mark.parametrize("dim", [256, 37, 1024])
def test_one_slice_is_whole_rows_bitwise(cl, gi, empty_keep, dim):
    g = graphs()[gi]
    want = run(cl, g, dim, 3, 11, 0, empty_keep=empty_keep)
    for cols in (dim + 3 - (dim + 3) % 4, 4096):  # at least the padded width
        got = run(cl, g, dim, 3, 11, cols, empty_keep=empty_keep)
        assert np.array_equal(got, want), cols


def test_resume_replay_and_schedules_bitwise(cl):
    g = graphs()[0]
    ref = run(cl, g, 256, 5, 3, 64)
    # resumption: 5 = 2 + 3 = 1 + 1 + 1 + 1 + 1 (single steps are not captured)
    assert np.array_equal(run(cl, g, 256, 5, 3, 64, steps=[2, 3]), ref)
    assert np.array_equal(run(cl, g, 256, 5, 3, 64, steps=[1] * 5), ref)
    with cl.Context(0) as ctx:  # eager launches (timing on) against the captured graph
        ctx.set_slices(64)
        ctx.build_graph(g).init(256, "f32", 3)
        ctx.set_timing(True)
        ctx.propagate(5)
        ctx.set_timing(False)
        assert ctx.kernel_time()["spmm_launches"] == 5 * 4  # four slices per iteration
        assert np.array_equal(ctx.embedding().cpu().numpy(), ref)
    for pack, persistent in [(16, 1), (64, 2), (0, 0)]:
        with cl.Context(0) as ctx:
            ctx.set_slices(64)
            ctx.set_schedule(pack, persistent)
            ctx.build_graph(g).init(256, "f32", 3).propagate(5)
            assert np.array_equal(ctx.embedding().cpu().numpy(), ref), (pack, persistent)


def test_previous_buffer_is_complete(cl):
    # T_{t-1} (the other buffer) is scaled like T_t: what new-node rows read
    import ctypes
    import torch
    g = graphs()[1]
    want = run(cl, g, 256, 4, 3, 64)
    hip = ctypes.CDLL("libamdhip64.so")  # the runtime torch already loaded
    with cl.Context(0) as ctx:
        ctx.set_slices(64)
        ctx.build_graph(g).init(256, "f32", 3).propagate(5)
        ptr, ld = ctx.embedding_ptr(previous=True)
        assert ld == 256
        prev = torch.empty((g.n, ld), device="cuda")
        torch.cuda.synchronize()
        assert hip.hipMemcpy(ctypes.c_void_p(prev.data_ptr()), ctypes.c_void_p(ptr),
                             ctypes.c_size_t(g.n * ld * 4), 4) == 0
        assert np.array_equal(prev.cpu().numpy(), want)


def test_batch_equals_solo_with_slices(cl):
    gs = [gen.chung_lu(3000, 20_000, 2.1, 50 + i) for i in range(3)] + [star(1500)]
    seeds = [7, 8, 9, 10]
    with cl.Context(0) as ctx:
        ctx.set_slices(32)
        outs = cl.embed_batch(ctx, gs, 128, 3, seeds)
    for g, sd, out in zip(gs, seeds, outs):
        solo = run(cl, g, 128, 3, sd, 32)
        assert np.array_equal(out.cpu().numpy(), solo)


def test_bf16_ignores_slices(cl):
    g = graphs()[0]
    a = run(cl, g, 256, 3, 4, 64, dtype="bf16")
    b = run(cl, g, 256, 3, 4, 0, dtype="bf16")
    assert np.array_equal(a, b)


def test_set_slices_rejects_bad_values(cl):
    from paper_2102_02302_amd import _lib
    with cl.Context(0) as ctx:
        for cols in (-1, 6, 4100):
            with pytest.raises(cl.CleoraError) as e:
                ctx.set_slices(cols)
            assert e.value.code == _lib.E_INVAL
        ctx.set_slices(0)
        ctx.set_slices(4096)


def test_embed_with_slices(cl):
    g = graphs()[0]
    got = cl.embed(g, 256, 3, 4, slices=64).cpu().numpy()
    assert np.array_equal(got, run(cl, g, 256, 3, 4, 64))


def test_release_scratch_keeps_a_sliced_embedding(cl):
    g = graphs()[1]
    want = run(cl, g, 256, 3, 6, 64)
    with cl.Context(0) as ctx:
        ctx.set_slices(64)
        ctx.build_graph(g).init(256, "f32", 6).propagate(2)
        ctx.release_scratch()  # the slice buffers belong to the embedding
        ctx.propagate(1)
        assert np.array_equal(ctx.embedding().cpu().numpy(), want)
