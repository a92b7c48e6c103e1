"""GPU parity of column-sliced iterations (cleora_set_slices): each
iteration gathers a slice of columns at a time and stores rows unscaled;
the next iteration multiplies by M diag(1/norm); each call ends with the
normalised T_k written out of place.  Through the C ABI, against the FP64
oracle and the whole-row path.

Bars: float32 within max-abs 1e-5 of the oracle and 2e-6 of whole rows;
bfloat16 within the stated bound of the oracle (max-abs 4e-3, minimum row
cosine 0.9999) and 4e-3 of whole rows; a slice at least as wide as the row
is whole rows (bit-identical); resumption, graph replay, eager launches,
schedules and batch = solo bit-exact within the sliced mode; whole rows by
default; the automatic mode keeps whole rows until the autotuner has
chosen, then runs bit-identically to the chosen width set by hand.
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
    """T_k with column slices `cols` wide (0: whole rows)."""
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


def test_previous_buffer_needs_whole_rows(cl):
    # sliced iterations keep T_t's unscaled rows in the other buffer, not
    # T_{t-1}: asking for it is a state error; whole rows keep it
    from paper_2102_02302_amd import _lib
    g = graphs()[1]
    with cl.Context(0) as ctx:
        ctx.set_slices(64)
        ctx.build_graph(g).init(256, "f32", 3).propagate(5)
        with pytest.raises(cl.CleoraError) as e:
            ctx.embedding_ptr(previous=True)
        assert e.value.code == _lib.E_STATE
        ctx.set_slices(0)
        ctx.init(256, "f32", 3).propagate(5)
        ptr, ld = ctx.embedding_ptr(previous=True)
        assert ptr and ld == 256


def test_widths(cl):
    # whole rows by default; a bfloat16 width rounds up to 16 bytes; a
    # slice as wide as the row is whole rows; 1024 columns in 128-column
    # slices stay within rounding of whole rows and of the oracle
    g = graphs()[0]
    with cl.Context(0) as ctx:
        ctx.build_graph(g).init(1024, "f32", 2)
        assert ctx.schedule()["slice_cols"] == 0
        ctx.set_slices(132)
        ctx.init(1024, "f32", 2)
        assert ctx.schedule()["slice_cols"] == 132
        ctx.init(1024, "bf16", 2)
        assert ctx.schedule()["slice_cols"] == 136
        ctx.init(132, "f32", 2)
        assert ctx.schedule()["slice_cols"] == 0
    got = run(cl, g, 1024, 3, 2, 128)
    assert np.abs(got - run(cl, g, 1024, 3, 2, 0)).max() <= 2e-6
    assert np.abs(got - oracle.embed(g, 1024, 3, 2)).max() <= F32_TOL


def test_step_multi_and_autotune_continue_from_normalised_rows(cl):
    # both discard a sliced context's unscaled rows: the context continues
    # from the normalised T_t, within rounding of the uninterrupted run
    g = graphs()[0]
    ref = run(cl, g, 256, 4, 9, 64)
    with cl.Context(0) as ctx:
        ctx.set_slices(64)
        ctx.build_graph(g).init(256, "f32", 9).propagate(2)
        cl.step_multi([ctx])
        ctx.propagate(1)
        assert np.abs(ctx.embedding().cpu().numpy() - ref).max() <= 2e-6
    with cl.Context(0) as ctx:
        ctx.set_slices(64)
        ctx.build_graph(g).init(256, "f32", 9).propagate(2)
        ctx.autotune()
        ctx.propagate(2)
        assert np.abs(ctx.embedding().cpu().numpy() - ref).max() <= 2e-6


def test_batch_equals_solo_with_slices(cl):
    gs = [gen.chung_lu(3000, 20_000, 2.1, 50 + i) for i in range(3)] + [star(1500)]
    seeds = [7, 8, 9, 10]
    with cl.Context(0) as ctx:
        ctx.set_slices(32)
        outs = cl.embed_batch(ctx, gs, 128, 3, seeds)
    for g, sd, out in zip(gs, seeds, outs):
        solo = run(cl, g, 128, 3, sd, 32)
        assert np.array_equal(out.cpu().numpy(), solo)


def bf16_report(got, want):
    err = float(np.abs(got - want).max())
    nz = np.linalg.norm(want, axis=1) > 0
    cos = (got[nz] * want[nz]).sum(1) / (np.linalg.norm(got[nz], axis=1) *
                                         np.linalg.norm(want[nz], axis=1))
    return err, float(cos.min())


@pytest.mark.parametrize("gi", [0, 1, 2, 3])
@pytest.mark.parametrize("dim,cols", [(1024, 256), (256, 64), (100, 36)])
def test_bf16_slices(cl, gi, dim, cols):
    # bfloat16 slices: unscaled rows rounded once, T_k rounded again when
    # it is written; within the stated bound of the oracle and close to
    # whole rows; resumption bit-exact
    g = graphs()[gi]
    got = run(cl, g, dim, 4, 5, cols, dtype="bf16")
    err, cmin = bf16_report(got, oracle.embed(g, dim, 4, 5))
    print(f"bf16 sliced {g.name} d={dim} cols={cols}: max-abs {err:.3e} min-cos {cmin:.7f}")
    assert err <= 4e-3 and cmin >= 0.9999
    assert np.abs(got - run(cl, g, dim, 4, 5, 0, dtype="bf16")).max() <= 4e-3
    assert np.array_equal(run(cl, g, dim, 4, 5, cols, dtype="bf16", steps=[1, 3]), got)


def test_set_slices_rejects_bad_values(cl):
    from paper_2102_02302_amd import _lib
    with cl.Context(0) as ctx:
        for cols in (-2, 6, 8196):
            with pytest.raises(cl.CleoraError) as e:
                ctx.set_slices(cols)
            assert e.value.code == _lib.E_INVAL
        ctx.set_slices(0)
        ctx.set_slices(8192)
        ctx.set_slices("auto")
        ctx.set_slices(_lib.SLICES_AUTO)


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


@pytest.mark.parametrize("dtype,dim,widths", [("f32", 1024, (128, 256)), ("bf16", 1024, (256, 512)),
                                              ("f32", 200, (128,)), ("f32", 100, ())])
def test_auto_slices(cl, dtype, dim, widths):
    # whole rows until the autotuner has timed both; then the fastest of
    # whole rows and 1 KiB or 512-byte slices (only those narrower than the
    # row), with
    # results bit-identical to setting that width by hand; another dim
    # returns to whole rows until the next autotune; the embedding the
    # autotuner ran on is unchanged
    g = graphs()[0]
    with cl.Context(0) as ctx:
        ctx.set_slices("auto")
        ctx.build_graph(g).init(dim, dtype, 4)
        assert ctx.schedule()["slice_cols"] == 0
        before = ctx.embedding().float().cpu().numpy()
        ctx.autotune()
        chosen = ctx.schedule()["slice_cols"]
        assert chosen in (0,) + widths, chosen
        assert np.array_equal(ctx.embedding().float().cpu().numpy(), before)
        ctx.propagate(1).propagate(3)
        got = ctx.embedding().float().cpu().numpy()
        ctx.init(dim, dtype, 4)  # same layout: the choice stays
        assert ctx.schedule()["slice_cols"] == chosen
        ctx.init(dim - 4, dtype, 4)
        assert ctx.schedule()["slice_cols"] == 0
    print(f"{dtype} d={dim}: autotuner chose slice width {chosen}")
    # the same 1 + 3 iterations from T_0 with the chosen width set by hand
    want = run(cl, g, dim, 4, 4, chosen, dtype=dtype, steps=[1, 3])
    assert np.array_equal(got, want)
