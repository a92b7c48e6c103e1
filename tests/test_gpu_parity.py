"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, on
the same seeded inputs, element by element.

Bars: integer CSR results bit-exact; T_0 bit-exact (float32, and bfloat16
after round-to-nearest-even); float32 embeddings within max-abs 1e-5 of the
FP64 oracle; bfloat16-storage embeddings within max-abs 4e-3 and minimum row
cosine 0.9999.
"""

import math

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


def gpu_embed(cl, g, dim, k, seed, dtype="f32", chunk=0, empty_keep=False):
    with cl.Context(0) as ctx:
        ctx.build_graph(g, empty_keep=empty_keep)
        if chunk:
            ctx.set_chunk(chunk)
        ctx.init(dim, dtype, seed)
        ctx.propagate(k)
        return ctx.embedding().float().cpu().numpy().astype(np.float64)


def oracle_embed(g, dim, k, seed, empty_keep=False):
    return oracle.embed(g, dim, k, seed, oracle.EMPTY_KEEP if empty_keep else 0)


def zoo():
    star = gen.Graph(20_001, np.zeros(20_000, np.int32), np.arange(1, 20_001, dtype=np.int32),
                     None, False, "star20k")
    return [
        gen.erdos_renyi(3000, 15_000, 1),
        gen.random_graph(500, 3000, 2, directed=True, weighted=True, loops=True, multi=True),
        gen.random_graph(700, 2000, 3, directed=False, weighted=True, loops=True, multi=True),
        gen.chung_lu(5000, 40_000, 2.1, 4),
        gen.bipartite_zipf(3000, 500, 30_000, 1.1, 5),
        star,
    ]


# ------------------------------------------------------------- init

@pytest.mark.parametrize("dim", [1, 3, 37, 128, 256, 1024])
def test_init_bitwise_f32(cl, dim):
    g = gen.erdos_renyi(600, 1500, 9)
    got = gpu_embed(cl, g, dim, 0, seed=123)
    want = oracle.init(123, g.n, dim)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dim", [5, 64, 512])
def test_init_bitwise_bf16(cl, dim):
    import torch
    g = gen.erdos_renyi(400, 1000, 9)
    with cl.Context(0) as ctx:
        ctx.build_graph(g).init(dim, "bf16", 77)
        got = ctx.embedding().cpu()
    want = torch.tensor(oracle.init(77, g.n, dim), dtype=torch.float32).to(torch.bfloat16)
    assert torch.equal(got.view(torch.int16), want.view(torch.int16))


# -------------------------------------------------------------- CSR

@pytest.mark.parametrize("gi", range(6))
def test_csr_matches_oracle(cl, gi):
    g = zoo()[gi]
    adj = oracle.build_graph(g)
    mval, deg = oracle.transition(adj)
    with cl.Context(0) as ctx:
        ctx.build_graph(g)
        csr = {k: v.cpu().numpy() for k, v in ctx.csr().items()}
    assert np.array_equal(csr["row_ptr"], adj.row_ptr)
    assert np.array_equal(csr["col"], adj.col)
    assert np.allclose(csr["deg"], deg, rtol=1e-15, atol=0)
    if g.w is None:
        assert np.array_equal(csr["deg"], deg)
    assert np.all(np.abs(csr["val"] - mval) <= mval * 2.0**-24 * 1.0001)


@pytest.mark.parametrize("n", [1, 2, 3, 1023, 1024, 1025, 65536])
def test_csr_key_width_boundaries(cl, n):
    # sort keys are row << bits(n_cols) | col with bits(n + 1) row bits: node
    # counts at and around powers of two, loops (whose second copy is an
    # invalid key) and repeated pairs
    for directed in (True, False):
        g = gen.random_graph(n, 4 * n + 8, 40 + n, directed=directed, weighted=True,
                             loops=True, multi=True)
        adj = oracle.build_graph(g)
        mval, deg = oracle.transition(adj)
        with cl.Context(0) as ctx:
            ctx.build_graph(g)
            csr = {k: v.cpu().numpy() for k, v in ctx.csr().items()}
        assert np.array_equal(csr["row_ptr"], adj.row_ptr), (n, directed)
        assert np.array_equal(csr["col"], adj.col), (n, directed)
        assert np.allclose(csr["deg"], deg, rtol=1e-15, atol=0)
        assert np.all(np.abs(csr["val"] - mval) <= mval * 2.0**-24 * 1.0001)


def test_csr_long_rows_weighted(cl):
    # one row of 40k entries (block radix sort), rows of ~5k (LDS sort),
    # repeated weighted pairs to merge
    rng = np.random.default_rng(8)
    n = 50_000
    hub = np.zeros(60_000, np.int32)
    tgt = rng.integers(1, n, 60_000).astype(np.int32)
    mid_src = rng.integers(1, 40, 100_000).astype(np.int32)
    mid_dst = rng.integers(0, n, 100_000).astype(np.int32)
    src = np.concatenate([hub, mid_src])
    dst = np.concatenate([tgt, mid_dst])
    w = rng.lognormal(0, 1, src.size).astype(np.float32)
    for directed in (True, False):
        g = gen.Graph(n, src, dst, w, directed)
        adj = oracle.build_graph(g)
        mval, deg = oracle.transition(adj)
        with cl.Context(0) as ctx:
            ctx.build_graph(g)
            csr = {k: v.cpu().numpy() for k, v in ctx.csr().items()}
        assert np.array_equal(csr["row_ptr"], adj.row_ptr)
        assert np.array_equal(csr["col"], adj.col)
        assert np.allclose(csr["deg"], deg, rtol=1e-14, atol=0)
        assert np.all(np.abs(csr["val"] - mval) <= mval * 2.0**-24 * 1.0001 + 1e-30)


def test_csr_runs_of_empty_rows(cl):
    # edges only among a few node ranges: long runs of empty rows at the
    # start, between the ranges and at the end (row pointers of a run of
    # 64 or more empty rows are written by a whole wave), loops, repeated
    # weighted pairs; undirected weighted and directed unweighted
    rng = np.random.default_rng(12)
    n = 20_000
    parts = []
    ranges = [(1000, 1100, 3000), (5000, 5010, 200), (5075, 5076, 5), (12_000, 12_400, 4000)]
    for lo, hi, m in ranges:  # (5075, 5076): loops only
        parts.append((rng.integers(lo, hi, m), rng.integers(lo, hi, m)))
    src = np.concatenate([a for a, _ in parts]).astype(np.int32)
    dst = np.concatenate([b for _, b in parts]).astype(np.int32)
    w = rng.lognormal(0, 1, src.size).astype(np.float32)
    cases = [gen.Graph(n, src, dst, w, False, "ranges"),
             gen.Graph(n, src, dst, None, True, "ranges-directed")]
    for g in cases:
        adj = oracle.build_graph(g)
        mval, deg = oracle.transition(adj)
        with cl.Context(0) as ctx:
            ctx.build_graph(g)
            csr = {k: v.cpu().numpy() for k, v in ctx.csr().items()}
        assert np.array_equal(csr["row_ptr"], adj.row_ptr), g.name
        assert np.array_equal(csr["col"], adj.col), g.name
        assert np.allclose(csr["deg"], deg, rtol=1e-14, atol=0)
        assert np.all(np.abs(csr["val"] - mval) <= mval * 2.0**-24 * 1.0001 + 1e-30)


# ------------------------------------------------------ propagation

@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("dim,chunk", [(128, 0), (256, 0), (37, 16), (1024, 0), (64, 8)])
def test_propagate_parity_f32(cl, gi, dim, chunk):
    g = zoo()[gi]
    got = gpu_embed(cl, g, dim, 3, seed=5, chunk=chunk)
    want = oracle_embed(g, dim, 3, 5)
    err = np.abs(got - want).max()
    assert err <= F32_TOL, (g.name, dim, chunk, err)


def test_er10k_workload_parity(cl):
    # the small Erdos-Renyi workload in full: N=10k, 50k edges, d=128, k=4
    g, dim, k, _ = gen.workload("er10k")
    got = gpu_embed(cl, g, dim, k, seed=2102)
    want = oracle_embed(g, dim, k, 2102)
    err = np.abs(got - want).max()
    print(f"er10k max-abs {err:.3e}")
    assert err <= F32_TOL


def test_empty_keep(cl):
    g = gen.random_graph(2000, 1500, 12, directed=True)
    for keep in (False, True):
        got = gpu_embed(cl, g, 48, 3, seed=3, empty_keep=keep)
        want = oracle_embed(g, 48, 3, 3, empty_keep=keep)
        assert np.abs(got - want).max() <= F32_TOL


def test_gpu_invariants(cl):
    g = gen.chung_lu(20_000, 150_000, 2.1, 13)
    adj = oracle.build_graph(g)
    deg = np.diff(adj.row_ptr)
    T = gpu_embed(cl, g, 256, 4, seed=1)
    nrm = np.linalg.norm(T, axis=1)
    assert np.all(np.abs(nrm[deg > 0] - 1) < 1e-5)
    assert np.all(T[deg == 0] == 0)


def test_resume_is_bitwise(cl):
    g = gen.chung_lu(20_000, 150_000, 2.1, 14)
    with cl.Context(0) as a, cl.Context(0) as b:
        a.build_graph(g).init(128, "f32", 9).propagate(4)
        b.build_graph(g).init(128, "f32", 9).propagate(1).propagate(0).propagate(3)
        assert a.info()["iteration"] == 4 == b.info()["iteration"]
        ea, eb = a.embedding().cpu().numpy(), b.embedding().cpu().numpy()
    assert np.array_equal(ea, eb)


def test_deterministic_rerun(cl):
    g = gen.bipartite_zipf(20_000, 3000, 200_000, 1.1, 15)
    a = gpu_embed(cl, g, 256, 4, seed=4, chunk=64)
    b = gpu_embed(cl, g, 256, 4, seed=4, chunk=64)
    assert np.array_equal(a, b)


# ------------------------------------------------------------ batched

def test_batch_equals_solo_bitwise(cl):
    graphs = [gen.chung_lu(3000, 20_000, 2.1, 20), gen.erdos_renyi(500, 2000, 21),
              gen.bipartite_zipf(2000, 300, 15_000, 1.1, 22), gen.chung_lu(8000, 60_000, 2.1, 23)]
    seeds = [5, 6, 7, 8]
    with cl.Context(0) as ctx:
        outs = cl.embed_batch(ctx, graphs, 96, 4, seeds)
        outs = [o.cpu().numpy() for o in outs]
    for g, s, o in zip(graphs, seeds, outs):
        solo = gpu_embed(cl, g, 96, 4, seed=s).astype(np.float32)
        assert np.array_equal(o, solo), g.name
        assert np.abs(o - oracle_embed(g, 96, 4, s)).max() <= F32_TOL


@pytest.mark.parametrize("persistent", [0, 1])
def test_step_multi_equals_solo_bitwise(cl, persistent):
    graphs = [gen.chung_lu(4000, 30_000, 2.1, 30), gen.erdos_renyi(900, 4000, 31),
              gen.chung_lu(12_000, 90_000, 2.1, 32)]
    ctxs = [cl.Context(0) for _ in graphs]
    try:
        for c, g, s in zip(ctxs, graphs, [1, 2, 3]):
            # the first context's grid choice applies to the shared launch
            c.set_schedule(0, persistent)
            c.build_graph(g).init(128, "f32", s)
            assert c.schedule()["persistent"] == persistent
        ctxs[0].propagate(1)  # requests at different iterations share a step
        for _ in range(3):
            cl.step_multi(ctxs)
        cl.step_multi(ctxs[1:])
        got = [c.embedding().cpu().numpy() for c in ctxs]
        its = [c.info()["iteration"] for c in ctxs]
    finally:
        for c in ctxs:
            c.close()
    assert its == [4, 4, 4]
    for g, s, o in zip(graphs, [1, 2, 3], got):
        assert np.array_equal(o, gpu_embed(cl, g, 128, 4, seed=s).astype(np.float32))


# --------------------------------------------------------------- bf16

def bf16_report(got, want):
    err = np.abs(got - want).max()
    nz = np.linalg.norm(want, axis=1) > 0
    cos = (got[nz] * want[nz]).sum(1) / (np.linalg.norm(got[nz], axis=1) *
                                         np.linalg.norm(want[nz], axis=1))
    return float(err), float(cos.min())


@pytest.mark.parametrize("gi", [0, 3, 4])
def test_bf16_error_bound(cl, gi):
    g = zoo()[gi]
    got = gpu_embed(cl, g, 256, 4, seed=6, dtype="bf16")
    want = oracle_embed(g, 256, 4, 6)
    err, cmin = bf16_report(got, want)
    print(f"bf16 {g.name}: max-abs {err:.3e} min-cos {cmin:.7f}")
    assert err <= BF16_MAXABS and cmin >= BF16_MINCOS


# ------------------------------------------------------------- errors

def test_invalid_inputs(cl):
    from paper_2102_02302_amd import _lib
    with cl.Context(0) as ctx:
        with pytest.raises(cl.CleoraError) as e:
            ctx.build_csr(10, [0, 11], [1, 2])
        assert e.value.code == _lib.E_INPUT
        with pytest.raises(cl.CleoraError) as e:
            ctx.build_csr(10, [0, 1], [1, 2], w=[1.0, -1.0])
        assert e.value.code == _lib.E_INPUT
        with pytest.raises(cl.CleoraError) as e:
            ctx.build_csr(10, [0, 1], [1, 2], w=[1.0, math.inf])
        assert e.value.code == _lib.E_INPUT
        with pytest.raises(cl.CleoraError) as e:
            ctx.init(16, "f32", 0)  # no graph after a failed build
        assert e.value.code == _lib.E_STATE
        ctx.build_csr(10, [0, 1], [1, 2])
        with pytest.raises(cl.CleoraError) as e:
            ctx.init(0, "f32", 0)
        assert e.value.code == _lib.E_INVAL
        with pytest.raises(cl.CleoraError) as e:
            ctx.propagate(1)
        assert e.value.code == _lib.E_STATE
        ctx.init(16, "f32", 0)
        with pytest.raises(cl.CleoraError):
            ctx.propagate(-1)
        ctx.propagate(2)
        assert ctx.info()["iteration"] == 2


def test_empty_graph_and_tiny(cl):
    g = gen.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), None, False)
    T = gpu_embed(cl, g, 8, 2, seed=1)
    assert np.all(T == 0)
    T = gpu_embed(cl, g, 8, 2, seed=1, empty_keep=True)
    assert np.abs(T - oracle_embed(g, 8, 2, 1, empty_keep=True)).max() <= F32_TOL
    g1 = gen.Graph(1, np.zeros(1, np.int32), np.zeros(1, np.int32), None, False)  # one loop
    assert np.abs(gpu_embed(cl, g1, 3, 3, seed=2) - oracle_embed(g1, 3, 3, 2)).max() <= F32_TOL


def test_graph_replays_match_eager(cl):
    # k >= 2 runs as a captured graph: replay it several times, with eager
    # single steps in between, and compare every result with all-eager steps
    g = gen.chung_lu(30_000, 200_000, 2.1, 40)
    with cl.Context(0) as a, cl.Context(0) as b:
        a.set_chunk(32)
        b.set_chunk(32)
        a.build_graph(g).init(96, "f32", 3)
        b.build_graph(g).init(96, "f32", 3)
        for rep in range(4):
            a.propagate(2)
            a.propagate(1)
            for _ in range(3):
                b.propagate(1)
            assert np.array_equal(a.embedding().cpu().numpy(), b.embedding().cpu().numpy()), rep
        assert a.info()["iteration"] == 12


def test_timed_graph_replays_match_untimed(cl):
    # timing on: the captured loop records events around its launches; the
    # bits are those of the untimed loop and of eager steps, and every
    # launch of every replay is timed
    g = gen.chung_lu(30_000, 200_000, 2.1, 41)
    with cl.Context(0) as a, cl.Context(0) as b:
        a.set_chunk(32)
        b.set_chunk(32)
        a.build_graph(g).init(128, "f32", 5)
        b.build_graph(g).init(128, "f32", 5)
        a.kernel_time()
        a.set_timing(True)
        for _ in range(3):
            a.propagate(4)
        a.set_timing(False)
        kt = a.kernel_time()
        assert kt["spmm_launches"] == 12 and kt["spmm_ms"] > 0
        assert kt["combine_launches"] == 12 and kt["combine_ms"] > 0
        for _ in range(12):
            b.propagate(1)
        assert np.array_equal(a.embedding().cpu().numpy(), b.embedding().cpu().numpy())
        a.propagate(4)  # untimed loop of the same k
        for _ in range(4):
            b.propagate(1)
        assert np.array_equal(a.embedding().cpu().numpy(), b.embedding().cpu().numpy())
        assert a.kernel_time()["spmm_launches"] == 0


def test_rebuilds_reuse_the_captured_loop(cl):
    # the same graph rebuilt and re-initialised (as every bench step and
    # batch does) replays the loop captured the first time; a graph of
    # another shape is captured anew, and its results are still right
    import torch
    g = gen.chung_lu(20_000, 150_000, 2.1, 42)
    h = gen.erdos_renyi(9_000, 40_000, 43)
    dev = torch.device("cuda", 0)
    gs, gd = torch.as_tensor(g.src).to(dev), torch.as_tensor(g.dst).to(dev)
    hs, hd = torch.as_tensor(h.src).to(dev), torch.as_tensor(h.dst).to(dev)
    with cl.Context(0) as ctx:
        outs = []
        for _ in range(4):
            ctx.build_init(g.n, gs, gd, None, 64, "f32", seed=7)
            ctx.propagate(4)
            outs.append(ctx.embedding().cpu().numpy())
        st = ctx.launch_stats()
        assert st == {"graph_instantiations": 1, "graph_launches": 4}, st
        assert all(np.array_equal(outs[0], o) for o in outs[1:])
        ctx.build_init(h.n, hs, hd, None, 64, "f32", seed=7)
        ctx.propagate(4)
        got_h = ctx.embedding().cpu().numpy()
        assert ctx.launch_stats()["graph_instantiations"] == 2
        ctx.build_init(g.n, gs, gd, None, 64, "f32", seed=7)
        ctx.propagate(4)
        assert np.array_equal(ctx.embedding().cpu().numpy(), outs[0])
    assert np.abs(outs[0] - oracle_embed(g, 64, 4, 7)).max() <= F32_TOL
    assert np.abs(got_h - oracle_embed(h, 64, 4, 7)).max() <= F32_TOL


@pytest.mark.parametrize("dim,dtype", [(32, "f32"), (128, "f32"), (256, "bf16"), (1024, "f32")])
def test_persistent_grid_same_bits(cl, dim, dtype):
    # a persistent grid only changes which wave runs which work item
    import torch
    g = gen.chung_lu(30_000, 250_000, 2.1, 71)  # 175 rows longer than 256 entries
    ref = cl.embed(g, dim, 3, 9, dtype=dtype)
    for pack, persistent in [(0, 1), (16, 1), (64, 2), (0, 0)]:
        with cl.Context(0) as c:
            c.set_schedule(pack, persistent)
            c.build_graph(g).init(dim, dtype, 9)
            sch = c.schedule()
            assert sch["persistent"] == persistent and sch["split_rows"] > 0
            if pack:
                assert sch["pack"] == pack
            c.propagate(3)
            assert torch.equal(c.embedding(), ref), (pack, persistent)


def test_set_schedule_rejects_bad_values(cl):
    with cl.Context(0) as c:
        for pack, persistent in [(8, -1), (1 << 21, -1), (0, 9), (0, -2)]:
            with pytest.raises(cl.CleoraError):
                c.set_schedule(pack, persistent)


def test_autotune_keeps_results(cl):
    # the packing size only moves rows between waves: same bits before and
    # after tuning, and the tuned choice is reused by later inits
    g = gen.chung_lu(40_000, 300_000, 2.1, 70)
    with cl.Context(0) as a:
        a.build_graph(g).init(128, "f32", 4).propagate(2)
        before = a.embedding().cpu().numpy()
        tuned = a.autotune()
        assert 16 <= tuned["pack"] <= a.schedule()["chunk"]
        assert a.schedule()["pack"] == tuned["pack"]
        assert a.schedule()["persistent"] == int(tuned["persistent"])
        assert a.schedule()["packed_items"] > 0
        assert np.array_equal(a.embedding().cpu().numpy(), before)
        assert a.info()["iteration"] == 2
        a.propagate(2)
        after = a.embedding().cpu().numpy()
    with cl.Context(0) as b:
        b.build_graph(g).init(128, "f32", 4).propagate(4)
        assert np.array_equal(b.embedding().cpu().numpy(), after)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_build_init_equals_separate_calls(cl, dtype):
    import torch
    for g in (gen.chung_lu(20_000, 150_000, 2.1, 81),
              gen.random_graph(3000, 9000, 82, directed=True, weighted=True, loops=True,
                               multi=True)):
        with cl.Context(0) as a, cl.Context(0) as b:
            a.build_graph(g).init(96, dtype, 5).propagate(3)
            b.build_graph_init(g, 96, dtype, 5).propagate(3)
            assert torch.equal(a.embedding(), b.embedding()), g.name
            # k = 0 returns T_0 itself
            b.build_graph_init(g, 96, dtype, 6)
            a.init(96, dtype, 6)
            assert torch.equal(a.embedding(), b.embedding()), g.name


def test_build_init_bad_input_leaves_no_embedding(cl):
    g = gen.erdos_renyi(500, 2000, 83)
    bad = g.dst.copy()
    bad[10] = 500
    with cl.Context(0) as c:
        c.build_graph_init(g, 32, "f32", 1).propagate(1)
        with pytest.raises(cl.CleoraError) as e:
            c.build_init(g.n, g.src, bad, None, 32, "f32", 1)
        assert "E_INPUT" in str(e.value)
        with pytest.raises(cl.CleoraError):
            c.propagate(1)
        c.build_graph_init(g, 32, "f32", 1).propagate(2)
        want = cl.embed(g, 32, 2, 1)
        import torch
        assert torch.equal(c.embedding(), want)


def test_tune_cache_file_across_processes(cl, tmp_path):
    """CLEORA_TUNE_CACHE: a tuned choice is written once and picked up by
    later processes, also by inits that never call the autotuner."""
    import os
    import subprocess
    import sys
    code = (
        "import sys, gen, paper_2102_02302_amd as cl\n"
        "g = gen.chung_lu(20_000, 150_000, 2.1, 91)\n"
        "with cl.Context(0) as c:\n"
        "    c.build_graph_init(g, 64, 'f32', 1)\n"
        "    if sys.argv[1] == 'tune':\n"
        "        t = c.autotune()\n"
        "        print('RESULT', t['pack'], int(t['persistent']))\n"
        "    else:\n"
        "        s = c.schedule()\n"
        "        print('RESULT', s['pack'], s['persistent'])\n")
    path = tmp_path / "tune.txt"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CLEORA_TUNE_CACHE=str(path))

    def run(mode):
        r = subprocess.run([sys.executable, "-c", code, mode], cwd=root, env=env,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        return [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT")][0].split()[1:]

    tuned = run("tune")
    lines = path.read_text().strip().splitlines()
    assert len(lines) == 1 and len(lines[0].split()) == 8
    assert lines[0].split()[5:7] == tuned
    assert run("plain") == tuned   # planned from the file, no tuning
    assert run("tune") == tuned    # cached: nothing new appended
    assert len(path.read_text().strip().splitlines()) == 1


# ------------------------------------------------------ edge cases

def hub_graph(n, hub_degrees, extra_m, seed):
    """Hubs 0, 1, ... with exactly the given numbers of distinct neighbours,
    plus random edges among the other nodes."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for h, d in enumerate(hub_degrees):
        nb = rng.choice(np.arange(len(hub_degrees), n), d, replace=False)
        src.append(np.full(d, h))
        dst.append(nb)
    a = rng.integers(len(hub_degrees), n, extra_m)
    b = rng.integers(len(hub_degrees), n, extra_m)
    ok = a != b
    src.append(a[ok])
    dst.append(b[ok])
    return gen.Graph(n, np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32),
                     None, False, f"hubs{hub_degrees}")


@pytest.mark.parametrize("dim,dtype", [(64, "f32"), (256, "f32"), (96, "bf16"), (512, "bf16")])
def test_split_size_boundaries(cl, dim, dtype):
    # rows of exactly S - 1, S, S + 1, 2S, 2S + 1 entries (S = 512) and one
    # past the 4096-entry segmented row sums
    g = hub_graph(9000, [511, 512, 513, 1024, 1025, 4097], 20_000, 61)
    with cl.Context(0) as c:
        c.build_graph(g).init(dim, dtype, 7).propagate(3)
        assert c.schedule()["chunk"] == 512 and c.schedule()["split_rows"] >= 4
        got = c.embedding("f32").cpu().numpy().astype(np.float64)
    want = oracle_embed(g, dim, 3, 7)
    if dtype == "f32":
        assert np.abs(got - want).max() <= F32_TOL
    else:
        err, cmin = bf16_report(got, want)
        assert err <= BF16_MAXABS and cmin >= BF16_MINCOS, (err, cmin)


@pytest.mark.parametrize("dim,dtype", [(4096, "f32"), (8192, "bf16")])
def test_maximum_dimensions(cl, dim, dtype):
    g = hub_graph(1500, [700], 6000, 62)  # one split hub row
    with cl.Context(0) as c:
        c.build_graph(g).init(dim, dtype, 8).propagate(2)
        got = c.embedding("f32").cpu().numpy().astype(np.float64)
        with pytest.raises(cl.CleoraError):
            c.init(dim + 1, dtype, 8)
    want = oracle_embed(g, dim, 2, 8)
    if dtype == "f32":
        assert np.abs(got - want).max() <= F32_TOL
    else:
        err, cmin = bf16_report(got, want)
        assert err <= BF16_MAXABS and cmin >= BF16_MINCOS, (err, cmin)


@pytest.mark.parametrize("dim", [8, 24, 40, 200, 1000])
def test_bf16_odd_widths(cl, dim):
    # every group count of the narrow-row kernels (16, 16, 8, 2, 1 rows per
    # wave) and partial 16-byte vectors
    g = zoo()[3]
    got = gpu_embed(cl, g, dim, 3, seed=10, dtype="bf16")
    want = oracle_embed(g, dim, 3, 10)
    err, cmin = bf16_report(got, want)
    assert err <= BF16_MAXABS and cmin >= BF16_MINCOS, (dim, err, cmin)


@pytest.mark.parametrize("empty_keep", [False, True])
def test_batch_directed_weighted_equals_solo(cl, empty_keep):
    graphs = [gen.random_graph(n, 4 * n, 70 + i, directed=True, weighted=True, loops=True,
                               multi=True) for i, n in enumerate((300, 1200, 50, 4000))]
    seeds = [11, 12, 13, 14]
    with cl.Context(0) as ctx:
        outs = cl.embed_batch(ctx, graphs, 40, 3, seeds, directed=True, empty_keep=empty_keep)
        outs = [o.cpu().numpy() for o in outs]
    for g, s, o in zip(graphs, seeds, outs):
        solo = gpu_embed(cl, g, 40, 3, seed=s, empty_keep=empty_keep).astype(np.float32)
        assert np.array_equal(o, solo), g.name
        want = oracle_embed(g, 40, 3, s, empty_keep=empty_keep)
        assert np.abs(o - want).max() <= F32_TOL


def test_batch_status_names_the_bad_graphs(cl):
    # one graph with an id out of range, one with a negative weight: the
    # call fails with E_INPUT, the status names them, the rest go again
    from paper_2102_02302_amd import _lib
    gs = [gen.erdos_renyi(300, 900, 70 + i) for i in range(4)]
    bad_id = gen.Graph(gs[1].n, gs[1].src.copy(), gs[1].dst.copy(), None, False, "bad id")
    bad_id.dst[7] = gs[1].n
    w = np.ones(gs[3].m, np.float32)
    w[5] = -1.0
    bad_w = gen.Graph(gs[3].n, gs[3].src, gs[3].dst, w, False, "bad weight")
    batch = [gs[0], bad_id, gs[2], bad_w]
    with cl.Context(0) as ctx:
        with pytest.raises(cl.CleoraError):
            cl.batch_status(ctx, 4)  # no batch call yet
        with pytest.raises(cl.CleoraError) as e:
            cl.embed_batch(ctx, batch, 32, 2, [1, 2, 3, 4])
        assert e.value.code == _lib.E_INPUT
        assert cl.batch_status(ctx, 4) == [_lib.OK, _lib.E_INPUT, _lib.OK, _lib.E_INPUT]
        with pytest.raises(cl.CleoraError):
            cl.batch_status(ctx, 3)  # not the last call's count
        outs = cl.embed_batch(ctx, [gs[0], gs[2]], 32, 2, [1, 3])
        assert cl.batch_status(ctx, 2) == [_lib.OK, _lib.OK]
    for g, sd, out in ((gs[0], 1, outs[0]), (gs[2], 3, outs[1])):
        assert np.array_equal(out.cpu().numpy(), gpu_embed(cl, g, 32, 2, sd))
