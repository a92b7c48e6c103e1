"""Served form on the GPU: requests that arrive while others run are admitted
as slots and budget free up, share steps with requests at other iterations,
and each result equals the same request embedded alone -- bit for bit, and
within the stated tolerance of the FP64 oracle."""

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


def jobs_for(trace, graphs, time_scale):
    from paper_2102_02302_amd.serve import Job
    return [Job(index=r.index, arrival_s=r.arrival_s * time_scale, n=g.n, m=g.m, seed=r.seed,
                payload=g) for r, g in zip(trace, graphs)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_served_results_equal_solo(cl, dtype):
    """Poisson arrivals about every 20 us (well inside one request's build
    and steps, so requests are always in flight together), groups of at
    most two: requests join while others step, and every result equals the
    request embedded alone, bit for bit, and is within the stated tolerance
    of the FP64 oracle."""
    from paper_2102_02302_amd.serve import latency_stats, run_native
    trace = gen.served_trace(24, 1.0, n_lo=100, n_hi=20_000)
    graphs = gen.materialize(trace)
    dim, k = 64, 4
    jobs = jobs_for(trace, graphs, 0.00002)
    done = run_native(jobs, dim, dtype, k, slots=6, budget_bytes=1 << 30, builders=2,
                      keep_results=True, max_group=2)
    assert len(done) == len(jobs)
    st = run_native.last_stats
    assert st["max_active_groups"] >= 2, "requests never overlapped"
    print(f"{dtype}: {latency_stats(done, k, dim, lambda j: 2 * j.m)}, {st}")
    for j in done:
        g = j.payload
        solo = cl.embed(g, dim, k, j.seed, dtype=dtype)
        assert torch_equal(j.result, solo), j.index
        want = oracle.embed(g, dim, k, j.seed)
        err = np.abs(j.result.float().cpu().numpy() - want).max()
        assert err <= (1e-5 if dtype == "f32" else 4e-3), (j.index, err)


def test_native_server_memory_within_budget(cl):
    """A budget of about 2.5 of the largest request's charge: idle slots give
    their buffers back to make room, the charged memory never exceeds the
    budget, every build stays within its charge, and results are still
    those of the requests embedded alone."""
    from paper_2102_02302_amd.serve import NativeServer, run_native
    trace = gen.served_trace(40, 1.0, n_lo=100, n_hi=30_000)
    graphs = gen.materialize(trace)
    dim, k = 64, 4
    charge = [cl.footprint_bytes(g.n, g.m, dim, "f32") + 12 * g.m + 1024 for g in graphs]
    budget = int(2.5 * max(charge))
    srv = NativeServer(dim, "f32", k, slots=6, budget_bytes=budget, builders=2, max_group=4)
    try:
        done = run_native(jobs_for(trace, graphs, 0.0002), dim, "f32", k, keep_results=True,
                          server=srv)
        mem = srv.memory()
    finally:
        srv.close()
    print(f"budget {budget}: {mem}, {run_native.last_stats}")
    assert len(done) == len(graphs)
    assert mem["budget_bytes"] == budget
    assert mem["peak_charged_bytes"] <= budget
    assert mem["bound_exceeded"] == 0
    for j in done[::5]:
        assert torch_equal(j.result, cl.embed(j.payload, dim, k, j.seed)), j.index


def test_one_at_a_time_baseline(cl):
    from paper_2102_02302_amd.serve import one_at_a_time
    trace = gen.served_trace(6, 1.0, n_lo=100, n_hi=5000)
    graphs = gen.materialize(trace)
    jobs = jobs_for(trace, graphs, 0.0)
    done = one_at_a_time(jobs, 32, 4, keep_results=True)
    for j in done:
        want = oracle.embed(j.payload, 32, 4, j.seed)
        assert np.abs(j.result.numpy() - want).max() <= 1e-5


@pytest.mark.parametrize("dtype,max_group", [("f32", 1), ("f32", 8), ("bf16", 8)])
def test_native_server_results_equal_solo(cl, dtype, max_group):
    from paper_2102_02302_amd.serve import latency_stats, run_native
    trace = gen.served_trace(30, 1.0, n_lo=100, n_hi=20_000)
    graphs = gen.materialize(trace)
    dim, k = 64, 4
    jobs = jobs_for(trace, graphs, 0.0)
    # all at t = 0 so that groups of several requests form
    done = run_native(jobs, dim, dtype, k, slots=3, budget_bytes=1 << 30, builders=2,
                      keep_results=True, max_group=max_group)
    assert len(done) == len(jobs)
    stats = latency_stats(done, k, dim, lambda j: 2 * j.m)
    print(f"native {dtype} group {max_group}: {stats} {run_native.last_stats}")
    if max_group == 1:
        assert run_native.last_stats["max_active_groups"] >= 2, "requests never overlapped"
    else:
        assert run_native.last_stats["groups"] < len(jobs), "no request was grouped"
    for j in done:
        solo = cl.embed(j.payload, dim, k, j.seed, dtype=dtype)
        assert torch_equal(j.result, solo), j.index


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a.view(torch.int16) if a.dtype == torch.bfloat16 else a,
                            b.view(torch.int16) if b.dtype == torch.bfloat16 else b))


@pytest.mark.parametrize("max_group", [1, 4])
def test_native_server_reports_bad_requests(cl, max_group):
    """A bad request completes with E_INPUT; the requests built in the same
    group are still served, with their solo results.  Edge arrays may sit
    in host or device memory."""
    import torch
    from paper_2102_02302_amd import _lib
    from paper_2102_02302_amd.serve import NativeServer
    srv = NativeServer(16, "f32", 2, slots=2, budget_bytes=1 << 28, builders=1,
                       max_group=max_group)
    try:
        good = gen.erdos_renyi(50, 100, 3)
        other = gen.erdos_renyi(70, 300, 4)
        outs = [torch.empty((n, 16), device="cuda") for n in (50, 50, 70, 50)]
        bad_dst = good.dst.copy()
        bad_dst[3] = 50  # outside [0, n)
        bad_w = np.ones(len(good.src), np.float32)
        bad_w[7] = 0.0   # zero weights are rejected
        d_src = torch.as_tensor(other.src, device="cuda")
        d_dst = torch.as_tensor(other.dst, device="cuda")
        torch.cuda.synchronize()
        tickets = [srv.submit(50, good.src, bad_dst, None, 1, outs[0]),
                   srv.submit(50, good.src, good.dst, None, 1, outs[1]),
                   srv.submit(70, d_src, d_dst, None, 5, outs[2]),
                   srv.submit(50, good.src, good.dst, bad_w, 1, outs[3])]
        got = {}
        while len(got) < len(tickets):
            for c in srv.poll(8, 0.5):
                got[c[0]] = c[1]
        assert [got[t] for t in tickets] == [_lib.E_INPUT, 0, 0, _lib.E_INPUT]
        assert torch.equal(outs[1], cl.embed(good, 16, 2, 1))
        assert torch.equal(outs[2], cl.embed(other, 16, 2, 5))
        with pytest.raises(cl.CleoraError):
            srv.submit(0, good.src, good.dst, None, 1, outs[0])
    finally:
        srv.close()


def test_server_before_torch_in_fresh_process(cl):
    """A process whose first GPU user is the library (a server created
    before anything touches torch.cuda) can still allocate torch tensors."""
    import os
    import subprocess
    import sys
    code = (
        "from paper_2102_02302_amd.serve import NativeServer\n"
        "import numpy as np\n"
        "srv = NativeServer(16, 'f32', 2, slots=2, budget_bytes=1 << 28, builders=1)\n"
        "import torch\n"
        "out = torch.empty((3, 16), device='cuda')\n"
        "src = np.array([0, 1], np.int32); dst = np.array([1, 2], np.int32)\n"
        "t = srv.submit(3, src, dst, None, 5, out)\n"
        "got = []\n"
        "while not got:\n"
        "    got = srv.poll(4, 1.0)\n"
        "assert got[0][0] == t and got[0][1] == 0, got\n"
        "import paper_2102_02302_amd as cl, gen\n"
        "g = gen.Graph(3, src, dst, None, False)\n"
        "assert torch.equal(out, cl.embed(g, 16, 2, 5))\n"
        "srv.close()\n"
        "print('ok')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_native_server_concurrent_submitters(cl):
    """Four threads submit at once (ctypes releases the GIL in the calls);
    every ticket completes once, with its solo result."""
    import threading

    import torch
    from paper_2102_02302_amd.serve import NativeServer
    graphs = [gen.erdos_renyi(200 + 37 * i, 900 + 101 * i, 90 + i) for i in range(24)]
    outs = [torch.empty((g.n, 32), device="cuda") for g in graphs]
    torch.cuda.synchronize()
    srv = NativeServer(32, "f32", 3, slots=4, budget_bytes=1 << 30, builders=3, max_group=4)
    tickets = {}
    lock = threading.Lock()

    def submitter(part):
        for i in range(part, len(graphs), 4):
            g = graphs[i]
            t = srv.submit(g.n, g.src, g.dst, None, 1000 + i, outs[i])
            with lock:
                tickets[t] = i

    try:
        threads = [threading.Thread(target=submitter, args=(p,)) for p in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        done = {}
        while len(done) < len(graphs):
            for c in srv.poll(64, 0.5):
                assert c[0] not in done
                done[c[0]] = c[1]
        assert sorted(tickets) == sorted(done) and all(s == 0 for s in done.values())
    finally:
        srv.close()
    for t, i in tickets.items():
        assert torch.equal(outs[i], cl.embed(graphs[i], 32, 3, 1000 + i)), i


def test_native_server_budget_from_free_memory(cl):
    """budget 0: 80% of the free device memory.  A request whose footprint
    is above that is refused at submit; a normal one is served."""
    import torch
    from paper_2102_02302_amd.serve import NativeServer
    srv = NativeServer(32, "f32", 2, slots=2, budget_bytes=0, builders=1)
    try:
        g = gen.erdos_renyi(300, 1200, 95)
        out = torch.empty((g.n, 32), device="cuda")
        t = srv.submit(g.n, g.src, g.dst, None, 3, out)
        got = []
        while not got:
            got = srv.poll(4, 1.0)
        assert got[0][0] == t and got[0][1] == 0
        assert torch.equal(out, cl.embed(g, 32, 2, 3))
        tiny = np.zeros(4, np.int32)
        with pytest.raises(cl.CleoraError):  # about 600 GB of footprint
            srv.submit(2_000_000_000, tiny, tiny, None, 1, out)
    finally:
        srv.close()


def test_native_server_directed_weighted(cl):
    """A server for directed graphs: weighted requests with loops, repeated
    pairs and sinks, grouped, give their solo results."""
    import torch
    from paper_2102_02302_amd.serve import NativeServer
    graphs = [gen.random_graph(n, 3 * n, 120 + i, directed=True, weighted=True, loops=True,
                               multi=True) for i, n in enumerate((80, 900, 300, 2500, 40))]
    outs = [torch.empty((g.n, 24), device="cuda") for g in graphs]
    torch.cuda.synchronize()
    srv = NativeServer(24, "f32", 3, slots=2, budget_bytes=1 << 30, builders=1, max_group=4,
                       directed=True)
    try:
        tickets = {srv.submit(g.n, g.src, g.dst, g.w, 500 + i, outs[i]): i
                   for i, g in enumerate(graphs)}
        done = {}
        while len(done) < len(graphs):
            for c in srv.poll(8, 0.5):
                done[c[0]] = c[1]
        assert all(s == 0 for s in done.values())
    finally:
        srv.close()
    for t, i in tickets.items():
        assert torch.equal(outs[i], cl.embed(graphs[i], 24, 3, 500 + i)), i
