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
    from paper_2102_02302_amd.serve import GpuEngine, Scheduler, latency_stats
    trace = gen.served_trace(24, 1.0, n_lo=100, n_hi=20_000)
    graphs = gen.materialize(trace)
    dim, k = 64, 4
    jobs = jobs_for(trace, graphs, 0.0005)  # arrivals every ~0.5 ms on average
    eng = GpuEngine(dim, dtype, max_slots=6, keep_results=True)
    try:
        sched = Scheduler(eng, k=k, max_slots=6, budget_bytes=1 << 30)
        done = sched.run(jobs)
    finally:
        eng.close()
    assert len(done) == len(jobs)
    assert sched.max_active >= 2, "requests never overlapped"
    stats = latency_stats(done, k, dim, lambda j: 2 * j.m)
    print(f"{dtype}: {stats}, max active {sched.max_active}")
    for j in done:
        g = j.payload
        solo = cl.embed(g, dim, k, j.seed, dtype=dtype).float().cpu().numpy()
        got = j.result.float().numpy()
        assert np.array_equal(got, solo), j.index
        want = oracle.embed(g, dim, k, j.seed)
        err = np.abs(got - want).max()
        assert err <= (1e-5 if dtype == "f32" else 4e-3), (j.index, err)


def test_one_at_a_time_baseline(cl):
    from paper_2102_02302_amd.serve import one_at_a_time
    trace = gen.served_trace(6, 1.0, n_lo=100, n_hi=5000)
    graphs = gen.materialize(trace)
    jobs = jobs_for(trace, graphs, 0.0)
    done = one_at_a_time(jobs, 32, 4, keep_results=True)
    for j in done:
        want = oracle.embed(j.payload, 32, 4, j.seed)
        assert np.abs(j.result.numpy() - want).max() <= 1e-5
