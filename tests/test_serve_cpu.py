"""CPU tests of the served form's scheduling policy with a simulated engine
and a virtual clock: admission by slots and footprint budget, iteration-level
batching, retirement after k iterations."""

import pytest

from paper_2102_02302_amd.serve import Job, Scheduler


class FakeEngine:
    def __init__(self, clock, build_s=0.002, step_s=0.001, budget=None, slots=None):
        self.clock = clock
        self.build_s = build_s
        self.step_s = step_s
        self.building = []
        self.live_slots = set()
        self.live_bytes = 0
        self.budget = budget
        self.slots = slots
        self.stepped = {}
        self.max_concurrent = 0
        self.finishing = []
        self.copy_s = 0.0003

    def footprint(self, job):
        return job.m * 10

    def start_build(self, job, slot):
        assert slot not in self.live_slots, "slot reused while busy"
        self.live_slots.add(slot)
        assert self.slots is None or slot < self.slots
        self.live_bytes += self.footprint(job)
        assert self.budget is None or self.live_bytes <= self.budget, "budget exceeded"
        self.building.append((self.clock.t + self.build_s, job))

    def poll_ready(self):
        ready = [j for t, j in self.building if t <= self.clock.t]
        self.building = [(t, j) for t, j in self.building if t > self.clock.t]
        return ready

    def step(self, jobs):
        self.max_concurrent = max(self.max_concurrent, len(jobs))
        for j in jobs:
            self.stepped[j.index] = self.stepped.get(j.index, 0) + 1
        self.clock.t += self.step_s

    def start_finish(self, job):
        self.finishing.append((self.clock.t + self.copy_s, job))

    def poll_finished(self):
        out = [j for t, j in self.finishing if t <= self.clock.t]
        self.finishing = [(t, j) for t, j in self.finishing if t > self.clock.t]
        for job in out:
            self.live_slots.discard(job.slot)
            self.live_bytes -= self.footprint(job)
            job.result = ("done", job.index)
        return out

    def idle_wait(self, s):
        self.clock.t += max(s, 1e-5)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def make_jobs(n, gap, m=100):
    return [Job(index=i, arrival_s=i * gap, n=10, m=m + i, seed=i) for i in range(n)]


def test_every_job_runs_k_iterations_and_finishes():
    clock = Clock()
    eng = FakeEngine(clock)
    sched = Scheduler(eng, k=4, max_slots=8, budget_bytes=10**9, clock=clock)
    done = sched.run(make_jobs(50, 0.0005))
    assert len(done) == 50
    assert all(eng.stepped[j.index] == 4 for j in done)
    assert all(j.result == ("done", j.index) for j in done)
    for j in done:
        assert j.arrival_s <= j.admitted_s <= j.ready_s <= j.done_s
        assert j.latency_s >= eng.build_s + 4 * eng.step_s - 1e-12


def test_continuous_batching_mixes_requests_at_different_iterations():
    clock = Clock()
    eng = FakeEngine(clock, build_s=0.0005, step_s=0.001)
    sched = Scheduler(eng, k=4, max_slots=16, budget_bytes=10**9, clock=clock)
    sched.run(make_jobs(40, 0.0004))
    # arrivals every 0.4 ms, one step per 1 ms: requests overlap in steps
    assert eng.max_concurrent >= 3
    assert max(sched.step_sizes) == eng.max_concurrent


def test_slots_and_budget_are_respected():
    clock = Clock()
    budget = 5 * 10 * 120
    eng = FakeEngine(clock, budget=budget, slots=3)
    sched = Scheduler(eng, k=2, max_slots=3, budget_bytes=budget, clock=clock)
    done = sched.run(make_jobs(30, 0.0))  # all at once: admission must queue
    assert len(done) == 30
    assert sched.peak_used <= budget
    assert sched.max_active <= 3


def test_request_larger_than_budget_is_refused():
    clock = Clock()
    eng = FakeEngine(clock)
    sched = Scheduler(eng, k=2, max_slots=2, budget_bytes=500, clock=clock)
    with pytest.raises(ValueError):
        sched.run(make_jobs(3, 0.0, m=100))


def test_arrival_order_admission_and_k_zero():
    clock = Clock()
    eng = FakeEngine(clock)
    sched = Scheduler(eng, k=0, max_slots=1, budget_bytes=10**9, clock=clock)
    done = sched.run(make_jobs(5, 0.001))
    assert [j.index for j in done] == list(range(5))
    assert not eng.stepped
