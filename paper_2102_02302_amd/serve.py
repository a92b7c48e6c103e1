"""Served form: continuous batching of independent embedding requests.

Each request is a whole graph to embed (T_k of Algorithm 1 for its own
graph and seed).  The server

* admits waiting requests in arrival order while a slot (a library context)
  is free and the HBM footprint of everything admitted stays within a
  budget (``cleora_footprint_bytes``);
* builds an admitted request's CSR and T_0 on a side stream, in a builder
  thread, while the running requests keep stepping;
* advances every running request by one iteration per step, all of them in
  the same kernel launches (``cleora_step_multi``), whatever iteration each
  is at: a request joins at the next iteration boundary after its build and
  leaves as soon as it has done its k iterations, freeing its slot and its
  share of the budget;
* records latency = completion - arrival per request.

The scheduling policy (``Scheduler``) is plain Python and is tested on the
CPU with a simulated engine; ``GpuEngine`` is the MI355X implementation.
"""

from __future__ import annotations

import collections
import ctypes
import dataclasses
import queue
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence


@dataclasses.dataclass
class Job:
    index: int
    arrival_s: float
    n: int
    m: int
    seed: int
    payload: object = None          # host-side graph (src, dst, w, directed)
    footprint: int = 0
    admitted_s: float = -1.0
    ready_s: float = -1.0
    done_s: float = -1.0
    iteration: int = 0
    slot: int = -1
    result: object = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class Scheduler:
    """Admission and iteration-level batching, independent of the device.

    ``engine`` provides: footprint(job) -> bytes; start_build(job, slot)
    (asynchronous); poll_ready() -> list of jobs whose build finished;
    step(jobs) (one iteration each, synchronous); start_finish(job)
    (asynchronous copy of the result); poll_finished() -> list of jobs whose
    result is out; idle_wait(seconds)."""

    def __init__(self, engine, k: int, max_slots: int, budget_bytes: int,
                 clock: Callable[[], float] = time.perf_counter):
        self.engine = engine
        self.k = k
        self.max_slots = max_slots
        self.budget = budget_bytes
        self.clock = clock
        self.used = 0
        self.peak_used = 0
        self.max_active = 0
        self.steps = 0
        self.step_sizes: List[int] = []

    def run(self, jobs: Sequence[Job]) -> List[Job]:
        jobs = sorted(jobs, key=lambda j: (j.arrival_s, j.index))
        for j in jobs:
            j.footprint = int(self.engine.footprint(j))
            if j.footprint > self.budget:
                raise ValueError(f"request {j.index} needs {j.footprint} bytes, "
                                 f"more than the whole budget {self.budget}")
        free_slots = collections.deque(range(self.max_slots))
        pending: collections.deque = collections.deque()
        building: Dict[int, Job] = {}
        retiring: Dict[int, Job] = {}
        active: List[Job] = []
        done: List[Job] = []
        nxt = 0
        t0 = self.clock()
        while len(done) < len(jobs):
            now = self.clock() - t0
            while nxt < len(jobs) and jobs[nxt].arrival_s <= now:
                pending.append(jobs[nxt])
                nxt += 1
            # admission: arrival order, a free slot, and the budget
            while pending and free_slots and self.used + pending[0].footprint <= self.budget:
                j = pending.popleft()
                j.slot = free_slots.popleft()
                j.admitted_s = self.clock() - t0
                self.used += j.footprint
                self.peak_used = max(self.peak_used, self.used)
                building[j.index] = j
                self.engine.start_build(j, j.slot)
            for j in self.engine.poll_finished():
                retiring.pop(j.index)
                j.done_s = self.clock() - t0
                self.used -= j.footprint
                free_slots.append(j.slot)
                done.append(j)
            for j in self.engine.poll_ready():
                building.pop(j.index)
                j.ready_s = self.clock() - t0
                if self.k == 0:
                    retiring[j.index] = j
                    self.engine.start_finish(j)
                else:
                    active.append(j)
            if active:
                self.max_active = max(self.max_active, len(active))
                self.engine.step(active)
                self.steps += 1
                self.step_sizes.append(len(active))
                still = []
                for j in active:
                    j.iteration += 1
                    if j.iteration >= self.k:
                        retiring[j.index] = j
                        self.engine.start_finish(j)
                    else:
                        still.append(j)
                active = still
            else:
                wait = 0.0002 if (building or retiring) else 0.0005
                if nxt < len(jobs) and not building and not pending and not retiring:
                    wait = max(0.0, min(0.01, jobs[nxt].arrival_s - (self.clock() - t0)))
                self.engine.idle_wait(wait)
        return done


class GpuEngine:
    """Requests on one MI355X: one library context per slot (reused, so its
    device buffers are reused), builds on a side stream in a worker thread,
    steps with ``step_multi`` on the main stream."""

    def __init__(self, dim: int, dtype: str, max_slots: int, device: int = 0,
                 keep_results: bool = False, builders: int = 4):
        import torch

        from . import Context, footprint_bytes
        self.torch = torch
        self.dim, self.dtype = dim, dtype
        self.keep_results = keep_results
        self._footprint = footprint_bytes
        self.ctxs = [Context(device) for _ in range(max_slots)]
        self.main = torch.cuda.Stream(device=device)
        self._todo: queue.Queue = queue.Queue()
        self._ready: queue.Queue = queue.Queue()
        self._err: Optional[BaseException] = None
        self._retiring: list = []
        # several builders, each with its own stream, so that the host-side
        # latency of one build (launches, two synchronisations) overlaps others
        self._workers = []
        for _ in range(max(1, builders)):
            t = threading.Thread(target=self._build_loop,
                                 args=(torch.cuda.Stream(device=device),), daemon=True)
            t.start()
            self._workers.append(t)

    def footprint(self, job: Job) -> int:
        g = job.payload
        return self._footprint(job.n, job.m, self.dim, self.dtype, directed=g.directed)

    def start_build(self, job: Job, slot: int) -> None:
        self._todo.put(job)

    def _build_loop(self, side) -> None:
        torch = self.torch
        while True:
            job = self._todo.get()
            if job is None:
                return
            try:
                ctx = self.ctxs[job.slot]
                g = job.payload
                with torch.cuda.stream(side):
                    ctx.build_csr(g.n, g.src, g.dst, g.w, directed=g.directed, stream=side)
                    ctx.init(self.dim, self.dtype, job.seed, stream=side)
                    ctx.sync(side)
                self._ready.put(job)
            except BaseException as e:  # surfaced by poll_ready
                self._err = e
                self._ready.put(None)

    def poll_ready(self) -> List[Job]:
        out = []
        while True:
            try:
                j = self._ready.get_nowait()
            except queue.Empty:
                break
            if j is None:
                raise RuntimeError("request build failed") from self._err
            out.append(j)
        return out

    def step(self, jobs: List[Job]) -> None:
        from . import step_multi
        step_multi([self.ctxs[j.slot] for j in jobs], stream=self.main)

    def start_finish(self, job: Job) -> None:
        """Copy the result to pinned host memory on the copy stream; the
        slot is released when the copy's event has completed."""
        torch = self.torch
        ctx = self.ctxs[job.slot]
        inf = ctx.info()
        tdt = torch.float32 if inf["dtype"] == 0 else torch.bfloat16
        host = torch.empty((inf["n"], inf["dim"]), dtype=tdt, pin_memory=True)
        from . import _lib
        _lib.check(ctx._lib.cleora_get_embedding(ctx.handle, host.data_ptr(), inf["dim"],
                                                 inf["dtype"], ctypes.c_void_p(self.main.cuda_stream)))
        ev = torch.cuda.Event()
        ev.record(self.main)
        self._retiring.append((ev, job, host))

    def poll_finished(self) -> List[Job]:
        out, keep = [], []
        for ev, job, host in self._retiring:
            if ev.query():
                job.result = host if self.keep_results else None
                out.append(job)
            else:
                keep.append((ev, job, host))
        self._retiring = keep
        return out

    def idle_wait(self, seconds: float) -> None:
        if seconds > 0:
            time.sleep(seconds)

    def close(self) -> None:
        for _ in self._workers:
            self._todo.put(None)
        for t in self._workers:
            t.join(timeout=10)
        for c in self.ctxs:
            c.close()


def one_at_a_time(jobs: Sequence[Job], dim: int, k: int, dtype: str = "f32", device: int = 0,
                  keep_results: bool = False,
                  clock: Callable[[], float] = time.perf_counter,
                  result_on_device: bool = False) -> List[Job]:
    """Baseline: the same arrivals served one request after another by a
    single context with the plain path (build, init, k iterations, copy of
    the result to pinned host memory, or to device memory)."""
    import torch

    from . import Context, _lib
    jobs = sorted(jobs, key=lambda j: (j.arrival_s, j.index))
    out = []
    with Context(device) as ctx:
        t0 = clock()
        for j in jobs:
            wait = j.arrival_s - (clock() - t0)
            if wait > 0:
                time.sleep(wait)
            j.admitted_s = clock() - t0
            g = j.payload
            ctx.build_csr(g.n, g.src, g.dst, g.w, directed=g.directed)
            ctx.init(dim, dtype, j.seed)
            ctx.propagate(k)
            # result straight into pinned host (or device) memory, as the servers do
            tdt = torch.float32 if dtype in ("f32", "float32") else torch.bfloat16
            host = (torch.empty((g.n, dim), dtype=tdt, device=ctx.device) if result_on_device
                    else torch.empty((g.n, dim), dtype=tdt, pin_memory=True))
            _lib.check(ctx._lib.cleora_get_embedding(ctx.handle, host.data_ptr(), dim,
                                                     0 if tdt == torch.float32 else 1, None))
            ctx.sync()
            j.result = host if keep_results else None
            j.done_s = clock() - t0
            out.append(j)
        torch.cuda.synchronize()
    return out


def latency_stats(done: Sequence[Job], k: int, dim: int, nnz_of: Callable[[Job], int]) -> dict:
    import numpy as np
    lat = np.array([j.latency_s for j in done]) * 1e3
    span = max(j.done_s for j in done) - min(j.arrival_s for j in done)
    edge_dims = sum(nnz_of(j) for j in done) * float(k) * dim
    out = {"requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3),
           "req_per_s": round(len(done) / span, 2),
           "gedge_dims_per_s": round(edge_dims / span / 1e9, 3), "span_s": round(span, 3)}
    if all(j.admitted_s >= 0 and j.ready_s >= 0 for j in done):
        # where the time goes: waiting for admission, build + init, k steps
        # and the copy of the result
        phases = {"queue": [j.admitted_s - j.arrival_s for j in done],
                  "build": [j.ready_s - j.admitted_s for j in done],
                  "steps": [j.done_s - j.ready_s for j in done]}
        out["phases_ms"] = {name: {"p50": round(float(np.percentile(v, 50)) * 1e3, 3),
                                   "p99": round(float(np.percentile(v, 99)) * 1e3, 3)}
                            for name, v in phases.items()}
    return out


class NativeServer:
    """The C++ request server of the library (``cleora_server_*``): the same
    policy as ``Scheduler``, with native scheduler and builder threads."""

    def __init__(self, dim: int, dtype: str, k: int, slots: int = 64,
                 budget_bytes: int = 64 << 30, builders: int = 3, device: int = 0,
                 directed: bool = False, max_group: int = 16):
        from . import DIRECTED, _dtype_code, _lib
        self._lib = _lib.load()
        self._check = _lib.check
        self._Request, self._Completion = _lib.Request, _lib.Completion
        self.dim, self.dtype, self.k = dim, dtype, k
        self.code = _dtype_code(dtype)
        h = ctypes.c_void_p()
        self._check(self._lib.cleora_server_create(ctypes.byref(h), device, dim, self.code, k,
                                                   slots, budget_bytes, builders, max_group,
                                                   DIRECTED if directed else 0))
        self._h = h
        self._keep: Dict[int, tuple] = {}

    def now(self) -> float:
        return float(self._lib.cleora_server_now(self._h))

    def submit(self, n: int, src, dst, w, seed: int, out) -> int:
        """src/dst/w: contiguous host (numpy) or device (torch) arrays; out: a
        device or pinned host tensor of n x dim.  Returns the ticket."""
        import numpy as np

        def ptr(a):
            if a is None:
                return None
            return a.ctypes.data if isinstance(a, np.ndarray) else a.data_ptr()

        req = self._Request(n, len(src), ptr(src), ptr(dst), ptr(w), seed & (2**64 - 1),
                            out.data_ptr())
        t = ctypes.c_int64()
        self._check(self._lib.cleora_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (src, dst, w, out)
        return t.value

    def poll(self, max_n: int = 256, wait_s: float = 0.0) -> list:
        buf = (self._Completion * max_n)()
        n = ctypes.c_int32()
        self._check(self._lib.cleora_server_poll(self._h, buf, max_n, ctypes.byref(n), wait_s))
        out = []
        for i in range(n.value):
            c = buf[i]
            self._keep.pop(c.ticket, None)
            out.append((c.ticket, c.status, c.submit_s, c.admit_s, c.ready_s, c.done_s))
        return out

    def stats(self) -> dict:
        a, b, d, e, f = (ctypes.c_int64() for _ in range(5))
        c = ctypes.c_int32()
        self._check(self._lib.cleora_server_stats(self._h, ctypes.byref(a), ctypes.byref(b),
                                                  ctypes.byref(c), ctypes.byref(d),
                                                  ctypes.byref(e), ctypes.byref(f)))
        return {"steps": a.value, "request_steps": b.value, "max_active_groups": c.value,
                "peak_footprint_bytes": d.value, "groups": e.value, "in_system": f.value}

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.cleora_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_native(jobs: Sequence[Job], dim: int, dtype: str, k: int, slots: int = 64,
               budget_bytes: int = 64 << 30, builders: int = 3, device: int = 0,
               keep_results: bool = False, server: Optional[NativeServer] = None,
               max_group: int = 16) -> List[Job]:
    """Serve ``jobs`` (arrival times in seconds from the start) with the
    native server; results land in device memory.  Job times are relative
    to the start of the trace; latency = result ready - arrival."""
    import numpy as np
    import torch
    jobs = sorted(jobs, key=lambda j: (j.arrival_s, j.index))
    tdt = torch.float32 if dtype in ("f32", "float32") else torch.bfloat16
    dev = torch.device("cuda", device)
    own = server is None
    srv = server or NativeServer(dim, dtype, k, slots, budget_bytes, builders, device,
                                 directed=jobs[0].payload.directed if jobs else False,
                                 max_group=max_group)
    arrays, outs = {}, {}
    for j in jobs:
        g = j.payload
        arrays[j.index] = (np.ascontiguousarray(g.src, np.int32),
                           np.ascontiguousarray(g.dst, np.int32),
                           None if g.w is None else np.ascontiguousarray(g.w, np.float32))
        outs[j.index] = torch.empty((g.n, dim), dtype=tdt, device=dev)
    torch.cuda.synchronize()
    by_ticket, done = {}, []
    try:
        s0 = srv.stats()
        t0 = srv.now()

        def drain(wait):
            for ticket, status, _s, a, r, d in srv.poll(256, wait):
                j = by_ticket.pop(ticket)
                if status != 0:
                    raise RuntimeError(f"request {j.index} failed with status {status}")
                j.admitted_s, j.ready_s, j.done_s = a - t0, r - t0, d - t0
                j.iteration = k
                if keep_results:
                    j.result = outs[j.index]
                done.append(j)

        for j in jobs:
            while srv.now() - t0 < j.arrival_s:
                drain(0.0)
                lag = j.arrival_s - (srv.now() - t0)
                if lag > 0.0002:
                    time.sleep(min(lag - 0.0001, 0.002))
            src, dst, w = arrays[j.index]
            by_ticket[srv.submit(j.payload.n, src, dst, w, j.seed, outs[j.index])] = j
        while by_ticket:
            drain(0.05)
        # counters of this run (a long-lived server accumulates them); the
        # maxima are over the server's life
        st = srv.stats()
        for key in ("steps", "request_steps", "groups"):
            st[key] -= s0[key]
        run_native.last_stats = st
    finally:
        if own:
            srv.close()
    return done
