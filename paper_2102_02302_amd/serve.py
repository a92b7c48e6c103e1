"""Served form: continuous batching of independent embedding requests.

Each request is a whole graph to embed (T_k of Algorithm 1 for its own
graph and seed).  Serving is the library's native server
(``cleora_server_*``, wrapped by ``NativeServer``): requests are admitted
in arrival order as groups built together as one block-diagonal graph,
while a slot is free and the device memory charged to the slots stays
within a budget; built groups advance one iteration per step in shared
launches and retire after k iterations.  Its admission and grouping policy
is host-only C++ (``csrc/admission.hpp``), unit-tested on the CPU.

This module drives that server over a request trace (``run_native``),
serves the same trace one request at a time with the plain path as the
baseline (``one_at_a_time``), and summarises latencies (``latency_stats``).
"""

from __future__ import annotations

import ctypes
import dataclasses
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
    """The C++ request server of the library (``cleora_server_*``): native
    builder and scheduler threads, admission by charged device memory."""

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
                "peak_charged_bytes": d.value, "groups": e.value, "in_system": f.value}

    def memory(self) -> dict:
        """Budget, bytes charged now and at most, and builds whose slot held
        more than it was charged (0 when every footprint bounded its build)."""
        a, b, c, d = (ctypes.c_int64() for _ in range(4))
        self._check(self._lib.cleora_server_memory(self._h, ctypes.byref(a), ctypes.byref(b),
                                                   ctypes.byref(c), ctypes.byref(d)))
        return {"budget_bytes": a.value, "charged_bytes": b.value, "peak_charged_bytes": c.value,
                "bound_exceeded": d.value}

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
