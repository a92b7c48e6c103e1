"""Benchmark of the Cleora propagation hot path on one MI355X.

One step = the whole path on one synthetic graph whose edge list is already
in HBM: build M = D^-1 A (CSR, FP64 row sums), initialise T_0, run k
iterations of multiply + row L2 normalisation.  Throughput is edge-dims per
second: k * nnz * d / step time (nnz = stored entries of M).

Prints one JSON line.  The roofline object describes the fused SpMM +
normalise kernel (HBM-bound): its algorithmic bytes per launch

    nnz * (4 + 4)                  column index + M value per entry
  + nnz * d * s                    one gathered row of T per entry
  + (N - n_split_rows) * d * s     one written row of T per row it finishes

divided by its average launch time, measured with HIP events on the launch
stream during the timed steps.  That model counts every gathered row as
read from memory; hub rows that hit in L2 or the Infinity Cache make its
rate exceed what HBM delivers on graphs whose T fits in those caches'
reach, so two more figures stand beside it: ``compulsory_frac`` (each row
of T read once, the floor of any schedule) and, from the committed
rocprofv3 counter summary when it was taken on the current kernel source,
``traffic`` (measured DRAM-side bytes per launch) with
``hbm_measured_frac``, the fraction of HBM peak the kernel really moves.

Default workload: the largest single-GPU configuration (Chung-Lu
gamma = 2.2, N = 10M, 400M stored entries, d = 1024, k = 5) in FP32, with
BF16 storage measured beside it on the same graph.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GEdge-dims/s per iteration (nnz·d/s) + % HBM peak; p50/p99 served latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2102_02302_amd", "csrc", "propagate.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "spmm_norm_{workload}_{dtype}_pmc.json")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


SPMM = "k_spmm_norm"


def summarize_trace(trace_dir: str, out: str, last: int, command: str) -> None:
    """Per-kernel summary (calls, average and total duration) of a
    rocprofv3 --kernel-trace --output-format csv run, as a short text file,
    plus the SpMM kernel over its last `last` dispatches only: the timed
    steps, after the autotuner's trial launches (0: every dispatch)."""
    import csv
    import glob
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {trace_dir}")
    agg, spmm = {}, []
    for f in files:
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"]
            t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            dur = (t1 - t0) / 1e6
            a = agg.setdefault(name, [0, 0.0])
            a[0] += 1
            a[1] += dur
            if SPMM in name:
                spmm.append((t0, dur))
    rows = sorted(agg.items(), key=lambda kv: -kv[1][1])
    spmm.sort()
    tail = spmm[-last:] if last > 0 else spmm
    with open(out, "w") as f:
        f.write(f"# rocprofv3 kernel trace summary\n# command: {command}\n")
        f.write(f"# kernel source sha256[:16]: {kernel_source_hash()}\n")
        if tail:
            f.write(f"# {SPMM}, last {len(tail)} dispatches (the timed steps): "
                    f"avg {sum(d for _, d in tail) / len(tail):.4f} ms, "
                    f"min {min(d for _, d in tail):.4f}, max {max(d for _, d in tail):.4f}\n")
        f.write("# all dispatches (autotuner trials and warm-up included):\n")
        f.write(f"{'calls':>6} {'avg_ms':>10} {'total_ms':>10}  kernel\n")
        for name, (n, tot) in rows:
            f.write(f"{n:6d} {tot / n:10.4f} {tot:10.3f}  {name[:150]}\n")


def summarize_counters(pmc_dir: str, out: str, last: int, command: str) -> None:
    """Per-dispatch averages of every counter of a rocprofv3 --pmc run over
    the SpMM kernel's last `last` dispatches (the timed steps)."""
    import csv
    import glob
    files = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {pmc_dir}")
    per = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if SPMM in r["Kernel_Name"]:
                per.setdefault(r["Counter_Name"], []).append(
                    (int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    res = {"command": command, "kernel_source_sha256_16": kernel_source_hash(), "counters": {}}
    for name, vals in sorted(per.items()):
        vals.sort()
        v = [x for _, x in vals][-last:] if last > 0 else [x for _, x in vals]
        res["counters"][name] = {"per_dispatch": sum(v) / len(v), "dispatches": len(v)}
    c = {k: v["per_dispatch"] for k, v in res["counters"].items()}
    if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
        res["l2_hit_rate"] = c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"])
    if "TCC_EA0_RDREQ_sum" in c and "TCC_EA0_RDREQ_DRAM_sum" in c:
        res["dram_share_of_l2_read_requests"] = c["TCC_EA0_RDREQ_DRAM_sum"] / c["TCC_EA0_RDREQ_sum"]
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


def summarize_markers(trace_dir: str, out: str, command: str) -> None:
    """Per-range summary of a rocprofv3 --marker-trace run: the library's
    named ranges around its entry points, host-side durations."""
    import csv
    import glob
    files = glob.glob(os.path.join(trace_dir, "**", "*marker_api_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no marker_api_trace.csv under {trace_dir}")
    agg = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
            a = agg.setdefault(r["Function"], [0, 0.0, 0.0])
            a[0] += 1
            a[1] += d
            a[2] = max(a[2], d)
    with open(out, "w") as f:
        f.write(f"# rocprofv3 marker (roctx range) summary\n# command: {command}\n")
        f.write("# host time from entering to leaving each entry point: calls that\n"
                "# synchronise (build, init, autotune) include their GPU work and wait for\n"
                "# work queued before them (the previous step's iterations); propagate\n"
                "# only queues its graph launch\n")
        f.write(f"{'calls':>6} {'avg_ms':>10} {'max_ms':>10} {'total_ms':>10}  range\n")
        for name, (n, tot, mx) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            f.write(f"{n:6d} {tot / n:10.4f} {mx:10.4f} {tot:10.3f}  {name}\n")


def summarize_pmc(fetch_dir: str, write_dir: str, out: str, command: str,
                  copy_bytes: int, last: int) -> None:
    """HBM-side traffic per launch of the SpMM kernel from two rocprofv3
    --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by
    what the same counter reads for a plain device copy of copy_bytes.
    Only the SpMM kernel's last `last` dispatches count (the timed steps;
    0: every dispatch)."""
    import csv
    import glob

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        rows = [r for fn in f for r in csv.DictReader(open(fn)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    res = {"command": command, "kernel_source_sha256_16": kernel_source_hash()}
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = load(d, counter)
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        ref = max(copies) * 1024.0  # the calibration copy is the largest copy
        scale = copy_bytes / ref
        spmm = [float(r["Counter_Value"]) for r in rows if SPMM in r["Kernel_Name"]]
        if last > 0:
            spmm = spmm[-last:]
        res[f"{tag}_kib_per_launch_raw"] = sum(spmm) / len(spmm)
        res[f"{tag}_copy_kib_raw"] = ref / 1024.0
        res[f"{tag}_scale"] = scale
        res[f"{tag}_bytes_per_launch"] = sum(spmm) / len(spmm) * 1024.0 * scale
        res[f"{tag}_launches"] = len(spmm)
    res["hbm_bytes_per_launch"] = res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


def served_main(args, trace=None, graphs=None) -> dict:
    """Served stream: Poisson arrivals of independent Chung-Lu requests
    (N log-uniform in [100, 200k], mean degree U(5, 30), d = 128, k = 4).
    1. capacity of the continuous-batching server (the library's native
       server, BF16, co-admitted requests built together as one
       block-diagonal graph): every request submitted at t = 0;
    2. the same requests arriving as a Poisson process at `load` x that
       capacity, served with continuous batching;
    3. the same arrivals served one request at a time by the plain FP32
       path.  Results land in device memory in every case; latency is
       arrival -> result ready."""
    import gen
    from paper_2102_02302_amd.serve import Job, NativeServer, run_native

    dim, k = 128, 4
    if trace is None:
        trace, graphs = served_inputs(args.requests)

    def jobs(scale):
        return [Job(index=r.index, arrival_s=r.arrival_s * scale, n=g.n, m=g.m, seed=r.seed,
                    payload=g) for r, g in zip(trace, graphs)]

    nnz = {r.index: (g.m if g.directed else 2 * g.m) for r, g in zip(trace, graphs)}
    nnz_of = lambda j: nnz[j.index]  # noqa: E731
    servers = {}

    def server(max_group):
        # one long-lived server per grouping, warmed up once with the whole
        # trace at t = 0 so that its slots have grown their buffers, as in
        # steady-state serving
        if max_group not in servers:
            srv = NativeServer(dim, args.served_dtype, k, args.slots, args.budget_gib << 30,
                               args.builders, max_group=max_group)
            run_native(jobs(0.0), dim, args.served_dtype, k, server=srv)
            servers[max_group] = srv
        return servers[max_group]

    try:
        out = _served_runs(args, jobs, nnz_of, graphs, dim, k, server)
    finally:
        for srv in servers.values():
            srv.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _served_cpu_baseline(trace, graphs, dim, k)
    return out


def served_inputs(n_requests: int):
    """The served stream's requests and their graphs (drawn in worker
    processes: call before the GPU is used)."""
    import gen
    t0 = time.time()
    trace = gen.served_trace(n_requests, 1.0)
    graphs = gen.materialize(trace, workers=min(16, os.cpu_count() or 1))
    print(f"[served] generated {len(graphs)} requests in {time.time() - t0:.1f}s", flush=True)
    return trace, graphs


def _served_cpu_baseline(trace, graphs, dim: int, k: int, n_sample: int = 200) -> dict:
    """The FP64 oracle on the host cores over a seeded random sample of the
    stream's requests, one after another, whole path each (adjacency, M,
    T_0, k iterations)."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(2102)
    idx = rng.choice(len(graphs), size=min(n_sample, len(graphs)), replace=False)
    t0 = time.perf_counter()
    edge_dims = 0
    for i in idx:
        g = graphs[i]
        oracle.embed(g, dim, k, trace[i].seed)
        edge_dims += k * (g.m if g.directed else 2 * g.m) * dim
    dt = time.perf_counter() - t0
    return {"value": round(len(idx) / dt, 2), "unit": "req/s", "cores": oracle.get_threads(),
            "kind": "oracle", "gedge_dims_per_s": round(edge_dims / dt / 1e9, 4),
            "sample": f"{len(idx)} random requests of the stream (seed 2102), whole path each, "
                      f"FP64, {dt:.1f}s (edge-dims counted before repeated pairs merge)"}


def _served_runs(args, jobs, nnz_of, graphs, dim, k, server) -> dict:
    from paper_2102_02302_amd.serve import latency_stats, one_at_a_time, run_native
    opts = dict(server=server(args.max_group))
    cap = latency_stats(run_native(jobs(0.0), dim, args.served_dtype, k, **opts), k, dim, nnz_of)
    cap.update(run_native.last_stats)
    rate = args.load * cap["req_per_s"]
    print(f"[served] capacity {cap['req_per_s']} req/s; offered {rate:.1f} req/s", flush=True)
    batched = latency_stats(run_native(jobs(1.0 / rate), dim, args.served_dtype, k, **opts),
                            k, dim, nnz_of)
    batched.update(run_native.last_stats)
    batched["dtype"] = args.served_dtype
    base = latency_stats(one_at_a_time(jobs(1.0 / rate), dim, k, "f32", result_on_device=True),
                         k, dim, nnz_of)
    base["dtype"] = "f32"
    other_loads = []
    for ld in [float(x) for x in args.loads.split(",") if x]:
        r = ld * cap["req_per_s"]
        st = latency_stats(run_native(jobs(1.0 / r), dim, args.served_dtype, k, **opts),
                           k, dim, nnz_of)
        row = {"load": ld, "offered_req_per_s": round(r, 2),
               "continuous_batching": {key: st[key] for key in ("p50_ms", "p99_ms", "req_per_s")}}
        st = latency_stats(one_at_a_time(jobs(1.0 / r), dim, k, "f32", result_on_device=True),
                           k, dim, nnz_of)
        row["one_at_a_time_f32"] = {key: st[key] for key in ("p50_ms", "p99_ms", "req_per_s")}
        print(f"[served] load {ld}: {row}", flush=True)
        other_loads.append(row)
    sweep = []
    for r in [float(x) for x in args.rates.split(",") if x]:
        row = {"offered_req_per_s": r}
        for g in sorted({1, args.max_group}):
            st = latency_stats(run_native(jobs(1.0 / r), dim, args.served_dtype, k,
                                          server=server(g)), k, dim, nnz_of)
            row[f"group{g}"] = {key: st[key] for key in ("p50_ms", "p99_ms", "req_per_s")}
            row[f"group{g}"]["groups"] = run_native.last_stats["groups"]
        st = latency_stats(one_at_a_time(jobs(1.0 / r), dim, k, "f32", result_on_device=True),
                           k, dim, nnz_of)
        row["one_at_a_time_f32"] = {key: st[key] for key in ("p50_ms", "p99_ms", "req_per_s")}
        print(f"[served] rate {r}: {row}", flush=True)
        sweep.append(row)
    out = {"requests": len(graphs), "dim": dim, "k": k, "offered_req_per_s": round(rate, 2),
           "load": args.load, "slots": args.slots, "builders": args.builders,
           "max_group": args.max_group,
           "saturated_capacity": cap, "continuous_batching": batched,
           "one_at_a_time_f32": base}
    if other_loads:
        out["other_loads"] = other_loads
    if sweep:
        out["rate_sweep"] = sweep
    return out


def blocked_main(args) -> dict:
    """Column-blocked form (cleora_embed_blocked): the workload's T_k computed
    ``--blocked`` columns at a time, against init + propagate on the same
    graph (both after one CSR build, which is not timed).  The blocked form
    runs k(k+1)/2 + k block iterations for k of the whole width; its device
    buffers are two N x block embeddings instead of two N x d."""
    import torch

    import gen
    import paper_2102_02302_amd as cl

    spec = gen.WORKLOADS[args.workload]
    dim, block = spec["dim"], args.blocked
    k = args.k if args.k is not None else spec["k"]
    dtype = args.dtype or spec["dtype"]
    g = _cached_graph(args.graph_cache, args.workload, spec)
    print(f"[blocked] {args.workload}: n={g.n} m={g.m} d={dim} block={block} k={k}", flush=True)
    dev = torch.device("cuda", 0)
    src = torch.as_tensor(g.src).to(dev)
    dst = torch.as_tensor(g.dst).to(dev)
    w = torch.as_tensor(g.w).to(dev) if g.w is not None else None
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    ctx = cl.Context(0)
    ctx.build_csr(g.n, src, dst, w, directed=g.directed)
    nnz = ctx.info()["nnz"]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps

    def plain():
        ctx.init(dim, dtype, 2102)
        ctx.propagate(k)

    out_dev = torch.empty((g.n, dim), dtype=tdt, device=dev)
    out_host = torch.empty((g.n, dim), dtype=tdt, pin_memory=True)
    plain_ms = timed(plain)
    print(f"[blocked] init + propagate: {plain_ms:.3f} ms", flush=True)
    ref = ctx.embedding()
    dev_ms = timed(lambda: ctx.embed_blocked(dim, block, k, dtype, 2102, out=out_dev))
    print(f"[blocked] blocked, device output: {dev_ms:.3f} ms", flush=True)
    host_ms = timed(lambda: ctx.embed_blocked(dim, block, k, dtype, 2102, out=out_host))
    print(f"[blocked] blocked, pinned host output: {host_ms:.3f} ms", flush=True)
    diff = float((out_dev.float() - ref.float()).abs().max())
    same_host = bool(torch.equal(out_host, out_dev.cpu()))
    ctx.close()
    esz = 2 if dtype == "bf16" else 4
    ld_b = -(-min(block, dim) * esz // 16) * 16 // esz
    ld = -(-dim * esz // 16) * 16 // esz
    n_blocks = -(-dim // block)
    return {"workload": args.workload, "n_nodes": g.n, "nnz": nnz, "dim": dim, "block": block,
            "blocks": n_blocks, "k": k, "dtype": dtype,
            "plain_ms": round(plain_ms, 3), "blocked_ms": round(dev_ms, 3),
            "blocked_host_out_ms": round(host_ms, 3),
            "slowdown": round(dev_ms / plain_ms, 3),
            "block_iterations_ratio": (k * (k + 1) // 2 + k) / k,
            "embedding_buffers_bytes": {"plain": 2 * g.n * ld * esz,
                                        "blocked": 2 * g.n * ld_b * esz},
            "max_abs_vs_plain": diff, "host_output_same_bits": same_host}


def batched_main(args, trace=None, graphs=None) -> dict:
    """Batched form: many independent graphs of uneven size (shapes of the
    served stream: Chung-Lu, N log-uniform in [100, 200k], mean degree
    U(5, 30); d = 128, k = 4), edge lists already on the device.
    1. plain FP32 path, one graph after another (build and T_0, k
       iterations);
    2. one cleora_embed_batch call (one block-diagonal build, k iterations
       over all graphs, results copied to one tensor per graph), FP32;
    3. the same in BF16."""
    import torch

    import gen
    import paper_2102_02302_amd as cl

    dim, k = 128, 4
    if trace is None:
        t0 = time.time()
        trace = gen.served_trace(args.batch, 1.0)
        graphs = gen.materialize(trace, workers=min(16, os.cpu_count() or 1))
        print(f"[batched] generated {len(graphs)} graphs in {time.time() - t0:.1f}s", flush=True)
    dev = torch.device("cuda", 0)
    dgraphs = [gen.Graph(g.n, torch.as_tensor(g.src).to(dev), torch.as_tensor(g.dst).to(dev),
                         None, g.directed) for g in graphs]
    seeds = [r.seed for r in trace]
    nnz = sum(2 * g.m for g in graphs)
    edge_dims = float(k) * nnz * dim
    torch.cuda.synchronize()
    ctx = cl.Context(0)

    def plain():
        for g, sd in zip(dgraphs, seeds):
            ctx.build_init(g.n, g.src, g.dst, None, dim, "f32", sd)
            ctx.propagate(k)

    def batched(dtype):
        return lambda: cl.embed_batch(ctx, dgraphs, dim, k, seeds, dtype)

    def timed(fn, reps):
        fn()  # warm-up (buffers grow, kernels load)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - ta) / reps

    res = {}
    for name, fn in (("one_at_a_time_f32", plain), ("embed_batch_f32", batched("f32")),
                     ("embed_batch_bf16", batched("bf16"))):
        sec = timed(fn, args.steps)
        res[name] = {"ms": round(sec * 1e3, 3), "graphs_per_s": round(len(graphs) / sec, 1),
                     "gedge_dims_per_s": round(edge_dims / sec / 1e9, 2)}
        print(f"[batched] {name}: {res[name]}", flush=True)
    ctx.close()
    base = res["one_at_a_time_f32"]["ms"]
    out = {"graphs": len(graphs), "nodes": sum(g.n for g in graphs), "nnz": nnz, "dim": dim,
           "k": k, "results": res,
           "speedup_vs_one_at_a_time_f32": {n: round(base / r["ms"], 2) for n, r in res.items()}}
    if not args.no_cpu_baseline:
        # the oracle over a seeded sample of the batch's graphs, in graphs/s
        cb = _served_cpu_baseline(trace, graphs, dim, k, n_sample=100)
        cb["unit"] = "graphs/s"
        cb["sample"] = cb["sample"].replace("requests of the stream", "graphs of the batch")
        out["cpu_baseline"] = cb
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chunglu10m",
                    help="er10k | chunglu1m | chunglu10m | bipartite6m")
    ap.add_argument("--dtype", default=None, help="override the workload's dtype (f32|bf16)")
    ap.add_argument("--also-dtype", default=None,
                    help="storage type measured beside the headline (default: the other of "
                         "f32/bf16; '' for none)")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--dim", type=int, default=None,
                    help="override the workload's d (e.g. one GPU's share of the columns)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--slices", default="auto",
                    help="column slices of each iteration: 'auto' (the autotuner times whole "
                         "rows against 512-byte slices on this process's buffers and keeps "
                         "the faster; whole rows with --no-autotune), 0 whole rows, or a "
                         "width in columns")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the library's schedule autotuner (run once per graph "
                         "shape, before the timed steps)")
    ap.add_argument("--served", action="store_true",
                    help="run the served-stream benchmark instead (p50/p99 latency)")
    ap.add_argument("--batched", action="store_true",
                    help="run the batched-form benchmark instead (many graphs per call)")
    ap.add_argument("--batch", type=int, default=512, help="graphs in the batched benchmark")
    ap.add_argument("--blocked", type=int, default=0,
                    help="run the column-blocked form instead, this many columns per block")
    ap.add_argument("--requests", type=int, default=10_000)
    ap.add_argument("--served-requests", type=int, default=2000,
                    help="requests of the reduced served stream reported beside the default "
                         "line (0: none)")
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gib", type=int, default=64)
    ap.add_argument("--builders", type=int, default=3,
                    help="server build threads (3: with the stepping stream, one per hardware "
                         "queue of the process)")
    ap.add_argument("--max-group", type=int, default=16,
                    help="most requests the server builds together as one block-diagonal graph")
    ap.add_argument("--served-dtype", default="bf16")
    ap.add_argument("--loads", default="0.5,0.9",
                    help="further offered loads (multiples of the measured capacity) to report "
                         "beside --load")
    ap.add_argument("--rates", default="",
                    help="comma-separated offered rates (req/s): latency at each, grouped and "
                         "ungrouped, beside one-at-a-time FP32")
    ap.add_argument("--graph-cache", default="",
                    help="directory to keep drawn workload graphs in (reused by later runs)")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="launch one plain device copy of this many GiB first "
                         "(reference kernel for HBM counter scaling)")
    return ap.parse_args()


def main():
    # summarize-trace TRACE_DIR OUT LAST COMMAND...
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-trace":
        summarize_trace(sys.argv[2], sys.argv[3], int(sys.argv[4]), " ".join(sys.argv[5:]))
        return
    # summarize-counters PMC_DIR OUT LAST COMMAND...
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-counters":
        summarize_counters(sys.argv[2], sys.argv[3], int(sys.argv[4]), " ".join(sys.argv[5:]))
        return
    # summarize-markers TRACE_DIR OUT COMMAND...
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-markers":
        summarize_markers(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
        return
    # summarize-pmc FETCH_DIR WRITE_DIR OUT COPY_BYTES LAST COMMAND...
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-pmc":
        summarize_pmc(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[7:]),
                      int(sys.argv[5]), int(sys.argv[6]))
        return
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1 "
                                   "(the multi-GPU column split is a design, not code)"}))
        sys.exit(2)

    if args.batched:
        res = batched_main(args)
        b = res["results"]["embed_batch_bf16"]
        print(json.dumps({"metric": "batched throughput (many graphs, one block-diagonal build)",
                          "value": b["gedge_dims_per_s"], "unit": "GEdge-dims/s",
                          "higher_is_better": True, "n_gpus": 1, "steps": args.steps,
                          "dtype": "bf16", "data": "synthetic",
                          "config": {"workload": "batch of Chung-Lu graphs",
                                     "graphs": res["graphs"]},
                          "cpu_baseline": res.pop("cpu_baseline", None),
                          "batched": res}), flush=True)
        return
    if args.blocked:
        res = blocked_main(args)
        print(json.dumps({"metric": "column-blocked T_k (useful nnz·d·k per second)",
                          "value": round(res["k"] * res["nnz"] * res["dim"]
                                         / (res["blocked_ms"] * 1e-3) / 1e9, 3),
                          "unit": "GEdge-dims/s", "higher_is_better": True, "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": res["blocked_ms"], "dtype": res["dtype"],
                          "data": "synthetic",
                          "config": {"workload": args.workload, "block": args.blocked},
                          "blocked": res}), flush=True)
        return
    if args.served:
        res = served_main(args)
        b = res["continuous_batching"]
        print(json.dumps({"metric": "served latency p50/p99 (continuous batching)",
                          "value": b["p50_ms"], "unit": "ms", "higher_is_better": False,
                          "p99_ms": b["p99_ms"], "n_gpus": 1, "dtype": args.served_dtype,
                          "data": "synthetic", "config": {"workload": "served Chung-Lu stream"},
                          "cpu_baseline": res.pop("cpu_baseline", None),
                          "served": res}), flush=True)
        return

    import torch

    import gen
    import paper_2102_02302_amd as cl

    spec = gen.WORKLOADS[args.workload]
    dim = args.dim or spec["dim"]
    k = args.k if args.k is not None else spec["k"]
    dtype = args.dtype or spec["dtype"]

    t0 = time.time()
    g = _cached_graph(args.graph_cache, args.workload, spec)
    gen_s = time.time() - t0
    print(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {gen_s:.1f}s", flush=True)
    served_in = served_inputs(args.served_requests) if args.served_requests > 0 else None

    dev = torch.device("cuda", 0)
    if args.calibrate_copy_gib > 0:
        nb = int(args.calibrate_copy_gib * (1 << 30)) // 4
        a = torch.ones(nb, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    src = torch.as_tensor(g.src).to(dev)
    dst = torch.as_tensor(g.dst).to(dev)
    w = torch.as_tensor(g.w).to(dev) if g.w is not None else None
    torch.cuda.synchronize()

    ctx = cl.Context(0)
    if args.chunk:
        ctx.set_chunk(args.chunk)
    if args.slices == "auto":
        ctx.set_slices("auto")
    elif int(args.slices):
        ctx.set_slices(int(args.slices))

    main_run = _measure(ctx, g, src, dst, w, dim, k, dtype, args.steps, args.warmup,
                        not args.no_autotune, args.workload,
                        traffic_ok=dim == spec["dim"])
    n, nnz = main_run["n"], main_run["nnz"]
    out = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "GEdge-dims/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "desc": spec["desc"], "n_nodes": n,
                   "n_edges": g.m, "nnz": nnz, "dim": dim, "k": k,
                   "step": "build CSR + FP64 row sums + init T_0 + k iterations",
                   "column_slices": main_run["n_slices"], "slice_mode": str(args.slices),
                   "parallelism": "single GPU"},
        "propagate_only": main_run["propagate_only"],
        "phases_ms": main_run["phases_ms"],
        "launch_path": main_run["launch_path"],
        "roofline": main_run["roofline"],
    }
    # the other storage type beside the headline (same graph, same GPU)
    other = args.also_dtype if args.also_dtype is not None else (
        "bf16" if dtype == "f32" else "f32")
    if other and other != dtype and args.steps > 0:
        o_steps = max(3, args.steps // 2)
        o = _measure(ctx, g, src, dst, w, dim, k, other, o_steps, max(1, args.warmup // 2),
                     not args.no_autotune, args.workload,
                     traffic_ok=dim == spec["dim"])
        out[other] = {"value": o["value"], "unit": "GEdge-dims/s", "steps": o_steps,
                      "ms_per_step": o["ms_per_step"],
                      "speedup_vs_" + dtype: round(o["value"] / main_run["value"], 3),
                      "column_slices": o["n_slices"],
                      "propagate_only": o["propagate_only"], "phases_ms": o["phases_ms"],
                      "roofline": o["roofline"]}
    ctx.close()
    del ctx, src, dst, w
    torch.cuda.empty_cache()
    if served_in is not None:
        out["served"] = _served_summary(args, *served_in)
        nb = min(256, len(served_in[1]))
        out["batched"] = _batched_summary(args, served_in[0][:nb], served_in[1][:nb])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(g, dim, k)
    print(json.dumps(out), flush=True)


def _batched_summary(args, trace, graphs) -> dict:
    """The batched form beside the default line: the first requests of the
    served trace as one batch (one cleora_embed_batch call, FP32 and BF16)
    against the plain FP32 path one graph after another."""
    import copy
    a = copy.copy(args)
    a.steps, a.no_cpu_baseline = 3, True
    res = batched_main(a, trace, graphs)
    return {"graphs": res["graphs"], "nodes": res["nodes"], "nnz": res["nnz"], "dim": res["dim"],
            "k": res["k"], "results": res["results"],
            "speedup_vs_one_at_a_time_f32": res["speedup_vs_one_at_a_time_f32"],
            "batch": f"the first {res['graphs']} requests of the served trace, edge lists "
                     f"on the device; 3 timed calls after one warm-up"}


def _served_summary(args, trace, graphs) -> dict:
    """The reduced served stream beside the default line: the native
    server's saturated capacity, then p50/p99 latency and throughput at
    0.7 x that capacity (continuous batching, BF16) against the same
    arrivals served one at a time by the plain FP32 path."""
    import copy
    a = copy.copy(args)
    a.requests, a.loads, a.rates, a.no_cpu_baseline = len(graphs), "", "", True
    res = served_main(a, trace, graphs)
    keys = ("p50_ms", "p99_ms", "req_per_s", "gedge_dims_per_s")
    cb, base = res["continuous_batching"], res["one_at_a_time_f32"]
    return {"requests": res["requests"], "dim": res["dim"], "k": res["k"],
            "saturated_req_per_s": res["saturated_capacity"]["req_per_s"],
            "load": res["load"], "offered_req_per_s": res["offered_req_per_s"],
            "continuous_batching": {"dtype": cb["dtype"], **{x: cb[x] for x in keys}},
            "one_at_a_time_f32": {x: base[x] for x in keys},
            "stream": "Poisson arrivals, Chung-Lu requests (gamma 2.1), N log-uniform in "
                      "[100, 200k], mean degree U(5, 30), seeded; a reduced trace of the "
                      "10,000-request stream of --served"}


def _measure(ctx, g, src, dst, w, dim, k, dtype, steps, warmup, autotune, workload,
             traffic_ok) -> dict:
    """Timed steps of the whole path in one storage type, then the phases
    one by one (untimed by the headline), and the roofline of the SpMM."""
    import torch
    esz = 2 if dtype == "bf16" else 4

    def step():
        # CSR build and T_0 in one call (T_0 written while the CSR is built)
        ctx.build_init(g.n, src, dst, w, dim, dtype, seed=2102, directed=g.directed)
        ctx.propagate(k)

    tuned = None
    if autotune:
        step()
        tuned = ctx.autotune()
        print(f"[bench] {dtype} autotune: {tuned}", flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps: the production launch path (k iterations as one
    # captured graph, reused from step to step), with HIP events on the
    # launch stream around each graph replay
    launches0 = ctx.launch_stats()
    loop_events = []
    t_start = time.perf_counter()
    for _ in range(steps):
        ctx.build_init(g.n, src, dst, w, dim, dtype, seed=2102, directed=g.directed)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.propagate(k)
        b.record()
        loop_events.append((a, b))
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    launches1 = ctx.launch_stats()
    loop_ms = sum(a.elapsed_time(b) for a, b in loop_events) / max(steps, 1)
    # kernel durations: the same steps with every SpMM and combine launch
    # between two HIP events (eager launches of the same kernels and
    # arguments: events inside a graph carry no time)
    kernel_steps = max(2, steps // 4)
    ctx.kernel_time()  # reset
    ctx.set_timing(True)
    for _ in range(kernel_steps):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(False)
    kt = ctx.kernel_time()
    info = ctx.info()
    nnz, n = info["nnz"], info["n"]

    # separate measurement of the phases (not part of the timed steps)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    ctx.build_csr(g.n, src, dst, w, directed=g.directed)
    torch.cuda.synchronize()
    tb2 = time.perf_counter()
    ctx.init(dim, dtype, seed=2102)
    torch.cuda.synchronize()
    tb3 = time.perf_counter()
    ctx.propagate(k)
    torch.cuda.synchronize()
    tb4 = time.perf_counter()
    ctx.build_init(g.n, src, dst, w, dim, dtype, seed=2102, directed=g.directed)
    torch.cuda.synchronize()
    tb5 = time.perf_counter()
    phase = {"build_ms": (tb2 - tb) * 1e3, "init_ms": (tb3 - tb2) * 1e3,
             "propagate_ms": (tb4 - tb3) * 1e3, "build_init_fused_ms": (tb5 - tb4) * 1e3}

    ms_per_step = (t_end - t_start) * 1e3 / max(steps, 1)
    edge_dims = float(k) * nnz * dim
    value = edge_dims / (ms_per_step * 1e-3) / 1e9

    # dominant kernel: fused SpMM + normalise, per launch; with column
    # slices one iteration is S launches, each gathering its slice of the
    # rows and reading every entry's column index and value
    sched = ctx.schedule()
    ld = -(-dim * esz // 16) * 16 // esz
    n_slices = -(-ld // sched["slice_cols"]) if sched["slice_cols"] else 1
    spmm_ms = kt["spmm_ms"] / max(kt["spmm_launches"], 1)
    comb_ms = (kt["combine_ms"] / max(kt["combine_launches"], 1)
               if kt["combine_launches"] else 0.0)
    split_rows = sched["split_rows"]
    spmm_bytes = (n_slices * nnz * 8 + nnz * dim * esz + (n - split_rows) * dim * esz) / n_slices
    # compulsory bytes: every entry's index and value once, every row of
    # T_{t-1} read once and every finished row of T_t written once
    compulsory = (n_slices * nnz * 8 + n * dim * esz + (n - split_rows) * dim * esz) / n_slices
    achieved = spmm_bytes / (spmm_ms * 1e-3) / 1e9
    # the counter summaries are of the workload's own d
    traffic = _traffic(workload, dtype, sched["slice_cols"]) if traffic_ok else None
    # one iteration on the production path: the captured loop's time over k
    iter_ms = loop_ms / max(k, 1)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_spmm_norm" if n_slices == 1 else
                          f"k_spmm_norm, one of {n_slices} column slices of "
                          f"{sched['slice_cols']} per iteration (figures per launch)",
                "bytes_per_launch": int(spmm_bytes),
                "avg_launch_ms": round(spmm_ms, 4), "launches": kt["spmm_launches"],
                "kernel_timing": f"HIP events around each launch over {kernel_steps} steps "
                                 f"after the timed ones",
                "combine_avg_ms": round(comb_ms, 4),
                "graph_iteration_ms": round(loop_ms / max(k, 1), 4),
                "compulsory_bytes_per_launch": int(compulsory),
                "compulsory_frac": round(compulsory / (spmm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "schedule": sched, "autotune": tuned}
    if traffic:
        # measured DRAM-side bytes over the same launch time: the HBM fraction
        roofline["hbm_measured_gbs"] = round(traffic / (spmm_ms * 1e-3) / 1e9, 1)
        roofline["hbm_measured_frac"] = round(traffic / (spmm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    model_it = nnz * 8 + nnz * dim * esz + n * dim * esz
    return {"n": n, "nnz": nnz, "value": round(value, 3), "ms_per_step": round(ms_per_step, 3),
            "n_slices": n_slices,
            "launch_path": {"graph_replays": launches1["graph_launches"] - launches0["graph_launches"],
                            "graph_instantiations": launches1["graph_instantiations"]
                            - launches0["graph_instantiations"],
                            "loop_ms_per_step": round(loop_ms, 4)},
            "propagate_only": {"ms_per_iteration": round(iter_ms, 4),
                               "gedge_dims_per_s": round(nnz * dim / (iter_ms * 1e-3) / 1e9, 2),
                               "model_bytes_per_iteration": int(model_it),
                               "model_bytes_rate_over_hbm_peak": round(
                                   model_it / (iter_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "phases_ms": {kk: round(v, 3) for kk, v in phase.items()},
            "roofline": roofline}


def _traffic(workload: str, dtype: str, slice_cols: int = 0):
    """Measured HBM bytes per SpMM launch from the committed counter summary
    of this workload, storage type and slicing (per slice launch when
    sliced), or None if there is none for the current kernel source."""
    tag = dtype if not slice_cols else f"{dtype}_slices{slice_cols}"
    path = PMC_SUMMARY.format(workload=workload, dtype=tag)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        s = json.load(f)
    if s.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return s.get("hbm_bytes_per_launch")


def _cached_graph(cache_dir: str, name: str, spec: dict):
    """The workload's seeded graph; with a cache directory, drawn once and
    then loaded from DIR/<name>.npz (the draw is deterministic)."""
    import numpy as np

    import gen
    path = os.path.join(cache_dir, f"{name}.npz") if cache_dir else ""
    if path and os.path.exists(path):
        z = np.load(path)
        w = z["w"] if z["w"].size else None
        return gen.Graph(int(z["n"]), z["src"], z["dst"], w, bool(z["directed"]), name)
    gen.graphs.PROGRESS = True  # large graphs take minutes to draw
    try:
        g = spec["make"]()
    finally:
        gen.graphs.PROGRESS = False
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(path, n=g.n, src=g.src, dst=g.dst, directed=g.directed,
                 w=g.w if g.w is not None else np.zeros(0, np.float32))
    return g


def _cpu_baseline(g, dim: int, k: int, budget_s: float = 15.0) -> dict:
    """The FP64 oracle on the host cores.  Small graphs: the same whole path
    (adjacency, M, T_0, k iterations) on the same graph, timed once.  Large
    graphs (the whole path would take hours and two N x d FP64 buffers):
    a bounded sample, the oracle's iteration (multiply + row normalise) over
    a prefix of the rows, repeated for about ``budget_s`` seconds."""
    if float(k) * g.nnz_upper() * dim > 4e11:
        return _cpu_baseline_sampled(g, dim, budget_s)
    import numpy as np

    import oracle
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    adj = oracle.build_graph(g)
    mval, _ = oracle.transition(adj)
    T0 = oracle.init(2102, g.n, dim)
    oracle.propagate(adj, mval, T0, k)
    dt = time.perf_counter() - t0
    # one thread: one iteration over the first N/16 rows (propagation only)
    T1 = np.empty_like(T0)
    r1 = max(1, g.n // 16)
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.step_rows(adj, mval, T0, T1, 0, r1)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    ed1 = int(adj.row_ptr[r1]) * dim
    return {"value": round(k * adj.nnz * dim / dt / 1e9, 4), "unit": "GEdge-dims/s",
            "cores": threads, "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"whole path on the full graph (n={g.n}, nnz={adj.nnz}, d={dim}, k={k}), "
                      f"FP64, {dt:.1f}s",
            "single_thread": {"value": round(ed1 / dt1 / 1e9, 4), "unit": "GEdge-dims/s",
                              "sample": f"one FP64 iteration over rows [0, {r1}), "
                                        f"propagation only, {dt1:.1f}s"}}


def _cpu_baseline_sampled(g, dim: int, budget_s: float) -> dict:
    """The oracle's FP64 iteration over rows [0, N/256) of the graph (node
    ids are a seeded random permutation, so a prefix is a uniform sample of
    rows): their exact adjacency rows, M values and the T_0 rows of every
    neighbour they read, then repeated iterations of those rows, timed.
    The rate (entries x d per second) is the oracle's propagation rate; it
    leaves out the CSR build and T_0, which the whole path also pays."""
    import numpy as np

    import oracle
    threads = oracle.get_threads()
    n_rows = max(1, g.n // 256)
    tp = time.perf_counter()
    sub = oracle.adjacency_rows(g, np.arange(n_rows, dtype=np.int32))
    cols, inv = np.unique(sub.col, return_inverse=True)
    adj = oracle.Adjacency(n_rows, sub.row_ptr, inv.astype(np.int32), sub.aval)
    del sub
    mval, _ = oracle.transition(adj)
    T_in = oracle.init_ids(2102, cols.astype(np.int32), dim)
    T_out = np.empty((n_rows, dim), np.float64)
    prep = time.perf_counter() - tp
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.step_rows(adj, mval, T_in, T_out, 0, n_rows)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    nnz_total = g.nnz_upper()
    return {"value": round(reps * adj.nnz * dim / dt / 1e9, 4), "unit": "GEdge-dims/s",
            "cores": threads, "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"FP64 iterations (multiply + row normalise) of rows [0, {n_rows}) "
                      f"(N/256; ids are randomly permuted, so a uniform row sample), "
                      f"{adj.nnz} entries (~{adj.nnz / nnz_total:.2%} of nnz), reading the "
                      f"T_0 rows of their {cols.size} distinct neighbours; {reps} repetitions "
                      f"in {dt:.1f}s (set-up {prep:.1f}s untimed); rate = entries x d x "
                      f"repetitions / time, propagation only (the whole path adds the "
                      f"build and T_0)"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
