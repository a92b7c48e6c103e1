"""Host logic of bench.py (no GPU): profile summaries, the graph cache and
the one-GPU guard."""

import csv
import json
import os
import subprocess
import sys

import numpy as np

import bench
import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_csv(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_trace_uses_the_last_dispatches(tmp_path):
    # autotuner trials (slow) first, then the timed launches (2 ms each)
    rows, t = [], 0
    for i, dur_us in enumerate([5000] * 6 + [2000] * 4):
        rows.append({"Kernel_Name": "void k_spmm_norm<float, 1, 1, 8>(...)",
                     "Start_Timestamp": t, "End_Timestamp": t + dur_us * 1000})
        t += dur_us * 1000 + 10
        rows.append({"Kernel_Name": "k_other", "Start_Timestamp": t,
                     "End_Timestamp": t + 1000})
        t += 2000
    write_csv(str(tmp_path / "run" / "t_kernel_trace.csv"),
              ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = tmp_path / "summary.txt"
    bench.summarize_trace(str(tmp_path / "run"), str(out), 4, "the command")
    text = out.read_text()
    assert "# command: the command" in text
    assert "last 4 dispatches (the timed steps): avg 2.0000 ms" in text
    # the whole-run table counts every dispatch
    line = [ln for ln in text.splitlines() if "k_spmm_norm<float" in ln and "avg" not in ln][0]
    assert line.split()[0] == "10" and abs(float(line.split()[1]) - 3.8) < 1e-9


def test_summarize_pmc_scales_by_the_copy(tmp_path):
    # FETCH_SIZE reads half of the copy's true bytes, WRITE_SIZE all of them
    copy_bytes = 1 << 30
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    fetch = [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer",
              "Counter_Name": "FETCH_SIZE", "Counter_Value": copy_bytes / 2 / 1024}]
    write = [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer",
              "Counter_Name": "WRITE_SIZE", "Counter_Value": copy_bytes / 1024}]
    for d, (f_kib, w_kib) in enumerate([(999.0, 999.0), (100.0, 10.0), (300.0, 30.0)], 2):
        fetch.append({"Dispatch_Id": d, "Kernel_Name": "k_spmm_norm<float>",
                      "Counter_Name": "FETCH_SIZE", "Counter_Value": f_kib})
        write.append({"Dispatch_Id": d, "Kernel_Name": "k_spmm_norm<float>",
                      "Counter_Name": "WRITE_SIZE", "Counter_Value": w_kib})
    write_csv(str(tmp_path / "f" / "p_counter_collection.csv"), fields, fetch)
    write_csv(str(tmp_path / "w" / "p_counter_collection.csv"), fields, write)
    out = tmp_path / "pmc.json"
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(out), "cmd", copy_bytes, 2)
    r = json.loads(out.read_text())
    assert r["fetch_launches"] == 2 and r["write_launches"] == 2
    assert abs(r["fetch_scale"] - 2.0) < 1e-12 and abs(r["write_scale"] - 1.0) < 1e-12
    assert abs(r["fetch_bytes_per_launch"] - 200.0 * 1024 * 2) < 1e-6
    assert abs(r["write_bytes_per_launch"] - 20.0 * 1024) < 1e-6
    assert r["hbm_bytes_per_launch"] == r["fetch_bytes_per_launch"] + r["write_bytes_per_launch"]


def test_graph_cache_round_trip(tmp_path):
    for name, make in (("er", lambda: gen.erdos_renyi(500, 2000, 3)),
                       ("bip", lambda: gen.bipartite_zipf(300, 50, 3000, 1.1, 4)),
                       ("dir", lambda: gen.random_graph(200, 800, 5, directed=True))):
        spec = {"make": make}
        a = bench._cached_graph(str(tmp_path), name, spec)
        assert (tmp_path / f"{name}.npz").exists()
        b = bench._cached_graph(str(tmp_path), name, spec)
        assert a.n == b.n and a.directed == b.directed
        assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
        assert (a.w is None and b.w is None) or np.array_equal(a.w, b.w)
        assert b.src.dtype == np.int32 and (b.w is None or b.w.dtype == np.float32)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_cpu_baseline_on_a_small_graph():
    g = gen.erdos_renyi(2000, 8000, 6)
    r = bench._cpu_baseline(g, 16, 2)
    assert r["kind"] == "oracle" and r["unit"] == "GEdge-dims/s" and r["value"] > 0
    assert r["cores"] >= 1 and r["single_thread"]["value"] > 0


def test_traffic_only_while_the_kernel_source_matches(tmp_path, monkeypatch):
    # the committed counter summaries are of the current SpMM source
    for dt in ("f32", "bf16"):
        t = bench._traffic("chunglu1m", dt)
        assert t is not None and t > 0, dt
    # a summary of another source is not used
    stale = tmp_path / "spmm_norm_chunglu1m_f32_pmc.json"
    stale.write_text(json.dumps({"kernel_source_sha256_16": "0" * 16,
                                 "hbm_bytes_per_launch": 1.0}))
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(tmp_path / "spmm_norm_{workload}_{dtype}_pmc.json"))
    assert bench._traffic("chunglu1m", "f32") is None
    stale.write_text(json.dumps({"kernel_source_sha256_16": bench.kernel_source_hash(),
                                 "hbm_bytes_per_launch": 5.0}))
    assert bench._traffic("chunglu1m", "f32") == 5.0
    assert bench._traffic("chunglu10m", "f32") is None  # no summary for that workload
    # sliced iterations use the summary of their own slicing (per slice launch)
    sliced = tmp_path / "spmm_norm_chunglu1m_f32_slices128_pmc.json"
    sliced.write_text(json.dumps({"kernel_source_sha256_16": bench.kernel_source_hash(),
                                  "hbm_bytes_per_launch": 7.0}))
    assert bench._traffic("chunglu1m", "f32", 128) == 7.0
    assert bench._traffic("chunglu1m", "f32", 256) is None
    assert bench._traffic("chunglu1m", "f32", 0) == 5.0


def test_committed_sliced_counter_summaries():
    # the slicings the autotuner may keep at the 10M-node workload have
    # counter summaries of the current source
    for dt, widths in (("f32", (128, 256)), ("bf16", (256, 512))):
        for w in widths:
            t = bench._traffic("chunglu10m", dt, w)
            assert t is not None and t > 0, (dt, w)


def test_every_trace_summary_is_of_the_current_source():
    # profiles/ holds one source's figures: each summary names the hash
    prof = os.path.join(ROOT, "profiles")
    h = bench.kernel_source_hash()
    for name in sorted(os.listdir(prof)):
        text = open(os.path.join(prof, name)).read()
        if name.endswith("_trace.txt") or name.endswith(".json"):
            assert h in text, name


def test_served_cpu_baseline_on_a_small_stream():
    trace = gen.served_trace(6, 1.0, seed=3, n_hi=400)
    graphs = gen.materialize(trace)
    r = bench._served_cpu_baseline(trace, graphs, 16, 2, n_sample=4)
    assert r["kind"] == "oracle" and r["unit"] == "req/s" and r["value"] > 0
    assert r["cores"] >= 1 and r["sample"].startswith("4 random requests")
