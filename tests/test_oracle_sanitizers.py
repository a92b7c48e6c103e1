"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host only): every entry point runs on small graphs with loops,
repeated pairs, weights, directed edges, empty rows, chunks and hyperedges,
and the sanitizers must report nothing."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cleora_oracle.c")

SCRIPT = r"""
import numpy as np
import gen, oracle
for seed, directed in ((1, True), (2, False), (3, True)):
    g = gen.random_graph(150, 900, seed, directed=directed, weighted=True, loops=True,
                         multi=True)
    for flags in (0, oracle.EMPTY_KEEP):
        T = oracle.embed(g, 7, 3, seed, flags)
        assert np.isfinite(T).all()
    rows = np.array([0, 5, 149, 77], np.int32)
    oracle.t1_rows(g, rows, 7, seed)
    adj = oracle.adjacency_rows(g, rows)
    assert adj.n == rows.size
g = gen.random_graph(120, 700, 4, weighted=True)
chunks = np.array_split(np.random.default_rng(0).permutation(g.m), 3)
oracle.embed_chunked(g, chunks, 5, 2, 9)
off = np.array([0, 3, 3, 7, 8], np.int64)
mem = np.array([1, 2, 3, 0, 4, 4, 5, 6], np.int32)
oracle.expand_clique(off, mem)
oracle.expand_star(10, off, mem)
oracle.init_ids(5, np.array([0, 9, 3], np.int32), 6)
oracle.uniform(1, 2, 3, 4)
empty = gen.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), None, False)
oracle.embed(empty, 4, 2, 1)
print("sanitized ok")
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fPIC",
                           "-shared", "-std=c11", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-o", lib, SRC, "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "sanitized ok" in r.stdout
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
