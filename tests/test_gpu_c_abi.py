"""The C ABI from a plain C program (gcc; no Python or torch in the
process): a small graph embedded through include/cleora.h matches the FP64
oracle, the column-blocked form of the same embedding agrees with it, and
an edge id out of range comes back as CLEORA_E_INPUT with a message."""

import os
import subprocess
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "c_abi"))


def c_graph(n):
    src, dst = [], []
    for i in range(n):
        for b in ((i + 1) % n, (7 * i + 3) % n):
            if b != i:
                src.append(i)
                dst.append(b)
    return gen.Graph(n, np.array(src, np.int32), np.array(dst, np.int32), None, False, "c_abi")


def test_c_program_matches_oracle():
    import build_smoke
    exe = build_smoke.build()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.strip().splitlines()
    n, d = map(int, lines[0].split())
    got = np.array([[float(x) for x in ln.split()] for ln in lines[1:1 + n]])
    assert got.shape == (n, d)
    want = oracle.embed(c_graph(n), d, 3, 42)
    err = float(np.abs(got - want).max())
    print(f"C program: max-abs {err:.3e}")
    assert err <= 1e-5
    tag, diff = lines[1 + n].split()
    assert tag == "blocked_maxdiff" and float(diff) <= 2e-6
    _, code, msg = lines[-1].split(" ", 2)
    assert int(code) == 5 and "outside" in msg
