"""The native server's admission and grouping policy (csrc/admission.hpp),
host-only C++, unit-tested on the CPU under AddressSanitizer and
UndefinedBehaviorSanitizer: budget edges, the group size limit, arrival
order, the int32 node range of a group, trimming of idle slots, misuse,
and random simulations against a fake engine whose slots hold what exact
buffer growth really holds."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "admission", "admission_test.cpp")
CSRC = os.path.join(ROOT, "paper_2102_02302_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_policy_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "admission_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-I", CSRC, "-o", exe, SRC])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "admission ok" in r.stdout
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
