"""Compile embed_smoke.c (plain C, gcc) against include/cleora.h and the
in-tree libcleora.so.  Usage: python tests/c_abi/build_smoke.py"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "embed_smoke.c")
EXE = os.path.join(HERE, "embed_smoke")
LIBDIR = os.path.join(ROOT, "paper_2102_02302_amd")


def build(force: bool = False) -> str:
    lib = os.path.join(LIBDIR, "libcleora.so")
    if (not force and os.path.exists(EXE)
            and os.path.getmtime(EXE) >= max(os.path.getmtime(SRC), os.path.getmtime(lib))):
        return EXE
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), SRC, "-L", LIBDIR, "-lcleora", "-L/opt/rocm/lib",
           "-lamdhip64", "-Wl,-rpath,$ORIGIN/../../paper_2102_02302_amd",
           "-Wl,-rpath,/opt/rocm/lib", "-o", EXE]
    subprocess.check_call(cmd)
    return EXE


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
