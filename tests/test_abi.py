"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and its pure functions answer without a GPU."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cleora.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cleora_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2102_02302_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libcleora.so is not built (python -m paper_2102_02302_amd.build)")
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["cleora_build_csr", "cleora_init", "cleora_propagate", "cleora_embed_batch",
                 "cleora_get_embedding", "cleora_step_multi", "cleora_last_error"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2102_02302_amd import _lib
    names = declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(cleora_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)
    assert sorted(_lib.EXPORTS) == names


def test_header_compiles_as_c():
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c",
                        HEADER], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_footprint_is_pure_and_monotone(lib):
    f = lib.cleora_footprint_bytes
    a = f(1_000_000, 20_000_000, 0, 256, 0)
    b = f(1_000_000, 20_000_000, 0, 256, 1)
    c = f(1_000_000, 40_000_000, 0, 256, 0)
    # two N x d float32 buffers at least (Section 4.5 memory model)
    assert a >= 2 * 1_000_000 * 256 * 4
    assert b < a < c
    assert f(0, 10, 0, 256, 0) == 0 and f(10, 10, 0, 0, 0) == 0 and f(10, 10, 0, 8, 7) == 0


def test_error_paths_without_gpu(lib):
    import ctypes
    from paper_2102_02302_amd import _lib
    assert lib.cleora_create(None, 0) == _lib.E_INVAL
    assert b"NULL" in lib.cleora_last_error()
    assert lib.cleora_propagate(None, 1, None) == _lib.E_INVAL
    assert lib.cleora_step_multi(None, -1, None) == _lib.E_INVAL
    lib.cleora_destroy(None)
    h = ctypes.c_void_p()
    # on a machine without a GPU there is no device 0
    import torch
    if not torch.cuda.is_available():
        assert lib.cleora_create(ctypes.byref(h), 0) == _lib.E_DEVICE


def test_more_error_paths_without_gpu(lib):
    """Argument checks that answer before any device work."""
    import ctypes
    from paper_2102_02302_amd import _lib
    null = None
    assert lib.cleora_build_init(null, 10, 0, null, null, null, 0, 16, 0, 1, null) == _lib.E_INVAL
    assert lib.cleora_set_schedule(null, 0, -1) == _lib.E_INVAL
    assert lib.cleora_autotune(null, null, null, null, null) == _lib.E_INVAL
    assert lib.cleora_schedule_info(null, null, null, null, null, null, null, null) == _lib.E_INVAL
    assert lib.cleora_set_chunk(null, 0) == _lib.E_INVAL
    assert lib.cleora_embed_blocked(null, 16, 4, 0, 1, 2, null, 16, null) == _lib.E_INVAL
    assert lib.cleora_release_scratch(null) == _lib.E_INVAL
    assert lib.cleora_set_slices(null, 64) == _lib.E_INVAL
    assert lib.cleora_batch_status(null, 1, null) == _lib.E_INVAL
    # server: null out, and bad parameters, rejected before any context is made
    assert lib.cleora_server_create(null, 0, 16, 0, 2, 2, 1 << 20, 1, 1, 0) == _lib.E_INVAL
    h = ctypes.c_void_p()
    for args in ((0, 0, 0, 2, 2, 1 << 20, 1, 1, 0),      # dim 0
                 (0, 4097, 0, 2, 2, 1 << 20, 1, 1, 0),   # dim above the FP32 maximum
                 (0, 8193, 1, 2, 2, 1 << 20, 1, 1, 0),   # dim above the BF16 maximum
                 (0, 16, 7, 2, 2, 1 << 20, 1, 1, 0),     # bad dtype
                 (0, 16, 0, -1, 2, 1 << 20, 1, 1, 0),    # k < 0
                 (0, 16, 0, 2, 0, 1 << 20, 1, 1, 0),     # no slots
                 (0, 16, 0, 2, 2, -1, 1, 1, 0),          # negative budget
                 (0, 16, 0, 2, 2, 1 << 20, 0, 1, 0),     # no builders
                 (0, 16, 0, 2, 2, 1 << 20, 1, 0, 0),     # groups of 0
                 (0, 16, 0, 2, 2, 1 << 20, 1, 1, 64)):   # unknown flag
        assert lib.cleora_server_create(ctypes.byref(h), *args) == _lib.E_INVAL, args
        assert not h.value
    assert lib.cleora_server_submit(null, null, null) == _lib.E_INVAL
    n = ctypes.c_int32()
    assert lib.cleora_server_poll(null, null, 0, ctypes.byref(n), 0.0) == _lib.E_INVAL
    assert lib.cleora_server_stats(null, null, null, null, null, null, null) == _lib.E_INVAL
    assert lib.cleora_server_now(null) == 0.0
    lib.cleora_server_destroy(null)


def test_noalloc_limits_without_gpu(lib):
    """The no-allocation entry point refuses sizes above its limits (and
    bad arguments) before any device work; the limits of the binding are
    the header's."""
    from paper_2102_02302_amd import _lib
    text = open(HEADER).read()
    for name in ("MAX_ROWS", "MAX_EDGES", "MAX_ROW_BYTES"):
        m = re.search(rf"#define CLEORA_NOALLOC_{name} (\d+)", text)
        assert m and int(m.group(1)) == getattr(_lib, f"NOALLOC_{name}"), name
    f = lib.cleora_propagate_rows_noalloc
    T, out, ids = 1 << 12, 1 << 13, 1 << 14  # aligned stand-ins, never dereferenced
    R, M = _lib.NOALLOC_MAX_ROWS, _lib.NOALLOC_MAX_EDGES
    assert f(0, R + 1, 10, 5, ids, ids, None, T, 16, 16, 0, out, 16, None) == _lib.E_INVAL
    assert b"limits" in lib.cleora_last_error()
    assert f(0, R, 10, M + 1, ids, ids, None, T, 16, 16, 0, out, 16, None) == _lib.E_INVAL
    # 1028 float32 columns: a 4112-byte row
    assert f(0, 10, 10, 5, ids, ids, None, T, 1028, 1028, 0, out, 1028, None) == _lib.E_INVAL
    assert f(0, 10, 10, 5, ids, ids, None, None, 16, 16, 0, out, 16, None) == _lib.E_INVAL
    assert f(0, 10, 10, 5, ids, ids, None, T, 20, 16, 0, out, 16, None) == _lib.E_INVAL  # ld_in
    assert f(0, 10, 10, 5, None, ids, None, T, 16, 16, 0, out, 16, None) == _lib.E_INVAL


def test_binding_constants_match_the_header():
    """Flags, storage types and the automatic slice width of the binding are
    the header's."""
    from paper_2102_02302_amd import _lib
    text = open(HEADER).read()
    want = {"CLEORA_SLICES_AUTO": _lib.SLICES_AUTO, "CLEORA_DIRECTED": _lib.DIRECTED,
            "CLEORA_EMPTY_KEEP": _lib.EMPTY_KEEP, "CLEORA_F32": _lib.F32, "CLEORA_BF16": _lib.BF16}
    for name, value in want.items():
        m = re.search(rf"#define {name} \(?(-?\d+)", text) or re.search(
            rf"\b{name}\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == value, name
