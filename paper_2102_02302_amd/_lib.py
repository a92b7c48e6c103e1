"""ctypes binding of libcleora.so (the C ABI in include/cleora.h).

Argument marshalling only: every step of the embedding runs in the HIP
library.  Loading fails loudly when the library has not been built; there is
no fallback path.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CLEORA_LIB", os.path.join(_HERE, "libcleora.so"))

OK, E_INVAL, E_STATE, E_NOMEM, E_DEVICE, E_INPUT = range(6)
F32, BF16 = 0, 1
DIRECTED, EMPTY_KEEP = 1, 2
SLICES_AUTO = -1  # cleora_set_slices: the autotuner chooses whole rows or slices
MAX_DIM = {F32: 4096, BF16: 8192}

_CODES = {E_INVAL: "E_INVAL", E_STATE: "E_STATE", E_NOMEM: "E_NOMEM",
          E_DEVICE: "E_DEVICE", E_INPUT: "E_INPUT"}

# limits of cleora_propagate_rows_noalloc (cleora.h)
NOALLOC_MAX_ROWS = 8192
NOALLOC_MAX_EDGES = 524288
NOALLOC_MAX_ROW_BYTES = 4096

EXPORTS = [
    "cleora_create", "cleora_destroy", "cleora_footprint_bytes", "cleora_build_csr",
    "cleora_build_init",
    "cleora_init", "cleora_propagate", "cleora_embed_blocked", "cleora_release_scratch",
    "cleora_get_embedding",
    "cleora_embedding_ptr",
    "cleora_previous_embedding_ptr", "cleora_propagate_rows", "cleora_propagate_rows_noalloc",
    "cleora_get_csr", "cleora_info",
    "cleora_schedule_info", "cleora_sync", "cleora_set_chunk", "cleora_set_schedule",
    "cleora_set_slices",
    "cleora_set_timing",
    "cleora_kernel_time", "cleora_launch_stats", "cleora_autotune", "cleora_expand_clique",
    "cleora_expand_star",
    "cleora_build_chunk", "cleora_chunk_info", "cleora_merge_chunk", "cleora_merge_finish",
    "cleora_embed_batch", "cleora_batch_status", "cleora_step_multi", "cleora_server_create",
    "cleora_server_submit",
    "cleora_server_poll", "cleora_server_stats", "cleora_server_memory", "cleora_server_now",
    "cleora_server_destroy",
    "cleora_last_error",
]


class CleoraError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Graph(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("seed", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("out", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32),
                ("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("ready_s", ctypes.c_double), ("done_s", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2102_02302_amd.build`")
    # torch first: the library then binds to the HIP runtime torch loaded.
    # Loaded the other way round, torch could not initialise its GPU
    # afterwards in the same process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_uint64)
    sig = {
        "cleora_create": (ctypes.c_int, [ctypes.POINTER(p), ctypes.c_int]),
        "cleora_destroy": (None, [p]),
        "cleora_footprint_bytes": (ctypes.c_size_t, [i64, i64, u32, i32, i32]),
        "cleora_build_csr": (ctypes.c_int, [p, i64, i64, p, p, p, u32, p]),
        "cleora_build_init": (ctypes.c_int, [p, i64, i64, p, p, p, u32, i32, i32, u64, p]),
        "cleora_init": (ctypes.c_int, [p, i32, i32, u64, p]),
        "cleora_propagate": (ctypes.c_int, [p, i32, p]),
        "cleora_embed_blocked": (ctypes.c_int, [p, i32, i32, i32, u64, i32, p, i64, p]),
        "cleora_release_scratch": (ctypes.c_int, [p]),
        "cleora_set_slices": (ctypes.c_int, [p, i32]),
        "cleora_get_embedding": (ctypes.c_int, [p, p, i64, i32, p]),
        "cleora_embedding_ptr": (ctypes.c_int, [p, ctypes.POINTER(p), ctypes.POINTER(i64)]),
        "cleora_previous_embedding_ptr": (ctypes.c_int, [p, ctypes.POINTER(p),
                                                         ctypes.POINTER(i64)]),
        "cleora_propagate_rows": (ctypes.c_int, [p, i64, i64, i64, p, p, p, p, i64, i32, i32, p,
                                                 i64, p]),
        "cleora_propagate_rows_noalloc": (ctypes.c_int, [ctypes.c_int, i64, i64, i64, p, p, p, p,
                                                         i64, i32, i32, p, i64, p]),
        "cleora_get_csr": (ctypes.c_int, [p, p, p, p, p, p]),
        "cleora_info": (ctypes.c_int, [p, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                       ctypes.POINTER(i32), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32)]),
        "cleora_schedule_info": (ctypes.c_int, [p, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                                ctypes.POINTER(i64), ctypes.POINTER(i64),
                                                ctypes.POINTER(i32), ctypes.POINTER(i32),
                                                ctypes.POINTER(i32)]),
        "cleora_sync": (ctypes.c_int, [p, p]),
        "cleora_set_chunk": (ctypes.c_int, [p, i32]),
        "cleora_set_schedule": (ctypes.c_int, [p, i32, i32]),
        "cleora_set_timing": (ctypes.c_int, [p, ctypes.c_int]),
        "cleora_kernel_time": (ctypes.c_int, [p, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(i64),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(i64)]),
        "cleora_launch_stats": (ctypes.c_int, [p, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "cleora_autotune": (ctypes.c_int, [p, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                           ctypes.POINTER(ctypes.c_float), p]),
        "cleora_expand_clique": (ctypes.c_int, [p, i64, p, p, p, p, i64, ctypes.POINTER(i64), p]),
        "cleora_expand_star": (ctypes.c_int, [p, i64, i64, p, p, p, p, i64, ctypes.POINTER(i64),
                                              p]),
        "cleora_build_chunk": (ctypes.c_int, [p, i64, i64, p, p, p, u32, p]),
        "cleora_chunk_info": (ctypes.c_int, [p, ctypes.POINTER(i64), p, p, p]),
        "cleora_merge_chunk": (ctypes.c_int, [p, p, i64, p, p]),
        "cleora_merge_finish": (ctypes.c_int, [ctypes.c_int, p, i64, p, i64, i32, p, i64, i32, p]),
        "cleora_batch_status": (ctypes.c_int, [p, i32, p]),
        "cleora_embed_batch": (ctypes.c_int, [p, i32, ctypes.POINTER(Graph), u32, i32, i32, i32,
                                              ctypes.POINTER(p), p]),
        "cleora_step_multi": (ctypes.c_int, [ctypes.POINTER(p), i32, p]),
        "cleora_server_create": (ctypes.c_int, [ctypes.POINTER(p), ctypes.c_int, i32, i32, i32, i32,
                                                i64, i32, i32, u32]),
        "cleora_server_submit": (ctypes.c_int, [p, ctypes.POINTER(Request), ctypes.POINTER(i64)]),
        "cleora_server_poll": (ctypes.c_int, [p, ctypes.POINTER(Completion), i32,
                                              ctypes.POINTER(i32), ctypes.c_double]),
        "cleora_server_stats": (ctypes.c_int, [p, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                               ctypes.POINTER(i32), ctypes.POINTER(i64),
                                               ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "cleora_server_memory": (ctypes.c_int, [p, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                                ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "cleora_server_now": (ctypes.c_double, [p]),
        "cleora_server_destroy": (None, [p]),
        "cleora_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != OK:
        msg = load().cleora_last_error()
        raise CleoraError(rc, msg.decode() if msg else "")
