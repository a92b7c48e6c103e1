"""FP64 CPU oracle for Cleora propagation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of ``bench.py`` may
import this package.  The GPU library never calls it and shares no code with
it.  The arithmetic lives in ``cleora_oracle.c`` (plain C, FP64); this module
compiles it with gcc on first use and marshals numpy arrays.

Functions follow the paper (arXiv 2102.02302):
  * ``build_adjacency`` -- e_ab counts / weight sums (Section 3.2)
  * ``transition``      -- M = D^-1 A (Section 3.2, Algorithm 1)
  * ``init``            -- T_0 ~ U(-1, 1) (Section 3.2)
  * ``propagate``       -- I iterations of multiply + row L2 normalise
                           (Algorithm 1)
  * ``embed_chunked``   -- Algorithm 1's chunks and weighted merge
  * ``t1_rows``         -- the first iteration for sampled rows, from the seed
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cleora_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

EMPTY_KEEP = 1
NO_NORM = 2

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        # ORACLE_LIB: an already built copy of the same source (the
        # sanitizer test loads an instrumented build this way)
        path = os.environ.get("ORACLE_LIB") or build()
        lib = ctypes.CDLL(path)
        i64, i32, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        p = ctypes.c_void_p
        lib.oracle_splitmix64.restype = u64
        lib.oracle_splitmix64.argtypes = [u64]
        lib.oracle_uniform.restype = ctypes.c_double
        lib.oracle_uniform.argtypes = [u64, i64, i32, i32]
        lib.oracle_init.restype = None
        lib.oracle_init.argtypes = [u64, i64, i64, i32, p]
        lib.oracle_init_ids.restype = None
        lib.oracle_init_ids.argtypes = [u64, p, i64, i32, p]
        lib.oracle_entry_bound.restype = i64
        lib.oracle_entry_bound.argtypes = [i64, ctypes.c_int]
        lib.oracle_build_adjacency.restype = ctypes.c_int
        lib.oracle_build_adjacency.argtypes = [i64, i64, p, p, p, ctypes.c_int, p, p, p,
                                               ctypes.POINTER(i64)]
        lib.oracle_transition.restype = None
        lib.oracle_transition.argtypes = [i64, p, p, p, p]
        lib.oracle_step_rows.restype = None
        lib.oracle_step_rows.argtypes = [i64, i64, i32, p, p, p, p, p, ctypes.c_uint]
        lib.oracle_propagate.restype = None
        lib.oracle_propagate.argtypes = [i64, i32, p, p, p, p, p, ctypes.c_int, ctypes.c_uint]
        lib.oracle_adjacency_rows.restype = ctypes.c_int
        lib.oracle_adjacency_rows.argtypes = [i64, i64, p, p, p, ctypes.c_int, p, i64, p, p, p,
                                              i64, ctypes.POINTER(i64)]
        lib.oracle_t1_rows.restype = None
        lib.oracle_t1_rows.argtypes = [i64, p, i32, u64, p, p, p, p, ctypes.c_uint]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_get_threads.restype = ctypes.c_int
        lib.oracle_get_threads.argtypes = []
        _lib = lib
        return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def splitmix64(x: int) -> int:
    return int(_load().oracle_splitmix64(ctypes.c_uint64(x & (2**64 - 1))))


def uniform(seed: int, i: int, d: int, j: int) -> float:
    return float(_load().oracle_uniform(seed & (2**64 - 1), i, d, j))


def init(seed: int, n: int, d: int, row0: int = 0) -> np.ndarray:
    """T_0 rows row0 .. row0+n-1 (graph-local indices), float64 n x d."""
    T = np.empty((n, d), np.float64)
    _load().oracle_init(seed & (2**64 - 1), row0, n, d, _ptr(T))
    return T


class Adjacency:
    """A in CSR: row_ptr int64[n+1], col int32[nnz], aval float64[nnz]."""

    def __init__(self, n, row_ptr, col, aval):
        self.n = n
        self.row_ptr = row_ptr
        self.col = col
        self.aval = aval

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def build_adjacency(n: int, src: np.ndarray, dst: np.ndarray, w: Optional[np.ndarray],
                    directed: bool) -> Adjacency:
    lib = _load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    if w is not None:
        w = np.ascontiguousarray(w, np.float32)
    m = src.size
    cap = max(1, int(lib.oracle_entry_bound(m, int(directed))))
    row_ptr = np.empty(n + 1, np.int64)
    col = np.empty(cap, np.int32)
    aval = np.empty(cap, np.float64)
    nnz = ctypes.c_int64(0)
    rc = lib.oracle_build_adjacency(n, m, _ptr(src), _ptr(dst), _ptr(w), int(directed),
                                    _ptr(row_ptr), _ptr(col), _ptr(aval), ctypes.byref(nnz))
    if rc == -1:
        raise ValueError("edge id outside [0, n) or weight not finite and positive")
    if rc != 0:
        raise MemoryError("oracle adjacency build ran out of memory")
    k = nnz.value
    return Adjacency(n, row_ptr, col[:k].copy(), aval[:k].copy())


def build_graph(g) -> Adjacency:
    """Adjacency of a ``gen.Graph``."""
    return build_adjacency(g.n, g.src, g.dst, g.w, g.directed)


def transition(adj: Adjacency) -> tuple[np.ndarray, np.ndarray]:
    """(mval float64[nnz], deg float64[n]) with mval = aval / deg[row]."""
    mval = np.empty(max(1, adj.nnz), np.float64)
    deg = np.empty(adj.n, np.float64)
    _load().oracle_transition(adj.n, _ptr(adj.row_ptr), _ptr(adj.aval), _ptr(mval), _ptr(deg))
    return mval[:adj.nnz], deg


def step_rows(adj: Adjacency, mval: np.ndarray, T_in: np.ndarray, T_out: np.ndarray,
              r0: int, r1: int, flags: int = 0) -> None:
    """One iteration for rows [r0, r1) into T_out (other rows untouched)."""
    assert T_in.dtype == np.float64 and T_in.flags.c_contiguous
    assert T_out.dtype == np.float64 and T_out.flags.c_contiguous
    d = T_in.shape[1]
    _load().oracle_step_rows(r0, r1, d, _ptr(adj.row_ptr), _ptr(adj.col), _ptr(mval),
                             _ptr(T_in), _ptr(T_out), flags)


def propagate(adj: Adjacency, mval: np.ndarray, T0: np.ndarray, k: int,
              flags: int = 0) -> np.ndarray:
    """T_k from T_0 (float64 n x d); returns a new array."""
    T = np.array(T0, dtype=np.float64, order="C", copy=True)
    tmp = np.empty_like(T)
    n, d = T.shape
    assert n == adj.n
    _load().oracle_propagate(n, d, _ptr(adj.row_ptr), _ptr(adj.col), _ptr(mval), _ptr(T),
                             _ptr(tmp), int(k), flags)
    return T


def adjacency_rows(g, rows: np.ndarray) -> Adjacency:
    """A restricted to the listed rows (any order, no repeats): a CSR whose
    row i is row rows[i] of the full adjacency."""
    lib = _load()
    rows = np.ascontiguousarray(rows, np.int32)
    in_sample = np.zeros(g.n, np.int64)
    in_sample[rows] = np.arange(1, rows.size + 1)
    src = np.ascontiguousarray(g.src, np.int32)
    dst = np.ascontiguousarray(g.dst, np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, np.float32)
    # capacity: every edge touching a sampled row, in both directions
    touch = int(np.count_nonzero(in_sample[src])) + int(np.count_nonzero(in_sample[dst]))
    cap = max(1, touch)
    sub_ptr = np.empty(rows.size + 1, np.int64)
    col = np.empty(cap, np.int32)
    aval = np.empty(cap, np.float64)
    nnz = ctypes.c_int64(0)
    rc = lib.oracle_adjacency_rows(g.n, src.size, _ptr(src), _ptr(dst), _ptr(w),
                                   int(g.directed), _ptr(in_sample), rows.size, _ptr(sub_ptr),
                                   _ptr(col), _ptr(aval), cap, ctypes.byref(nnz))
    if rc == -1:
        raise ValueError("edge id outside [0, n) or weight not finite and positive")
    if rc != 0:
        raise MemoryError(f"oracle_adjacency_rows failed ({rc})")
    k = nnz.value
    return Adjacency(rows.size, sub_ptr, col[:k].copy(), aval[:k].copy())


def t1_rows(g, rows: np.ndarray, d: int, seed: int, flags: int = 0) -> np.ndarray:
    """T_1 for the listed rows, computed from the graph and the seed alone."""
    rows = np.ascontiguousarray(rows, np.int32)
    sub = adjacency_rows(g, rows)
    out = np.empty((rows.size, d), np.float64)
    _load().oracle_t1_rows(rows.size, _ptr(rows), d, seed & (2**64 - 1), _ptr(sub.row_ptr),
                           _ptr(sub.col), _ptr(sub.aval), _ptr(out), flags)
    return out


def expand_clique(offsets, members):
    """Clique expansion (Section 3.2): every pair of members, i < j, of
    each hyperedge, hyperedge by hyperedge.  Plain loops."""
    src, dst = [], []
    for h in range(len(offsets) - 1):
        mem = list(members[offsets[h]:offsets[h + 1]])
        for i in range(len(mem)):
            for j in range(i + 1, len(mem)):
                src.append(mem[i])
                dst.append(mem[j])
    return np.array(src, np.int32), np.array(dst, np.int32)


def expand_star(n_nodes, offsets, members):
    """Star expansion (Section 3.2): hyperedge h becomes node n_nodes + h
    linked to each member."""
    src, dst = [], []
    for h in range(len(offsets) - 1):
        for m in members[offsets[h]:offsets[h + 1]]:
            src.append(n_nodes + h)
            dst.append(m)
    return np.array(src, np.int32), np.array(dst, np.int32)


def init_ids(seed: int, ids: np.ndarray, d: int) -> np.ndarray:
    """T_0 rows of the given global ids."""
    ids = np.ascontiguousarray(ids, np.int32)
    T = np.empty((ids.size, d), np.float64)
    _load().oracle_init_ids(seed & (2**64 - 1), _ptr(ids), ids.size, d, _ptr(T))
    return T


def embed_chunked(g, chunks, d: int, k: int, seed: int, flags: int = 0) -> np.ndarray:
    """Algorithm 1 with Q chunks: ``chunks`` lists the edge indices of each
    chunk.  Chunk q is embedded on the nodes its edges touch (T_0 rows of
    their global ids); node v's result is sum_q w_qv T^q_v with
    w_qv = occ_q(v) / sum_q occ_q(v), occ_q(v) = v's stored entries in chunk
    q before repeated pairs are merged."""
    acc = np.zeros((g.n, d))
    wsum = np.zeros(g.n)
    for idx in chunks:
        src, dst = g.src[idx], g.dst[idx]
        w = None if g.w is None else g.w[idx]
        nodes = np.unique(np.concatenate([src, dst]))
        lid = np.full(g.n, -1, np.int64)
        lid[nodes] = np.arange(nodes.size)
        ls, ld = lid[src].astype(np.int32), lid[dst].astype(np.int32)
        adj = build_adjacency(nodes.size, ls, ld, w, g.directed)
        mval, _ = transition(adj)
        Tq = propagate(adj, mval, init_ids(seed, nodes, d), k, flags)
        occ = np.bincount(ls, minlength=nodes.size).astype(np.float64)
        if not g.directed:
            occ += np.bincount(ld[ls != ld], minlength=nodes.size)
        acc[nodes] += occ[:, None] * Tq
        wsum[nodes] += occ
    out = np.zeros_like(acc)
    nz = wsum > 0
    out[nz] = acc[nz] / wsum[nz, None]
    return out


def embed(g, d: int, k: int, seed: int, flags: int = 0) -> np.ndarray:
    """Whole path for one graph: A -> M -> T_0(seed) -> T_k."""
    adj = build_graph(g)
    mval, _ = transition(adj)
    T0 = init(seed, g.n, d)
    return propagate(adj, mval, T0, k, flags)
