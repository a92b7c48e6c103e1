"""MI355X (gfx950) implementation of Cleora's propagation hot path.

Cleora (Rychalska et al., arXiv 2102.02302, Section 3.2, Algorithm 1) embeds
a graph by repeating T_i = normalise_rows(M . T_{i-1}) with M = D^-1 A and
T_0 ~ U(-1, 1).  The work runs in the HIP library ``libcleora.so`` behind the
C ABI of ``include/cleora.h``; this package only marshals torch tensors
(device memory) and streams into those calls.
"""

from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

from . import _lib
from ._lib import BF16, DIRECTED, EMPTY_KEEP, F32, CleoraError, load  # noqa: F401

__all__ = ["Context", "embed", "embed_batch", "batch_status", "embed_blocked", "embed_chunked",
           "embed_new_nodes", "step_multi",
           "footprint_bytes", "CleoraError",
           "F32", "BF16", "DIRECTED", "EMPTY_KEEP", "load"]


def _torch():
    import torch
    return torch


def _dtype_code(dtype) -> int:
    if dtype in (F32, "f32", "float32", "fp32"):
        return F32
    if dtype in (BF16, "bf16", "bfloat16"):
        return BF16
    torch = _torch()
    if dtype is torch.float32:
        return F32
    if dtype is torch.bfloat16:
        return BF16
    raise ValueError(f"unknown dtype {dtype!r}")


def _stream(stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_i32(x, device):
    torch = _torch()
    t = torch.as_tensor(x)
    return t.to(device=device, dtype=torch.int32).contiguous()


def _dev_f32(x, device):
    if x is None:
        return None
    torch = _torch()
    return torch.as_tensor(x).to(device=device, dtype=torch.float32).contiguous()


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def footprint_bytes(n_nodes: int, n_edges: int, dim: int, dtype="f32",
                    directed: bool = False) -> int:
    return int(load().cleora_footprint_bytes(n_nodes, n_edges, DIRECTED if directed else 0, dim,
                                             _dtype_code(dtype)))


class Context:
    """One graph and its embedding on one GPU (a ``cleora_ctx``)."""

    def __init__(self, device: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        self._lib = load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _lib.check(self._lib.cleora_create(ctypes.byref(h), device))
        self._h = h
        self._keep = []  # inputs that must outlive queued work

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            self._lib.cleora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    # -- calls
    def build_csr(self, n_nodes: int, src, dst, w=None, directed: bool = False,
                  empty_keep: bool = False, stream=None) -> "Context":
        s = _dev_i32(src, self.device)
        d = _dev_i32(dst, self.device)
        wt = _dev_f32(w, self.device)
        flags = (DIRECTED if directed else 0) | (EMPTY_KEEP if empty_keep else 0)
        _lib.check(self._lib.cleora_build_csr(self._h, int(n_nodes), int(s.numel()), _ptr(s),
                                              _ptr(d), _ptr(wt), flags, _stream(stream)))
        self._keep = [s, d, wt]
        return self

    def build_graph(self, g, empty_keep: bool = False, stream=None) -> "Context":
        """Build from a ``gen.Graph``-like object (n, src, dst, w, directed)."""
        return self.build_csr(g.n, g.src, g.dst, g.w, g.directed, empty_keep, stream)

    def build_init(self, n_nodes: int, src, dst, w=None, dim: int = 128, dtype="f32",
                   seed: int = 0, directed: bool = False, empty_keep: bool = False,
                   stream=None) -> "Context":
        """build_csr + init in one call, T_0 written while the CSR is built."""
        s = _dev_i32(src, self.device)
        d = _dev_i32(dst, self.device)
        wt = _dev_f32(w, self.device)
        flags = (DIRECTED if directed else 0) | (EMPTY_KEEP if empty_keep else 0)
        _lib.check(self._lib.cleora_build_init(self._h, int(n_nodes), int(s.numel()), _ptr(s),
                                               _ptr(d), _ptr(wt), flags, int(dim),
                                               _dtype_code(dtype), int(seed) & (2**64 - 1),
                                               _stream(stream)))
        self._keep = [s, d, wt]
        return self

    def build_graph_init(self, g, dim: int, dtype="f32", seed: int = 0,
                         empty_keep: bool = False, stream=None) -> "Context":
        """build_init from a ``gen.Graph``-like object."""
        return self.build_init(g.n, g.src, g.dst, g.w, dim, dtype, seed, g.directed, empty_keep,
                               stream)

    def set_chunk(self, chunk: int) -> None:
        _lib.check(self._lib.cleora_set_chunk(self._h, int(chunk)))

    def set_slices(self, cols) -> None:
        """Column slices of the next init's iterations: 0 whole rows (the
        default), else ``cols`` wide (results differ from whole rows in
        rounding only); ``"auto"``: whole rows until ``autotune`` has timed
        both on this embedding and kept the faster (``schedule()["slice_cols"]``
        reports the width in use)."""
        code = _lib.SLICES_AUTO if cols == "auto" else int(cols)
        _lib.check(self._lib.cleora_set_slices(self._h, code))

    def set_schedule(self, pack: int = 0, persistent: int = -1) -> None:
        """Fix the packing size (0: automatic) and SpMM grid (-1: automatic,
        0: one wave per item, m: m x the resident waves) for the next init."""
        _lib.check(self._lib.cleora_set_schedule(self._h, int(pack), int(persistent)))

    def init(self, dim: int, dtype="f32", seed: int = 0, stream=None) -> "Context":
        _lib.check(self._lib.cleora_init(self._h, int(dim), _dtype_code(dtype),
                                         int(seed) & (2**64 - 1), _stream(stream)))
        return self

    def propagate(self, k: int, stream=None) -> "Context":
        _lib.check(self._lib.cleora_propagate(self._h, int(k), _stream(stream)))
        return self

    def embed_blocked(self, dim: int, block: int, k: int, dtype="f32", seed: int = 0, out=None,
                      stream=None):
        """T_k of the context's graph computed ``block`` columns at a time
        (for embeddings too wide for two N x dim device buffers): the result
        of init(dim, dtype, seed) + propagate(k) up to float32 summation
        order.  ``out`` is an N x dim tensor of the dtype
        (device, or pinned host memory for graphs larger than the device);
        a device tensor is allocated when it is None.  The context keeps its
        graph and holds no embedding afterwards."""
        torch = _torch()
        code = _dtype_code(dtype)
        tdt = torch.float32 if code == F32 else torch.bfloat16
        n = self.info()["n"]
        if out is None:
            out = torch.empty((n, dim), dtype=tdt, device=self.device)
        if out.dtype != tdt or out.dim() != 2 or out.shape[0] != n or out.shape[1] < dim \
                or out.stride(1) != 1:
            raise ValueError("out must be an N x dim tensor of the dtype with unit column stride")
        _lib.check(self._lib.cleora_embed_blocked(self._h, int(dim), int(block), code,
                                                  int(seed) & (2**64 - 1), int(k),
                                                  out.data_ptr(), out.stride(0), _stream(stream)))
        return out

    def release_scratch(self) -> "Context":
        """Free the build's temporaries (and the embedding buffers when the
        context holds no embedding); the graph stays."""
        _lib.check(self._lib.cleora_release_scratch(self._h))
        return self

    def sync(self, stream=None) -> None:
        _lib.check(self._lib.cleora_sync(self._h, _stream(stream)))

    def info(self) -> dict:
        n, nnz = ctypes.c_int64(), ctypes.c_int64()
        dim, dt, it = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self._lib.cleora_info(self._h, ctypes.byref(n), ctypes.byref(nnz),
                                         ctypes.byref(dim), ctypes.byref(dt), ctypes.byref(it)))
        return {"n": n.value, "nnz": nnz.value, "dim": dim.value, "dtype": dt.value,
                "iteration": it.value}

    def schedule(self) -> dict:
        chunk, pack, persist, sl = (ctypes.c_int32() for _ in range(4))
        ns, nl, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self._lib.cleora_schedule_info(self._h, ctypes.byref(chunk), ctypes.byref(ns),
                                                  ctypes.byref(nl), ctypes.byref(nb),
                                                  ctypes.byref(pack), ctypes.byref(persist),
                                                  ctypes.byref(sl)))
        return {"chunk": chunk.value, "split_chunks": ns.value, "split_rows": nl.value,
                "packed_items": nb.value, "pack": pack.value, "persistent": persist.value,
                "slice_cols": sl.value}

    def embedding(self, dtype=None, stream=None):
        """Copy of the current N x dim embedding as a device tensor."""
        torch = _torch()
        inf = self.info()
        code = inf["dtype"] if dtype is None else _dtype_code(dtype)
        tdt = torch.float32 if code == F32 else torch.bfloat16
        out = torch.empty((inf["n"], inf["dim"]), dtype=tdt, device=self.device)
        _lib.check(self._lib.cleora_get_embedding(self._h, out.data_ptr(), inf["dim"], code,
                                                  _stream(stream)))
        return out

    def embedding_ptr(self, previous: bool = False):
        """(device pointer, row stride) of T_t, or of T_{t-1} when previous."""
        ptr, ld = ctypes.c_void_p(), ctypes.c_int64()
        fn = (self._lib.cleora_previous_embedding_ptr if previous
              else self._lib.cleora_embedding_ptr)
        _lib.check(fn(self._h, ctypes.byref(ptr), ctypes.byref(ld)))
        return ptr.value, ld.value

    def propagate_rows(self, n_rows: int, n_cols: int, rows, cols, T_in, dim: int, dtype="f32",
                       w=None, ld_in: Optional[int] = None, out=None, stream=None):
        """One Algorithm-1 step for n_rows new rows against T_in (n_cols rows):
        out[i] = normalise(sum over edges i->b of w * T_in[b] / deg(i)).
        T_in is a device tensor, or a raw device pointer with ld_in."""
        torch = _torch()
        code = _dtype_code(dtype)
        tdt = torch.float32 if code == F32 else torch.bfloat16
        r = _dev_i32(rows, self.device)
        c = _dev_i32(cols, self.device)
        wt = _dev_f32(w, self.device)
        epv = 4 if code == F32 else 8
        ld_pad = (dim + epv - 1) // epv * epv
        if isinstance(T_in, int):
            ptr, ld = T_in, ld_in if ld_in is not None else ld_pad
        else:
            t = torch.as_tensor(T_in).to(device=self.device, dtype=tdt)
            if t.shape[1] != ld_pad:
                t = torch.nn.functional.pad(t[:, :dim], (0, ld_pad - dim))
            t = t.contiguous()
            ptr, ld = t.data_ptr(), ld_pad
            self._keep = [t]
        if out is None:
            out = torch.empty((n_rows, dim), dtype=tdt, device=self.device)
        _lib.check(self._lib.cleora_propagate_rows(
            self._h, int(n_rows), int(n_cols), int(r.numel()), _ptr(r), _ptr(c), _ptr(wt), ptr,
            ld, int(dim), code, out.data_ptr(), out.stride(0), _stream(stream)))
        return out

    def build_chunk(self, n_global: int, src, dst, w=None, directed: bool = False,
                    stream=None) -> "Context":
        """CSR of one chunk of a larger graph, on the nodes its edges touch."""
        s = _dev_i32(src, self.device)
        d = _dev_i32(dst, self.device)
        wt = _dev_f32(w, self.device)
        _lib.check(self._lib.cleora_build_chunk(self._h, int(n_global), int(s.numel()), _ptr(s),
                                                _ptr(d), _ptr(wt), DIRECTED if directed else 0,
                                                _stream(stream)))
        self._keep = [s, d, wt]
        return self

    def merge_chunk(self, acc, wsum, stream=None) -> None:
        """acc[v] += occ(v) * T[v], wsum[v] += occ(v) for the chunk's nodes."""
        _lib.check(self._lib.cleora_merge_chunk(self._h, acc.data_ptr(), acc.stride(0),
                                                wsum.data_ptr(), _stream(stream)))

    def expand(self, offsets, members, mode: str = "clique", n_nodes: int = 0, stream=None):
        """Hyperedges (CSR: offsets int64[H+1], members int32) -> edge list
        (src, dst) by clique or star expansion (Section 3.2)."""
        torch = _torch()
        off = torch.as_tensor(offsets).to(device=self.device, dtype=torch.int64).contiguous()
        mem = torch.as_tensor(members).to(device=self.device, dtype=torch.int32).contiguous()
        h = off.numel() - 1
        n = ctypes.c_int64()
        if mode == "clique":
            fn = lambda s_, d_, cap: self._lib.cleora_expand_clique(  # noqa: E731
                self._h, h, off.data_ptr(), mem.data_ptr(), s_, d_, cap, ctypes.byref(n),
                _stream(stream))
        elif mode == "star":
            fn = lambda s_, d_, cap: self._lib.cleora_expand_star(  # noqa: E731
                self._h, int(n_nodes), h, off.data_ptr(), mem.data_ptr(), s_, d_, cap,
                ctypes.byref(n), _stream(stream))
        else:
            raise ValueError(mode)
        _lib.check(fn(None, None, 0))
        src = torch.empty(max(n.value, 1), dtype=torch.int32, device=self.device)
        dst = torch.empty(max(n.value, 1), dtype=torch.int32, device=self.device)
        _lib.check(fn(src.data_ptr(), dst.data_ptr(), src.numel()))
        return src[:n.value], dst[:n.value]

    def csr(self, stream=None) -> dict:
        torch = _torch()
        inf = self.info()
        n, nnz = inf["n"], inf["nnz"]
        rp = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(nnz, 1), dtype=torch.float32, device=self.device)
        deg = torch.empty(n, dtype=torch.float64, device=self.device)
        _lib.check(self._lib.cleora_get_csr(self._h, rp.data_ptr(), col.data_ptr(),
                                            val.data_ptr(), deg.data_ptr(), _stream(stream)))
        return {"row_ptr": rp, "col": col[:nnz], "val": val[:nnz], "deg": deg}

    def autotune(self, stream=None) -> dict:
        """Pick the fastest packing size and SpMM grid (one wave per item or
        persistent) for this graph; results are unchanged."""
        pack, persistent, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        _lib.check(self._lib.cleora_autotune(self._h, ctypes.byref(pack), ctypes.byref(persistent),
                                             ctypes.byref(ms), _stream(stream)))
        return {"pack": pack.value, "persistent": bool(persistent.value), "step_ms": ms.value}

    # -- measurement
    def set_timing(self, on: bool) -> None:
        _lib.check(self._lib.cleora_set_timing(self._h, 1 if on else 0))

    def kernel_time(self) -> dict:
        a, b = ctypes.c_double(), ctypes.c_double()
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self._lib.cleora_kernel_time(self._h, ctypes.byref(a), ctypes.byref(na),
                                                ctypes.byref(b), ctypes.byref(nb)))
        return {"spmm_ms": a.value, "spmm_launches": na.value, "combine_ms": b.value,
                "combine_launches": nb.value}

    def launch_stats(self) -> dict:
        """Captured k-iteration graphs instantiated, and their replays, since
        the context was created."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self._lib.cleora_launch_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return {"graph_instantiations": a.value, "graph_launches": b.value}


def propagate_rows_noalloc(n_rows: int, n_cols: int, rows, cols, T_in, dim: int, dtype="f32",
                           w=None, out=None, device: int = 0, stream=None):
    """``Context.propagate_rows`` without a context and without device
    allocation inside the library (``cleora_propagate_rows_noalloc``; sizes
    within the CLEORA_NOALLOC_* limits).  T_in: device tensor whose row
    stride is dim rounded up to 16 bytes."""
    torch = _torch()
    code = _dtype_code(dtype)
    tdt = torch.float32 if code == F32 else torch.bfloat16
    r = _dev_i32(rows, device)
    c = _dev_i32(cols, device)
    wt = _dev_f32(w, device)
    epv = 4 if code == F32 else 8
    ld = (dim + epv - 1) // epv * epv
    assert T_in.dtype == tdt and T_in.is_contiguous() and T_in.shape[1] == ld
    if out is None:
        out = torch.empty((n_rows, dim), dtype=tdt, device=T_in.device)
    _lib.check(load().cleora_propagate_rows_noalloc(
        int(device), int(n_rows), int(n_cols), int(r.numel()), _ptr(r), _ptr(c), _ptr(wt),
        T_in.data_ptr(), ld, int(dim), code, out.data_ptr(), out.stride(0), _stream(stream)))
    return out


def embed(g, dim: int, k: int, seed: int = 0, dtype="f32", device: int = 0,
          empty_keep: bool = False, chunk: int = 0, slices=0):
    """Whole path for one graph: build M, initialise T_0, k iterations
    (``slices``: the column slices of the iterations, 0 whole rows; with
    ``"auto"`` the autotuner runs and chooses)."""
    with Context(device) as ctx:
        if chunk:
            ctx.set_chunk(chunk)
        if slices:
            ctx.set_slices(slices)
        ctx.build_graph_init(g, dim, dtype, seed, empty_keep=empty_keep)
        if slices == "auto":
            ctx.autotune()
        ctx.propagate(k)
        return ctx.embedding()


def embed_blocked(g, dim: int, block: int, k: int, seed: int = 0, dtype="f32",
                  device: int = 0, empty_keep: bool = False, out=None):
    """Whole path for one graph with the embedding computed ``block`` columns
    at a time (``Context.embed_blocked``); same result as ``embed`` up to
    float32 summation order."""
    with Context(device) as ctx:
        ctx.build_graph(g, empty_keep=empty_keep)
        return ctx.embed_blocked(dim, block, k, dtype, seed, out=out)


def embed_new_nodes(base: Context, n_new: int, new_ids, old_ids, w=None,
                    previous: bool = True, work: Optional[Context] = None):
    """Embeddings of nodes added after ``base`` was embedded (Section 3.2):
    each new node i averages the rows of its existing neighbours (edges
    new_ids[e] -> old_ids[e], optional weights), from iteration I-1 when
    ``previous`` (the paper's recommendation), else from iteration I."""
    inf = base.info()
    ptr, ld = base.embedding_ptr(previous=previous)
    own = work is None
    work = work or Context(base.device.index or 0)
    try:
        return work.propagate_rows(n_new, inf["n"], new_ids, old_ids, ptr, inf["dim"],
                                   inf["dtype"], w=w, ld_in=ld)
    finally:
        if own:
            work.close()


def embed_chunked(g, chunks, dim: int, k: int, seed: int = 0, dtype="f32", device: int = 0):
    """Algorithm 1 with chunks: ``chunks`` is a list of edge-index arrays (or
    an int Q: Q contiguous edge ranges).  Each chunk is embedded on its own
    nodes, then the chunk embeddings are merged per node, weighted by the
    node's occurrences in each chunk."""
    import numpy as np
    torch = _torch()
    if isinstance(chunks, int):
        chunks = np.array_split(np.arange(g.m), chunks)
    dev = torch.device("cuda", device)
    acc = torch.zeros((g.n, dim), dtype=torch.float32, device=dev)
    wsum = torch.zeros(g.n, dtype=torch.float32, device=dev)
    with Context(device) as ctx:
        for idx in chunks:
            w = None if g.w is None else g.w[idx]
            ctx.build_chunk(g.n, g.src[idx], g.dst[idx], w, g.directed)
            ctx.init(dim, dtype, seed).propagate(k)
            ctx.merge_chunk(acc, wsum)
    code = _dtype_code(dtype)
    out = torch.empty((g.n, dim), dtype=torch.float32 if code == F32 else torch.bfloat16,
                      device=dev)
    _lib.check(load().cleora_merge_finish(device, acc.data_ptr(), acc.stride(0),
                                          wsum.data_ptr(), g.n, dim, out.data_ptr(),
                                          out.stride(0), code, _stream(None)))
    return out


def embed_batch(ctx: Context, graphs: Sequence, dim: int, k: int, seeds: Sequence[int],
                dtype="f32", directed: bool = False, empty_keep: bool = False,
                stream=None) -> List:
    """Embed several graphs as one block-diagonal graph (cleora_embed_batch)."""
    torch = _torch()
    code = _dtype_code(dtype)
    tdt = torch.float32 if code == F32 else torch.bfloat16
    arr = (_lib.Graph * len(graphs))()
    keep, outs = [], []
    for i, g in enumerate(graphs):
        s = _dev_i32(g.src, ctx.device)
        d = _dev_i32(g.dst, ctx.device)
        w = _dev_f32(g.w, ctx.device)
        keep += [s, d, w]
        arr[i] = _lib.Graph(g.n, s.numel(), _ptr(s), _ptr(d), _ptr(w),
                            int(seeds[i]) & (2**64 - 1))
        outs.append(torch.empty((g.n, dim), dtype=tdt, device=ctx.device))
    out_ptrs = (ctypes.c_void_p * len(graphs))(*[o.data_ptr() for o in outs])
    flags = (DIRECTED if directed else 0) | (EMPTY_KEEP if empty_keep else 0)
    _lib.check(ctx._lib.cleora_embed_batch(ctx.handle, len(graphs), arr, flags, dim, code, k,
                                           out_ptrs, _stream(stream)))
    return outs


def batch_status(ctx: Context, n_graphs: int) -> List[int]:
    """Per-graph status codes of the last embed_batch call on ``ctx`` (after
    a failure with E_INPUT, E_INPUT marks the graphs with bad edges)."""
    arr = (ctypes.c_int32 * int(n_graphs))()
    _lib.check(ctx._lib.cleora_batch_status(ctx.handle, int(n_graphs), arr))
    return list(arr)


def step_multi(ctxs: Sequence[Context], stream=None) -> None:
    """One iteration for every context in a single set of launches."""
    if not ctxs:
        return
    arr = (ctypes.c_void_p * len(ctxs))(*[c.handle.value for c in ctxs])
    _lib.check(ctxs[0]._lib.cleora_step_multi(arr, len(ctxs), _stream(stream)))
