// Internal declarations shared by the translation units of the library.
#pragma once

#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.hpp"

namespace cleora {

// A named range on the profiler's timeline (rocprofv3 --marker-trace) for
// the lifetime of the object; cheap when no profiler is attached.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace cleora

namespace cleora {

// ------------------------------------------------------------------ scan

// Workspace (int64 elements) that exclusive_scan needs for n inputs.
size_t scan_workspace_elems(int64_t n);
// out[i] = sum of in[0..i), i = 0..n (out has n+1 entries; out[n] = total).
void exclusive_scan(const int32_t *in, int64_t n, int64_t *out, int64_t *ws, hipStream_t s);
void exclusive_scan(const uint8_t *in, int64_t n, int64_t *out, int64_t *ws, hipStream_t s);
void exclusive_scan(const int64_t *in, int64_t n, int64_t *out, int64_t *ws, hipStream_t s);

// ----------------------------------------------------- propagation step

// Everything one context contributes to a propagation launch.  Stored in
// device memory; a launch covers one or more contexts, each owning the
// waves [wave_begin, wave_begin + n_split + n_buckets) of the SpMM launch
// and the blocks [block_begin, block_begin + n_long) of the combine launch.
struct StepDesc {
    const int64_t *rp;        // CSR row pointers, N+1
    const int32_t *col;       // CSR columns
    const float *val;         // M values
    const void *Ein;          // T_{t-1}, N x ld
    void *Eout;               // T_t,     N x ld
    float *partial;           // n_split x ld float32 partial sums of split rows
    const int2 *split_items;  // (row, chunk index) of every split chunk
    const int32_t *bucket_row;  // n_buckets+1 row boundaries of the packed items
    const int32_t *long_rows;   // rows split into chunks, ascending
    const int64_t *chunk_base;  // N+1: first partial slot of each row
    int64_t wave_begin;
    int64_t block_begin;
    int64_t n_split;
    int64_t n_buckets;
    int64_t n_long;
    int32_t ld;
    int32_t chunk;
    uint32_t flags;
    int32_t persist;  // SpMM grid: 0 = one wave per item, m > 0 = m x the resident blocks
    // Column blocks and slices (both null otherwise, and in multi-context
    // launches): with row_ss, each row's squared norm is added to
    // row_ss[r] and the row is stored unscaled if keep_rows, else not at
    // all; with row_scale, row r is scaled by row_scale[r] instead of being
    // normalised.
    const float *row_scale;
    float *row_ss;
    int32_t keep_rows;
};

// Kernel variant for an embedding layout.
struct Variant {
    int dtype;  // CLEORA_F32 / CLEORA_BF16
    int cpr;    // 16-byte vectors per embedding row
    int G;      // rows of T gathered at once per wave (groups of 64/G lanes)
    int VPL;    // 16-byte vectors per lane
    int cprf;   // float4 vectors per partial (float32) row
    int VPLF;   // float4 vectors per lane in the combine kernel
};
Variant choose_variant(int dtype, int ld);

// One context: the descriptor's fields become kernel arguments.
void launch_spmm(const Variant &v, const StepDesc &one, hipStream_t s);
// Several contexts: `descs` is a device table with wave_begin prefixes.
void launch_spmm_multi(const Variant &v, const StepDesc *descs, int n_desc, int64_t total_waves,
                       int32_t persist, hipStream_t s);
// One-time set-up of a persistent SpMM grid for this variant (no launch);
// ext: the instantiation with the column-block epilogues.
void prime_spmm(const Variant &v, int32_t persist, bool ext = false);
void launch_combine(const Variant &v, const StepDesc *descs, int n_desc, int64_t total_blocks,
                    hipStream_t s);
// T_0 for rows of one or more graphs (row0[g]..row0[g+1] use seeds[g] and
// local indices), or a single graph when n_graphs == 1 and row0 == nullptr.
// With ids != nullptr, row i uses global index ids[i] (chunks of a graph).
// max_blocks caps the grid (0: as many blocks as the work allows), so that
// the init can run beside other work instead of filling every CU.  With
// dfull > 0 the rows are columns [j0, j0 + dim) of a dfull-wide T_0 (entry
// (i, j0 + j) keyed by i * dfull + j0 + j).
void launch_init(int dtype, void *E, int64_t n, int32_t dim, int32_t ld, const int64_t *row0,
                 const uint64_t *seeds, int n_graphs, uint64_t seed0, hipStream_t s,
                 const int32_t *ids = nullptr, int64_t max_blocks = 0, int32_t dfull = 0,
                 int32_t j0 = 0);

// Hypergraph expansion (expand.hip).  expand_clique returns the edge count
// (and writes nothing when src is null).
int64_t expand_clique(int64_t n_hyper, const int64_t *offsets, const int32_t *members,
                      int32_t *src, int32_t *dst, int64_t capacity, DevBuf &scratch,
                      int64_t *h_total, hipStream_t s);
void expand_star(int64_t n_nodes, int64_t n_hyper, const int64_t *offsets,
                 const int32_t *members, int32_t *src, int32_t *dst, hipStream_t s);

// Chunks of a graph (chunked.hip).
void build_chunk(cleora_ctx *c, int64_t n_global, int64_t m, const int32_t *src,
                 const int32_t *dst, const float *w, uint32_t flags, hipStream_t s);
void launch_merge_rows(int dtype, const void *E, int64_t n, int32_t dim, int32_t ld,
                       const int32_t *ids, const float *occ, float *acc, int64_t ld_acc,
                       float *wsum, hipStream_t s);
void launch_merge_finish(const float *acc, int64_t ld_acc, const float *wsum, int64_t n,
                         int32_t dim, void *out, int64_t ld_out, int out_dtype, hipStream_t s);
void launch_widen_bf16(const void *src, int64_t n, int32_t dim, int32_t ld_src, float *dst,
                       int64_t ld_dst, hipStream_t s);

// Row-norm helpers of column slices (blocked.hip): x = 0; inv = 1/sqrt(ss)
// (0 for a zero row); row r of the n x ld float32 matrix E times inv[r].
void launch_fill_zero(float *x, int64_t n, hipStream_t s);
void launch_inv_norm(const float *ss, float *inv, int64_t n, hipStream_t s);
void launch_scale_rows(float *E, int64_t n, int32_t ld, const float *inv, hipStream_t s);
// dst row r = src row r * inv[r] (n x ld, float32 or bfloat16 rounded to
// nearest even, out of place).
void launch_scale_rows_to(int dtype, const void *src, void *dst, int64_t n, int32_t ld,
                          const float *inv, hipStream_t s);
// out[e] = val[e] * inv[col[e]]: the values of M diag(inv).
void launch_scale_values(const float *val, const int32_t *col, const float *inv, int64_t nnz,
                         float *out, hipStream_t s);

}  // namespace cleora

// ------------------------------------------------------------------- ctx

namespace cleora {
// A captured k-iteration loop and the launch parameters it was captured
// with: it is replayed only while they are unchanged, so rebuilding a graph
// of the same shape into the same buffers reuses it.
struct LoopGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> sig;
    hipEvent_t done = nullptr;  // recorded after every replay
    bool launched = false;
};
}  // namespace cleora

struct cleora_ctx {
    int device = 0;

    // graph (CSR of M)
    bool has_graph = false;
    int64_t n = 0, n_cols = 0, nnz = 0, m_in = 0;
    uint32_t flags = 0;
    cleora::DevBuf rp, col, val, deg;
    // a chunk of a larger graph: local row -> global node, entry counts
    bool is_chunk = false;
    int64_t n_global = 0;
    cleora::DevBuf chunk_ids, chunk_occ, t_local, t_expand;

    // embedding
    bool has_emb = false;
    int32_t dim = 0, dtype = 0, ld = 0, iteration = 0, cur = 0;
    cleora::DevBuf E[2];

    // schedule
    int32_t chunk_req = 0, chunk = 0, pack = 0, pack_req = 0;
    int32_t persist = 0, persist_req = -1;  // SpMM grid (StepDesc::persist); -1: not forced
    int64_t n_split = 0, n_buckets = 0, n_long = 0;
    cleora::DevBuf split_items, bucket_row, long_rows, chunk_base, partial, desc;
    // column-blocked form: per-row 1/norm of iterations 1..k, squared norms
    cleora::DevBuf blk_norms;
    // column slices of each iteration (0: whole rows): requested
    // width, width in use, the slices' combine descriptors,
    // squared norms and 1/norm per row, and the values of M diag(1/norm)
    // that the next iteration reads.  `deferred`: E[cur] holds the
    // normalised T_t and E[cur ^ 1] the unscaled rows it was scaled from,
    // with their factors in slice_norms (the next iteration reads those).
    int32_t slice_req = 0, slice_cols = 0;
    // CLEORA_SLICES_AUTO: the autotuner's choice (0: whole rows) and the
    // embedding layout it was measured on
    int32_t slice_auto = 0, slice_auto_dim = 0, slice_auto_dtype = -1;
    int32_t last_k = 0;  // iterations of the last cleora_propagate call
    bool deferred = false;
    cleora::DevBuf slice_desc, slice_norms, val2;

    // build temporaries (grow-only)
    cleora::DevBuf t_edges, t_wts, t_cnt, t_off, t_keys, t_tmp, t_head, t_pos, t_esum, t_lists,
        t_scan, t_small, multi_desc;
    int64_t *h_small = nullptr;  // pinned host mirror of t_small

    // per-graph status of the last cleora_embed_batch call
    std::vector<int32_t> batch_status;

    // captured k-iteration graphs, keyed by (k, starting parity, deferred)
    std::map<std::tuple<int32_t, int, bool>, cleora::LoopGraph> graphs;
    int64_t graph_instantiations = 0, graph_launches = 0;
    hipStream_t cap_stream = nullptr;
    // side stream of cleora_build_init (T_0 written during the build)
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // timing (eager launches between events from a reused pool)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_spmm, ev_comb;
    size_t ev_next = 0;
};

namespace cleora {
// CSR build from edges already in device memory (build_csr.hip).
// Rows [0, n) and columns [0, n_cols); undirected graphs need n_cols == n.
// With occ != nullptr, occ[r] receives row r's entry count before merging.
void build_graph(cleora_ctx *c, int64_t n, int64_t n_cols, int64_t m, const int32_t *src,
                 const int32_t *dst, const float *w, uint32_t flags, hipStream_t s,
                 float *occ = nullptr);
// Propagation schedule for the current graph and chunk (propagate.hip).
void plan_schedule(cleora_ctx *c, hipStream_t s);
// Packing size the autotuner chose for a graph of this shape, or 0.
int32_t tuned_pack(const cleora_ctx *c);
// SpMM grid the autotuner chose for a graph of this shape (0 by default).
int32_t tuned_persist(const cleora_ctx *c);
// Fill the two per-parity step descriptors of a context.
void write_descs(cleora_ctx *c, hipStream_t s);
StepDesc host_desc(const cleora_ctx *c, int parity);
// Column slice starting at column c0 (slice_cols wide, or to ld) of
// buffer `parity`: unscaled rows out, squared norms added to slice_norms.
StepDesc slice_desc(const cleora_ctx *c, int parity, int32_t c0);
// runtime.hip helpers shared with the server
void step_contexts(cleora_ctx *const *ctxs, int32_t n, hipStream_t s);
// Several graphs as one block-diagonal graph: their edges concatenated in
// device memory (local ids, rewritten in place), graph g owning edges
// [eoff[g], eoff[g+1]) and rows [row0[g], row0[g+1]) and seed seeds[g].
void build_group_and_init(cleora_ctx *c, int32_t n_graphs, int64_t n_total, int64_t m_total,
                          int32_t *src, int32_t *dst, const float *w, const int64_t *d_row0,
                          const int64_t *d_eoff, const uint64_t *d_seeds, uint32_t flags,
                          int32_t dim, int32_t dtype, hipStream_t s);
void set_last_error(const std::string &msg);
// cleora_propagate_rows: argument checks (throwing E_INVAL), and the work on
// a context whose buffers serve as scratch (synchronises s).
void check_rows_args(int64_t n_rows, int64_t n_cols, int64_t m, const int32_t *rows,
                     const int32_t *cols, const void *T_in, int64_t ld_in, int32_t dim,
                     int32_t dtype, const void *out, int64_t ld_out);
void propagate_rows_into(cleora_ctx *c, int64_t n_rows, int64_t n_cols, int64_t m,
                         const int32_t *rows, const int32_t *cols, const float *w,
                         const void *T_in, int32_t dim, int32_t dtype, void *out, int64_t ld_out,
                         hipStream_t s);
// Every device buffer of a context; their summed capacity; exact growth for
// all of them (the server's memory accounting); release all but the status
// words (the context then holds no graph and no embedding).
std::vector<DevBuf *> ctx_buffers(cleora_ctx *c);
int64_t ctx_device_bytes(cleora_ctx *c);
void set_exact_growth(cleora_ctx *c);
void release_buffers(cleora_ctx *c);
// Column-blocked T_k (blocked.hip): dim columns, `block` at a time, into
// out (row stride ld_out elements).  The context's graph stays; its
// embedding buffers are reused as block buffers.
void embed_blocked(cleora_ctx *c, int32_t dim, int32_t block, int32_t dtype, uint64_t seed,
                   int32_t k, void *out, int64_t ld_out, hipStream_t s);
}  // namespace cleora
