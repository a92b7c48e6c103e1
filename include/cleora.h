/*
 * cleora.h -- C ABI of the MI355X (gfx950) Cleora propagation library.
 *
 * The method (Rychalska et al., "Cleora: A Simple, Strong and Scalable Graph
 * Embedding Scheme", arXiv 2102.02302, Section 3.2 and Algorithm 1):
 *   M = D^-1 A, the random-walk transition matrix of a graph, with
 *       A[a][b] = e_ab (number of a->b edges, or the sum of their weights)
 *       and D[a] = sum_b A[a][b];
 *   T_0 ~ U(-1, 1), an N x d matrix;
 *   repeat I times: T_i = M . T_{i-1}, then L2-normalise every row of T_i.
 *
 * Conventions for every call below:
 *   - All functions return CLEORA_OK (0) or one of the CLEORA_E_* codes and
 *     never throw; cleora_last_error() gives a message for the calling thread.
 *   - "device pointer" means memory the GPU of the context can read or write
 *     (hipMalloc / torch CUDA tensors).  "stream" is a hipStream_t passed as
 *     void*; NULL means the default stream.  Work is queued on that stream;
 *     calls return before it finishes unless stated otherwise.
 *   - Input buffers must stay alive and unchanged until the stream has
 *     passed the call.  Everything the library allocates belongs to the
 *     context and is released by cleora_destroy.
 *   - A context is not thread-safe.  Separate contexts are independent.
 */
#ifndef CLEORA_H
#define CLEORA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define CLEORA_OK 0
#define CLEORA_E_INVAL 1  /* bad argument (null pointer, size out of range) */
#define CLEORA_E_STATE 2  /* call out of order (no graph, no embedding)    */
#define CLEORA_E_NOMEM 3  /* device allocation failed                      */
#define CLEORA_E_DEVICE 4 /* HIP runtime error                             */
#define CLEORA_E_INPUT 5  /* edge id outside [0, n) or weight not finite>0  */

/* ---------------------------------------------------------- data types */
#define CLEORA_F32 0  /* embeddings stored as float32                     */
#define CLEORA_BF16 1 /* stored as bfloat16 (round to nearest even);
                         products, sums and row norms are float32         */

/* ---------------------------------------------------------------- flags */
#define CLEORA_DIRECTED 1u   /* edge (a,b) counts only for a->b; default:
                                undirected, stored as a->b and b->a, a loop
                                {a,a} once (Section 3.2, Section 4.5)       */
#define CLEORA_EMPTY_KEEP 2u /* a node with no out-edges keeps its previous
                                row (normalised); default: its row becomes
                                zero, since row a of M is zero              */

/* Largest embedding dimension supported: 4096 (float32) / 8192 (bf16). */
#define CLEORA_MAX_DIM_F32 4096
#define CLEORA_MAX_DIM_BF16 8192

typedef struct cleora_ctx cleora_ctx;

/* Create a context on HIP device `device`.  *out receives the handle.
 * Errors: E_INVAL (out NULL), E_DEVICE (no such device). */
int cleora_create(cleora_ctx **out, int device);

/* Release the context and all device memory it owns.  Waits for work the
 * context queued.  NULL is ignored. */
void cleora_destroy(cleora_ctx *ctx);

/* Device bytes a context needs to embed a graph with n_nodes nodes and
 * n_edges input edges at the given dim and dtype (the memory model of
 * Section 4.5 -- one sparse matrix plus two N x d embedding buffers -- plus
 * the build and hub-row scratch of this implementation).  An upper bound
 * for whole-row iterations, used for admission decisions; column slices
 * (cleora_set_slices) add 4 bytes per stored entry and 8 per node.
 * Returns 0 for invalid arguments. */
size_t cleora_footprint_bytes(int64_t n_nodes, int64_t n_edges, uint32_t flags, int32_t dim,
                              int32_t dtype);

/* Build M = D^-1 A (Section 3.2) on the GPU from an edge list.
 *   n_nodes  number of nodes N, 1 <= N < 2^31
 *   n_edges  number of edges m >= 0 (m = 0 gives an empty graph)
 *   src,dst  device int32[m]: edge a->b is (src[e], dst[e]); ids in [0, N)
 *   w        device float32[m] weights (finite, > 0), or NULL: every edge
 *            counts 1
 *   flags    CLEORA_DIRECTED and/or CLEORA_EMPTY_KEEP
 * Result (owned by ctx): CSR with rows ascending, columns ascending within
 * a row, repeated pairs merged by summing (e_ab), D[a] summed in float64,
 * M values rounded to float32.  Replaces any previous graph and embedding.
 * Synchronises the stream once at the end (to size the result).
 * Errors: E_INVAL (sizes, null pointers), E_INPUT (an id out of range or a
 * bad weight; the context then holds no graph), E_NOMEM, E_DEVICE. */
int cleora_build_csr(cleora_ctx *ctx, int64_t n_nodes, int64_t n_edges, const int32_t *src,
                     const int32_t *dst, const float *w, uint32_t flags, void *stream);

/* Initialise T_0 (Section 3.2: T_0 ~ U(-1, 1)) for the current graph:
 *   T_0[i][j] = k / 2^23 - 1,  k = splitmix64(seed ^ splitmix64(i*dim + j)) >> 40
 * (SplitMix64 output function of Steele, Lea and Flood, 2014), exact in
 * float32, rounded to nearest even for CLEORA_BF16.  Also plans the
 * propagation schedule for this dim, which synchronises the stream.
 * Resets the iteration count to 0.
 * Errors: E_STATE (no graph), E_INVAL (dim < 1 or above the maximum, bad
 * dtype), E_NOMEM, E_DEVICE. */
int cleora_init(cleora_ctx *ctx, int32_t dim, int32_t dtype, uint64_t seed, void *stream);

/* cleora_build_csr + cleora_init in one call (Section 3.2: M, then T_0),
 * with T_0 written on an internal stream while the CSR is built on
 * `stream` (T_0 depends only on n_nodes, dim and the seed).  `stream`
 * waits for both before any later work on it.  Arguments, results and
 * errors as the two calls; on failure no embedding is left (E_STATE for
 * cleora_propagate until the next successful build and init). */
int cleora_build_init(cleora_ctx *ctx, int64_t n_nodes, int64_t n_edges, const int32_t *src,
                      const int32_t *dst, const float *w, uint32_t flags, int32_t dim,
                      int32_t dtype, uint64_t seed, void *stream);

/* Run k more iterations of Algorithm 1 (multiply by M, then L2-normalise
 * each row; a row whose product is exactly zero becomes zero, see
 * CLEORA_EMPTY_KEEP).  k = 0 does nothing.  Calls continue from the current
 * iteration: propagate(a) then propagate(b) equals propagate(a + b) bit for
 * bit.  Errors: E_INVAL (k < 0), E_STATE (no embedding), E_DEVICE. */
int cleora_propagate(cleora_ctx *ctx, int32_t k, void *stream);

/* T_k of the context's graph for an embedding too wide to keep two N x dim
 * buffers in device memory (graphs larger than HBM, Section 3.2 and the
 * paper's memory limits in Section 5): the result of cleora_init(dim,
 * dtype, seed) + cleora_propagate(k), computed `block` columns at a time.
 * Columns interact only through the row norms, so pass t = 1..k runs each
 * block of T_0 through the t - 1 known row scalings and sums its share of
 * the squared row norms of iteration t; a final pass writes each block of
 * T_k.  Cost: k(k+1)/2 + k block iterations over dim/block blocks
 * (k iterations for the whole width otherwise).  Device memory: two
 * N x block embedding buffers, (k + 1) N floats and the schedule.
 *   block   columns per block, >= 1 (block >= dim: one block)
 *   out     N x dim (dtype), row stride ld_out >= dim elements; device or
 *           host memory (pinned for speed); written block by block
 * Results: T_0 entries are the same as cleora_init's (keyed by the full
 * width); every iteration differs from the unblocked one in float32
 * rounding only (a narrower block may gather several entries at once in
 * lane groups, and each squared norm is summed block by block), and with a
 * single block the result is bit-identical to init + propagate.  Rows
 * follow the graph's CLEORA_EMPTY_KEEP flag.  The context keeps its graph
 * and holds no embedding afterwards (E_STATE for cleora_propagate until
 * the next cleora_init).  Synchronises `stream`.
 * Errors: E_INVAL (NULL, dim/dtype, block < 1, k < 0, ld_out < dim),
 * E_STATE (no graph), E_NOMEM, E_DEVICE. */
int cleora_embed_blocked(cleora_ctx *ctx, int32_t dim, int32_t block, int32_t dtype, uint64_t seed,
                         int32_t k, void *out, int64_t ld_out, void *stream);

/* Free device memory the context keeps only for reuse by later calls: the
 * CSR build's temporaries (about 40 bytes per stored entry) always, and,
 * when the context holds no embedding (after cleora_embed_blocked, before
 * the first init, after a failed one), its embedding, schedule and
 * column-blocked buffers.  The graph (CSR, M values, degrees, a chunk's
 * nodes) and a current embedding stay usable; later calls allocate again
 * what they need.  Meant for graphs near the device's capacity, e.g.
 * between cleora_build_csr and cleora_embed_blocked.  Waits for all work on
 * the device.  Errors: E_INVAL (NULL), E_DEVICE. */
int cleora_release_scratch(cleora_ctx *ctx);

/* Copy the current N x dim embedding into dst (device or host memory; a
 * host destination should be pinned) with a row stride of ld elements
 * (ld >= dim).  dst_dtype must equal the context dtype, or be CLEORA_F32
 * for a CLEORA_BF16 context (widened on the GPU; device dst only).
 * Errors: E_STATE, E_INVAL, E_DEVICE. */
int cleora_get_embedding(cleora_ctx *ctx, void *dst, int64_t ld, int32_t dst_dtype, void *stream);

/* Device pointer and row stride (elements) of the current embedding
 * buffer; valid until the next propagate, init, build or destroy. */
int cleora_embedding_ptr(cleora_ctx *ctx, const void **ptr, int64_t *ld);

/* Device pointer and row stride of T_{t-1}, the embedding one iteration
 * before the current one (the other ping-pong buffer), valid while the
 * current iteration is >= 1 and until the next propagate, init, build or
 * destroy.  Errors: E_STATE (no embedding, or iteration 0). */
int cleora_previous_embedding_ptr(cleora_ctx *ctx, const void **ptr, int64_t *ld);

/* One iteration of Algorithm 1 for a set of rows against a given
 * embedding -- the paper's creation of embeddings for nodes added after
 * the graph was embedded (Section 3.2): each new node is the normalised
 * weighted average of its neighbours' rows, ideally taken from iteration
 * I-1.  Chaining calls (feeding new rows back in as columns) gives the
 * 2-hop reconstruction of Section 5.
 *   work      a context used as scratch (its graph and embedding are
 *             replaced)
 *   n_rows    number of new nodes R >= 1; n_cols: rows of T_in, C >= 1
 *   n_edges   m >= 0 edges rows[e] -> cols[e] (device int32, rows in
 *             [0, R), cols in [0, C)); w: device float32 weights or NULL
 *   T_in      device C x ld_in embedding (dtype), ld_in = dim rounded up to
 *             a multiple of 16 bytes (the library's own layout); padding
 *             elements must be zero
 *   out       device or host R x ld_out (dtype), ld_out >= dim
 * A row without edges becomes zero.  Result bit-identical to the matching
 * row of cleora_propagate over a graph holding the same edges.
 * Errors: E_INVAL, E_INPUT (ids out of range, bad weights), E_NOMEM,
 * E_DEVICE. */
int cleora_propagate_rows(cleora_ctx *work, int64_t n_rows, int64_t n_cols, int64_t n_edges,
                          const int32_t *rows, const int32_t *cols, const float *w,
                          const void *T_in, int64_t ld_in, int32_t dim, int32_t dtype, void *out,
                          int64_t ld_out, void *stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation):
 * cleora_propagate_rows without a context.  Arguments, result and errors
 * as cleora_propagate_rows, on HIP device `device`, within these limits:
 * n_rows <= CLEORA_NOALLOC_MAX_ROWS, n_edges <= CLEORA_NOALLOC_MAX_EDGES
 * and a row of T_in (ld_in elements) at most CLEORA_NOALLOC_MAX_ROW_BYTES;
 * above them it returns E_INVAL and does nothing.  It allocates no device
 * memory: its scratch (CSR build, schedule, partial sums, staging of the
 * rows) is a static device array of about 80 MB that every GPU the library
 * runs on holds until the process ends.  All calls on one GPU share that
 * array, so calls that overlap on one GPU (from several threads or
 * streams) race; each call synchronises `stream` before it returns, which
 * also makes it unsuitable for stream capture.  Errors: as
 * cleora_propagate_rows; E_DEVICE for a bad device. */
#define CLEORA_NOALLOC_MAX_ROWS 8192
#define CLEORA_NOALLOC_MAX_EDGES 524288
#define CLEORA_NOALLOC_MAX_ROW_BYTES 4096
int cleora_propagate_rows_noalloc(int device, int64_t n_rows, int64_t n_cols, int64_t n_edges,
                                  const int32_t *rows, const int32_t *cols, const float *w,
                                  const void *T_in, int64_t ld_in, int32_t dim, int32_t dtype,
                                  void *out, int64_t ld_out, void *stream);

/* Copy the built CSR into caller device buffers: row_ptr int64[N+1],
 * col int32[nnz], val float32[nnz] (M values), deg float64[N] (D).  Any of
 * them may be NULL.  Sizes come from cleora_info.  Errors: E_STATE. */
int cleora_get_csr(cleora_ctx *ctx, int64_t *row_ptr, int32_t *col, float *val, double *deg,
                   void *stream);

/* Sizes and state: any pointer may be NULL. */
int cleora_info(cleora_ctx *ctx, int64_t *n_nodes, int64_t *nnz, int32_t *dim, int32_t *dtype,
                int32_t *iteration);

/* Propagation schedule planned by the last cleora_init: split size, number
 * of split pieces, rows split into pieces (finished by the combine step),
 * packed work items, packing size, SpMM grid (0: one wave per work item,
 * m: m x the resident waves), column-slice width (0: whole rows).  Any
 * pointer may be NULL.  Errors: E_STATE (no embedding). */
int cleora_schedule_info(cleora_ctx *ctx, int32_t *chunk, int64_t *n_split_chunks,
                         int64_t *n_split_rows, int64_t *n_packed_items, int32_t *pack,
                         int32_t *persistent, int32_t *slice_cols);

/* Wait for the stream.  Errors: E_DEVICE. */
int cleora_sync(cleora_ctx *ctx, void *stream);

/* Per-context tuning: split size of the SpMM -- rows with more entries are
 * split into pieces of this many entries whose partial sums are added in a
 * fixed order (the packing of shorter rows into work items adapts to the
 * graph by itself).  It fixes the float32 summation order of long rows, so
 * contexts that must agree bit for bit must use the same value.  0
 * restores the default, 512 entries for every graph and layout.  Takes
 * effect at the next cleora_init.
 * Errors: E_INVAL (chunk < 0 or > 2^20). */
int cleora_set_chunk(cleora_ctx *ctx, int32_t chunk);

/* Column slices of the iterations, taking effect at the next cleora_init,
 * cleora_build_init or cleora_embed_batch on this context: cols = 0 (the
 * default) keeps whole rows, cols > 0 slices `cols` wide (rounded up to
 * 16 bytes for CLEORA_BF16; at least the padded row width: whole rows).
 * Each slice's SpMM gathers that part of the neighbour rows (a narrower
 * gather keeps more of the most-used rows of T in cache), stores its rows
 * unscaled and adds its share of each row's squared norm (Section 3.2's
 * normalisation is over the whole row).  The next iteration multiplies by
 * M diag(1/norm) (M's values scaled per column, one pass over them)
 * instead of scaling the rows, and each cleora_propagate call ends by
 * writing the normalised T_k out of place; the unscaled rows stay for the
 * next call.  Results differ from whole rows in rounding only (with
 * CLEORA_BF16 the stored rows are unscaled bfloat16 and T_k is rounded
 * once more when it is written); propagate resumption, graph replay and
 * batch = solo (with the same setting) hold bit for bit.  While the
 * unscaled rows are kept, T_{t-1} is not: cleora_previous_embedding_ptr
 * returns E_STATE.  cleora_step_multi steps whole rows from the normalised
 * T_t, and cleora_autotune's trial steps discard the unscaled rows: the
 * context continues from the normalised T_t.  cleora_propagate_rows uses
 * whole rows.
 * cols = CLEORA_SLICES_AUTO: whole rows until cleora_autotune has measured,
 * on this context's embedding and in this process, one whole-row iteration
 * against one iteration in slices of 1 KiB and of 512 bytes (256 and 128
 * float32, or 512 and 256 bfloat16 columns), each plus the final
 * out-of-place scaling spread over the iterations of the context's last
 * cleora_propagate call (4 if none), and kept the fastest slicing only if
 * it is at least 1% faster than whole rows (the choice is not
 * cached across processes: on large embeddings the time of both forms
 * depends on where the two buffers landed in physical memory); a later
 * cleora_init with another dim or dtype returns to whole rows until the
 * next cleora_autotune.  cleora_schedule_info reports the width in use.
 * Errors: E_INVAL (cols < -1, not a multiple of 4, or above 8192). */
#define CLEORA_SLICES_AUTO (-1)
int cleora_set_slices(cleora_ctx *ctx, int32_t cols);

/* Fix the propagation schedule instead of the autotuned or default one
 * (takes effect at the next cleora_init; cleora_autotune clears it).
 * pack: entries per work item for rows that are not split (0: automatic,
 * else 16 .. 2^20, capped at the split size).  persistent: SpMM grid (-1:
 * automatic, 0: one wave per work item, m in 1..8: m x the resident waves,
 * each looping over work items).  Neither changes results.
 * Errors: E_INVAL (out of range). */
int cleora_set_schedule(cleora_ctx *ctx, int32_t pack, int32_t persistent);

/* Autotuner: time one SpMM + combine step of the current embedding with
 * each candidate schedule and keep the fastest for this graph.  Candidates:
 * packing size (entries per work item for rows that are not split: 16 ..
 * the split size, powers of two) x SpMM grid (one wave per work item, or a
 * persistent grid of the resident waves, each looping over work items).
 * The choice never changes results -- only which wave handles which rows
 * -- and the embedding and iteration count are left as they were.
 * Choices are cached per (N, nnz, dim, dtype, split size) for the life of
 * the process, and every later cleora_init of a graph of that shape, in
 * any context, uses the cached choice.  With the environment variable
 * CLEORA_TUNE_CACHE naming a file, choices are also read from that file
 * (once per process, also by inits that never call the autotuner) and
 * each new choice is appended to it, one text line per graph shape.  With
 * cleora_set_slices(ctx, CLEORA_SLICES_AUTO) it then also chooses between
 * whole rows and column slices (see there).  Outputs (may be NULL): the
 * chosen packing size, 1 if the persistent grid won (else 0), and the time
 * per step in ms (whole rows).  Errors: E_STATE (no embedding), E_DEVICE. */
int cleora_autotune(cleora_ctx *ctx, int32_t *pack, int32_t *persistent, float *step_ms,
                    void *stream);

/* Kernel timing for measurement: when on, the library launches every
 * iteration eagerly (not as a captured graph: events recorded inside a
 * graph carry no time) and records HIP events around every SpMM+normalise
 * and combine launch on the launch stream, accumulating their durations;
 * cleora_kernel_time returns the total milliseconds and the number of
 * launches timed since the last reset (and resets).  The kernels and their
 * arguments are those of the captured graph. */
int cleora_set_timing(cleora_ctx *ctx, int on);
int cleora_kernel_time(cleora_ctx *ctx, double *spmm_ms, int64_t *spmm_launches,
                       double *combine_ms, int64_t *combine_launches);

/* Launch statistics since the context was created: captured k-iteration
 * graphs instantiated, and graph replays.  k >= 2 iterations (without
 * timing) run as one captured graph, kept per (k, starting buffer) together
 * with the launch parameters it was captured with; a later call replays it
 * whenever those are unchanged (e.g. a graph of the same shape rebuilt into
 * the same buffers) and captures anew otherwise.  Any pointer may be NULL.
 * Errors: E_INVAL (NULL ctx). */
int cleora_launch_stats(cleora_ctx *ctx, int64_t *graph_instantiations, int64_t *graph_launches);

/* ------------------------------------------------ hypergraph expansion */

/* Section 3.2 breaks every hyperedge into ordinary edges before embedding.
 * Hyperedges come in CSR form on the device: hyperedge h has members
 * members[offsets[h] .. offsets[h+1]) (int64 offsets, int32 node ids).
 * The edges are written to src/dst (device int32, `capacity` entries) in a
 * fixed order, hyperedge by hyperedge; pass src = NULL to get only the
 * count in *n_edges.  Feed the result to cleora_build_csr as an undirected
 * graph.  `ctx` provides the device and scratch memory (its graph and
 * embedding are kept).  Both synchronise the stream.
 *
 * Clique expansion: every pair (m_i, m_j), i < j, of a hyperedge with k
 * members: k(k-1)/2 edges; a member listed twice yields a loop.
 * Errors: E_INVAL (sizes, capacity below the count), E_DEVICE. */
int cleora_expand_clique(cleora_ctx *ctx, int64_t n_hyper, const int64_t *offsets,
                         const int32_t *members, int32_t *src, int32_t *dst, int64_t capacity,
                         int64_t *n_edges, void *stream);

/* Star expansion: hyperedge h becomes a new node n_nodes + h linked to each
 * of its members: k edges per hyperedge, n_nodes + n_hyper nodes in all
 * (must stay below 2^31).  Errors: as above. */
int cleora_expand_star(cleora_ctx *ctx, int64_t n_nodes, int64_t n_hyper, const int64_t *offsets,
                       const int32_t *members, int32_t *src, int32_t *dst, int64_t capacity,
                       int64_t *n_edges, void *stream);

/* ------------------------------------------ chunks (Algorithm 1 merge) */

/* Graphs processed in Q chunks (Algorithm 1): each chunk is an edge subset
 * embedded on the nodes it touches, and the chunk embeddings are merged
 * per node with weights w_qv = occurrences of v in chunk q / occurrences of
 * v in all chunks (occurrences = the node's stored entries before repeated
 * pairs are merged).
 *
 * cleora_build_chunk: like cleora_build_csr for the edges of one chunk of a
 * graph with n_global nodes (ids in [0, n_global)), but the CSR covers only
 * the touched nodes, numbered in increasing global id; the next
 * cleora_init keys each row's T_0 by its *global* id, so all chunks start
 * from the same vectors.  Errors: as cleora_build_csr; E_INVAL for a chunk
 * without edges. */
int cleora_build_chunk(cleora_ctx *ctx, int64_t n_global, int64_t n_edges, const int32_t *src,
                       const int32_t *dst, const float *w, uint32_t flags, void *stream);

/* Touched nodes of the chunk: *n_local, and optionally (device buffers of
 * n_local entries) their global ids and occurrence counts.
 * Errors: E_STATE (not a chunk). */
int cleora_chunk_info(cleora_ctx *ctx, int64_t *n_local, int32_t *ids, float *occ,
                      void *stream);

/* acc[v][j] += occ(v) * T[v][j] and wsum[v] += occ(v) for every touched
 * node v of the chunk (current embedding of ctx).  acc: device float32
 * n_global x ld_acc (ld_acc >= dim), wsum: device float32[n_global], both
 * zeroed by the caller before the first chunk.  Chunks merged on one stream
 * one after another give deterministic sums.  Errors: E_STATE, E_INVAL. */
int cleora_merge_chunk(cleora_ctx *ctx, float *acc, int64_t ld_acc, float *wsum, void *stream);

/* out[v] = acc[v] / wsum[v] (zero where wsum is 0), n_global x dim into out
 * (device, row stride ld_out, CLEORA_F32 or CLEORA_BF16) on `device`.
 * Errors: E_INVAL, E_DEVICE. */
int cleora_merge_finish(int device, const float *acc, int64_t ld_acc, const float *wsum,
                        int64_t n_global, int32_t dim, void *out, int64_t ld_out,
                        int32_t out_dtype, void *stream);

/* ------------------------------------------------------ batched form */

/* One graph of a batch.  Pointers are device pointers as in
 * cleora_build_csr; seed keys that graph's T_0 by its own node indices, so
 * a graph embeds to the same bits alone or in any batch. */
typedef struct {
    int64_t n_nodes;
    int64_t n_edges;
    const int32_t *src;
    const int32_t *dst;
    const float *w; /* NULL: unweighted */
    uint64_t seed;
} cleora_graph;

/* Embed n_graphs independent graphs as one block-diagonal graph: one CSR
 * build, one T_0 initialisation and k iterations over all of them at once
 * (Algorithm 1 per graph: a block-diagonal M propagates each block on its
 * own).  Besides unrelated graphs, this embeds the separate sparse matrix
 * the paper builds for every pair of entity columns of a relation
 * (Sections 4.2-4.3) in one call.
 * out[g] is a device float32/bf16 (per dtype) buffer of graphs[g].n_nodes x
 * dim elements, row stride dim.  The context's graph and embedding are
 * replaced by the block-diagonal ones.  Errors: as build/init/propagate;
 * any failure writes no output. */
int cleora_embed_batch(cleora_ctx *ctx, int32_t n_graphs, const cleora_graph *graphs,
                       uint32_t flags, int32_t dim, int32_t dtype, int32_t k, void *const *out,
                       void *stream);

/* Per-graph status of the last cleora_embed_batch call on this context
 * (n_graphs entries into host memory `status`): after a call that failed
 * with E_INPUT, CLEORA_E_INPUT for each graph with an id outside [0,
 * n_nodes) or a weight that is not finite and positive (found by a host
 * check of the edge arrays), CLEORA_OK for the others, which can be
 * submitted again without the bad ones; after a call that failed with
 * another error, that code for every graph; after a successful call,
 * CLEORA_OK for every graph.  Errors: E_INVAL (NULL, n_graphs not the last
 * call's count), E_STATE (no batch call yet). */
int cleora_batch_status(cleora_ctx *ctx, int32_t n_graphs, int32_t *status);

/* Continuous batching: advance each of n contexts (each with an embedding,
 * all with the same dim and dtype) by ONE iteration, every context's rows
 * in the same kernel launches.  Each context's result is bit-identical to
 * cleora_propagate(ctx, 1).  Errors: E_INVAL (mixed dim/dtype, n < 0),
 * E_STATE, E_DEVICE. */
int cleora_step_multi(cleora_ctx *const *ctxs, int32_t n, void *stream);

/* ------------------------------------------------------- served form */

/* A native request server on one device: continuous batching of
 * independent graphs.  Requests are admitted in submission order, as groups
 * of up to max_group requests, when a builder thread is free, a slot (a
 * context with its staging buffer) is free and the device memory charged
 * to the slots stays within budget_bytes (groups grow with the backlog).
 * A request's charge is its cleora_footprint_bytes plus 12 bytes per edge
 * (and 1 KiB) of staging.  Slots keep their buffers between groups: an
 * idle or running slot is charged what its buffers hold, a building slot
 * that plus its group's charge (slot buffers grow to the exact size asked
 * for), and idle slots release their buffers, largest first, when a group
 * needs the room.
 * Builder threads pack a group's edges into pinned staging,
 * copy them to the device once and build the group as one block-diagonal
 * graph (its CSR and T_0, each member's T_0 rows keyed by its own seed and
 * local ids) on their own streams, while built groups advance one
 * iteration per step, all of them in shared launches (as
 * cleora_step_multi).  A group that reached k iterations is copied out,
 * member by member, to the `out` buffers asynchronously and its slot reused
 * after the copies.  Every result is bit-identical to the same graph
 * embedded alone with cleora_build_csr + cleora_init + cleora_propagate
 * (Section 3.2: a block-diagonal M propagates each block independently;
 * the kernels compute each row the same way whatever else is in the
 * graph).  A group whose build fails on bad input is checked member by
 * member on the host: the bad members complete with E_INPUT, the rest are
 * rebuilt and served. */
typedef struct cleora_server cleora_server;

typedef struct {
    int64_t n_nodes;
    int64_t n_edges;
    const int32_t *src; /* host or device memory, unchanged until completion */
    const int32_t *dst;
    const float *w;     /* NULL: unweighted */
    uint64_t seed;
    void *out;          /* n_nodes x dim (server dtype), row stride dim; device or
                           pinned host memory, written when the request completes */
} cleora_request;

typedef struct {
    int64_t ticket;
    int32_t status;     /* CLEORA_OK or the build's error code (e.g. E_INPUT) */
    double submit_s;    /* seconds since the server was created */
    double admit_s;
    double ready_s;
    double done_s;      /* the result is in `out` */
} cleora_completion;

/* slots: contexts (groups in flight); budget_bytes: most device memory
 * charged to the slots (0: 80% of the device memory free at creation);
 * builders: build threads; max_group: most requests built together (1:
 * every request on its own).  flags: CLEORA_DIRECTED / CLEORA_EMPTY_KEEP
 * for every request.  Errors: E_INVAL (dim outside [1, CLEORA_MAX_DIM_*]
 * for the dtype, other bad parameters), E_DEVICE, E_NOMEM. */
int cleora_server_create(cleora_server **out, int device, int32_t dim, int32_t dtype, int32_t k,
                         int32_t slots, int64_t budget_bytes, int32_t builders, int32_t max_group,
                         uint32_t flags);
/* Thread-safe; returns at once.  Errors: E_INVAL (sizes, a footprint above
 * the whole budget), E_DEVICE (the server stopped after a device error). */
int cleora_server_submit(cleora_server *s, const cleora_request *req, int64_t *ticket);
/* Up to max completions (waiting up to wait_s seconds when none is ready). */
int cleora_server_poll(cleora_server *s, cleora_completion *out, int32_t max, int32_t *n_out,
                       double wait_s);
/* Steps run, request-steps run, most groups in one step, peak charged
 * device memory, groups built, requests submitted and not yet polled.  Any
 * output pointer may be NULL. */
int cleora_server_stats(cleora_server *s, int64_t *steps, int64_t *stepped, int32_t *max_active,
                        int64_t *peak_bytes, int64_t *groups, int64_t *in_system);
/* Memory accounting: the budget, the bytes charged now and at most so far
 * (the slots' buffers plus the charges of groups being built), and the
 * number of builds after which a slot held more than it was charged (0
 * unless a footprint failed to bound a build).  Any output may be NULL.
 * Errors: E_INVAL (NULL server). */
int cleora_server_memory(cleora_server *s, int64_t *budget, int64_t *charged, int64_t *peak,
                         int64_t *bound_exceeded);
/* Seconds since the server was created (the clock of the completions). */
double cleora_server_now(cleora_server *s);
/* Stops the threads (requests not yet completed are dropped) and frees
 * everything.  No other call on the same server may be in progress or
 * start afterwards (submit, poll and stats are thread-safe among
 * themselves, not against destroy).  NULL is ignored. */
void cleora_server_destroy(cleora_server *s);

/* Message for the last error on this thread ("" if none). */
const char *cleora_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLEORA_H */
