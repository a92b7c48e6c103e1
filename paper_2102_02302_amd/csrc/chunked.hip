// Graphs larger than one pass: Algorithm 1's chunks.  The edge set is split
// into Q chunks; each chunk is embedded on its own nodes (the nodes its
// edges touch, numbered locally), with T_0 rows keyed by the *global* node
// id so that every chunk starts from the same vectors; the chunk
// embeddings are then merged per node with weights w_qv = (occurrences of
// v in chunk q) / (occurrences of v in all chunks).
//
// build_chunk: flag the touched nodes, scan to local ids, relabel the
// edges, then the ordinary CSR build, which also counts each row's entries
// before merging (the node's occurrences in the chunk).
// k_merge_rows: acc[global(i)] += occ[i] * T[i], wsum[global(i)] += occ[i]
// (one wave per row; rows of one chunk touch distinct global rows, chunks
// are merged one after another, so the sums are deterministic).
// k_merge_finish: T[v] = acc[v] / wsum[v] (zero for untouched nodes).
#include "internal.hpp"

#include <algorithm>

namespace cleora {

namespace {

unsigned grid_for(int64_t items, int threads, int64_t cap = 1 << 16)
{
    int64_t g = ceil_div(items > 0 ? items : 1, threads);
    return (unsigned)std::min<int64_t>(g, cap);
}

__global__ void k_mark_used(int64_t m, const int32_t *__restrict__ src,
                            const int32_t *__restrict__ dst, int64_t n_global,
                            uint8_t *__restrict__ used)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = src[e], b = dst[e];
        if (a >= 0 && a < n_global) used[a] = 1;
        if (b >= 0 && b < n_global) used[b] = 1;
    }
}

__global__ void k_relabel(int64_t m, const int32_t *__restrict__ src,
                          const int32_t *__restrict__ dst, int64_t n_global,
                          const int64_t *__restrict__ lid, int32_t *__restrict__ lsrc,
                          int32_t *__restrict__ ldst)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = src[e], b = dst[e];
        // an id outside [0, n_global) stays invalid for the build to report
        lsrc[e] = (a >= 0 && a < n_global) ? (int32_t)lid[a] : -1;
        ldst[e] = (b >= 0 && b < n_global) ? (int32_t)lid[b] : -1;
    }
}

__global__ void k_local_ids(int64_t n_global, const uint8_t *__restrict__ used,
                            const int64_t *__restrict__ lid, int32_t *__restrict__ ids)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n_global;
         v += (int64_t)gridDim.x * blockDim.x)
        if (used[v]) ids[lid[v]] = (int32_t)v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_merge_rows(const T *__restrict__ E, int64_t n,
                                                    int32_t dim, int32_t ld,
                                                    const int32_t *__restrict__ ids,
                                                    const float *__restrict__ occ,
                                                    float *__restrict__ acc, int64_t ld_acc,
                                                    float *__restrict__ wsum)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const int64_t g = ids[row];
    const float w = occ[row];
    for (int32_t j = lane; j < dim; j += 64) {
        float x;
        if constexpr (sizeof(T) == 4) x = E[row * ld + j];
        else x = __uint_as_float((uint32_t)E[row * ld + j] << 16);
        acc[g * ld_acc + j] = fmaf(w, x, acc[g * ld_acc + j]);
    }
    if (lane == 0) wsum[g] += w;
}

__global__ void k_merge_finish(const float *__restrict__ acc, int64_t ld_acc,
                               const float *__restrict__ wsum, int64_t n, int32_t dim,
                               void *__restrict__ out, int64_t ld_out, int out_dtype)
{
    const int64_t total = n * dim;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = idx / dim;
        const int32_t j = (int32_t)(idx - v * dim);
        const float s = wsum[v];
        const float x = s > 0.0f ? acc[v * ld_acc + j] / s : 0.0f;
        if (out_dtype == CLEORA_BF16)
            reinterpret_cast<uint16_t *>(out)[v * ld_out + j] = (uint16_t)f32_to_bf16_rne(x);
        else
            reinterpret_cast<float *>(out)[v * ld_out + j] = x;
    }
}

}  // namespace

void build_chunk(cleora_ctx *c, int64_t n_global, int64_t m, const int32_t *src,
                 const int32_t *dst, const float *w, uint32_t flags, hipStream_t s)
{
    c->is_chunk = false;
    const int64_t m1 = std::max<int64_t>(m, 1);
    c->t_head.ensure((size_t)n_global);
    c->t_pos.ensure(sizeof(int64_t) * ((size_t)n_global + 1));
    c->t_scan.ensure(sizeof(int64_t) * scan_workspace_elems(n_global + 1));
    c->t_local.ensure(2 * sizeof(int32_t) * (size_t)m1);
    uint8_t *used = c->t_head.as<uint8_t>();
    int64_t *lid = c->t_pos.as<int64_t>();
    int32_t *lsrc = c->t_local.as<int32_t>(), *ldst = lsrc + m1;
    CLEORA_HIP(hipMemsetAsync(used, 0, (size_t)n_global, s));
    if (m > 0) {
        k_mark_used<<<grid_for(m, 256), 256, 0, s>>>(m, src, dst, n_global, used);
        CLEORA_LAUNCH_CHECK();
    }
    exclusive_scan(used, n_global, lid, c->t_scan.as<int64_t>(), s);
    CLEORA_HIP(hipMemcpyAsync(c->h_small + 4, lid + n_global, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    CLEORA_HIP(hipStreamSynchronize(s));
    const int64_t n_local = c->h_small[4];
    if (n_local < 1) throw Error(CLEORA_E_INVAL, "a chunk needs at least one edge");
    c->chunk_ids.ensure(sizeof(int32_t) * (size_t)n_local);
    c->chunk_occ.ensure(sizeof(float) * (size_t)n_local);
    k_local_ids<<<grid_for(n_global, 256), 256, 0, s>>>(n_global, used, lid,
                                                       c->chunk_ids.as<int32_t>());
    CLEORA_LAUNCH_CHECK();
    k_relabel<<<grid_for(m, 256), 256, 0, s>>>(m, src, dst, n_global, lid, lsrc, ldst);
    CLEORA_LAUNCH_CHECK();
    build_graph(c, n_local, n_local, m, lsrc, ldst, w, flags, s, c->chunk_occ.as<float>());
    c->is_chunk = true;
    c->n_global = n_global;
}

void launch_merge_rows(int dtype, const void *E, int64_t n, int32_t dim, int32_t ld,
                       const int32_t *ids, const float *occ, float *acc, int64_t ld_acc,
                       float *wsum, hipStream_t s)
{
    const unsigned blocks = (unsigned)ceil_div(n, 4);
    if (dtype == CLEORA_BF16)
        k_merge_rows<uint16_t><<<blocks, 256, 0, s>>>(reinterpret_cast<const uint16_t *>(E), n,
                                                      dim, ld, ids, occ, acc, ld_acc, wsum);
    else
        k_merge_rows<float><<<blocks, 256, 0, s>>>(reinterpret_cast<const float *>(E), n, dim,
                                                   ld, ids, occ, acc, ld_acc, wsum);
    CLEORA_LAUNCH_CHECK();
}

void launch_merge_finish(const float *acc, int64_t ld_acc, const float *wsum, int64_t n,
                         int32_t dim, void *out, int64_t ld_out, int out_dtype, hipStream_t s)
{
    k_merge_finish<<<grid_for(n * dim, 256), 256, 0, s>>>(acc, ld_acc, wsum, n, dim, out, ld_out,
                                                          out_dtype);
    CLEORA_LAUNCH_CHECK();
}

}  // namespace cleora
