// Hypergraph expansion (Section 3.2): every hyperedge becomes ordinary edges
// before embedding.
//   clique: all pairs (m_i, m_j), i < j, of the hyperedge's member list;
//           k members give k(k-1)/2 edges (undirected);
//   star:   a new node n_nodes + h for hyperedge h, linked to each member;
//           k members give k edges.
// Hyperedges are given in CSR form: offsets[h] .. offsets[h+1] index
// `members`.  Output positions come from an exclusive scan of the per-
// hyperedge edge counts, so the edge order is fixed: hyperedge by
// hyperedge, and within a clique row by row (i, then j).  A member listed
// twice in one hyperedge yields a loop, as the Cartesian product does.
#include "internal.hpp"

#include <algorithm>

namespace cleora {

namespace {

__global__ void k_clique_counts(int64_t n_hyper, const int64_t *__restrict__ offsets,
                                int64_t *__restrict__ counts)
{
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < n_hyper;
         h += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = offsets[h + 1] - offsets[h];
        counts[h] = k * (k - 1) / 2;
    }
}

// One wave per hyperedge: row i of the pair triangle, lanes over j > i.
__global__ __launch_bounds__(256) void k_clique_emit(int64_t n_hyper,
                                                     const int64_t *__restrict__ offsets,
                                                     const int32_t *__restrict__ members,
                                                     const int64_t *__restrict__ out_off,
                                                     int32_t *__restrict__ src,
                                                     int32_t *__restrict__ dst)
{
    const int64_t h = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (h >= n_hyper) return;
    const int lane = threadIdx.x & 63;
    const int64_t b = offsets[h], k = offsets[h + 1] - b, o = out_off[h];
    for (int64_t i = 0; i + 1 < k; ++i) {
        const int32_t a = members[b + i];
        const int64_t row = o + i * k - i * (i + 1) / 2;  // pairs before row i
        for (int64_t j = i + 1 + lane; j < k; j += 64) {
            src[row + (j - i - 1)] = a;
            dst[row + (j - i - 1)] = members[b + j];
        }
    }
}

__global__ __launch_bounds__(256) void k_star_emit(int64_t n_nodes, int64_t n_hyper,
                                                   const int64_t *__restrict__ offsets,
                                                   const int32_t *__restrict__ members,
                                                   int32_t *__restrict__ src,
                                                   int32_t *__restrict__ dst)
{
    const int64_t h = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (h >= n_hyper) return;
    const int lane = threadIdx.x & 63;
    const int64_t b = offsets[h], e = offsets[h + 1];
    for (int64_t p = b + lane; p < e; p += 64) {
        src[p - offsets[0]] = (int32_t)(n_nodes + h);
        dst[p - offsets[0]] = members[p];
    }
}

}  // namespace

int64_t expand_clique(int64_t n_hyper, const int64_t *offsets, const int32_t *members,
                      int32_t *src, int32_t *dst, int64_t capacity, DevBuf &scratch,
                      int64_t *h_total, hipStream_t s)
{
    scratch.ensure(sizeof(int64_t) * (2 * (size_t)n_hyper + 1 + scan_workspace_elems(n_hyper)));
    int64_t *counts = scratch.as<int64_t>(), *out_off = counts + n_hyper,
            *ws = out_off + n_hyper + 1;
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(std::max<int64_t>(n_hyper, 1), 256), 65536);
    k_clique_counts<<<g, 256, 0, s>>>(n_hyper, offsets, counts);
    CLEORA_LAUNCH_CHECK();
    exclusive_scan(counts, n_hyper, out_off, ws, s);
    CLEORA_HIP(hipMemcpyAsync(h_total, out_off + n_hyper, sizeof(int64_t), hipMemcpyDeviceToHost,
                              s));
    CLEORA_HIP(hipStreamSynchronize(s));
    const int64_t total = *h_total;
    if (!src) return total;  // size query
    if (total > capacity) throw Error(CLEORA_E_INVAL, "output capacity below the edge count");
    if (n_hyper > 0) {
        k_clique_emit<<<(unsigned)ceil_div(n_hyper, 4), 256, 0, s>>>(n_hyper, offsets, members,
                                                                    out_off, src, dst);
        CLEORA_LAUNCH_CHECK();
    }
    return total;
}

void expand_star(int64_t n_nodes, int64_t n_hyper, const int64_t *offsets,
                 const int32_t *members, int32_t *src, int32_t *dst, hipStream_t s)
{
    if (n_hyper > 0) {
        k_star_emit<<<(unsigned)ceil_div(n_hyper, 4), 256, 0, s>>>(n_nodes, n_hyper, offsets,
                                                                  members, src, dst);
        CLEORA_LAUNCH_CHECK();
    }
}

}  // namespace cleora
