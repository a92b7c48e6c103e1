// Graph -> CSR of M = D^-1 A on the GPU (Section 3.2 of the paper: e_ab is
// the number of a->b edges or the sum of their weights, M_ab = e_ab/deg(a);
// undirected edges are stored in both directions, Section 4.5).
//
// Pipeline (all on the caller's stream, one host synchronisation at the end):
//   count degrees -> scan -> scatter (col[, weight]) into rows ->
//   sort every row by (col, weight) -> mark the first entry of each run of
//   equal columns -> scan -> compact (e_ab summed in float64) ->
//   deg(a) in float64 -> M values rounded to float32.
// Rows are sorted by three kernels chosen by length: a wave-wide bitonic
// network (<= 64 entries), an LDS bitonic network (<= 64 KiB of keys) and a
// block-wide stable LSD radix sort over global memory (longer hub rows).
// The sort key includes the weight bits, so the merged sums (and everything
// after them) do not depend on the order the atomics placed entries in.
#include "internal.hpp"

#include <algorithm>

namespace cleora {

namespace {

constexpr uint32_t ERR_ID = 1u, ERR_WEIGHT = 2u;

// Sort keys: uint32 = column (unweighted graphs), uint64 = column << 32 |
// float bits of the weight (positive floats order like their bit patterns).
template <typename K>
__device__ __forceinline__ int32_t key_col(K k)
{
    if constexpr (sizeof(K) == 8) return (int32_t)(k >> 32);
    else return (int32_t)k;
}
template <typename K>
__device__ __forceinline__ double key_weight(K k)
{
    if constexpr (sizeof(K) == 8) return (double)__uint_as_float((uint32_t)(k & 0xffffffffu));
    else return 1.0;
}
template <typename K>
__device__ __forceinline__ K make_key(int32_t col, const float *w, int64_t e)
{
    if constexpr (sizeof(K) == 8)
        return ((uint64_t)(uint32_t)col << 32) | (uint64_t)__float_as_uint(w[e]);
    else
        return (uint32_t)col;
}

__device__ __forceinline__ bool edge_ok(int64_t e, int64_t n, const int32_t *src,
                                        const int32_t *dst, const float *w, uint32_t *err)
{
    int32_t a = src[e], b = dst[e];
    if (a < 0 || a >= n || b < 0 || b >= n) {
        atomicOr(err, ERR_ID);
        return false;
    }
    if (w) {
        float x = w[e];
        if (!(x > 0.0f && x <= 3.402823466e38f)) {  // finite and positive
            atomicOr(err, ERR_WEIGHT);
            return false;
        }
    }
    return true;
}

__global__ void k_count(int64_t m, int64_t n, const int32_t *__restrict__ src,
                        const int32_t *__restrict__ dst, const float *__restrict__ w,
                        int directed, int32_t *__restrict__ cnt, uint32_t *err)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (!edge_ok(e, n, src, dst, w, err)) continue;
        int32_t a = src[e], b = dst[e];
        atomicAdd(&cnt[a], 1);
        if (!directed && a != b) atomicAdd(&cnt[b], 1);
    }
}

template <typename K>
__global__ void k_scatter(int64_t m, int64_t n, const int32_t *__restrict__ src,
                          const int32_t *__restrict__ dst, const float *__restrict__ w,
                          int directed, const int64_t *__restrict__ off,
                          int32_t *__restrict__ cursor, K *__restrict__ keys, uint32_t *err)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = src[e], b = dst[e];
        bool ok = a >= 0 && a < n && b >= 0 && b < n;
        if (ok && w) ok = w[e] > 0.0f && w[e] <= 3.402823466e38f;
        if (!ok) continue;  // already flagged by k_count
        int64_t p = off[a] + atomicAdd(&cursor[a], 1);
        keys[p] = make_key<K>(b, w, e);
        if (!directed && a != b) {
            int64_t q = off[b] + atomicAdd(&cursor[b], 1);
            keys[q] = make_key<K>(a, w, e);
        }
    }
}

// Rows of 2..64 entries: one wave, one entry per lane, bitonic network.
template <typename K>
__global__ __launch_bounds__(256) void k_sort_small(int64_t n, const int64_t *__restrict__ off,
                                                    K *__restrict__ keys)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const int64_t lo = off[row], len = off[row + 1] - lo;
    if (len < 2 || len > 64) return;
    K key = lane < len ? keys[lo + lane] : ~K(0);
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            K other = __shfl_xor(key, j, WAVE);
            bool asc = (lane & k) == 0, lower = (lane & j) == 0;
            key = (asc == lower) ? (key < other ? key : other) : (key < other ? other : key);
        }
    }
    if (lane < len) keys[lo + lane] = key;
}

__global__ void k_classify(int64_t n, const int64_t *__restrict__ off, int64_t mid_cap,
                           int32_t *__restrict__ mid_list, int32_t *__restrict__ big_list,
                           int32_t *counts)
{
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * blockDim.x) {
        int64_t len = off[row + 1] - off[row];
        if (len > 64 && len <= mid_cap) mid_list[atomicAdd(&counts[0], 1)] = (int32_t)row;
        else if (len > mid_cap) big_list[atomicAdd(&counts[1], 1)] = (int32_t)row;
    }
}

// Rows of 65..CAP entries: one block, bitonic network in LDS.
template <typename K, int CAP>
__global__ __launch_bounds__(256) void k_sort_mid(const int64_t *__restrict__ off,
                                                  K *__restrict__ keys,
                                                  const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ count)
{
    __shared__ K s[CAP];
    const int cnt = *count;
    for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
        const int64_t row = list[li];
        const int64_t lo = off[row];
        const int len = (int)(off[row + 1] - lo);
        int P = 128;
        while (P < len) P <<= 1;
        for (int i = threadIdx.x; i < P; i += blockDim.x) s[i] = i < len ? keys[lo + i] : ~K(0);
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                    int a = 2 * i - (i & (j - 1)), b = a + j;
                    bool asc = (a & k) == 0;
                    K x = s[a], y = s[b];
                    if ((x > y) == asc) {
                        s[a] = y;
                        s[b] = x;
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < len; i += blockDim.x) keys[lo + i] = s[i];
        __syncthreads();
    }
}

// Rows longer than the LDS network: one block of 1024 threads runs a stable
// LSD radix sort (8-bit digits) over the row in global memory, ping-ponging
// with tmp.  Low digits first: the weight bits (uint64 keys), then the column.
template <typename K>
__global__ __launch_bounds__(1024) void k_sort_big(const int64_t *__restrict__ off,
                                                   K *__restrict__ keys, K *__restrict__ tmp,
                                                   const int32_t *__restrict__ list,
                                                   const int32_t *__restrict__ count,
                                                   int col_passes)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t tcount[256];
    __shared__ uint16_t wcnt[16][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wpass = sizeof(K) == 8 ? 4 : 0;
    const int npass = wpass + col_passes;
    const int cnt = *count;
    for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
        const int64_t row = list[li];
        const int64_t lo = off[row];
        const int64_t len = off[row + 1] - lo;
        K *from = keys + lo, *to = tmp + lo;
        for (int p = 0; p < npass; ++p) {
            const int shift = p < wpass ? 8 * p : (sizeof(K) == 8 ? 32 : 0) + 8 * (p - wpass);
            if (t < 256) hist[t] = 0;
            __syncthreads();
            for (int64_t i = t; i < len; i += 1024)
                atomicAdd(&hist[(uint32_t)(from[i] >> shift) & 255u], 1u);
            __syncthreads();
            if (t == 0) {
                uint32_t s = 0;
                for (int d = 0; d < 256; ++d) {
                    base[d] = s;
                    s += hist[d];
                }
            }
            __syncthreads();
            for (int64_t t0 = 0; t0 < len; t0 += 1024) {
                const int64_t i = t0 + t;
                const bool valid = i < len;
                const K key = valid ? from[i] : K(0);
                const uint32_t dg = valid ? ((uint32_t)(key >> shift) & 255u) : 0u;
                for (int x = t; x < 16 * 256; x += 1024) (&wcnt[0][0])[x] = 0;
                __syncthreads();
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bool bit = (dg >> b) & 1u;
                    const uint64_t m = __ballot(bit);
                    peers &= bit ? m : ~m;
                }
                const uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
                if (valid && rank == 0) wcnt[w][dg] = (uint16_t)__popcll(peers);
                __syncthreads();
                if (t < 256) {
                    uint32_t s = 0;
                    for (int x = 0; x < 16; ++x) {
                        uint32_t c = wcnt[x][t];
                        wcnt[x][t] = (uint16_t)s;
                        s += c;
                    }
                    tcount[t] = s;
                }
                __syncthreads();
                if (valid) to[base[dg] + wcnt[w][dg] + rank] = key;
                __syncthreads();
                if (t < 256) base[t] += tcount[t];
                __syncthreads();
            }
            K *sw = from;
            from = to;
            to = sw;
        }
        if (from != keys + lo)
            for (int64_t i = t; i < len; i += 1024) keys[lo + i] = from[i];
        __syncthreads();
    }
}

// head[i] = 1 for the first entry of each run of equal columns in a row.
template <typename K>
__global__ void k_mark_heads(int64_t total_ub, const int64_t *__restrict__ total_p,
                             const K *__restrict__ keys, uint8_t *__restrict__ head)
{
    const int64_t total = *total_p;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total_ub;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint8_t h = 0;
        if (i < total) h = (i == 0 || key_col(keys[i]) != key_col(keys[i - 1])) ? 1 : 0;
        head[i] = h;
    }
}

__global__ void k_mark_row_starts(int64_t n, const int64_t *__restrict__ off,
                                  uint8_t *__restrict__ head)
{
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * blockDim.x)
        if (off[row + 1] > off[row]) head[off[row]] = 1;
}

// One merged entry per run: its column and e_ab (count or weight sum, float64).
template <typename K>
__global__ void k_compact(int64_t total_ub, const int64_t *__restrict__ total_p,
                          const K *__restrict__ keys, const uint8_t *__restrict__ head,
                          const int64_t *__restrict__ pos, int32_t *__restrict__ col_u,
                          double *__restrict__ e_u)
{
    const int64_t total = *total_p;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!head[i]) continue;
        const int64_t u = pos[i];
        col_u[u] = key_col(keys[i]);
        double s = key_weight(keys[i]);
        for (int64_t j = i + 1; j < total && !head[j]; ++j) s += key_weight(keys[j]);
        e_u[u] = s;
    }
    (void)total_ub;
}

__global__ void k_rowptr(int64_t n, const int64_t *__restrict__ off,
                         const int64_t *__restrict__ pos, int64_t *__restrict__ rp)
{
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a <= n;
         a += (int64_t)gridDim.x * blockDim.x)
        rp[a] = pos[off[a]];
}

// deg(a) = sum_b e_ab in float64 and M_ab = e_ab / deg(a) rounded to float32.
// One wave per row (rows whose unmerged length is at most mid_cap); the
// per-lane partial sums are combined in a fixed butterfly order.
__global__ __launch_bounds__(256) void k_rowsum_wave(int64_t n, const int64_t *__restrict__ off,
                                                     int64_t mid_cap,
                                                     const int64_t *__restrict__ rp,
                                                     const double *__restrict__ e_u,
                                                     float *__restrict__ val,
                                                     double *__restrict__ deg)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    if (off[row + 1] - off[row] > mid_cap) return;
    const int lane = threadIdx.x & 63;
    const int64_t lo = rp[row], hi = rp[row + 1];
    double s = 0.0;
    for (int64_t j = lo + lane; j < hi; j += 64) s += e_u[j];
    s = wave_sum(s);
    if (lane == 0) deg[row] = s;
    for (int64_t j = lo + lane; j < hi; j += 64) val[j] = (float)(e_u[j] / s);
}

// Same for the long rows: one block of 1024 threads per row.
__global__ __launch_bounds__(1024) void k_rowsum_block(const int32_t *__restrict__ list,
                                                       const int32_t *__restrict__ count,
                                                       const int64_t *__restrict__ rp,
                                                       const double *__restrict__ e_u,
                                                       float *__restrict__ val,
                                                       double *__restrict__ deg)
{
    __shared__ double ws[16];
    __shared__ double total;
    const int cnt = *count;
    for (int li = blockIdx.x; li < cnt; li += gridDim.x) {
        const int64_t row = list[li];
        const int64_t lo = rp[row], hi = rp[row + 1];
        double s = 0.0;
        for (int64_t j = lo + threadIdx.x; j < hi; j += 1024) s += e_u[j];
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < 16; ++i) t += ws[i];
            total = t;
            deg[row] = t;
        }
        __syncthreads();
        const double d = total;
        for (int64_t j = lo + threadIdx.x; j < hi; j += 1024) val[j] = (float)(e_u[j] / d);
        __syncthreads();
    }
}

unsigned grid_for(int64_t items, int threads, int64_t cap = 1 << 20)
{
    int64_t g = ceil_div(items > 0 ? items : 1, threads);
    return (unsigned)std::min<int64_t>(g, cap);
}

template <typename K>
void build_typed(cleora_ctx *c, int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                 const float *w, uint32_t flags, hipStream_t s)
{
    const int directed = (flags & CLEORA_DIRECTED) ? 1 : 0;
    const int64_t total_ub = directed ? m : 2 * m;
    constexpr int64_t MID_CAP = 65536 / sizeof(K);

    c->t_cnt.ensure(sizeof(int32_t) * 2 * (size_t)n);
    c->t_off.ensure(sizeof(int64_t) * ((size_t)n + 1));
    c->t_keys.ensure(sizeof(K) * (size_t)std::max<int64_t>(total_ub, 1));
    c->t_tmp.ensure(sizeof(K) * (size_t)std::max<int64_t>(total_ub, 1));
    c->t_head.ensure((size_t)std::max<int64_t>(total_ub, 1));
    c->t_pos.ensure(sizeof(int64_t) * ((size_t)total_ub + 1));
    c->t_esum.ensure(sizeof(double) * (size_t)std::max<int64_t>(total_ub, 1));
    c->t_lists.ensure(sizeof(int32_t) * 2 * (size_t)n);
    c->t_scan.ensure(sizeof(int64_t) * scan_workspace_elems(std::max<int64_t>(n + 1, total_ub + 1)));
    c->rp.ensure(sizeof(int64_t) * ((size_t)n + 1));
    c->col.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(total_ub, 1));
    c->val.ensure(sizeof(float) * (size_t)std::max<int64_t>(total_ub, 1));
    c->deg.ensure(sizeof(double) * (size_t)n);

    int32_t *cnt = c->t_cnt.as<int32_t>(), *cursor = cnt + n;
    int64_t *off = c->t_off.as<int64_t>();
    K *keys = c->t_keys.as<K>(), *tmp = c->t_tmp.as<K>();
    uint8_t *head = c->t_head.as<uint8_t>();
    int64_t *pos = c->t_pos.as<int64_t>(), *ws = c->t_scan.as<int64_t>();
    double *esum = c->t_esum.as<double>();
    int32_t *mid_list = c->t_lists.as<int32_t>(), *big_list = mid_list + n;
    // t_small: [0] error word, [1] two int32 list counters
    int64_t *small = c->t_small.as<int64_t>();
    uint32_t *err = reinterpret_cast<uint32_t *>(small);
    int32_t *counts = reinterpret_cast<int32_t *>(small + 1);

    CLEORA_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * 2 * (size_t)n, s));
    CLEORA_HIP(hipMemsetAsync(small, 0, sizeof(int64_t) * 4, s));

    const unsigned ge = grid_for(m, 256, 65536);
    if (m > 0) {
        k_count<<<ge, 256, 0, s>>>(m, n, src, dst, w, directed, cnt, err);
        CLEORA_LAUNCH_CHECK();
    }
    exclusive_scan(cnt, n, off, ws, s);
    if (m > 0) {
        k_scatter<K><<<ge, 256, 0, s>>>(m, n, src, dst, w, directed, off, cursor, keys, err);
        CLEORA_LAUNCH_CHECK();
    }
    // sort rows
    k_sort_small<K><<<(unsigned)ceil_div(n, 4), 256, 0, s>>>(n, off, keys);
    CLEORA_LAUNCH_CHECK();
    k_classify<<<grid_for(n, 256, 65536), 256, 0, s>>>(n, off, MID_CAP, mid_list, big_list,
                                                        counts);
    CLEORA_LAUNCH_CHECK();
    k_sort_mid<K, (int)MID_CAP><<<(unsigned)std::min<int64_t>(std::max<int64_t>(n, 1), 8192), 256,
                                   0, s>>>(off, keys, mid_list, counts);
    CLEORA_LAUNCH_CHECK();
    int col_bits = 0;
    while (col_bits < 31 && ((int64_t)1 << col_bits) < n) ++col_bits;
    const int col_passes = std::max(1, (col_bits + 7) / 8);
    k_sort_big<K><<<512, 1024, 0, s>>>(off, keys, tmp, big_list, counts + 1, col_passes);
    CLEORA_LAUNCH_CHECK();
    // merge repeated (a, b) pairs
    const unsigned gt = grid_for(total_ub, 256, 65536);
    k_mark_heads<K><<<gt, 256, 0, s>>>(total_ub, off + n, keys, head);
    CLEORA_LAUNCH_CHECK();
    k_mark_row_starts<<<grid_for(n, 256, 65536), 256, 0, s>>>(n, off, head);
    CLEORA_LAUNCH_CHECK();
    exclusive_scan(head, total_ub, pos, ws, s);
    k_compact<K><<<gt, 256, 0, s>>>(total_ub, off + n, keys, head, pos, c->col.as<int32_t>(), esum);
    CLEORA_LAUNCH_CHECK();
    k_rowptr<<<grid_for(n + 1, 256, 65536), 256, 0, s>>>(n, off, pos, c->rp.as<int64_t>());
    CLEORA_LAUNCH_CHECK();
    // D and M values
    k_rowsum_wave<<<(unsigned)ceil_div(n, 4), 256, 0, s>>>(n, off, MID_CAP, c->rp.as<int64_t>(),
                                                           esum, c->val.as<float>(),
                                                           c->deg.as<double>());
    CLEORA_LAUNCH_CHECK();
    k_rowsum_block<<<512, 1024, 0, s>>>(big_list, counts + 1, c->rp.as<int64_t>(), esum,
                                        c->val.as<float>(), c->deg.as<double>());
    CLEORA_LAUNCH_CHECK();
    // read back: error word and nnz
    CLEORA_HIP(hipMemcpyAsync(c->h_small, small, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CLEORA_HIP(hipMemcpyAsync(c->h_small + 1, c->rp.as<int64_t>() + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    CLEORA_HIP(hipStreamSynchronize(s));
    const uint32_t e = (uint32_t)(c->h_small[0] & 0xffffffff);
    if (e) {
        throw Error(CLEORA_E_INPUT, (e & ERR_ID) ? "edge id outside [0, n_nodes)"
                                                 : "edge weight not finite and positive");
    }
    c->nnz = c->h_small[1];
}

}  // namespace

void build_graph(cleora_ctx *c, int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                 const float *w, uint32_t flags, hipStream_t s)
{
    c->has_graph = false;
    c->has_emb = false;
    c->t_small.ensure(sizeof(int64_t) * 8);
    if (w) build_typed<uint64_t>(c, n, m, src, dst, w, flags, s);
    else build_typed<uint32_t>(c, n, m, src, dst, w, flags, s);
    c->n = n;
    c->m_in = m;
    c->flags = flags;
    c->has_graph = true;
}

}  // namespace cleora
