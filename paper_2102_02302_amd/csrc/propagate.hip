// The propagation hot path (Algorithm 1 of the paper): T_t = M . T_{t-1}
// followed by an L2 normalisation of every row, as one fused kernel.
//
// Work decomposition.  A row with more than `chunk` entries (the split size)
// is split into chunks aligned to its own start; every chunk writes a
// float32 partial sum and a combine kernel adds a row's partials in chunk
// order, normalises and stores.  The other rows are packed into items of
// about `pack` units of work (one unit per stored entry, one per row for its
// write): an item is the set of rows whose position rp[r] + r falls into one
// pack-sized bucket.  The packing adapts to the graph's size; the split size
// does not.  Each row's summation order therefore depends only on the row
// (its entries, its length and `chunk`), never on where it sits in the graph
// or in a batch.
//
// Inner loop.  A wave (64 lanes) owns a row.  The row of T_{t-1} of each
// neighbour is gathered with 16-byte loads along d (d contiguous, coalesced);
// when a row of T is narrower than 1 KiB the wave is split into G groups
// that gather G neighbours at once and are summed at the end.  Products and
// sums are float32 FMAs; the row norm is a wave reduction in the epilogue,
// so T_t is written once and never re-read by this iteration.
//
// Column blocks and slices.  Columns of T interact only through the row
// norms, so a block of columns can be propagated on its own once the norms
// are known (an embedding too wide for device memory), and one iteration
// can run as column slices of the resident rows (narrower gathers keep more
// of the hot rows in cache).  For both the SpMM has more epilogues
// (template flag EXT): add the slice's share of each row's squared norm to
// a vector, storing nothing or the unscaled row; or scale each row by a
// given factor (1/norm of the whole row) instead of normalising it.
#include "internal.hpp"

#include <algorithm>

namespace cleora {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Rows of T_t are written once per iteration and read only by the next one:
// store them non-temporally.
__device__ __forceinline__ void store_stream(uint4 *p, uint4 x)
{
    u32x4 v = {x.x, x.y, x.z, x.w};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
}


// ----------------------------------------------------------------- init

__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    // SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// U(-1,1) entry of T_0 for the counter c = i * d + j: 24 random bits k,
// value k * 2^-23 - 1 (exact).
__device__ __forceinline__ float uniform_entry(uint64_t seed, uint64_t c)
{
    const uint64_t x = splitmix64(seed ^ splitmix64(c));
    return (float)(uint32_t)(x >> 40) * 0x1p-23f - 1.0f;
}

// T_0 rows (or columns [j0, j0 + dim) of rows of width dfull).  Thread t
// owns 16-byte vector v0 = t % vt of rows t / vt, t / vt + rps, ... (vt
// threads per row, rps rows per sweep; vectors v0 + vt, ... too when a row
// has more vectors than the grid has threads): the division happens once per
// thread, and each row's counter base i * dfull + j0 once per row.
template <typename T>
__global__ void k_init(T *__restrict__ E, int64_t n, int32_t dim, int32_t ld,
                       const int64_t *__restrict__ row0, const uint64_t *__restrict__ seeds,
                       int n_graphs, uint64_t seed0, const int32_t *__restrict__ ids,
                       int32_t dfull, int32_t j0, int32_t vt, int32_t rps)
{
    constexpr int EPV = 16 / sizeof(T);
    const int32_t vpr = ld / EPV;
    const int32_t tid = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t r0 = tid / vt;
    if (r0 >= rps) return;
    const int32_t v0 = tid - r0 * vt;
    for (int64_t row = r0; row < n; row += rps) {
        int64_t local = row;
        uint64_t seed = seed0;
        if (row0) {
            int lo = 0, hi = n_graphs - 1;  // last g with row0[g] <= row
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (row0[mid] <= row) lo = mid;
                else hi = mid - 1;
            }
            local = row - row0[lo];
            seed = seeds[lo];
        }
        if (ids) local = ids[row];
        const uint64_t cbase = (uint64_t)local * (uint64_t)dfull + (uint64_t)j0;
        uint4 *out_row = reinterpret_cast<uint4 *>(E + row * (int64_t)ld);
        for (int32_t v = v0; v < vpr; v += vt) {
            float x[EPV];
#pragma unroll
            for (int e = 0; e < EPV; ++e) {
                const int32_t j = v * EPV + e;
                x[e] = j < dim ? uniform_entry(seed, cbase + (uint64_t)j) : 0.0f;
            }
            uint4 out;
            if constexpr (sizeof(T) == 4) {
                out = make_uint4(__float_as_uint(x[0]), __float_as_uint(x[1]),
                                 __float_as_uint(x[2]), __float_as_uint(x[3]));
            } else {
                uint32_t p[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    p[q] = f32_to_bf16_rne(x[2 * q]) | (f32_to_bf16_rne(x[2 * q + 1]) << 16);
                out = make_uint4(p[0], p[1], p[2], p[3]);
            }
            out_row[v] = out;
        }
    }
}

__global__ void k_widen_bf16(const uint16_t *__restrict__ src, int64_t n, int32_t dim,
                             int32_t ld_src, float *__restrict__ dst, int64_t ld_dst)
{
    const int64_t total = n * dim;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / dim;
        const int32_t j = (int32_t)(idx - r * dim);
        dst[r * ld_dst + j] = __uint_as_float((uint32_t)src[r * ld_src + j] << 16);
    }
}

// ------------------------------------------------------------- schedule

__global__ void k_sched_count(int64_t n, const int64_t *__restrict__ rp, int32_t chunk,
                              int32_t *__restrict__ nch, uint8_t *__restrict__ is_long)
{
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n;
         a += (int64_t)gridDim.x * blockDim.x) {
        const int64_t len = rp[a + 1] - rp[a];
        const bool L = len > chunk;
        nch[a] = L ? (int32_t)((len + chunk - 1) / chunk) : 0;
        is_long[a] = L ? 1 : 0;
    }
}

__global__ void k_sched_fill(int64_t n, const int64_t *__restrict__ chunk_base,
                             const int64_t *__restrict__ long_pos, int2 *__restrict__ items,
                             int32_t *__restrict__ long_rows)
{
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n;
         a += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b0 = chunk_base[a], b1 = chunk_base[a + 1];
        if (b1 == b0) continue;
        long_rows[long_pos[a]] = (int32_t)a;
        for (int64_t i = b0; i < b1; ++i) items[i] = make_int2((int32_t)a, (int32_t)(i - b0));
    }
}

// bucket_row[k] = first row r with rp[r] + r >= k * chunk (n if none).
__global__ void k_buckets(int64_t n, const int64_t *__restrict__ rp, int32_t chunk, int64_t nb,
                          int32_t *__restrict__ bucket_row)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= nb;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t target = k * (int64_t)chunk;
        int64_t lo = 0, hi = n;  // answer in [0, n]
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (rp[mid] + mid >= target) hi = mid;
            else lo = mid + 1;
        }
        bucket_row[k] = (int32_t)lo;
    }
}

// ------------------------------------------------------------ SpMM+norm

template <typename T>
struct EmbT {
    static constexpr int EPV = 16 / sizeof(T);  // elements per 16-byte vector
};

template <typename T>
__device__ __forceinline__ void widen(const uint4 &r, float *x)
{
    if constexpr (sizeof(T) == 4) {
        x[0] = __uint_as_float(r.x);
        x[1] = __uint_as_float(r.y);
        x[2] = __uint_as_float(r.z);
        x[3] = __uint_as_float(r.w);
    } else {
        x[0] = bf16_lo(r.x);
        x[1] = bf16_hi(r.x);
        x[2] = bf16_lo(r.y);
        x[3] = bf16_hi(r.y);
        x[4] = bf16_lo(r.z);
        x[5] = bf16_hi(r.z);
        x[6] = bf16_lo(r.w);
        x[7] = bf16_hi(r.w);
    }
}

template <typename T>
__device__ __forceinline__ uint4 narrow(const float *x)
{
    if constexpr (sizeof(T) == 4) {
        return make_uint4(__float_as_uint(x[0]), __float_as_uint(x[1]), __float_as_uint(x[2]),
                          __float_as_uint(x[3]));
    } else {
        uint32_t p[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            p[q] = f32_to_bf16_rne(x[2 * q]) | (f32_to_bf16_rne(x[2 * q + 1]) << 16);
        return make_uint4(p[0], p[1], p[2], p[3]);
    }
}

__device__ __forceinline__ int find_desc(const StepDesc *descs, int n_desc, int64_t id,
                                         bool blocks)
{
    int di = 0;
    while (di + 1 < n_desc && id >= (blocks ? descs[di + 1].block_begin : descs[di + 1].wave_begin))
        ++di;
    return di;
}

// acc += sum_{j in [jb, je)} val[j] * T[col[j]], G entries at a time
// (group g takes j = jb + g, jb + g + G, ...), U-way unrolled.
template <typename T, int G, int VPL, int U>
__device__ __forceinline__ void gather_rows(float (&acc)[VPL][EmbT<T>::EPV], int64_t jb,
                                            int64_t je, const int32_t *__restrict__ col,
                                            const float *__restrict__ val,
                                            const uint4 *__restrict__ Ein, int64_t vrow, int grp,
                                            int gl, int cpr)
{
    constexpr int EPV = EmbT<T>::EPV;
    constexpr int LPG = WAVE / G;
    int64_t j = jb;
    for (; j + (int64_t)G * U <= je; j += (int64_t)G * U) {
        int32_t c[U];
        float w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = col[j + u * G + grp];
            w[u] = val[j + u * G + grp];
        }
        uint4 x[U][VPL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint4 *row = Ein + (int64_t)c[u] * vrow;
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const int ch = gl + v * LPG;
                x[u][v] = ch < cpr ? row[ch] : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                float f[EPV];
                widen<T>(x[u][v], f);
#pragma unroll
                for (int e = 0; e < EPV; ++e) acc[v][e] = fmaf(w[u], f[e], acc[v][e]);
            }
    }
    if constexpr (G == 1) {
        // one row per wave: other waves hide the latency of a short tail
        for (; j < je; ++j) {
            const int32_t c = col[j];
            const float w = val[j];
            const uint4 *row = Ein + (int64_t)c * vrow;
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const int ch = gl + v * LPG;
                if (ch < cpr) {
                    float f[EPV];
                    widen<T>(row[ch], f);
#pragma unroll
                    for (int e = 0; e < EPV; ++e) acc[v][e] = fmaf(w, f[e], acc[v][e]);
                }
            }
        }
    } else if (j < je) {
        // narrow rows, G per wave: the last < G*U entries in one predicated
        // round, all loads in flight together; each group still adds its
        // entries in ascending order
        int32_t c[U];
        float w[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t jj = j + u * G + grp;
            ok[u] = jj < je;
            const int64_t js = ok[u] ? jj : je - 1;  // an in-range index for the unused slots
            c[u] = col[js];
            w[u] = val[js];
        }
        uint4 x[U][VPL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint4 *row = Ein + (int64_t)c[u] * vrow;
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const int ch = gl + v * LPG;
                x[u][v] = (ok[u] && ch < cpr) ? row[ch] : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                float f[EPV];
                widen<T>(x[u][v], f);
#pragma unroll
                for (int e = 0; e < EPV; ++e)
                    acc[v][e] = ok[u] ? fmaf(w[u], f[e], acc[v][e]) : acc[v][e];
            }
    }
}

template <int G, int VPL, int EPV>
__device__ __forceinline__ void reduce_groups(float (&acc)[VPL][EPV])
{
    if constexpr (G > 1) {
        constexpr int LPG = WAVE / G;
#pragma unroll
        for (int off = LPG; off < WAVE; off <<= 1)
#pragma unroll
            for (int v = 0; v < VPL; ++v)
#pragma unroll
                for (int e = 0; e < EPV; ++e) acc[v][e] += __shfl_xor(acc[v][e], off, WAVE);
    }
}

// One wave's work item of the fused SpMM + normalise step: either a chunk
// of a split row (partial sum to `partial`) or a packed group of rows
// (normalised rows to Eout).  With EXT, the column-block epilogues: a
// non-null row_ss receives each row's squared norm (added; the row itself
// is stored unscaled when keep_rows, else not at all), else row r is
// scaled by row_scale[r].
template <typename T, int G, int VPL, int U, bool EXT>
__device__ __forceinline__ void spmm_item(
    int64_t wave, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
    const float *__restrict__ val, const uint4 *__restrict__ Ein, uint4 *__restrict__ Eout,
    float *__restrict__ partial, const int2 *__restrict__ split_items,
    const int32_t *__restrict__ bucket_row, int64_t n_split, int64_t n_buckets, int ld,
    int chunk, uint32_t flags, int cpr, const float *__restrict__ row_scale,
    float *__restrict__ row_ss, int keep_rows)
{
    constexpr int EPV = EmbT<T>::EPV;
    constexpr int LPG = WAVE / G;
    const int lane = threadIdx.x & 63;
    const int grp = G == 1 ? 0 : lane / LPG;
    const int gl = G == 1 ? lane : lane % LPG;
    const int64_t vrow = ld / EPV;  // 16-byte vectors per row of T

    float acc[VPL][EPV];
    if (wave < n_split) {
        const int2 it = split_items[wave];
        const int64_t hi = rp[it.x + 1];
        const int64_t jb = rp[it.x] + (int64_t)it.y * chunk;
        const int64_t je = min(jb + (int64_t)chunk, hi);
#pragma unroll
        for (int v = 0; v < VPL; ++v)
#pragma unroll
            for (int e = 0; e < EPV; ++e) acc[v][e] = 0.0f;
        gather_rows<T, G, VPL, U>(acc, jb, je, col, val, Ein, vrow, grp, gl, cpr);
        reduce_groups<G, VPL, EPV>(acc);
        if (grp == 0) {
            float4 *prow = reinterpret_cast<float4 *>(partial + wave * (int64_t)ld);
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const int ch = gl + v * LPG;
                if (ch < cpr) {
#pragma unroll
                    for (int q = 0; q < EPV / 4; ++q)
                        prow[ch * (EPV / 4) + q] = make_float4(acc[v][4 * q], acc[v][4 * q + 1],
                                                               acc[v][4 * q + 2], acc[v][4 * q + 3]);
                }
            }
        }
        return;
    }
    const int64_t k = wave - n_split;
    if (k >= n_buckets) return;
    const int32_t r0 = bucket_row[k], r1 = bucket_row[k + 1];
    for (int32_t r = r0; r < r1; ++r) {
        const int64_t lo = rp[r], hi = rp[r + 1];
        if (hi - lo > chunk) continue;  // split row: chunks + combine
#pragma unroll
        for (int v = 0; v < VPL; ++v)
#pragma unroll
            for (int e = 0; e < EPV; ++e) acc[v][e] = 0.0f;
        if (hi == lo) {
            if ((flags & CLEORA_EMPTY_KEEP) && grp == 0) {
#pragma unroll
                for (int v = 0; v < VPL; ++v) {
                    const int ch = gl + v * LPG;
                    if (ch < cpr) widen<T>(Ein[(int64_t)r * vrow + ch], acc[v]);
                }
            }
        } else {
            gather_rows<T, G, VPL, U>(acc, lo, hi, col, val, Ein, vrow, grp, gl, cpr);
        }
        reduce_groups<G, VPL, EPV>(acc);
        float ss = 0.0f;
#pragma unroll
        for (int v = 0; v < VPL; ++v)
#pragma unroll
            for (int e = 0; e < EPV; ++e) ss = fmaf(acc[v][e], acc[v][e], ss);
        ss = group_sum<LPG>(ss);
        float inv;
        if constexpr (EXT) {
            if (row_ss) {
                // every group holds the whole row's sum after reduce_groups
                if (lane == 0) row_ss[r] += ss;
                if (!keep_rows) continue;
                inv = 1.0f;  // the row's norm is known after its last slice
            } else {
                inv = row_scale[r];
            }
        } else {
            inv = ss > 0.0f ? 1.0f / sqrtf(ss) : 0.0f;
        }
        if (grp == 0) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const int ch = gl + v * LPG;
                if (ch < cpr) {
                    float o[EPV];
#pragma unroll
                    for (int e = 0; e < EPV; ++e) o[e] = acc[v][e] * inv;
                    // written once, read by the next iteration: keep it out of L2
                    store_stream(&Eout[(int64_t)r * vrow + ch], narrow<T>(o));
                }
            }
        }
    }
}

// The wave index is uniform: readfirstlane keeps it, and every address
// derived from it, in scalar registers.
__device__ __forceinline__ int64_t wave_id()
{
    return (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// One graph: plain restrict-qualified global pointers, so column/value
// loads of a wave become scalar loads and gathers global loads.  A wave
// takes items wave, wave + waves in grid, ...: with one wave per item the
// loop runs once; with a grid of the resident waves only, the kernel is
// persistent (which of the two is faster is the autotuner's call).
template <typename T, int G, int VPL, int U, bool EXT>
__global__ __launch_bounds__(256) void k_spmm_norm(
    const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
    const float *__restrict__ val, const uint4 *__restrict__ Ein, uint4 *__restrict__ Eout,
    float *__restrict__ partial, const int2 *__restrict__ split_items,
    const int32_t *__restrict__ bucket_row, int64_t n_split, int64_t n_buckets, int ld,
    int chunk, uint32_t flags, int cpr, const float *__restrict__ row_scale,
    float *__restrict__ row_ss, int keep_rows)
{
    const int64_t items = n_split + n_buckets, stride = (int64_t)gridDim.x * 4;
    for (int64_t w = wave_id(); w < items; w += stride)
        spmm_item<T, G, VPL, U, EXT>(w, rp, col, val, Ein, Eout, partial, split_items,
                                     bucket_row, n_split, n_buckets, ld, chunk, flags, cpr,
                                     row_scale, row_ss, keep_rows);
}

// Several graphs (continuous batching): each item's graph is found in the
// descriptor table.
template <typename T, int G, int VPL, int U>
__global__ __launch_bounds__(256) void k_spmm_norm_multi(const StepDesc *__restrict__ descs,
                                                         int n_desc, int64_t items, int cpr)
{
    const int64_t stride = (int64_t)gridDim.x * 4;
    for (int64_t w = wave_id(); w < items; w += stride) {
        const StepDesc &D = descs[find_desc(descs, n_desc, w, false)];
        spmm_item<T, G, VPL, U, false>(w - D.wave_begin, D.rp, D.col, D.val,
                                       reinterpret_cast<const uint4 *>(D.Ein),
                                       reinterpret_cast<uint4 *>(D.Eout), D.partial,
                                       D.split_items, D.bucket_row, D.n_split, D.n_buckets, D.ld,
                                       D.chunk, D.flags, cpr, nullptr, nullptr, 0);
    }
}

// Combine the partial sums of a split row in chunk order, normalise, store.
// WPB waves per block; wave w adds partials w, w + WPB, ...; the wave sums
// are then added in a fixed pairwise order through LDS.
template <typename T, int VPLF, int WPB>
__global__ __launch_bounds__(WPB * 64) void k_combine(const StepDesc *__restrict__ descs,
                                                      int n_desc, int cprf)
{
    __shared__ float4 red[WPB / 2 > 0 ? WPB / 2 : 1][VPLF * 64];
    const int64_t blk = blockIdx.x;
    const StepDesc &D = descs[find_desc(descs, n_desc, blk, true)];
    const int64_t li = blk - D.block_begin;
    if (li >= D.n_long) return;  // whole block leaves together
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t row = D.long_rows[li];
    const int64_t b0 = D.chunk_base[row], nch = D.chunk_base[row + 1] - b0;
    const float4 *__restrict__ P = reinterpret_cast<const float4 *>(D.partial);
    const int64_t prow = D.ld / 4;
    float4 acc[VPLF];
#pragma unroll
    for (int v = 0; v < VPLF; ++v) acc[v] = make_float4(0.f, 0.f, 0.f, 0.f);
    // wave w adds partials w, w + WPB, ... in that order; CU of them are
    // loaded together (a hub row has hundreds per wave)
    constexpr int CU = VPLF >= 8 ? 1 : 8 / VPLF;
    int64_t i = w;
    for (; i + (int64_t)(CU - 1) * WPB < nch; i += (int64_t)CU * WPB) {
        float4 p[CU][VPLF];
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
            for (int v = 0; v < VPLF; ++v) {
                const int ch = lane + v * 64;
                p[u][v] = ch < cprf ? P[(b0 + i + (int64_t)u * WPB) * prow + ch]
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
            for (int v = 0; v < VPLF; ++v) {
                acc[v].x += p[u][v].x;
                acc[v].y += p[u][v].y;
                acc[v].z += p[u][v].z;
                acc[v].w += p[u][v].w;
            }
    }
    for (; i < nch; i += WPB) {
#pragma unroll
        for (int v = 0; v < VPLF; ++v) {
            const int ch = lane + v * 64;
            if (ch < cprf) {
                const float4 p = P[(b0 + i) * prow + ch];
                acc[v].x += p.x;
                acc[v].y += p.y;
                acc[v].z += p.z;
                acc[v].w += p.w;
            }
        }
    }
    for (int half = WPB / 2; half > 0; half >>= 1) {
        if (w >= half && w < 2 * half)
#pragma unroll
            for (int v = 0; v < VPLF; ++v) red[w - half][v * 64 + lane] = acc[v];
        __syncthreads();
        if (w < half)
#pragma unroll
            for (int v = 0; v < VPLF; ++v) {
                const float4 q = red[w][v * 64 + lane];
                acc[v].x += q.x;
                acc[v].y += q.y;
                acc[v].z += q.z;
                acc[v].w += q.w;
            }
        __syncthreads();
    }
    if (w != 0) return;
    float ss = 0.0f;
#pragma unroll
    for (int v = 0; v < VPLF; ++v) {
        ss = fmaf(acc[v].x, acc[v].x, ss);
        ss = fmaf(acc[v].y, acc[v].y, ss);
        ss = fmaf(acc[v].z, acc[v].z, ss);
        ss = fmaf(acc[v].w, acc[v].w, ss);
    }
    ss = wave_sum(ss);
    float inv;
    if (D.row_ss) {  // column blocks and slices: the squared norm, the row unscaled
        if (lane == 0) D.row_ss[row] += ss;
        if (!D.keep_rows) return;
        inv = 1.0f;
    } else {
        inv = D.row_scale ? D.row_scale[row] : (ss > 0.0f ? 1.0f / sqrtf(ss) : 0.0f);
    }
#pragma unroll
    for (int v = 0; v < VPLF; ++v) {
        const int ch = lane + v * 64;
        if (ch >= cprf) continue;
        const float o0 = acc[v].x * inv, o1 = acc[v].y * inv, o2 = acc[v].z * inv,
                    o3 = acc[v].w * inv;
        if constexpr (sizeof(T) == 4) {
            reinterpret_cast<float4 *>(D.Eout)[(int64_t)row * prow + ch] =
                make_float4(o0, o1, o2, o3);
        } else {
            reinterpret_cast<uint2 *>(D.Eout)[(int64_t)row * prow + ch] =
                make_uint2(f32_to_bf16_rne(o0) | (f32_to_bf16_rne(o1) << 16),
                           f32_to_bf16_rne(o2) | (f32_to_bf16_rne(o3) << 16));
        }
    }
}

unsigned grid_for(int64_t items, int threads, int64_t cap = 1 << 20)
{
    int64_t g = ceil_div(items > 0 ? items : 1, threads);
    return (unsigned)std::min<int64_t>(g, cap);
}

// Blocks of `kernel` (256 threads) resident on the whole device at once.
template <typename K>
int64_t resident_blocks(K kernel)
{
    int dev = 0, cus = 0, per_cu = 0;
    CLEORA_HIP(hipGetDevice(&dev));
    CLEORA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CLEORA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0));
    return (int64_t)std::max(cus, 1) * std::max(per_cu, 1);
}

template <typename T, int G, int VPL, int U, bool EXT>
void spmm_launch(const StepDesc *host, const StepDesc *descs, int n_desc, int64_t waves, int cpr,
                 int32_t persist, hipStream_t s)
{
    int64_t blocks = ceil_div(waves, 4);
    if (persist > 0) {
        // per kernel instance, queried once (at init: see prime_spmm); every
        // device this library runs on is a gfx950
        static const int64_t res1 = resident_blocks(k_spmm_norm<T, G, VPL, U, EXT>);
        static const int64_t resm = resident_blocks(k_spmm_norm_multi<T, G, VPL, U>);
        blocks = std::min(blocks, (int64_t)persist * (host ? res1 : resm));
    }
    if (blocks <= 0) return;
    if (blocks > 0x7fffffffLL) throw Error(CLEORA_E_INVAL, "propagation grid too large");
    if (host) {
        const StepDesc &D = *host;
        k_spmm_norm<T, G, VPL, U, EXT><<<(unsigned)blocks, 256, 0, s>>>(
            D.rp, D.col, D.val, reinterpret_cast<const uint4 *>(D.Ein),
            reinterpret_cast<uint4 *>(D.Eout), D.partial, D.split_items, D.bucket_row, D.n_split,
            D.n_buckets, D.ld, D.chunk, D.flags, cpr, D.row_scale, D.row_ss, D.keep_rows);
    } else {
        k_spmm_norm_multi<T, G, VPL, U><<<(unsigned)blocks, 256, 0, s>>>(descs, n_desc, waves,
                                                                         cpr);
    }
    CLEORA_LAUNCH_CHECK();
}

template <typename T, bool EXT>
void spmm_dispatch_ext(const Variant &v, const StepDesc *host, const StepDesc *descs, int n_desc,
                       int64_t waves, int32_t persist, hipStream_t s)
{
    const int c = v.cpr;
    if (v.VPL == 1) {
        switch (v.G) {
        case 1: return spmm_launch<T, 1, 1, 8, EXT>(host, descs, n_desc, waves, c, persist, s);
        case 2: return spmm_launch<T, 2, 1, 4, EXT>(host, descs, n_desc, waves, c, persist, s);
        case 4: return spmm_launch<T, 4, 1, 2, EXT>(host, descs, n_desc, waves, c, persist, s);
        case 8: return spmm_launch<T, 8, 1, 1, EXT>(host, descs, n_desc, waves, c, persist, s);
        case 16: return spmm_launch<T, 16, 1, 1, EXT>(host, descs, n_desc, waves, c, persist, s);
        default: break;
        }
    } else {
        switch (v.VPL) {
        case 2: return spmm_launch<T, 1, 2, 4, EXT>(host, descs, n_desc, waves, c, persist, s);
        case 4: return spmm_launch<T, 1, 4, 2, EXT>(host, descs, n_desc, waves, c, persist, s);
        case 8: return spmm_launch<T, 1, 8, 1, EXT>(host, descs, n_desc, waves, c, persist, s);
        case 16: return spmm_launch<T, 1, 16, 1, EXT>(host, descs, n_desc, waves, c, persist, s);
        default: break;
        }
    }
    throw Error(CLEORA_E_INVAL, "no kernel variant for this embedding width");
}

// The column-blocked epilogues exist for single-graph launches only.
template <typename T>
void spmm_dispatch(const Variant &v, const StepDesc *host, const StepDesc *descs, int n_desc,
                   int64_t waves, int32_t persist, hipStream_t s)
{
    if (host && (host->row_scale || host->row_ss))
        spmm_dispatch_ext<T, true>(v, host, descs, n_desc, waves, persist, s);
    else
        spmm_dispatch_ext<T, false>(v, host, descs, n_desc, waves, persist, s);
}

template <typename T, int VPLF>
void combine_launch(const StepDesc *descs, int n_desc, int64_t blocks, int cprf, hipStream_t s)
{
    constexpr int WPB = VPLF <= 4 ? 16 : (64 / VPLF > 1 ? 64 / VPLF : 1);
    if (blocks <= 0) return;
    if (blocks > 0x7fffffffLL) throw Error(CLEORA_E_INVAL, "combine grid too large");
    k_combine<T, VPLF, WPB><<<(unsigned)blocks, WPB * 64, 0, s>>>(descs, n_desc, cprf);
    CLEORA_LAUNCH_CHECK();
}

template <typename T>
void combine_dispatch(const Variant &v, const StepDesc *descs, int n_desc, int64_t blocks,
                      hipStream_t s)
{
    switch (v.VPLF) {
    case 1: return combine_launch<T, 1>(descs, n_desc, blocks, v.cprf, s);
    case 2: return combine_launch<T, 2>(descs, n_desc, blocks, v.cprf, s);
    case 4: return combine_launch<T, 4>(descs, n_desc, blocks, v.cprf, s);
    case 8: return combine_launch<T, 8>(descs, n_desc, blocks, v.cprf, s);
    case 16: return combine_launch<T, 16>(descs, n_desc, blocks, v.cprf, s);
    case 32: return combine_launch<T, 32>(descs, n_desc, blocks, v.cprf, s);
    default: break;
    }
    throw Error(CLEORA_E_INVAL, "no combine variant for this embedding width");
}

int pow2_ceil(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

Variant choose_variant(int dtype, int ld)
{
    Variant v;
    v.dtype = dtype;
    const int esz = dtype == CLEORA_BF16 ? 2 : 4;
    v.cpr = ld * esz / 16;
    if (v.cpr <= 64) {
        v.VPL = 1;
        v.G = std::min(16, 64 / pow2_ceil(v.cpr));
    } else {
        v.G = 1;
        v.VPL = pow2_ceil((int)ceil_div(v.cpr, 64));
    }
    v.cprf = ld / 4;
    v.VPLF = pow2_ceil((int)ceil_div(v.cprf, 64));
    return v;
}

void launch_spmm(const Variant &v, const StepDesc &one, hipStream_t s)
{
    const int64_t waves = one.n_split + one.n_buckets;
    if (v.dtype == CLEORA_BF16) spmm_dispatch<uint16_t>(v, &one, nullptr, 1, waves, one.persist, s);
    else spmm_dispatch<float>(v, &one, nullptr, 1, waves, one.persist, s);
}

// Runs the one-time occupancy queries of a persistent grid now, so that
// none happens inside a graph capture (no kernel is launched).
void prime_spmm(const Variant &v, int32_t persist, bool ext)
{
    if (persist <= 0) return;
    StepDesc none{};
    if (v.dtype == CLEORA_BF16) {
        if (ext) spmm_dispatch_ext<uint16_t, true>(v, &none, nullptr, 1, 0, persist, nullptr);
        else spmm_dispatch_ext<uint16_t, false>(v, &none, nullptr, 1, 0, persist, nullptr);
    } else {
        if (ext) spmm_dispatch_ext<float, true>(v, &none, nullptr, 1, 0, persist, nullptr);
        else spmm_dispatch_ext<float, false>(v, &none, nullptr, 1, 0, persist, nullptr);
    }
}

void launch_spmm_multi(const Variant &v, const StepDesc *descs, int n_desc, int64_t total_waves,
                       int32_t persist, hipStream_t s)
{
    if (v.dtype == CLEORA_BF16)
        spmm_dispatch<uint16_t>(v, nullptr, descs, n_desc, total_waves, persist, s);
    else spmm_dispatch<float>(v, nullptr, descs, n_desc, total_waves, persist, s);
}

void launch_combine(const Variant &v, const StepDesc *descs, int n_desc, int64_t total_blocks,
                    hipStream_t s)
{
    if (v.dtype == CLEORA_BF16) combine_dispatch<uint16_t>(v, descs, n_desc, total_blocks, s);
    else combine_dispatch<float>(v, descs, n_desc, total_blocks, s);
}

void launch_init(int dtype, void *E, int64_t n, int32_t dim, int32_t ld, const int64_t *row0,
                 const uint64_t *seeds, int n_graphs, uint64_t seed0, hipStream_t s,
                 const int32_t *ids, int64_t max_blocks, int32_t dfull, int32_t j0)
{
    if (dfull <= 0) dfull = dim;
    const int epv = dtype == CLEORA_BF16 ? 8 : 4;
    const int64_t vpr = ld / epv, total = n * vpr;
    const unsigned g = grid_for(total, 256, max_blocks > 0 ? max_blocks : 1 << 16);
    // vt threads per row, rps rows per sweep (vt * rps <= the grid's threads)
    const int64_t threads = (int64_t)g * 256;
    const int32_t vt = (int32_t)std::max<int64_t>(1, std::min<int64_t>(vpr, threads));
    const int32_t rps = (int32_t)std::max<int64_t>(1, threads / vt);
    if (dtype == CLEORA_BF16)
        k_init<uint16_t><<<g, 256, 0, s>>>(reinterpret_cast<uint16_t *>(E), n, dim, ld, row0,
                                           seeds, n_graphs, seed0, ids, dfull, j0, vt, rps);
    else
        k_init<float><<<g, 256, 0, s>>>(reinterpret_cast<float *>(E), n, dim, ld, row0, seeds,
                                        n_graphs, seed0, ids, dfull, j0, vt, rps);
    CLEORA_LAUNCH_CHECK();
}

void launch_widen_bf16(const void *src, int64_t n, int32_t dim, int32_t ld_src, float *dst,
                       int64_t ld_dst, hipStream_t s)
{
    k_widen_bf16<<<grid_for(n * dim, 256, 1 << 16), 256, 0, s>>>(
        reinterpret_cast<const uint16_t *>(src), n, dim, ld_src, dst, ld_dst);
    CLEORA_LAUNCH_CHECK();
}

void plan_schedule(cleora_ctx *c, hipStream_t s)
{
    const int64_t n = c->n;
    const int32_t C = c->chunk;  // split size: rows longer than this are split
    // packing size: enough items to keep every SIMD busy several times over
    // (no effect on results: a packed row is summed the same way in any item)
    // explicit (autotuner trial) > autotuned for this graph shape > formula
    const int32_t tuned = c->pack_req > 0 ? c->pack_req : tuned_pack(c);
    c->persist = c->persist_req >= 0 ? c->persist_req : tuned_persist(c);
    prime_spmm(choose_variant(c->dtype, c->ld), c->persist);
    c->pack = tuned > 0
                  ? (int32_t)std::min<int64_t>(C, tuned)
                  : (int32_t)std::min<int64_t>(C, std::max<int64_t>(16, (c->nnz + n) / 32768));
    const int32_t P = c->pack;
    c->t_cnt.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
    c->t_head.ensure((size_t)std::max<int64_t>(n, 1));
    c->chunk_base.ensure(sizeof(int64_t) * ((size_t)n + 1));
    c->t_pos.ensure(sizeof(int64_t) * ((size_t)n + 1));
    c->t_scan.ensure(sizeof(int64_t) * scan_workspace_elems(n + 1));
    int32_t *nch = c->t_cnt.as<int32_t>();
    uint8_t *is_long = c->t_head.as<uint8_t>();
    int64_t *long_pos = c->t_pos.as<int64_t>();
    const int64_t *rp = c->rp.as<int64_t>();
    k_sched_count<<<grid_for(n, 256, 65536), 256, 0, s>>>(n, rp, C, nch, is_long);
    CLEORA_LAUNCH_CHECK();
    exclusive_scan(nch, n, c->chunk_base.as<int64_t>(), c->t_scan.as<int64_t>(), s);
    exclusive_scan(is_long, n, long_pos, c->t_scan.as<int64_t>(), s);
    CLEORA_HIP(hipMemcpyAsync(c->h_small + 2, c->chunk_base.as<int64_t>() + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    CLEORA_HIP(hipMemcpyAsync(c->h_small + 3, long_pos + n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    CLEORA_HIP(hipStreamSynchronize(s));
    c->n_split = c->h_small[2];
    c->n_long = c->h_small[3];
    c->n_buckets = (c->nnz + n) / P + 1;
    c->split_items.ensure(sizeof(int2) * (size_t)std::max<int64_t>(c->n_split, 1));
    c->long_rows.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(c->n_long, 1));
    c->bucket_row.ensure(sizeof(int32_t) * ((size_t)c->n_buckets + 1));
    k_sched_fill<<<grid_for(n, 256, 65536), 256, 0, s>>>(n, c->chunk_base.as<int64_t>(), long_pos,
                                                         c->split_items.as<int2>(),
                                                         c->long_rows.as<int32_t>());
    CLEORA_LAUNCH_CHECK();
    k_buckets<<<grid_for(c->n_buckets + 1, 256, 65536), 256, 0, s>>>(
        n, rp, P, c->n_buckets, c->bucket_row.as<int32_t>());
    CLEORA_LAUNCH_CHECK();
}

StepDesc host_desc(const cleora_ctx *c, int parity)
{
    StepDesc d{};
    d.rp = c->rp.as<int64_t>();
    d.col = c->col.as<int32_t>();
    d.val = c->val.as<float>();
    d.Ein = c->E[parity].p;
    d.Eout = c->E[parity ^ 1].p;
    d.partial = c->partial.as<float>();
    d.split_items = c->split_items.as<int2>();
    d.bucket_row = c->bucket_row.as<int32_t>();
    d.long_rows = c->long_rows.as<int32_t>();
    d.chunk_base = c->chunk_base.as<int64_t>();
    d.wave_begin = 0;
    d.block_begin = 0;
    d.n_split = c->n_split;
    d.n_buckets = c->n_buckets;
    d.n_long = c->n_long;
    d.ld = c->ld;
    d.chunk = c->chunk;
    d.flags = c->flags;
    d.persist = c->persist;
    return d;
}

void write_descs(cleora_ctx *c, hipStream_t s)
{
    StepDesc h[2] = {host_desc(c, 0), host_desc(c, 1)};
    c->desc.ensure(sizeof(h));
    CLEORA_HIP(hipMemcpyAsync(c->desc.p, h, sizeof(h), hipMemcpyHostToDevice, s));
    std::vector<StepDesc> sl;
    if (c->slice_cols > 0) {
        // column slices: entry p * S + j reads buffer p, columns of slice j
        c->slice_norms.ensure(2 * sizeof(float) * (size_t)std::max<int64_t>(c->n, 1));
        c->val2.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->nnz, 1));
        for (int p = 0; p < 2; ++p)
            for (int32_t c0 = 0; c0 < c->ld; c0 += c->slice_cols) {
                sl.push_back(slice_desc(c, p, c0));
                // a persistent grid's occupancy query, outside any capture
                if (p == 0)
                    prime_spmm(choose_variant(c->dtype, std::min(c->slice_cols, c->ld - c0)),
                               c->persist, true);
            }
        c->slice_desc.ensure(sizeof(StepDesc) * sl.size());
        CLEORA_HIP(hipMemcpyAsync(c->slice_desc.p, sl.data(), sizeof(StepDesc) * sl.size(),
                                  hipMemcpyHostToDevice, s));
    }
    CLEORA_HIP(hipStreamSynchronize(s));
}

StepDesc slice_desc(const cleora_ctx *c, int parity, int32_t c0)
{
    StepDesc d = host_desc(c, parity);  // the row stride stays ld
    const size_t off = (size_t)c0 * (c->dtype == CLEORA_BF16 ? 2 : 4);
    d.Ein = static_cast<const char *>(d.Ein) + off;
    d.Eout = static_cast<char *>(d.Eout) + off;
    d.row_ss = c->slice_norms.as<float>();
    d.keep_rows = 1;
    return d;
}

}  // namespace cleora
