// Graph -> CSR of M = D^-1 A on the GPU (Section 3.2 of the paper: e_ab is
// the number of a->b edges or the sum of their weights, M_ab = e_ab/deg(a);
// undirected edges are stored in both directions, Section 4.5).
//
// Pipeline (caller's stream, one host synchronisation at the end):
//   1. one 64-bit key per stored entry, key = row << cb | col (cb = bits of
//      the column count - 1); a loop's second copy and invalid edges get
//      the key of row n, column 0, above every valid one; optional float32
//      weight as payload.  Rows and columns may number differently (new
//      nodes against existing ones); undirected graphs are square;
//   2. stable LSD radix sort of the keys (8-bit digits over bits(n + 1) +
//      cb bits, reduce-then-scan: per-tile digit counts, one device scan,
//      stable scatter through LDS, each wave ranking its own part of the
//      tile) -- no global atomics, so hub rows cost no more than other rows,
//      and repeated (a, b) pairs keep their input order;
//   3. mark the first entry of each run of equal keys, scan, compact: one
//      merged entry per pair with e_ab summed in float64 in input order;
//   4. row pointers by binary search over the merged keys;
//   5. deg(a) = sum_b e_ab in float64 and M_ab = e_ab / deg(a) in float32
//      (four rows per wave; rows over LONG_ROW entries in LONG_ROW-entry
//      segments, one wave each, added in segment order: a fixed reduction
//      order everywhere).
#include "internal.hpp"

#include <algorithm>

namespace cleora {

namespace {

constexpr uint32_t ERR_ID = 1u, ERR_WEIGHT = 2u;

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 32;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // keys per block and pass
constexpr int MG_ITEMS = 16;
constexpr int MG_TILE = RS_THREADS * MG_ITEMS;  // entries per block of the merge
constexpr int LONG_ROW = 4096;                  // rows summed in segments

__device__ __forceinline__ int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ bool weight_ok(float x)
{
    return x > 0.0f && x <= 3.402823466e38f;  // finite and positive
}

// Keys of the stored entries: entry 2e is edge e as given, entry 2e+1 its
// reverse (undirected graphs); directed graphs use entry e only.  Invalid
// edges and a loop's second copy get invalid_key, which sorts last; the
// number of valid entries is found after the sort.  Block b makes entries
// [b * RS_TILE, (b + 1) * RS_TILE), one radix tile, and also counts their
// first digits as the sort's first counting pass would:
// count[d * nblk + b] = entries of tile b whose low 8 bits are d.
__global__ __launch_bounds__(RS_THREADS) void k_make_keys(
    int64_t m, int64_t n_rows, int64_t n_cols, const int32_t *__restrict__ src,
    const int32_t *__restrict__ dst, const float *__restrict__ w, int directed, int cb,
    uint64_t invalid_key, int64_t total, int64_t nblk, uint64_t *__restrict__ keys,
    float *__restrict__ wout, int32_t *__restrict__ count, uint32_t *err)
{
    __shared__ uint32_t h[RS_THREADS / WAVE][256];
    const int t = threadIdx.x, w_ = t >> 6;
    for (int i = t; i < (RS_THREADS / WAVE) * 256; i += RS_THREADS) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = base + i * RS_THREADS + t;  // entry
        const bool valid = idx < total;
        uint64_t key = 0;
        if (valid) {
            const int64_t e = directed ? idx : idx >> 1;
            const bool rev = !directed && (idx & 1);
            const int32_t a = src[e], b = dst[e];
            bool ok = a >= 0 && a < n_rows && b >= 0 && b < n_cols;
            if (!ok && !rev) atomicOr(err, ERR_ID);
            float x = 1.0f;
            if (w) {
                x = w[e];
                if (ok && !weight_ok(x)) {
                    if (!rev) atomicOr(err, ERR_WEIGHT);
                    ok = false;
                }
            }
            if (rev) key = ok && a != b ? ((uint64_t)b << cb) | (uint64_t)a : invalid_key;
            else key = ok ? ((uint64_t)a << cb) | (uint64_t)b : invalid_key;
            keys[idx] = key;
            if (wout) wout[idx] = x;
        }
        if (valid) atomicAdd(&h[w_][(uint32_t)key & 255u], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
    for (int q = 0; q < RS_THREADS / WAVE; ++q) c += h[q][t];
    count[(int64_t)t * nblk + blockIdx.x] = (int32_t)c;
    (void)m;
}

// n_valid = number of sorted keys below invalid_key (one thread).
__global__ void k_count_valid(int64_t total, const uint64_t *__restrict__ keys,
                              uint64_t invalid_key, unsigned long long *n_valid)
{
    int64_t lo = 0, hi = total;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] >= invalid_key) hi = mid;
        else lo = mid + 1;
    }
    *n_valid = (unsigned long long)lo;
}

// Radix pass, step 1: count[d * nblk + b] = keys of tile b with digit d.
__global__ __launch_bounds__(RS_THREADS) void k_rs_count(const uint64_t *__restrict__ keys,
                                                         int64_t n, int shift, int64_t nblk,
                                                         int32_t *__restrict__ count)
{
    __shared__ uint32_t h[RS_THREADS / WAVE][256];
    const int t = threadIdx.x, w = t >> 6;
    for (int i = t; i < (RS_THREADS / WAVE) * 256; i += RS_THREADS) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    // all of the tile's loads are issued before any digit is counted
    uint64_t key[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = base + i * RS_THREADS + t;
        key[i] = idx < n ? keys[idx] : 0;
    }
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        // one LDS add per key into the wave's own counts (finding a lane's
        // digit peers by ballots first costs more VALU work than the
        // conflicting adds it saves)
        if (base + i * RS_THREADS + t < n)
            atomicAdd(&h[w][(uint32_t)(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    uint32_t s = 0;
    for (int q = 0; q < RS_THREADS / WAVE; ++q) s += h[q][t];
    count[(int64_t)t * nblk + blockIdx.x] = (int32_t)s;
}

// Radix pass, step 3: stable scatter.  Wave w ranks the w-th quarter of
// the tile's keys in rounds of 64 (by round, then lane), keeping running
// per-digit counts in its own LDS row, so ranking needs no block barrier;
// one per-digit prefix over the waves then gives every key its place in
// the tile in input order.  Keys are staged in LDS in digit order and
// written out run by run.
template <bool PAYLOAD>
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const float *__restrict__ pin, int64_t n, int shift,
    int64_t nblk, const int64_t *__restrict__ offs, uint64_t *__restrict__ kout,
    float *__restrict__ pout)
{
    constexpr int NW = RS_THREADS / WAVE;  // waves per block
    constexpr int CHUNK = RS_TILE / NW;    // keys per wave
    static_assert(RS_THREADS == 256, "one thread per digit");
    __shared__ uint64_t sk[RS_TILE];
    __shared__ float sp[PAYLOAD ? RS_TILE : 1];
    // per-wave digit counts, then per-wave digit starts, then (as int64)
    // each digit's output position minus its start in the tile
    __shared__ __align__(16) uint32_t wc[NW][256];
    __shared__ uint32_t total[256];
    __shared__ uint32_t dstart[256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const int64_t wbase = base + (int64_t)w * CHUNK;
    // where this tile's keys of digit t go (loaded now, used at the end)
    const int64_t goff = offs[(int64_t)t * nblk + blockIdx.x];
    uint64_t key[RS_ITEMS];
    float pay[PAYLOAD ? RS_ITEMS : 1];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = wbase + i * WAVE + lane;
        key[i] = idx < n ? kin[idx] : 0;
        if constexpr (PAYLOAD) pay[i] = idx < n ? pin[idx] : 0.0f;
    }
    for (int q = lane; q < 256; q += WAVE) wc[w][q] = 0;
    uint32_t rank[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const bool valid = wbase + i * WAVE + lane < n;
        const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t mk = __ballot(bit);
            peers &= bit ? mk : ~mk;
        }
        const uint32_t below = (uint32_t)__popcll(peers & ((1ull << lane) - 1ull));
        // the wave's own row: earlier writes by other lanes of this wave
        // must be seen, later ones must not be read early
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t before = wc[w][d];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) wc[w][d] = before + (uint32_t)__popcll(peers);
        rank[i] = valid ? before + below : 0xffffffffu;
    }
    __syncthreads();
    {
        // digit t: exclusive prefix over the waves
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const uint32_t c = wc[q][t];
            wc[q][t] = s;
            s += c;
        }
        total[t] = s;
    }
    __syncthreads();
    // local digit starts: exclusive scan of total[] (256 entries, one wave)
    if (w == 0) {
        uint32_t v[4], tot = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = total[lane * 4 + q];
            tot += v[q];
        }
        uint32_t x = tot;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        uint32_t s = x - tot;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            dstart[lane * 4 + q] = s;
            s += v[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        if (rank[i] == 0xffffffffu) continue;
        const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
        const uint32_t lp = dstart[d] + wc[w][d] + rank[i];
        sk[lp] = key[i];
        if constexpr (PAYLOAD) sp[lp] = pay[i];
    }
    __syncthreads();
    int64_t *gbase = reinterpret_cast<int64_t *>(&wc[0][0]);  // wc is free now
    gbase[t] = goff - (int64_t)dstart[t];
    __syncthreads();
    const int64_t cnt = min((int64_t)RS_TILE, n - base);
    for (int j = t; j < cnt; j += RS_THREADS) {
        const uint64_t k = sk[j];
        const int64_t g = gbase[(uint32_t)(k >> shift) & 255u] + j;
        kout[g] = k;
        if constexpr (PAYLOAD) pout[g] = sp[j];
    }
}

// Merging repeated pairs of the sorted keys (entries [0, total), invalid
// keys last).  Entry i starts a merged entry (a run of equal keys) when it
// is valid and differs from entry i - 1.  Block b covers indices
// [b * MG_TILE, (b + 1) * MG_TILE) of [0, total], index total standing for
// the end; wave w of the block a contiguous quarter of that, in rounds of 64.
// A wave loads its keys once; entry i - 1 (and i + 1) come from the
// neighbouring lane or round, and from memory only at the chunk's edges.
struct MergeChunk {
    uint64_t key[MG_ITEMS], prev[MG_ITEMS], hb[MG_ITEMS];
};

__device__ __forceinline__ void load_chunk(const uint64_t *__restrict__ keys, int64_t wbase,
                                           int64_t total, uint64_t invalid_key, int lane,
                                           MergeChunk &c)
{
#pragma unroll
    for (int i = 0; i < MG_ITEMS; ++i) {
        const int64_t idx = wbase + i * WAVE + lane;
        c.key[i] = idx < total ? keys[idx] : 0;
    }
    const uint64_t edge = wbase > 0 && wbase <= total ? keys[wbase - 1] : 0;
#pragma unroll
    for (int i = 0; i < MG_ITEMS; ++i) {
        const int64_t idx = wbase + i * WAVE + lane;
        const uint64_t up = __shfl_up(c.key[i], 1, WAVE);
        const uint64_t carry = i == 0 ? edge : __shfl(c.key[i > 0 ? i - 1 : 0], WAVE - 1, WAVE);
        c.prev[i] = lane == 0 ? carry : up;
        c.hb[i] = __ballot(idx < total && c.key[i] < invalid_key &&
                           (idx == 0 || c.prev[i] != c.key[i]));
    }
}

// hcount[b] = merged entries starting in block b.
__global__ __launch_bounds__(RS_THREADS) void k_merge_count(const uint64_t *__restrict__ keys,
                                                            int64_t total, uint64_t invalid_key,
                                                            int64_t *__restrict__ hcount)
{
    constexpr int NW = RS_THREADS / WAVE, CHUNK = MG_TILE / NW;
    __shared__ uint32_t wsum[NW];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t wbase = (int64_t)blockIdx.x * MG_TILE + (int64_t)w * CHUNK;
    MergeChunk c;
    load_chunk(keys, wbase, total, invalid_key, lane, c);
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < MG_ITEMS; ++i) cnt += (uint32_t)__popcll(c.hb[i]);
    if (lane == 0) wsum[w] = cnt;
    __syncthreads();
    if (t == 0) {
        int64_t sum = 0;
        for (int q = 0; q < NW; ++q) sum += wsum[q];
        hcount[blockIdx.x] = sum;
    }
}

// One merged entry per run, at hoff[b] + (runs before it in the block):
// column and e_ab (count, or float64 sum of the run's weights in input
// order).  Row pointers come from the same pass: where the row changes
// between index i - 1 and i (the end and invalid keys count as row n),
// rows (row(i - 1), row(i)] start at the number of merged entries before i.
__global__ __launch_bounds__(RS_THREADS) void k_merge(
    const uint64_t *__restrict__ keys, const float *__restrict__ wts, int64_t total,
    uint64_t invalid_key, int cb, int64_t n, const int64_t *__restrict__ hoff,
    int32_t *__restrict__ col_u, double *__restrict__ e_u, int64_t *__restrict__ rp)
{
    constexpr int NW = RS_THREADS / WAVE, CHUNK = MG_TILE / NW;
    __shared__ uint32_t wsum[NW];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t wbase = (int64_t)blockIdx.x * MG_TILE + (int64_t)w * CHUNK;
    const uint64_t cmask = ((uint64_t)1 << cb) - 1;
    MergeChunk c;
    load_chunk(keys, wbase, total, invalid_key, lane, c);
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < MG_ITEMS; ++i) cnt += (uint32_t)__popcll(c.hb[i]);
    if (lane == 0) wsum[w] = cnt;
    __syncthreads();
    int64_t u0 = hoff[blockIdx.x];
    for (int q = 0; q < w; ++q) u0 += wsum[q];
    const uint64_t lt = (1ull << lane) - 1ull;
    // entry after the chunk (for the last lane of the last round)
    const int64_t after = wbase + CHUNK;
    const uint64_t edge_next = after < total ? keys[after] : 0;
#pragma unroll
    for (int i = 0; i < MG_ITEMS; ++i) {
        const int64_t idx = wbase + i * WAVE + lane;
        const int64_t u = u0 + __popcll(c.hb[i] & lt);  // merged entries before idx
        u0 += __popcll(c.hb[i]);
        const uint64_t k = c.key[i];
        const uint64_t down = __shfl_down(k, 1, WAVE);
        const uint64_t carry =
            i + 1 < MG_ITEMS ? __shfl(c.key[i + 1 < MG_ITEMS ? i + 1 : i], 0, WAVE) : edge_next;
        const uint64_t next = lane == WAVE - 1 ? carry : down;
        if ((c.hb[i] >> lane) & 1ull) {
            col_u[u] = (int32_t)(k & cmask);
            double sum = wts ? (double)wts[idx] : 1.0;
            if (idx + 1 < total && next == k) {  // a repeated pair: add up its run
                for (int64_t j = idx + 1; j < total && keys[j] == k; ++j)
                    sum += wts ? (double)wts[j] : 1.0;
            }
            e_u[u] = sum;
        }
        // rows starting at idx (indices past the end start none)
        int64_t r_lo = 0, r_hi = -1;
        if (idx <= total) {
            const uint64_t pk = c.prev[i];
            const int64_t row = idx < total && k < invalid_key ? (int64_t)(k >> cb) : n;
            const int64_t prow = idx == 0 ? -1 : pk < invalid_key ? (int64_t)(pk >> cb) : n;
            r_lo = prow + 1;
            r_hi = row;
        }
        if (r_hi - r_lo < WAVE) {
            for (int64_t r = r_lo; r <= r_hi; ++r) rp[r] = u;
        }
        // a long run of empty rows: the whole wave writes it
        uint64_t big = __ballot(r_hi - r_lo >= WAVE);
        while (big) {
            const int l = __ffsll((unsigned long long)big) - 1;
            big &= big - 1;
            const int64_t lo = __shfl(r_lo, l), hi = __shfl(r_hi, l), ul = __shfl(u, l);
            for (int64_t r = lo + lane; r <= hi; r += WAVE) rp[r] = ul;
        }
    }
}

// occ[r] = stored entries of row r before repeated pairs are merged (the
// row's endpoint occurrences in the edge list), by binary search over the
// n_valid sorted keys.
__global__ void k_row_counts(int64_t n, const unsigned long long *__restrict__ n_valid,
                             const uint64_t *__restrict__ keys, int cb, float *__restrict__ occ)
{
    const int64_t nv = (int64_t)*n_valid;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t bound[2];
        for (int q = 0; q < 2; ++q) {
            const uint64_t target = (uint64_t)(r + q) << cb;
            int64_t lo = 0, hi = nv;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (keys[mid] >= target) hi = mid;
                else lo = mid + 1;
            }
            bound[q] = lo;
        }
        occ[r] = (float)(bound[1] - bound[0]);
    }
}

// deg(a) and M values, four rows per wave.  Rows of at most 16 (32)
// entries are summed by 16- (32-) lane groups, whatever the other rows of
// the wave hold: a 64-lane butterfly over a row that short only adds exact
// zeros in its first steps, so the grouping gives the same bits.  Longer
// rows take one 64-lane pass each, with the first 64 entries of all of
// them loaded before any is reduced; rows longer than LONG_ROW are listed
// for the segmented kernels.
__global__ __launch_bounds__(256) void k_rowsum_wave(int64_t n, const int64_t *__restrict__ rp,
                                                     const double *__restrict__ e_u,
                                                     float *__restrict__ val,
                                                     double *__restrict__ deg,
                                                     int32_t *__restrict__ long_list,
                                                     int32_t *__restrict__ long_count)
{
    const int64_t r0 =
        ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * 4;
    if (r0 >= n) return;
    const int lane = threadIdx.x & 63;
    const int nr = (int)min((int64_t)4, n - r0);
    int64_t lo[4], hi[4];
    bool mid = false, big = false;  // rows of 17..32, and of more than 32 entries
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        lo[q] = q < nr ? rp[r0 + q] : 0;
        hi[q] = q < nr ? rp[r0 + q + 1] : 0;
        mid |= hi[q] - lo[q] > 16 && hi[q] - lo[q] <= 32;
        big |= hi[q] - lo[q] > 32;
    }
    {
        // rows of at most 16 entries: 16 lanes each, all four at once
        const int q = lane >> 4, gl = lane & 15;
        const int64_t l = q == 0 ? lo[0] : q == 1 ? lo[1] : q == 2 ? lo[2] : lo[3];
        const int64_t h = q == 0 ? hi[0] : q == 1 ? hi[1] : q == 2 ? hi[2] : hi[3];
        const bool mine = q < nr && h - l <= 16;
        const bool has = mine && l + gl < h;
        const double e = has ? e_u[l + gl] : 0.0;
        const double sum = group_sum<16>(e);
        if (mine && gl == 0) deg[r0 + q] = sum;
        if (has) val[l + gl] = (float)(e / sum);
    }
    if (mid) {
        // rows of 17..32 entries: 32 lanes each, two at a time
        const int half = lane >> 5, gl = lane & 31;
        double e[2];
        int64_t at[2];
        bool mine[2], has[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int q = 2 * p + half;
            const int64_t l = half ? lo[2 * p + 1] : lo[2 * p];
            const int64_t h = half ? hi[2 * p + 1] : hi[2 * p];
            mine[p] = q < nr && h - l > 16 && h - l <= 32;
            at[p] = l + gl;
            has[p] = mine[p] && at[p] < h;
            e[p] = has[p] ? e_u[at[p]] : 0.0;
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const double sum = group_sum<32>(e[p]);
            if (mine[p] && gl == 0) deg[r0 + 2 * p + half] = sum;
            if (has[p]) val[at[p]] = (float)(e[p] / sum);
        }
    }
    if (!big) return;
    // longer rows: the first 64 entries of all of them are loaded before
    // any is reduced (independent loads in flight, not one after another)
    double first[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t len = hi[q] - lo[q];
        first[q] = q < nr && len > 32 && len <= LONG_ROW && lo[q] + lane < hi[q]
                       ? e_u[lo[q] + lane]
                       : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= nr) break;
        const int64_t row = r0 + q;
        if (hi[q] - lo[q] <= 32) continue;
        if (hi[q] - lo[q] > LONG_ROW) {
            if (lane == 0) long_list[atomicAdd(long_count, 1)] = (int32_t)row;
            continue;
        }
        double s = first[q];
        for (int64_t j = lo[q] + 64 + lane; j < hi[q]; j += 64) s += e_u[j];
        s = wave_sum(s);
        if (lane == 0) deg[row] = s;
        if (lo[q] + lane < hi[q]) val[lo[q] + lane] = (float)(first[q] / s);
        for (int64_t j = lo[q] + 64 + lane; j < hi[q]; j += 64) val[j] = (float)(e_u[j] / s);
    }
}

// Long rows: segment q of a listed row (LONG_ROW entries each) is summed by
// one wave in a fixed order into seg[...]; k_rowsum_long then adds a row's
// segment sums in order and writes deg and the M values.  Listed rows get
// consecutive segment slots from an exclusive scan of their segment counts.
// nseg[i] = segments of listed row i, zero for i in [count, n).
__global__ void k_long_segments(int64_t n, const int32_t *__restrict__ list,
                                const int32_t *__restrict__ count,
                                const int64_t *__restrict__ rp, int32_t *__restrict__ nseg)
{
    const int cnt = *count;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = 0;
        if (i < cnt) {
            const int64_t r = list[i];
            v = (int32_t)ceil_div_dev(rp[r + 1] - rp[r], LONG_ROW);
        }
        nseg[i] = v;
    }
}

__global__ __launch_bounds__(256) void k_rowsum_segments(
    const int32_t *__restrict__ list, const int32_t *__restrict__ count,
    const int64_t *__restrict__ seg_base, const int64_t *__restrict__ rp,
    const double *__restrict__ e_u, double *__restrict__ seg)
{
    const int cnt = *count;
    const int64_t nseg_total = cnt > 0 ? seg_base[cnt] : 0;
    const int lane = threadIdx.x & 63;
    for (int64_t q = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
         q < nseg_total; q += (int64_t)gridDim.x * 4) {
        int lo = 0, hi = cnt - 1;  // the listed row owning segment q
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (seg_base[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        const int64_t r = list[lo];
        const int64_t b = rp[r] + (q - seg_base[lo]) * LONG_ROW;
        const int64_t e = min(b + (int64_t)LONG_ROW, rp[r + 1]);
        double acc = 0.0;
        for (int64_t j = b + lane; j < e; j += 64) acc += e_u[j];
        acc = wave_sum(acc);
        if (lane == 0) seg[q] = acc;
    }
}

// deg of each listed row: its segment sums added in segment order.
__global__ void k_rowsum_long(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                              const int64_t *__restrict__ seg_base,
                              const double *__restrict__ seg, double *__restrict__ deg)
{
    const int cnt = *count;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x) {
        double d = 0.0;
        for (int64_t q = seg_base[i]; q < seg_base[i + 1]; ++q) d += seg[q];
        deg[list[i]] = d;
    }
}

// M values of the listed rows, one wave per segment (a hub row of 200k
// entries is spread over 49 waves instead of one block).
__global__ __launch_bounds__(256) void k_long_values(
    const int32_t *__restrict__ list, const int32_t *__restrict__ count,
    const int64_t *__restrict__ seg_base, const int64_t *__restrict__ rp,
    const double *__restrict__ e_u, const double *__restrict__ deg, float *__restrict__ val)
{
    const int cnt = *count;
    const int64_t nseg_total = cnt > 0 ? seg_base[cnt] : 0;
    const int lane = threadIdx.x & 63;
    for (int64_t q = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
         q < nseg_total; q += (int64_t)gridDim.x * 4) {
        int lo = 0, hi = cnt - 1;  // the listed row owning segment q
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (seg_base[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        const int64_t r = list[lo];
        const int64_t b = rp[r] + (q - seg_base[lo]) * LONG_ROW;
        const int64_t e = min(b + (int64_t)LONG_ROW, rp[r + 1]);
        const double d = deg[r];
        for (int64_t j = b + lane; j < e; j += 64) val[j] = (float)(e_u[j] / d);
    }
}

unsigned grid_for(int64_t items, int threads, int64_t cap = 1 << 20)
{
    int64_t g = ceil_div(items > 0 ? items : 1, threads);
    return (unsigned)std::min<int64_t>(g, cap);
}

int bits_for(int64_t n)
{
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n) ++b;
    return b;
}

}  // namespace

void build_graph(cleora_ctx *c, int64_t n, int64_t n_cols, int64_t m, const int32_t *src,
                 const int32_t *dst, const float *w, uint32_t flags, hipStream_t s, float *occ)
{
    c->has_graph = false;
    c->has_emb = false;
    const int directed = (flags & CLEORA_DIRECTED) ? 1 : 0;
    if (!directed && n_cols != n) throw Error(CLEORA_E_INVAL, "undirected graphs are square");
    const int64_t total = directed ? m : 2 * m;  // stored entries before merging
    const int64_t tot1 = std::max<int64_t>(total, 1);
    // key = row << cb | col; the invalid key is row n, col 0: above every
    // valid key, and inside rb = bits(n + 1) row bits, so it costs no pass
    const int cb = bits_for(n_cols), rb = bits_for(n + 1);
    const int key_bits = rb + cb;
    const uint64_t invalid_key = (uint64_t)n << cb;
    const int64_t nblk = ceil_div(tot1, RS_TILE);

    c->t_small.ensure(sizeof(int64_t) * 8);
    c->t_keys.ensure(sizeof(uint64_t) * (size_t)tot1);
    c->t_tmp.ensure(sizeof(uint64_t) * (size_t)tot1);
    c->t_esum.ensure(sizeof(double) * (size_t)tot1);
    // digit counts of a radix pass, later the long-row list and its segment counts
    c->t_cnt.ensure(sizeof(int32_t) * std::max(256 * (size_t)nblk, 2 * (size_t)n));
    const int64_t scan_max = std::max<int64_t>(std::max<int64_t>(tot1 + 1, 256 * nblk + 1), n + 1);
    c->t_pos.ensure(sizeof(int64_t) * (size_t)scan_max);
    c->t_scan.ensure(sizeof(int64_t) * scan_workspace_elems(scan_max));
    // weight payload (kept apart from t_edges, which may hold the input edges)
    c->t_wts.ensure(w ? 2 * sizeof(float) * (size_t)tot1 : 256);
    c->rp.ensure(sizeof(int64_t) * ((size_t)n + 1));
    c->col.ensure(sizeof(int32_t) * (size_t)tot1);
    c->val.ensure(sizeof(float) * (size_t)tot1);
    c->deg.ensure(sizeof(double) * (size_t)n);

    int64_t *small = c->t_small.as<int64_t>();
    uint32_t *err = reinterpret_cast<uint32_t *>(small);                     // [0]
    unsigned long long *n_valid = reinterpret_cast<unsigned long long *>(small + 1);
    int32_t *long_count = reinterpret_cast<int32_t *>(small + 2);
    uint64_t *keys = c->t_keys.as<uint64_t>(), *tmpk = c->t_tmp.as<uint64_t>();
    float *wa = w ? c->t_wts.as<float>() : nullptr, *wb = w ? wa + tot1 : nullptr;
    int32_t *count = c->t_cnt.as<int32_t>();
    int64_t *pos = c->t_pos.as<int64_t>(), *ws = c->t_scan.as<int64_t>();

    CLEORA_HIP(hipMemsetAsync(small, 0, sizeof(int64_t) * 4, s));
    // stable LSD radix sort of the keys (and weights); the first pass's
    // digit counts come with the keys
    if (total > 0) {
        k_make_keys<<<(unsigned)nblk, RS_THREADS, 0, s>>>(m, n, n_cols, src, dst, w, directed, cb,
                                                          invalid_key, total, nblk, keys, wa,
                                                          count, err);
        CLEORA_LAUNCH_CHECK();
        for (int shift = 0; shift < key_bits; shift += 8) {
            if (shift > 0) {
                k_rs_count<<<(unsigned)nblk, RS_THREADS, 0, s>>>(keys, total, shift, nblk, count);
                CLEORA_LAUNCH_CHECK();
            }
            exclusive_scan(count, 256 * nblk, pos, ws, s);
            if (w)
                k_rs_scatter<true><<<(unsigned)nblk, RS_THREADS, 0, s>>>(keys, wa, total, shift,
                                                                          nblk, pos, tmpk, wb);
            else
                k_rs_scatter<false><<<(unsigned)nblk, RS_THREADS, 0, s>>>(
                    keys, nullptr, total, shift, nblk, pos, tmpk, nullptr);
            CLEORA_LAUNCH_CHECK();
            std::swap(keys, tmpk);
            std::swap(wa, wb);
        }
    }
    // merge repeated pairs; row pointers
    const int64_t nblk_m = ceil_div(total + 1, MG_TILE);  // indices [0, total]
    int64_t *hcount = pos, *hoff = pos + nblk_m;           // nblk_m + (nblk_m + 1) entries
    k_merge_count<<<(unsigned)nblk_m, RS_THREADS, 0, s>>>(keys, total, invalid_key, hcount);
    CLEORA_LAUNCH_CHECK();
    exclusive_scan(hcount, nblk_m, hoff, ws, s);
    if (occ) {
        if (total > 0) {
            k_count_valid<<<1, 1, 0, s>>>(total, keys, invalid_key, n_valid);
            CLEORA_LAUNCH_CHECK();
        }
        k_row_counts<<<grid_for(n, 256, 65536), 256, 0, s>>>(n, n_valid, keys, cb, occ);
        CLEORA_LAUNCH_CHECK();
    }
    double *esum = c->t_esum.as<double>();
    k_merge<<<(unsigned)nblk_m, RS_THREADS, 0, s>>>(keys, wa, total, invalid_key, cb, n, hoff,
                                                    c->col.as<int32_t>(), esum,
                                                    c->rp.as<int64_t>());
    CLEORA_LAUNCH_CHECK();
    // deg(a) and M values
    int32_t *long_list = count;  // the digit counts are no longer needed
    k_rowsum_wave<<<(unsigned)ceil_div(n, 16), 256, 0, s>>>(n, c->rp.as<int64_t>(), esum,
                                                           c->val.as<float>(), c->deg.as<double>(),
                                                           long_list, long_count);
    CLEORA_LAUNCH_CHECK();
    {
        // long rows: per-segment sums, then per-row totals in segment order
        int32_t *nseg = long_list + n;  // the count buffer holds >= 2n entries
        int64_t *seg_base = pos;        // merged positions are not needed any more
        double *seg = reinterpret_cast<double *>(c->t_keys.p);  // sorted keys are done too
        k_long_segments<<<grid_for(n, 256, 65536), 256, 0, s>>>(n, long_list, long_count,
                                                                c->rp.as<int64_t>(), nseg);
        CLEORA_LAUNCH_CHECK();
        exclusive_scan(nseg, n, seg_base, ws, s);
        k_rowsum_segments<<<1024, 256, 0, s>>>(long_list, long_count, seg_base,
                                               c->rp.as<int64_t>(), esum, seg);
        CLEORA_LAUNCH_CHECK();
        k_rowsum_long<<<64, 256, 0, s>>>(long_list, long_count, seg_base, seg,
                                         c->deg.as<double>());
        CLEORA_LAUNCH_CHECK();
        k_long_values<<<1024, 256, 0, s>>>(long_list, long_count, seg_base, c->rp.as<int64_t>(),
                                           esum, c->deg.as<double>(), c->val.as<float>());
        CLEORA_LAUNCH_CHECK();
    }
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
    c->n = n;
    c->n_cols = n_cols;
    c->m_in = m;
    c->flags = flags;
    c->has_graph = true;
}

}  // namespace cleora
