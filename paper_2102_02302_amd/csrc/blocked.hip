// Column-blocked propagation: T_k of a graph whose N x d embedding does not
// fit in device memory, computed `block` columns at a time.
//
// Columns of T interact only through the row norms (Section 3.2: each
// iteration multiplies by M, which acts on every column alike, then
// normalises each row), so with s_t[a] = 1 / ||(M T_{t-1})_a||
//     T_t = diag(s_t) M T_{t-1},
// and a block of columns follows its own chain once s_1 .. s_{t-1} are
// known.  Pass t (t = 1 .. k) runs every block from T_0 through t - 1
// scaled steps and one more SpMM whose epilogue adds the block's share of
// each row's squared norm to a vector; after the last block the vector
// becomes s_t.  A final pass runs every block through all k scaled steps
// and copies it out.  That is k(k+1)/2 + k block iterations instead of k,
// with two N x block buffers (plus k + 1 float vectors of N) in place of
// two N x d buffers.  Empty rows follow the graph's flag: zero, or (with
// CLEORA_EMPTY_KEEP) the previous row, whose squared norm is what the SpMM
// epilogue sees for that row.
//
// With a single block the arithmetic is that of init + k fused iterations
// step for step (the squared norm is added to zero, 1/sqrt is taken with
// the same expression, and the product with the row is the same), so the
// result is bit-identical to it.
//
// The same row-norm helpers (zeroing, 1/sqrt, scaling rows) serve the
// column-slice option of ordinary iterations, whose loop is in the runtime.
#include "internal.hpp"

#include <algorithm>
#include <vector>

namespace cleora {

namespace {

// s[a] = 1 / sqrt(ss[a]), 0 for an all-zero row: the fused kernel's
// normalisation factor, taken over the whole row.
__global__ void k_inv_norm(int64_t n, const float *__restrict__ ss, float *__restrict__ inv)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float x = ss[i];
        inv[i] = x > 0.0f ? 1.0f / sqrtf(x) : 0.0f;
    }
}

__global__ void k_fill_zero(int64_t n, float *__restrict__ x)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0f;
}

// One wave per row: the row's float4 vectors times its factor (the fused
// kernel's `acc * inv`, applied to the stored unscaled row).
__global__ void k_scale_rows(float4 *__restrict__ E, int64_t n, int32_t vpr,
                             const float *__restrict__ inv)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < n;
         r += waves) {
        const float f = inv[r];
        float4 *row = E + r * vpr;
        for (int32_t j = lane; j < vpr; j += 64) {
            float4 x = row[j];
            x.x *= f;
            x.y *= f;
            x.z *= f;
            x.w *= f;
            row[j] = x;
        }
    }
}

// One wave per row, out of place: dst row r = src row r times its factor.
__global__ void k_scale_rows_to(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                int64_t n, int32_t vpr, const float *__restrict__ inv)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < n;
         r += waves) {
        const float f = inv[r];
        const float4 *a = src + r * vpr;
        float4 *b = dst + r * vpr;
        for (int32_t j = lane; j < vpr; j += 64) {
            float4 x = a[j];
            x.x *= f;
            x.y *= f;
            x.z *= f;
            x.w *= f;
            b[j] = x;
        }
    }
}

// The same for bfloat16 rows: widened, scaled in float32, rounded to
// nearest even (eight elements per 16-byte vector).
__global__ void k_scale_rows_to_bf16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                     int64_t n, int32_t vpr, const float *__restrict__ inv)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < n;
         r += waves) {
        const float f = inv[r];
        const uint4 *a = src + r * vpr;
        uint4 *b = dst + r * vpr;
        for (int32_t j = lane; j < vpr; j += 64) {
            const uint4 x = a[j];
            uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                w[q] = f32_to_bf16_rne(bf16_lo(w[q]) * f) | (f32_to_bf16_rne(bf16_hi(w[q]) * f) << 16);
            b[j] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

// M diag(inv): every stored value times the factor of its column's row.
__global__ void k_scale_values(int64_t nnz, const float *__restrict__ val,
                               const int32_t *__restrict__ col, const float *__restrict__ inv,
                               float *__restrict__ out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = val[e] * inv[col[e]];
}

unsigned grid_for_rows(int64_t n, int per_block)
{
    return (unsigned)std::min<int64_t>(std::max<int64_t>((n + per_block - 1) / per_block, 1),
                                       65536);
}

}  // namespace

void launch_fill_zero(float *x, int64_t n, hipStream_t s)
{
    k_fill_zero<<<grid_for_rows(n, 256), 256, 0, s>>>(n, x);
    CLEORA_LAUNCH_CHECK();
}

void launch_inv_norm(const float *ss, float *inv, int64_t n, hipStream_t s)
{
    k_inv_norm<<<grid_for_rows(n, 256), 256, 0, s>>>(n, ss, inv);
    CLEORA_LAUNCH_CHECK();
}

void launch_scale_rows(float *E, int64_t n, int32_t ld, const float *inv, hipStream_t s)
{
    k_scale_rows<<<grid_for_rows(n, 4), 256, 0, s>>>(reinterpret_cast<float4 *>(E), n, ld / 4,
                                                     inv);
    CLEORA_LAUNCH_CHECK();
}

void launch_scale_rows_to(int dtype, const void *src, void *dst, int64_t n, int32_t ld,
                          const float *inv, hipStream_t s)
{
    if (dtype == CLEORA_BF16)
        k_scale_rows_to_bf16<<<grid_for_rows(n, 4), 256, 0, s>>>(
            reinterpret_cast<const uint4 *>(src), reinterpret_cast<uint4 *>(dst), n, ld / 8, inv);
    else
        k_scale_rows_to<<<grid_for_rows(n, 4), 256, 0, s>>>(
            reinterpret_cast<const float4 *>(src), reinterpret_cast<float4 *>(dst), n, ld / 4, inv);
    CLEORA_LAUNCH_CHECK();
}

void launch_scale_values(const float *val, const int32_t *col, const float *inv, int64_t nnz,
                         float *out, hipStream_t s)
{
    if (nnz <= 0) return;
    k_scale_values<<<grid_for_rows(nnz, 256), 256, 0, s>>>(nnz, val, col, inv, out);
    CLEORA_LAUNCH_CHECK();
}

void embed_blocked(cleora_ctx *c, int32_t dim, int32_t block, int32_t dtype, uint64_t seed,
                   int32_t k, void *out, int64_t ld_out, hipStream_t s)
{
    const int64_t n = c->n;
    const size_t es = dtype == CLEORA_BF16 ? 2 : 4;
    const int32_t epv = (int32_t)(16 / es);
    c->blk_norms.ensure(sizeof(float) * (size_t)n * ((size_t)k + 1));
    float *scale = c->blk_norms.as<float>();  // row t - 1: s_t, t = 1 .. k
    float *ss = scale + (size_t)n * k;        // squared norms being summed
    const int32_t *ids = c->is_chunk ? c->chunk_ids.as<int32_t>() : nullptr;

    // Descriptors of one block width: entry 2m + p reads buffer p; mode
    // m < k scales by s_{m+1}, mode k sums squared norms.  The combine
    // kernel reads them from device memory.
    std::vector<StepDesc> tab;
    int32_t tab_ld = -1;
    auto set_width = [&](int32_t w) {
        const int32_t ld = (w + epv - 1) / epv * epv;
        if (ld == tab_ld) return;
        c->ld = ld;
        tab.assign(2 * ((size_t)k + 1), StepDesc{});
        for (int32_t m = 0; m <= k; ++m)
            for (int p = 0; p < 2; ++p) {
                StepDesc d = host_desc(c, p);
                d.row_scale = m < k ? scale + (size_t)m * n : nullptr;
                d.row_ss = m == k ? ss : nullptr;
                tab[2 * (size_t)m + p] = d;
            }
        c->desc.ensure(sizeof(StepDesc) * tab.size());
        CLEORA_HIP(hipMemcpyAsync(c->desc.p, tab.data(), sizeof(StepDesc) * tab.size(),
                                  hipMemcpyHostToDevice, s));
        CLEORA_HIP(hipStreamSynchronize(s));  // tab is rewritten for the next width
        tab_ld = ld;
    };
    // T_0 columns [c0, c0 + w) into buffer 0
    auto start_block = [&](int32_t c0, int32_t w) {
        set_width(w);
        launch_init(dtype, c->E[0].p, n, w, c->ld, nullptr, nullptr, 1, seed, s, ids, 0, dim, c0);
    };
    // one iteration of the current block in mode m (see tab)
    auto step = [&](const Variant &v, int32_t m, int &cur) {
        const size_t i = 2 * (size_t)m + cur;
        launch_spmm(v, tab[i], s);
        if (c->n_long > 0) launch_combine(v, c->desc.as<StepDesc>() + i, 1, c->n_long, s);
        if (m < k) cur ^= 1;  // the squared-norm mode stores no rows
    };

    const int32_t nb = (dim + block - 1) / block;
    const unsigned ng = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    for (int32_t t = 1; t <= k; ++t) {
        CLEORA_HIP(hipMemsetAsync(ss, 0, sizeof(float) * (size_t)n, s));
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t c0 = b * block, w = std::min(block, dim - c0);
            start_block(c0, w);
            const Variant v = choose_variant(dtype, c->ld);
            int cur = 0;
            for (int32_t m = 0; m + 1 < t; ++m) step(v, m, cur);
            step(v, k, cur);
        }
        k_inv_norm<<<ng, 256, 0, s>>>(n, ss, scale + (size_t)(t - 1) * n);
        CLEORA_LAUNCH_CHECK();
    }
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t c0 = b * block, w = std::min(block, dim - c0);
        start_block(c0, w);
        const Variant v = choose_variant(dtype, c->ld);
        int cur = 0;
        for (int32_t m = 0; m < k; ++m) step(v, m, cur);
        CLEORA_HIP(hipMemcpy2DAsync(static_cast<char *>(out) + (size_t)c0 * es,
                                    (size_t)ld_out * es, c->E[cur].p, (size_t)c->ld * es,
                                    (size_t)w * es, (size_t)n, hipMemcpyDefault, s));
    }
    CLEORA_HIP(hipStreamSynchronize(s));
}

}  // namespace cleora
