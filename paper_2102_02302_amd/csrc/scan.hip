// Device-wide exclusive prefix sums (reduce, scan the block sums, scan the
// tiles).  Used to lay out the CSR and the propagation schedule.
#include "internal.hpp"

namespace cleora {

namespace {

constexpr int ST = 256;            // threads per block
constexpr int SI = 16;             // items per thread
constexpr int STILE = ST * SI;     // items per block

template <typename In>
__global__ __launch_bounds__(ST) void k_scan_reduce(const In *__restrict__ in, int64_t n,
                                                    int64_t *__restrict__ sums)
{
    __shared__ int64_t wsum[ST / WAVE];
    const int64_t base = (int64_t)blockIdx.x * STILE;
    int64_t s = 0;
    for (int i = threadIdx.x; i < STILE; i += ST) {
        int64_t idx = base + i;
        if (idx < n) s += (int64_t)in[idx];
    }
    s = wave_sum(s);
    if ((threadIdx.x & (WAVE - 1)) == 0) wsum[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < ST / WAVE; ++w) t += wsum[w];
        sums[blockIdx.x] = t;
    }
}

// Exclusive scan of one tile plus the block's offset; the block holding the
// last item also writes out[n] = total.
template <typename In>
__global__ __launch_bounds__(ST) void k_scan_tile(const In *__restrict__ in, int64_t n,
                                                  const int64_t *__restrict__ offsets,
                                                  int64_t *__restrict__ out)
{
    __shared__ int64_t tile[STILE];
    __shared__ int64_t wtot[ST / WAVE];
    const int64_t base = (int64_t)blockIdx.x * STILE;
    for (int i = threadIdx.x; i < STILE; i += ST) {
        int64_t idx = base + i;
        tile[i] = idx < n ? (int64_t)in[idx] : 0;
    }
    __syncthreads();
    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
    int64_t run = 0;
    for (int k = 0; k < SI; ++k) {
        int64_t v = tile[t * SI + k];
        tile[t * SI + k] = run;
        run += v;
    }
    int64_t x = run;  // inclusive scan of per-thread totals within the wave
    for (int off = 1; off < WAVE; off <<= 1) {
        int64_t y = __shfl_up(x, off, WAVE);
        if (lane >= off) x += y;
    }
    if (lane == WAVE - 1) wtot[w] = x;
    __syncthreads();
    int64_t wprefix = 0;
    for (int i = 0; i < w; ++i) wprefix += wtot[i];
    const int64_t excl = (offsets ? offsets[blockIdx.x] : 0) + wprefix + x - run;
    for (int k = 0; k < SI; ++k) tile[t * SI + k] += excl;
    __syncthreads();
    for (int i = threadIdx.x; i < STILE; i += ST) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = tile[i];
    }
    if (t == ST - 1 && base + STILE >= n) out[n] = excl + run;
}

__global__ void k_fill_zero_i64(int64_t *p) { *p = 0; }

template <typename In>
void scan_impl(const In *in, int64_t n, int64_t *out, int64_t *ws, hipStream_t s)
{
    if (n <= 0) {
        k_fill_zero_i64<<<1, 1, 0, s>>>(out);
        CLEORA_LAUNCH_CHECK();
        return;
    }
    const int64_t nb = ceil_div(n, STILE);
    if (nb == 1) {
        k_scan_tile<In><<<1, ST, 0, s>>>(in, n, nullptr, out);
        CLEORA_LAUNCH_CHECK();
        return;
    }
    int64_t *sums = ws, *offs = ws + nb, *rest = offs + nb + 1;
    k_scan_reduce<In><<<(unsigned)nb, ST, 0, s>>>(in, n, sums);
    CLEORA_LAUNCH_CHECK();
    scan_impl<int64_t>(sums, nb, offs, rest, s);
    k_scan_tile<In><<<(unsigned)nb, ST, 0, s>>>(in, n, offs, out);
    CLEORA_LAUNCH_CHECK();
}

}  // namespace

size_t scan_workspace_elems(int64_t n)
{
    size_t t = 1;
    int64_t nb = ceil_div(n > 0 ? n : 1, STILE);
    while (nb > 1) {
        t += 2 * (size_t)nb + 1;
        nb = ceil_div(nb, STILE);
    }
    return t;
}

void exclusive_scan(const int32_t *in, int64_t n, int64_t *out, int64_t *ws, hipStream_t s)
{
    scan_impl<int32_t>(in, n, out, ws, s);
}
void exclusive_scan(const uint8_t *in, int64_t n, int64_t *out, int64_t *ws, hipStream_t s)
{
    scan_impl<uint8_t>(in, n, out, ws, s);
}
void exclusive_scan(const int64_t *in, int64_t n, int64_t *out, int64_t *ws, hipStream_t s)
{
    scan_impl<int64_t>(in, n, out, ws, s);
}

}  // namespace cleora
