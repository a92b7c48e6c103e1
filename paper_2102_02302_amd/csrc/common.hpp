// Shared device/host helpers of the gfx950 Cleora library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "cleora.h"

namespace cleora {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define CLEORA_HIP(expr)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::cleora::Error(e_ == hipErrorOutOfMemory ? CLEORA_E_NOMEM : CLEORA_E_DEVICE, \
                                  std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

#define CLEORA_LAUNCH_CHECK() CLEORA_HIP(hipGetLastError())

constexpr int WAVE = 64;

// ------------------------------------------------------------------ bf16

__device__ __forceinline__ float bf16_lo(uint32_t pair) { return __uint_as_float(pair << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t pair) { return __uint_as_float(pair & 0xffff0000u); }

// float32 -> bfloat16 with round-to-nearest-even (NaN kept quiet).
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// ------------------------------------------------------- wave reductions

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

// Sum over aligned groups of `width` lanes (width a power of two <= 64).
template <int WIDTH, typename T>
__device__ __forceinline__ T group_sum(T x)
{
#pragma unroll
    for (int off = WIDTH / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

// ------------------------------------------------------------- host side

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Grow-only device buffer owned by a context.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    bool exact = false;  // grow to the size asked for (no 1.5x step)
    bool fixed = false;  // a view into memory the buffer does not own: never reallocated
    // A regrowth asks for at least 1.5x the old size (the exact size if
    // that fails, or with `exact`), so a buffer reused for slowly growing
    // sizes reallocates O(log) times: each free waits for the device.
    void ensure(size_t bytes)
    {
        if (bytes <= cap && p) return;
        if (fixed)
            throw Error(CLEORA_E_INVAL, "needs " + std::to_string(bytes) +
                                            " bytes of a fixed scratch region of " +
                                            std::to_string(cap));
        const size_t grown = cap && !exact ? cap + cap / 2 : 0;
        release();
        size_t b = std::max<size_t>(bytes, 256);
        hipError_t e = hipErrorMemoryAllocation;
        if (grown > b) {
            e = hipMalloc(&p, grown);
            if (e == hipSuccess) b = grown;
            else (void)hipGetLastError();
        }
        if (e != hipSuccess) e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            cap = 0;
            (void)hipGetLastError();
            throw Error(CLEORA_E_NOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        }
        cap = b;
    }
    void release()
    {
        if (fixed) return;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T *as() const
    {
        return reinterpret_cast<T *>(p);
    }
};

}  // namespace cleora
