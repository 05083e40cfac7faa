// Shared helpers of the RTSDF gfx950 library (one translation unit: every
// .hip file of this directory is included by rtsdf_lib.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "rtsdf.h"

namespace rtsdf {

constexpr int kWave = 64;
// triangle references of a scene (after splitting) at most: record offsets (48 B each) are formed with the
// full-rate 24-bit multiply
constexpr int kMaxRefs = 1 << 24;
__device__ __forceinline__ uint32_t rec48(int i) { return __umul24((uint32_t)i, 48u); }

// Per-device error word (bits RTSDF_ERR_*), set by kernels, read and cleared
// by rtsdf_sync_status.
__device__ unsigned int g_error_word;

__device__ __forceinline__ void raise_error(unsigned int bit) { atomicOr(&g_error_word, bit); }

// Float operations that are rounded exactly once (round to nearest even) and
// never fused with a neighbour into an FMA: the texel centres, ray directions,
// coarse SDF values and shadow marches must be reproducible bit for bit.
// (HIP's __fadd_rn/__fmul_rn are plain operators that the compiler may
// contract, and its __fsqrt_rn is the approximate native square root; the
// builtin square root and division below are correctly rounded under hipcc's
// default fp32 settings.)
__device__ __forceinline__ float rn_add(float a, float b)
{
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ float rn_sub(float a, float b)
{
#pragma clang fp contract(off)
    return a - b;
}
__device__ __forceinline__ float rn_mul(float a, float b)
{
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ float rn_div(float a, float b)
{
#pragma clang fp contract(off)
    return a / b;
}
__device__ __forceinline__ float rn_sqrt(float a) { return __builtin_sqrtf(a); }

inline hipStream_t as_stream(rtsdf_stream s) { return reinterpret_cast<hipStream_t>(s); }

inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

inline int ilog2(int64_t x)
{
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= x) ++l;
    return l;
}

inline bool grid_ok(const rtsdf_grid &g)
{
    return g.n > 0 && g.h > 0.0f && g.h == g.h && g.lo[0] == g.lo[0] && g.lo[1] == g.lo[1] && g.lo[2] == g.lo[2];
}

#define RTSDF_CHECK_LAUNCH()                                        \
    do {                                                            \
        if (hipGetLastError() != hipSuccess) return RTSDF_EHIP;     \
    } while (0)

#define RTSDF_TRY(expr)                                             \
    do {                                                            \
        if ((expr) != hipSuccess) return RTSDF_EHIP;                \
    } while (0)

inline int num_cus()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

// Fill kernel (used instead of hipMemsetAsync so the calls stay safe inside
// captured graphs).
template <typename T>
__global__ void fill_kernel(T *p, T v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

template <typename T>
inline int launch_fill(T *p, T v, int64_t n, hipStream_t s)
{
    if (n <= 0) return RTSDF_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    fill_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(p, v, n);
    RTSDF_CHECK_LAUNCH();
    return RTSDF_OK;
}

// Morton helpers (bit b of x, y, z -> bits 3b, 3b+1, 3b+2).
__host__ __device__ __forceinline__ uint32_t part1by2(uint32_t x)
{
    x &= 0x000003ffu;
    x = (x | (x << 16)) & 0xff0000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__host__ __device__ __forceinline__ uint32_t compact1by2(uint32_t x)
{
    x &= 0x09249249u;
    x = (x ^ (x >> 2)) & 0x030c30c3u;
    x = (x ^ (x >> 4)) & 0x0300f00fu;
    x = (x ^ (x >> 8)) & 0xff0000ffu;
    x = (x ^ (x >> 16)) & 0x000003ffu;
    return x;
}

__host__ __device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}

}  // namespace rtsdf
