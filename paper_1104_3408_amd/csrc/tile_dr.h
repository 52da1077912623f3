// Radial-derivative tile shared by the derivative kernels (derivs.hip) and
// the BF16x3 one-launch form (bf16x3.hip).
#pragma once

#include "internal.h"

namespace sg {

namespace {

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// d_r: 64 lines per workgroup; wave w computes k = w R + r, r < R.  The tile
// is [n_r][65]: the odd row stride keeps the transposing stores and loads of
// consecutive k (consecutive threads) on different LDS banks.
constexpr int kDrStride = 65;
constexpr int kDrPer = (64 * 80 + 64 * kMinWaves - 1) / (64 * kMinWaves);   // tile loads per thread

template <int R>
__device__ __forceinline__ void dr_tile(long long tile, const double* __restrict__ in, double* __restrict__ out,
                                        const double* __restrict__ Db, int n_r, long long n_lines,
                                        double* __restrict__ sm) {   // sm: [n_r][kDrStride]
    const long long line0 = tile * 64;
    const int nl = (int)min((long long)64, n_lines - line0);
    const double* src = in + line0 * n_r;
    const int ne = nl * n_r;
    // e = l n_r + k split without an integer division: e < 64 n_r <= 5120, so
    // (e + 1/2)/n_r in FP32 is at least 1/(2 n_r) from an integer and its
    // rounding error (< 1e-5) cannot move the floor
    const float inv_nr = 1.0f / (float)n_r;
    {
        const int nt = blockDim.x;   // >= 64 kMinWaves, so kDrPer slots cover 64 N_r <= 64 * 80
        double v[kDrPer];
#pragma unroll
        for (int t = 0; t < kDrPer; ++t) {
            const int e = threadIdx.x + t * nt;
            v[t] = (e < ne) ? src[e] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kDrPer; ++t) {
            const int e = threadIdx.x + t * nt;
            if (e < 64 * n_r) {
                const int l = (int)(((float)e + 0.5f) * inv_nr), k = e - l * n_r;
                sm[k * kDrStride + l] = v[t];
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const double* Dw = Db + (long long)w * n_r * R;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    #pragma unroll 4   // operator loads run ahead of the FMAs (measured against 1, 2, default)
    for (int kk = 0; kk < n_r; ++kk) {
        const double v = sm[kk * kDrStride + lane];
        const double* d = Dw + kk * R;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(d[r], v, acc[r]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = w * R + r;
        if (k < n_r) sm[k * kDrStride + lane] = acc[r];
    }
    __syncthreads();
    double* dst = out + line0 * n_r;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const int l = (int)(((float)e + 0.5f) * inv_nr), k = e - l * n_r;
        dst[e] = sm[k * kDrStride + l];
    }
}

}  // namespace

}  // namespace sg
