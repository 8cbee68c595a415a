// tv2d_common.h -- pieces shared by the single-image and batched 2D solvers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvc {

// Threads per block of the gap reductions (four wave64 rows per block).
constexpr int kGapBlock = 256;
// Rows per block of the column prefix sums of the gap.  The single-image and
// batched solvers sum in the same order (within a block from zero, blocks
// added left to right), so their gaps agree bit for bit.
constexpr int kGapRows = 64;

// b_i of the row step; shared by the row chain source and the gap kernel so
// both see bit-identical values.
template <typename T>
__device__ __forceinline__ T row_data(T f, T x, T y, T tau, T inv1p) {
    return (tau * f + x - tau * y) * inv1p;
}

// Store a clipped dual value in precision T, rounded toward zero so that the
// stored value still satisfies |p| <= lambda.
template <typename T> __device__ __forceinline__ T store_feasible(double p);
template <> __device__ __forceinline__ double store_feasible<double>(double p) { return p; }
template <> __device__ __forceinline__ float store_feasible<float>(double p) { return __double2float_rz(p); }

__device__ __forceinline__ double clipd(double v, double lam) { return v < -lam ? -lam : (v > lam ? lam : v); }

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *__restrict__ dst, int64_t n, T v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = v;
}

// Copy between a dense H x W buffer and a strided one (leading dimension ld).
template <typename T>
__global__ __launch_bounds__(256) void k_copy2d(const T *__restrict__ src, int64_t lds, T *__restrict__ dst,
                                                int64_t ldd, int64_t H, int64_t W) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= H * W) return;
    const int64_t r = i / W, c = i % W;
    dst[r * ldd + c] = src[r * lds + c];
}

}  // namespace tvc
