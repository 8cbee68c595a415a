// chain_core.h -- device core of the exact O(n) chain TV prox (Sec. 4.1 of
// Kolmogorov, Pock, Rolinek, "Total variation on a tree"), one chain per lane.
//
// Problem (eq. (1D-ROF)): x = argmin sum_e w_e |x_{e+1} - x_e| + 1/2 sum_i (x_i - y_i)^2.
// This is Algorithm 2 on a chain with a_i = 1, b_i = y_i, w^-_e = -w_e,
// w^+_e = +w_e, and a virtual zero-weight edge above the root (the last node).
//
// Message representation.  The derivative of the message entering node s
// (1-based step) is a non-decreasing piecewise-linear function, kept as its
// sorted breakpoints lam_1 <= ... <= lam_t.  The paper's implicit slopes
// s_p + Abar_s become exact integers here: with a_i = 1, Abar_s = s, and every
// stored slope is -Abar_k for the step k at which that segment was a flat end,
// so each breakpoint carries the integer "birth step" k of the segment to its
// right and the true slope of that segment at step s is s - k (the end
// segments, flat after the clip, have slope 1 once g_s = z - y_s is added,
// i.e. tag s - 1).  Slopes are therefore exact and never zero.
//
// General unaries and asymmetric weights (a_i > 0, w^-_e <= w^+_e): the same
// representation with real-valued tags.  A breakpoint's tag is the prefix sum
// Abar_k of the step at which its right segment was a flat end, kept in FP64
// and read from a precomputed FP64 prefix array, so the slope Abar_s - Abar_k
// is one FP64 subtraction (rounded once to the working precision) and every
// run over a node sees the same bits; the end segments have slope
// Abar_s - Abar_{s-1} (= a_s).

#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvc {

// Every rounded operation of the DP is the one written: no multiply-add
// contraction (FMAs are explicit), so each step rounds the same in every
// kernel that inlines it and in every build, which the bit-for-bit comparison
// of segment states and the segmented = sequential results rely on.
#pragma clang fp contract(off)


template <typename T> __device__ __forceinline__ T recip(T v);
template <> __device__ __forceinline__ float recip<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ __forceinline__ double recip<double>(double v) { return 1.0 / v; }

// Four consecutive elements as one 16-byte access (two for double).  Only the
// element alignment is assumed: gfx950 runs in unaligned-access mode, and the
// compiler emits dwordx4 accesses for these copies at any 4-byte alignment.
__device__ __forceinline__ void vload4(const float *p, float (&o)[4]) {
    float4 v;
    __builtin_memcpy(&v, __builtin_assume_aligned(p, 4), 16);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void vload4(const double *p, double (&o)[4]) {
    double2 a, b;
    __builtin_memcpy(&a, __builtin_assume_aligned(p, 8), 16);
    __builtin_memcpy(&b, __builtin_assume_aligned(p + 2, 8), 16);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void vstore4(float *p, const float (&v)[4]) {
    const float4 t = make_float4(v[0], v[1], v[2], v[3]);
    __builtin_memcpy(__builtin_assume_aligned(p, 4), &t, 16);
}
__device__ __forceinline__ void vstore4(double *p, const double (&v)[4]) {
    const double2 a = make_double2(v[0], v[1]), b = make_double2(v[2], v[3]);
    __builtin_memcpy(__builtin_assume_aligned(p, 8), &a, 16);
    __builtin_memcpy(__builtin_assume_aligned(p + 2, 8), &b, 16);
}
// Element alignment (what the 16-byte accesses above need).
template <typename T> __device__ __forceinline__ bool elem_aligned(const T *p) { return ((uintptr_t)p % sizeof(T)) == 0; }

// Clip of v to [lo, hi] for lo <= hi (every call site guarantees the order:
// brackets of sorted breakpoints, and lambda^- <= lambda^+).  FP32 uses the
// median-of-three instruction (one VALU op, no NaN canonicalisation).
__device__ __forceinline__ float clampv(float v, float lo, float hi) { return __builtin_amdgcn_fmed3f(v, lo, hi); }
__device__ __forceinline__ double clampv(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Inputs of one DP step at node i (1-based step s = i + 1).  sf / sprev are
// the prefix sums Abar_s / Abar_{s-1} (s and s - 1 when a_i = 1); yi is b_i;
// lop / hip are w^-, w^+ of the edge entering the node (0 at the first node);
// lo / hi are w^-, w^+ of the edge leaving it (0 at the root, Algorithm 2's
// virtual zero-weight edge above the root).
template <typename T, typename G>
struct StepIn {
    G sf, sprev;
    T yi, lop, hip, lo, hi;
};

// Slope of the segment whose tag is k, and the end-segment slope a_s with its
// reciprocal.  With a_i = 1 (kGen false) they are exact: s - k in the working
// precision, and 1.
template <typename T, typename G>
__device__ __forceinline__ T slope_of(G sf, G k) {
    return (T)(sf - k);
}
template <typename T, typename G, bool kGen>
struct EndSlope {
    T a, ra;
    __device__ __forceinline__ EndSlope(G sf, G sprev) {
        if constexpr (kGen) {
            a = (T)(sf - sprev);
            ra = recip(a);
        } else {
            a = (T)1;
            ra = (T)1;
        }
    }
    // d / a_s and a_s * v (the identity when a_i = 1)
    __device__ __forceinline__ T div(T d) const {
        if constexpr (kGen) return d * ra;
        else return d;
    }
    __device__ __forceinline__ T mul(T v) const {
        if constexpr (kGen) return a * v;
        else return v;
    }
};

#pragma clang fp contract(fast)
}  // namespace tvc
