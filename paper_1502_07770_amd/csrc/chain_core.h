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
// Deques.  RingDeque keeps the breakpoints of one lane in a power-of-two ring
// in LDS, laid out slot-major / lane-minor, so that 64 lanes touching any
// per-lane slots hit 64 distinct banks.  GlobalDeque is the exact fallback
// for chains whose deque outgrows the ring: a per-lane array of 2n + 4 entries
// in HBM, starting in its middle and growing both ways (the 4n + O(1) array of
// Sec. 4.1, with two numbers per breakpoint).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvc {

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

// Per-lane ring of K entries in LDS.  lam/tag point at this lane's column:
// slot j lives at lam[j * LANES].
template <typename T, int K, int LANES>
struct RingDeque {
    T *lam;
    int *tag;
    int head;  // slot of the front entry
    int size;
    __device__ __forceinline__ void init(T *lam_base, int *tag_base, int lane) {
        lam = lam_base + lane;
        tag = tag_base + lane;
        head = 0;
        size = 0;
    }
    __device__ __forceinline__ int slot(int j) const { return ((head + j) & (K - 1)) * LANES; }
    __device__ __forceinline__ bool full() const { return size >= K; }
    __device__ __forceinline__ T front_lam() const { return lam[slot(0)]; }
    __device__ __forceinline__ int front_tag() const { return tag[slot(0)]; }
    __device__ __forceinline__ T back_lam() const { return lam[slot(size - 1)]; }
    __device__ __forceinline__ int back_tag() const { return tag[slot(size - 1)]; }
    __device__ __forceinline__ void pop_front() { head = (head + 1) & (K - 1); --size; }
    __device__ __forceinline__ void pop_back() { --size; }
    __device__ __forceinline__ void push_front(T l, int k) {
        head = (head + K - 1) & (K - 1);
        ++size;
        lam[slot(0)] = l;
        tag[slot(0)] = k;
    }
    __device__ __forceinline__ void set_back_tag(int k) { tag[slot(size - 1)] = k; }
    __device__ __forceinline__ void push_back(T l) {
        ++size;
        lam[slot(size - 1)] = l;
    }
    __device__ __forceinline__ void clear() { head = 0; size = 0; }
    __device__ __forceinline__ T lam_at(int j) const { return lam[slot(j)]; }
    __device__ __forceinline__ int tag_at(int j) const { return tag[slot(j)]; }
    // Fill from a saved state: entry j at base[j * stride] (head reset to 0).
    __device__ __forceinline__ void load(const T *l, const int *t, int n, int64_t stride) {
        head = 0;
        size = n;
        for (int j = 0; j < n; ++j) {
            lam[j * LANES] = l[j * stride];
            tag[j * LANES] = t[j * stride];
        }
    }
    __device__ __forceinline__ void save(T *l, int *t, int64_t stride) const {
        for (int j = 0; j < size; ++j) {
            l[j * stride] = lam_at(j);
            t[j * stride] = tag_at(j);
        }
    }
};

// Two deques hold the same message iff they hold the same breakpoints and the
// same slope tags (the back entry's tag is never read, so it is ignored).  Equal
// deques make every later step of the DP compute bit-identical values.
template <class DQ>
__device__ __forceinline__ bool deq_equal(const DQ &A, const DQ &B) {
    if (A.size != B.size) return false;
    if (A.size == 0) return true;
    if (A.back_lam() != B.back_lam() || A.front_lam() != B.front_lam()) return false;
    for (int j = 0; j < A.size; ++j) {
        if (A.lam_at(j) != B.lam_at(j)) return false;
        if (j + 1 < A.size && A.tag_at(j) != B.tag_at(j)) return false;
    }
    return true;
}

// Per-lane array of cap entries in global memory (fallback path).
template <typename T>
struct GlobalDeque {
    T *lam;
    int *tag;
    int64_t head, size, cap;
    __device__ __forceinline__ void init(T *lam_base, int *tag_base, int64_t capacity) {
        lam = lam_base;
        tag = tag_base;
        cap = capacity;
        head = capacity / 2;
        size = 0;
    }
    __device__ __forceinline__ bool full() const { return head <= 0 || head + size >= cap; }
    __device__ __forceinline__ T front_lam() const { return lam[head]; }
    __device__ __forceinline__ int front_tag() const { return tag[head]; }
    __device__ __forceinline__ T back_lam() const { return lam[head + size - 1]; }
    __device__ __forceinline__ int back_tag() const { return tag[head + size - 1]; }
    __device__ __forceinline__ void pop_front() { ++head; --size; }
    __device__ __forceinline__ void pop_back() { --size; }
    __device__ __forceinline__ void push_front(T l, int k) {
        --head;
        ++size;
        lam[head] = l;
        tag[head] = k;
    }
    __device__ __forceinline__ void set_back_tag(int k) { tag[head + size - 1] = k; }
    __device__ __forceinline__ void push_back(T l) {
        lam[head + size] = l;
        ++size;
    }
};

// One forward step of the DP at 1-based step s (transformations (a) and (b)
// of the message update, Sec. 4.1 "Forward pass").  wprev is the weight of the
// edge entering node s (0 at s = 1), w the weight of the edge leaving it
// (0 at the root).  On return lm / lp are lambda^-_s / lambda^+_s, the
// points where the node's message derivative equals -w / +w.  At the root
// only lm (the zero of the derivative, i.e. x_n) is computed and the deque is
// left as is.  Returns false if a push found the deque full.
template <typename T, class DQ>
__device__ __forceinline__ bool dp_step(DQ &dq, int s, T yi, T wprev, T w, bool root, T &lm, T &lp) {
    const T lo = -w, hi = w;
    if (dq.size == 0) {
        // No incoming breakpoints (the first node of a chain, or the start of a
        // segment run from an assumed zero message): the derivative is z - y_s,
        // so the segment between lm and lp has slope 1, i.e. tag s - 1.
        lm = yi + lo;
        lp = yi + hi;
        if (root) return true;
        if (dq.full()) return false;
        dq.push_front(lm, s - 1);
        if (dq.full()) return false;
        dq.push_back(lp);
        return true;
    }
    // Left end: walk the breakpoints from the left while the derivative stays
    // below -w; values follow from the flat left end (-wprev) plus the
    // integer slopes times the breakpoint gaps.
    int tnew;
    {
        T l1 = dq.front_lam();
        T v = l1 - wprev - yi;
        if (v >= lo) {
            lm = l1 - (v - lo);  // zero on the left end segment (slope 1)
            tnew = s - 1;
        } else {
            for (;;) {
                T lpv = dq.front_lam();
                int kp = dq.front_tag();
                dq.pop_front();
                if (dq.size == 0) {  // right end segment, slope 1
                    lm = lpv + (lo - v);
                    tnew = s - 1;
                    break;
                }
                T lq = dq.front_lam();
                T slope = (T)(s - kp);
                T vn = v + slope * (lq - lpv);
                if (vn >= lo) {
                    lm = clampv(lpv + (lo - v) * recip(slope), lpv, lq);
                    tnew = kp;
                    break;
                }
                v = vn;
            }
        }
    }
    if (root) return true;
    if (dq.full()) return false;
    dq.push_front(lm, tnew);
    // Right end, symmetric from the flat right end (+wprev), never popping the
    // breakpoint lm pushed just now.
    if (dq.size == 1) {
        lp = lm + (hi - lo);  // tnew == s - 1: slope 1
        if (dq.full()) return false;
        dq.push_back(lp);
        return true;
    }
    {
        T lt = dq.back_lam();
        T v = lt + wprev - yi;
        if (v <= hi) {
            lp = lt + (hi - v);  // zero on the right end segment (slope 1)
            dq.set_back_tag(s - 1);
        } else {
            for (;;) {
                T lr = dq.back_lam();
                dq.pop_back();
                T lq = dq.back_lam();
                T slope = (T)(s - dq.back_tag());
                if (dq.size == 1) {  // segment starting at lm
                    lp = lm + (hi - lo) * recip(slope);
                    if (lp > lr) lp = lr;
                    break;
                }
                T vp = v - slope * (lr - lq);
                if (vp <= hi) {
                    lp = clampv(lr - (v - hi) * recip(slope), lq, lr);
                    break;
                }
                v = vp;
            }
        }
    }
    if (dq.full()) return false;
    dq.push_back(lp);
    return true;
}

// Source / sink interface used by run_chain:
//   T   src.data(i)    -- the chain's data value at node i (forward order)
//   T   src.weight(i)  -- weight of edge (i, i+1), i < n - 1
//   void sink.emit(i, x) -- solution value at node i (called for i = n-1 .. 0)
// lam_lo / lam_hi: the lambda stream, node i at ws_base + i * ws_stride.
// Returns false on deque overflow; nothing is emitted then.
template <typename T, class DQ, class Src, class Sink>
__device__ __forceinline__ bool run_chain(DQ &dq, int64_t n, Src &src, Sink &sink,
                                          T *__restrict__ lam_lo, T *__restrict__ lam_hi,
                                          int64_t ws_base, int64_t ws_stride) {
    if (n <= 0) return true;
    T wprev = (T)0;
    T ynext = src.data(0);
    T wnext = (n > 1) ? src.weight(0) : (T)0;
    T xroot = (T)0;
    for (int64_t i = 0; i < n; ++i) {
        const T yi = ynext;
        const T wi = wnext;
        const bool root = (i == n - 1);
        if (i + 1 < n) {
            ynext = src.data(i + 1);
            wnext = (i + 2 < n) ? src.weight(i + 1) : (T)0;
        }
        T lm, lp;
        if (!dp_step<T>(dq, (int)(i + 1), yi, wprev, root ? (T)0 : wi, root, lm, lp)) return false;
        if (root) {
            xroot = lm;
        } else {
            const int64_t o = ws_base + i * ws_stride;
            lam_lo[o] = lm;
            lam_hi[o] = lp;
        }
        wprev = wi;
    }
    // Backward pass of Algorithm 2: x_i = clip(x_{i+1}, lam^-_i, lam^+_i).
    T x = xroot;
    sink.emit(n - 1, x);
    int64_t i = n - 2;
    for (; i >= 7; i -= 8) {
        T lo[8], hi[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t o = ws_base + (i - j) * ws_stride;
            lo[j] = lam_lo[o];
            hi[j] = lam_hi[o];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            x = clampv(x, lo[j], hi[j]);
            sink.emit(i - j, x);
        }
    }
    for (; i >= 0; --i) {
        const int64_t o = ws_base + i * ws_stride;
        x = clampv(x, lam_lo[o], lam_hi[o]);
        sink.emit(i, x);
    }
    return true;
}

}  // namespace tvc
