// chain_dp.hip -- the Sec. 4.1 chain DP with general quadratic unaries
// f_i(x) = a_i x^2 / 2 - b_i x (a_i > 0) and asymmetric pairwise terms
// f_e(z) = w^-_e z (z < 0), w^+_e z (z >= 0), z = x_{e+1} - x_e, w^-_e <= w^+_e,
// on the segmented kernels of seg_kernels.h.
//
// The slopes of the message are the sums Abar_s - Abar_k of the a_i between
// two steps, formed from FP64 prefix sums Abar_i that every run over a node
// (halo, segment, repair, fix-up, overflow) must reproduce bit for bit.  A
// prefix pass stores one FP64 anchor per group of kAnchor nodes, the sum of a
// before the group (blocks of kPrefixBlock nodes summed from zero, block
// totals added left to right); inside a group Abar_i is the anchor plus the
// group's a_j up to i, added left to right in FP64.  Runs start at multiples
// of the tile (a multiple of kAnchor), and a run starting elsewhere rebuilds
// Abar_{i-1} the same way, so the segmented output stays bit-identical to the
// sequential one, as for a_i = 1.
#include "kernels.h"
#include "seg_kernels.h"

namespace tvc {

// Nodes per anchor and per block of the prefix pass.
constexpr int64_t kAnchor = 8;
constexpr int64_t kPrefixBlock = 256;
static_assert(kPrefixBlock % kAnchor == 0, "blocks hold whole anchor groups");
static_assert(kTile % kAnchor == 0, "runs start on anchor groups");
constexpr int kAnchorShift = 3;
static_assert((int64_t(1) << kAnchorShift) == kAnchor, "anchor groups are a power of two");

template <typename T>
struct GenProb {
    using Tag = double;  // FP64 prefix sums
    static constexpr bool kGen = true;
    struct Params {
        const T *a, *b, *wm, *wp;  // a may be null (a_i = 1)
        const double *anchor;      // [ceil(n / kAnchor)][C]
        T *x;
        int64_t es, cs, C;
        const int64_t *offsets;
    };
    struct Pre {
        double s;  // anchor of the node's group
        T a, b, wm, wp;
    };
    struct SinkPre {};
    // Node offsets here are node indices: the element offset (base + i es) and
    // the anchor offset ((i / kAnchor) C + c) both follow from it.
    struct Src {
        const T *__restrict__ a;
        const T *__restrict__ b;
        const T *__restrict__ wm;
        const T *__restrict__ wp;
        const double *__restrict__ anchor;
        int64_t base, es, C, c;
        bool vec;  // unit stride and element-aligned: load4 may be used
        __device__ __forceinline__ Src(const Params &p, int64_t base_, int64_t es_, int64_t c_)
            : a(p.a), b(p.b), wm(p.wm), wp(p.wp), anchor(p.anchor), base(base_), es(es_), C(p.C), c(c_),
              vec(es_ == 1 && (!p.a || elem_aligned(p.a + base_)) && elem_aligned(p.b + base_) &&
                  elem_aligned(p.wm + base_) && elem_aligned(p.wp + base_)) {}
        __device__ __forceinline__ T av(int64_t o) const { return a ? a[o] : (T)1; }
        __device__ __forceinline__ Pre load(int64_t i) const { return load_off(i); }
        __device__ __forceinline__ int64_t off(int64_t i) const { return i; }
        __device__ __forceinline__ int64_t step() const { return 1; }
        __device__ __forceinline__ Pre load_off(int64_t i) const {
            const int64_t o = base + i * es;
            Pre p;
            p.s = anchor[(i >> kAnchorShift) * C + c];
            p.a = av(o);
            p.b = b[o];
            p.wm = wm[o];
            p.wp = wp[o];
            return p;
        }
        // nodes i .. i+3 (i a multiple of 4, vec set): one anchor group
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const {
            T va[4] = {(T)1, (T)1, (T)1, (T)1}, vb[4], vm[4], vp[4];
            if (a) vload4(a + base + i, va);
            vload4(b + base + i, vb);
            vload4(wm + base + i, vm);
            vload4(wp + base + i, vp);
            const double s = anchor[(i >> kAnchorShift) * C + c];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                o[k].s = s;
                o[k].a = va[k];
                o[k].b = vb[k];
                o[k].wm = vm[k];
                o[k].wp = vp[k];
            }
        }
        __device__ __forceinline__ T data(const Pre &p) const { return p.b; }
        __device__ __forceinline__ T wlo(const Pre &p) const { return p.wm; }
        __device__ __forceinline__ T whi(const Pre &p) const { return p.wp; }
        // Abar_i from Abar_{i-1} (or, at a group start, from the anchor)
        __device__ __forceinline__ double prefix(const Pre &p, int64_t i, double sprev) const {
            return ((i & (kAnchor - 1)) == 0 ? p.s : sprev) + (double)p.a;
        }
        // Abar_{i-1} for a run starting at node i > 0, summed as prefix() sums it
        __device__ __forceinline__ double prefix_before(int64_t i) const {
            const int64_t g = (i - 1) >> kAnchorShift;
            double s = anchor[g * C + c];
            for (int64_t j = g * kAnchor; j < i; ++j) s += (double)av(base + j * es);
            return s;
        }
    };
    struct Sink {
        T *__restrict__ x;
        int64_t base, es;
        bool vec;  // unit stride and element-aligned: store4 may be used
        __device__ __forceinline__ Sink(T *x_, int64_t base_, int64_t es_)
            : x(x_), base(base_), es(es_), vec(es_ == 1 && elem_aligned(x_ + base_)) {}
        __device__ __forceinline__ SinkPre load(int64_t) const { return SinkPre{}; }
        __device__ __forceinline__ void load4(int64_t, SinkPre *) const {}
        __device__ __forceinline__ void store(int64_t i, T v, const SinkPre &) const { x[base + i * es] = v; }
        __device__ __forceinline__ void store4(int64_t i, const T (&v)[4], const SinkPre (&)[4]) const {
            vstore4(x + base + i, v);
        }
    };
    static __device__ __forceinline__ ChainSpan span(const Params &p, int64_t c, int64_t nmax) {
        ChainSpan sp;
        sp.aux = c;
        if (p.offsets) {
            const int64_t o0 = p.offsets[c], len = p.offsets[c + 1] - o0;
            sp.base = o0;
            sp.es = 1;
            sp.n = len < 0 ? 0 : (len < nmax ? len : nmax);
        } else {
            sp.base = c * p.cs;
            sp.es = p.es;
            sp.n = nmax;
        }
        return sp;
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) {
        return Src(p, sp.base, sp.es, sp.aux);
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{p.x, sp.base, sp.es};
    }
};

// ---------------------------------------------------------------------------
// Prefix pass.  Lane (block j, chain c) sums a over the block in FP64 from
// zero, writing the sum before each of its anchor groups (pass 1) and the
// block total; one lane per chain turns the block totals into block starts
// (pass 2); every anchor then gets its block's start added (pass 3).
// a == nullptr stands for a_i = 1.
// ---------------------------------------------------------------------------
struct PrefixGeom {
    int64_t C, n, ngrp, nblk, es, cs;
    const int64_t *offsets;
};

__device__ __forceinline__ void chain_extent(const PrefixGeom &g, int64_t c, int64_t *base, int64_t *es,
                                             int64_t *len) {
    if (g.offsets) {
        const int64_t o0 = g.offsets[c], l = g.offsets[c + 1] - o0;
        *base = o0;
        *es = 1;
        *len = l < 0 ? 0 : (l < g.n ? l : g.n);
    } else {
        *base = c * g.cs;
        *es = g.es;
        *len = g.n;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_anchor_blocks(PrefixGeom g, const T *__restrict__ a,
                                                       double *__restrict__ anchor, double *__restrict__ part) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= g.nblk * g.C) return;
    const int64_t c = l % g.C, j = l / g.C;
    int64_t base, es, len;
    chain_extent(g, c, &base, &es, &len);
    const int64_t i0 = j * kPrefixBlock;
    const int64_t i1 = (i0 + kPrefixBlock < len) ? i0 + kPrefixBlock : len;
    const bool vec = a && es == 1 && elem_aligned(a + base);
    double acc = 0.0;
    for (int64_t i = i0; i < i1; i += kAnchor) {
        anchor[(i / kAnchor) * g.C + c] = acc;
        if (i + kAnchor <= i1) {
            T v[kAnchor];
            if (vec) {
#pragma unroll
                for (int k = 0; k < kAnchor; k += 4) {
                    T q[4];
                    vload4(a + base + i + k, q);
#pragma unroll
                    for (int m = 0; m < 4; ++m) v[k + m] = q[m];
                }
            } else {
#pragma unroll
                for (int k = 0; k < kAnchor; ++k) v[k] = a ? a[base + (i + k) * es] : (T)1;
            }
#pragma unroll
            for (int k = 0; k < kAnchor; ++k) acc += (double)v[k];
        } else {
            for (int64_t k = i; k < i1; ++k) acc += a ? (double)a[base + k * es] : 1.0;
        }
    }
    part[j * g.C + c] = acc;
}

__global__ __launch_bounds__(256) void k_prefix_starts(PrefixGeom g, double *__restrict__ part) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= g.C) return;
    double acc = 0.0;
    for (int64_t j = 0; j < g.nblk; ++j) {
        const double t = part[j * g.C + c];
        part[j * g.C + c] = acc;
        acc += t;
    }
}

__global__ __launch_bounds__(256) void k_anchor_add(PrefixGeom g, const double *__restrict__ part,
                                                    double *__restrict__ anchor) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= g.ngrp * g.C) return;
    const int64_t c = l % g.C, q = l / g.C;
    anchor[l] += part[(q / (kPrefixBlock / kAnchor)) * g.C + c];
}

// Workspace: [anchors ngrp x C doubles][block sums nblk x C doubles][segments].
static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

template <typename T>
size_t chain_dp_ws_bytes(int64_t C, int64_t n, size_t seg_bytes) {
    const int64_t ngrp = (n + kAnchor - 1) / kAnchor, nblk = (n + kPrefixBlock - 1) / kPrefixBlock;
    return al256(sizeof(double) * (size_t)(ngrp * C)) + al256(sizeof(double) * (size_t)(nblk * C)) + seg_bytes;
}

template <typename T>
hipError_t launch_chain_dp(const ChainBatch &bt, const T *a, const T *b, const T *wm, const T *wp, T *x,
                           void *workspace, const SegPlan &plan, hipStream_t stream) {
    const int64_t C = bt.num_chains, n = bt.n;
    if (C <= 0) return hipSuccess;
    const int64_t ngrp = (n + kAnchor - 1) / kAnchor, nblk = (n + kPrefixBlock - 1) / kPrefixBlock;
    char *p = (char *)workspace;
    double *anchor = (double *)p;
    p += al256(sizeof(double) * (size_t)(ngrp * C));
    double *part = (double *)p;
    p += al256(sizeof(double) * (size_t)(nblk * C));
    const PrefixGeom g{C, n, ngrp, nblk, bt.es, bt.cs, bt.offsets};
    hipLaunchKernelGGL((k_anchor_blocks<T>), dim3((unsigned)((nblk * C + 255) / 256)), dim3(256), 0, stream, g, a,
                       anchor, part);
    hipLaunchKernelGGL(k_prefix_starts, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, stream, g, part);
    hipLaunchKernelGGL(k_anchor_add, dim3((unsigned)((ngrp * C + 255) / 256)), dim3(256), 0, stream, g, part,
                       anchor);
    typename GenProb<T>::Params pp{a, b, wm, wp, anchor, x, bt.es, bt.cs, C, bt.offsets};
    return seg_run<T, GenProb<T>, kTile>(p, C, n, plan, pp, stream);
}

template size_t chain_dp_ws_bytes<float>(int64_t, int64_t, size_t);
template size_t chain_dp_ws_bytes<double>(int64_t, int64_t, size_t);
template hipError_t launch_chain_dp<float>(const ChainBatch &, const float *, const float *, const float *,
                                           const float *, float *, void *, const SegPlan &, hipStream_t);
template hipError_t launch_chain_dp<double>(const ChainBatch &, const double *, const double *, const double *,
                                            const double *, double *, void *, const SegPlan &, hipStream_t);

}  // namespace tvc
