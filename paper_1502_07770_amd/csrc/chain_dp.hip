// chain_dp.hip -- the Sec. 4.1 chain DP with general quadratic unaries
// f_i(x) = a_i x^2 / 2 - b_i x (a_i > 0) and asymmetric pairwise terms
// f_e(z) = w^-_e z (z < 0), w^+_e z (z >= 0), z = x_{e+1} - x_e, w^-_e <= w^+_e,
// on the segmented kernels of seg_kernels.h.
//
// The slopes of the message are the sums Abar_s - Abar_k of the a_i between
// two steps.  A prefix pass writes Abar_i = a_0 + ... + a_i in FP64, node-major
// [i][chain], in a fixed summation order (blocks of kPrefixBlock nodes from
// zero, block totals added left to right), and the DP reads it: every run over
// a node (halo, segment, repair, fix-up, overflow) sees the same bits, so the
// segmented output is bit-identical to the sequential one as for a_i = 1.
#include "kernels.h"
#include "seg_kernels.h"

namespace tvc {

// Nodes per block of the prefix pass.
constexpr int64_t kPrefixBlock = 256;

template <typename T>
struct GenProb {
    using Tag = double;  // FP64 prefix sums
    static constexpr bool kGen = true;
    struct Params {
        const T *b, *wm, *wp;
        const double *abar;  // [n][C]
        T *x;
        int64_t es, cs, C;
        const int64_t *offsets;
    };
    struct Pre {
        double s;
        T b, wm, wp;
    };
    struct SinkPre {};
    // Node offsets here are node indices: the element offset (base + i es) and
    // the prefix offset (i C + c) both follow from it.
    struct Src {
        const T *__restrict__ b;
        const T *__restrict__ wm;
        const T *__restrict__ wp;
        const double *__restrict__ abar;
        int64_t base, es, C, c;
        bool vec;  // unit stride and element-aligned: load4 may be used
        __device__ __forceinline__ Src(const Params &p, int64_t base_, int64_t es_, int64_t c_)
            : b(p.b), wm(p.wm), wp(p.wp), abar(p.abar), base(base_), es(es_), C(p.C), c(c_),
              vec(es_ == 1 && elem_aligned(p.b + base_) && elem_aligned(p.wm + base_) &&
                  elem_aligned(p.wp + base_)) {}
        __device__ __forceinline__ Pre load(int64_t i) const { return load_off(i); }
        __device__ __forceinline__ int64_t off(int64_t i) const { return i; }
        __device__ __forceinline__ int64_t step() const { return 1; }
        __device__ __forceinline__ Pre load_off(int64_t i) const {
            const int64_t o = base + i * es;
            Pre p;
            p.s = abar[i * C + c];
            p.b = b[o];
            p.wm = wm[o];
            p.wp = wp[o];
            return p;
        }
        // nodes i .. i+3 (i a multiple of 4, vec set)
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const {
            T vb[4], vm[4], vp[4];
            vload4(b + base + i, vb);
            vload4(wm + base + i, vm);
            vload4(wp + base + i, vp);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                o[k].s = abar[(i + k) * C + c];
                o[k].b = vb[k];
                o[k].wm = vm[k];
                o[k].wp = vp[k];
            }
        }
        __device__ __forceinline__ T data(const Pre &p) const { return p.b; }
        __device__ __forceinline__ double prefix(const Pre &p) const { return p.s; }
        __device__ __forceinline__ T wlo(const Pre &p) const { return p.wm; }
        __device__ __forceinline__ T whi(const Pre &p) const { return p.wp; }
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
// Prefix pass.  Lane (block j, chain c): the FP64 sum of a over the block
// (pass 1); one lane per chain turns the block sums into block starts (pass 2);
// lane (j, c) writes the running sums of its block from its start (pass 3).
// a == nullptr stands for a_i = 1.
// ---------------------------------------------------------------------------
struct PrefixGeom {
    int64_t C, n, nblk, es, cs;
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

template <typename T, bool kWrite>
__device__ __forceinline__ double block_scan(const PrefixGeom &g, const T *__restrict__ a, int64_t c, int64_t j,
                                             double acc, double *__restrict__ abar) {
    int64_t base, es, len;
    chain_extent(g, c, &base, &es, &len);
    const int64_t i0 = j * kPrefixBlock;
    const int64_t i1 = (i0 + kPrefixBlock < len) ? i0 + kPrefixBlock : len;
    constexpr int U = 8;
    int64_t i = i0;
    for (; i + U <= i1; i += U) {
        double v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = a ? (double)a[base + (i + k) * es] : 1.0;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            acc += v[k];
            if (kWrite) abar[(i + k) * g.C + c] = acc;
        }
    }
    for (; i < i1; ++i) {
        acc += a ? (double)a[base + i * es] : 1.0;
        if (kWrite) abar[i * g.C + c] = acc;
    }
    return acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_prefix_blocks(PrefixGeom g, const T *__restrict__ a,
                                                       double *__restrict__ part) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= g.nblk * g.C) return;
    const int64_t c = l % g.C, j = l / g.C;
    part[j * g.C + c] = block_scan<T, false>(g, a, c, j, 0.0, nullptr);
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

template <typename T>
__global__ __launch_bounds__(256) void k_prefix_write(PrefixGeom g, const T *__restrict__ a,
                                                      const double *__restrict__ part, double *__restrict__ abar) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= g.nblk * g.C) return;
    const int64_t c = l % g.C, j = l / g.C;
    block_scan<T, true>(g, a, c, j, part[j * g.C + c], abar);
}

// Workspace: [prefix sums n x C doubles][block sums nblk x C doubles][segments].
static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

template <typename T>
size_t chain_dp_ws_bytes(int64_t C, int64_t n, size_t seg_bytes) {
    const int64_t nblk = (n + kPrefixBlock - 1) / kPrefixBlock;
    return al256(sizeof(double) * (size_t)(n * C)) + al256(sizeof(double) * (size_t)(nblk * C)) + seg_bytes;
}

template <typename T>
hipError_t launch_chain_dp(const ChainBatch &bt, const T *a, const T *b, const T *wm, const T *wp, T *x,
                           void *workspace, const SegPlan &plan, hipStream_t stream) {
    const int64_t C = bt.num_chains, n = bt.n;
    if (C <= 0) return hipSuccess;
    const int64_t nblk = (n + kPrefixBlock - 1) / kPrefixBlock;
    char *p = (char *)workspace;
    double *abar = (double *)p;
    p += al256(sizeof(double) * (size_t)(n * C));
    double *part = (double *)p;
    p += al256(sizeof(double) * (size_t)(nblk * C));
    const PrefixGeom g{C, n, nblk, bt.es, bt.cs, bt.offsets};
    const unsigned pb = (unsigned)((nblk * C + 255) / 256);
    hipLaunchKernelGGL((k_prefix_blocks<T>), dim3(pb), dim3(256), 0, stream, g, a, part);
    hipLaunchKernelGGL(k_prefix_starts, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, stream, g, part);
    hipLaunchKernelGGL((k_prefix_write<T>), dim3(pb), dim3(256), 0, stream, g, a, part, abar);
    typename GenProb<T>::Params pp{b, wm, wp, abar, x, bt.es, bt.cs, C, bt.offsets};
    return seg_run<T, GenProb<T>, kTile>(p, C, n, plan, pp, stream);
}

template size_t chain_dp_ws_bytes<float>(int64_t, int64_t, size_t);
template size_t chain_dp_ws_bytes<double>(int64_t, int64_t, size_t);
template hipError_t launch_chain_dp<float>(const ChainBatch &, const float *, const float *, const float *,
                                           const float *, float *, void *, const SegPlan &, hipStream_t);
template hipError_t launch_chain_dp<double>(const ChainBatch &, const double *, const double *, const double *,
                                            const double *, double *, void *, const SegPlan &, hipStream_t);

}  // namespace tvc
