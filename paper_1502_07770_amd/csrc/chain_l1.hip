// chain_l1.hip -- TV-l1 chain prox (Sec. 4.2, piecewise-quadratic unaries) on
// the segmented kernels of seg_kernels.h:
//
//     x = argmin_x  sum_e w_e |x_{e+1} - x_e| + sum_i (x_i - y_i)^2 / 2 + sum_i c_i |x_i - d_i|,
//
// the row subproblem of the TV-l1 primal-dual iteration (eq. (prox-pq), with
// the quadratic weight normalised to 1).  The message step is l1_step
// (l1_core.h) on the LDS ring, whose entries hold (lambda, slope tag, jump);
// segments, halos, repair, fix-up, overflow fallbacks and the backward pass are
// the ones of the chain prox, and segment boundaries compare sets bit for bit,
// so the output is the sequential run's for every plan.  The set is FP64 for
// FP32 data too (WideL1: its jumps carry running sums).  The data, d, c and w
// are read in the caller's precision and x written in it.
#include "kernels.h"
#include "seg_kernels.h"

namespace tvc {

template <typename T>
struct L1Prob {
    using Tag = TagJ<T>;
    static constexpr bool kGen = false;
    static constexpr bool kL1 = true;
    struct Params {
        const T *y, *d, *w, *c;  // w, c may be null (scalars)
        T w_scalar, c_scalar;
        T *x;
        int64_t es, cs;
        const int64_t *offsets;
    };
    struct Pre {
        T y, d, c, w;
    };
    struct SinkPre {};
    struct Src {
        const T *__restrict__ y;
        const T *__restrict__ d;
        const T *__restrict__ w;
        const T *__restrict__ c;
        T ws, cs;
        int64_t base, es;
        bool vec;  // unit stride and element-aligned: load4 may be used
        __device__ __forceinline__ Src(const Params &p, int64_t base_, int64_t es_)
            : y(p.y), d(p.d), w(p.w), c(p.c), ws(p.w_scalar), cs(p.c_scalar), base(base_), es(es_),
              vec(es_ == 1 && elem_aligned(p.y + base_) && elem_aligned(p.d + base_) &&
                  (!p.w || elem_aligned(p.w + base_)) && (!p.c || elem_aligned(p.c + base_))) {}
        __device__ __forceinline__ Pre load(int64_t i) const { return load_off(base + i * es); }
        __device__ __forceinline__ int64_t off(int64_t i) const { return base + i * es; }
        __device__ __forceinline__ int64_t step() const { return es; }
        __device__ __forceinline__ Pre load_off(int64_t o) const {
            Pre p;
            p.y = y[o];
            p.d = d[o];
            p.c = c ? c[o] : cs;
            p.w = w ? w[o] : ws;
            return p;
        }
        // nodes i .. i+3 (i a multiple of 4, vec set)
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const {
            T vy[4], vd[4], vw[4] = {ws, ws, ws, ws}, vc[4] = {cs, cs, cs, cs};
            vload4(y + base + i, vy);
            vload4(d + base + i, vd);
            if (w) vload4(w + base + i, vw);
            if (c) vload4(c + base + i, vc);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                o[k].y = vy[k];
                o[k].d = vd[k];
                o[k].w = vw[k];
                o[k].c = vc[k];
            }
        }
        __device__ __forceinline__ T data(const Pre &p) const { return p.y; }
        __device__ __forceinline__ T dval(const Pre &p) const { return p.d; }
        __device__ __forceinline__ T cval(const Pre &p) const { return p.c; }
        __device__ __forceinline__ T weight(const Pre &p) const { return p.w; }
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
        sp.aux = 0;
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
        return Src(p, sp.base, sp.es);
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{p.x, sp.base, sp.es};
    }
};

template <typename T>
size_t chain_l1_ws_bytes(int64_t C, int64_t n) {
    return seg_bytes_max<double, TagJ<double>>(C, n, kPlanL1);
}

template <typename T>
hipError_t launch_chain_l1(const ChainBatch &bt, const T *y, const T *d, const T *w, T w_scalar, const T *c,
                           T c_scalar, T *x, void *workspace, hipStream_t stream) {
    if (bt.num_chains <= 0) return hipSuccess;
    const SegPlan plan = seg_plan(bt.num_chains, bt.n, kPlanL1);
    using R = typename L1Run<L1Prob, T>::Prob;
    typename R::Params pp{y, d, w, c, w_scalar, c_scalar, x, bt.es, bt.cs, bt.offsets};
    return seg_run<double, R, kTile>(workspace, bt.num_chains, bt.n, plan, pp, stream);
}

// Build parts: 1 FP32, 2 FP64.
#if TVC_IN_PART(1)
template size_t chain_l1_ws_bytes<float>(int64_t, int64_t);
template hipError_t launch_chain_l1<float>(const ChainBatch &, const float *, const float *, const float *, float,
                                           const float *, float, float *, void *, hipStream_t);
#endif
#if TVC_IN_PART(2)
template size_t chain_l1_ws_bytes<double>(int64_t, int64_t);
template hipError_t launch_chain_l1<double>(const ChainBatch &, const double *, const double *, const double *,
                                            double, const double *, double, double *, void *, hipStream_t);
#endif

}  // namespace tvc
