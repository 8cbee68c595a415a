// chain_kernels.hip -- batched exact chain TV prox and its adjoint for gfx950.
//
// The prox runs on the segmented kernels of seg_kernels.h (lane = segment of a
// chain, deque in an LDS ring, lambda stream node-major [i][chain]); the
// adjoint runs one chain per lane.
#include "kernels.h"
#include "seg_kernels.h"

namespace tvc {

// ---------------------------------------------------------------------------
// Plain chain prox as a problem policy of the segmented kernels.
// ---------------------------------------------------------------------------
template <typename T, bool EDGE_W>
struct PlainProb {
    struct Params {
        const T *y;
        const T *w;
        T w_scalar;
        T *x;
        int64_t es, cs;
        const int64_t *offsets;
    };
    struct Pre {
        T y, w;
    };
    struct SinkPre {};
    struct Src {
        const T *__restrict__ y;
        const T *__restrict__ w;
        T ws;
        int64_t base, es;
        bool vec;  // unit stride and 16-byte aligned: load4 may be used
        __device__ __forceinline__ Src(const T *y_, const T *w_, T ws_, int64_t base_, int64_t es_)
            : y(y_), w(w_), ws(ws_), base(base_), es(es_),
              vec(es_ == 1 && aligned16(y_ + base_) && (!EDGE_W || aligned16(w_ + base_))) {}
        __device__ __forceinline__ Pre load(int64_t i) const {
            Pre p;
            p.y = y[base + i * es];
            p.w = EDGE_W ? w[base + i * es] : ws;
            return p;
        }
        // nodes i .. i+3 (i a multiple of 4, vec set)
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const {
            T a[4], c[4];
            vload4(y + base + i, a);
            if (EDGE_W) vload4(w + base + i, c);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                o[k].y = a[k];
                o[k].w = EDGE_W ? c[k] : ws;
            }
        }
        __device__ __forceinline__ T data(const Pre &p) const { return p.y; }
        __device__ __forceinline__ T weight(const Pre &p) const { return p.w; }
    };
    struct Sink {
        T *__restrict__ x;
        int64_t base, es;
        bool vec;  // unit stride and 16-byte aligned: load4 / store4 may be used
        __device__ __forceinline__ Sink(T *x_, int64_t base_, int64_t es_)
            : x(x_), base(base_), es(es_), vec(es_ == 1 && aligned16(x_ + base_)) {}
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
        return Src{p.y, p.w, p.w_scalar, sp.base, sp.es};
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{p.x, sp.base, sp.es};
    }
};

// ---------------------------------------------------------------------------
// Several batches of chains in one launch (e.g. the row and the column chains
// of an image).  Global chain c belongs to the last batch b with c0[b] <= c;
// each batch has its own buffers, strides, length and scalar weight.  The
// per-node work is PlainProb's: only the lane's setup picks its batch.
// ---------------------------------------------------------------------------
constexpr int kMaxBatches = kMaxChainBatches;

template <typename T, bool EDGE_W>
struct MultiProb {
    using Base = PlainProb<T, EDGE_W>;
    struct Params {
        int nb;
        int64_t c0[kMaxBatches];  // first global chain of each batch
        const T *y[kMaxBatches];
        const T *w[kMaxBatches];
        T *x[kMaxBatches];
        T ws[kMaxBatches];
        int64_t n[kMaxBatches], es[kMaxBatches], cs[kMaxBatches];
    };
    using Pre = typename Base::Pre;
    using SinkPre = typename Base::SinkPre;
    using Src = typename Base::Src;
    using Sink = typename Base::Sink;
    // value of arr[b] for a per-lane b, without dynamic indexing of the kernel
    // arguments (selects over the batches)
    template <typename V>
    static __device__ __forceinline__ V pick(const V (&arr)[kMaxBatches], int b) {
        V v = arr[0];
#pragma unroll
        for (int j = 1; j < kMaxBatches; ++j) v = (b == j) ? arr[j] : v;
        return v;
    }
    static __device__ __forceinline__ int batch_of(const Params &p, int64_t c) {
        int b = 0;
#pragma unroll
        for (int j = 1; j < kMaxBatches; ++j) b += (j < p.nb && c >= p.c0[j]) ? 1 : 0;
        return b;
    }
    static __device__ __forceinline__ ChainSpan span(const Params &p, int64_t c, int64_t) {
        const int b = batch_of(p, c);
        ChainSpan sp;
        sp.aux = b;
        sp.base = (c - pick(p.c0, b)) * pick(p.cs, b);
        sp.es = pick(p.es, b);
        sp.n = pick(p.n, b);
        return sp;
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) {
        const int b = (int)sp.aux;
        return Src{pick(p.y, b), pick(p.w, b), pick(p.ws, b), sp.base, sp.es};
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{pick(p.x, (int)sp.aux), sp.base, sp.es};
    }
};

// ---------------------------------------------------------------------------
// Adjoint.  Pass 1 (left to right): run sums of g in FP64; at the end of each
// run its mean goes to grad_y at the run's last node, and the boundary edge
// that closed the previous run gets s_e (mean_prev - mean) in grad_w; edges
// inside runs get 0.  Pass 2 (right to left): spread each run's mean over the
// run.  Runs are detected by exact equality of consecutive x.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_chain_adjoint(ChainBatch b, const T *__restrict__ x,
                                                      const T *__restrict__ g, T *__restrict__ gy,
                                                      T *__restrict__ gw, int w_per_edge) {
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= b.num_chains) return;
    const ChainSpan a = PlainProb<T, false>::span(
        typename PlainProb<T, false>::Params{nullptr, nullptr, (T)0, nullptr, b.es, b.cs, b.offsets}, c, b.n);
    const int64_t n = a.n;
    if (n <= 0) {
        if (gw && !w_per_edge) gw[c] = (T)0;
        return;
    }
    double run_sum = 0.0, prev_mean = 0.0, wsum = 0.0;
    int64_t run_len = 0, prev_end = -1;
    T xprev_end_val = (T)0, xi = x[a.base];
    for (int64_t i = 0; i < n; ++i) {
        const T xn = (i + 1 < n) ? x[a.base + (i + 1) * a.es] : xi;
        run_sum += (double)g[a.base + i * a.es];
        ++run_len;
        const bool end = (i + 1 == n) || (xn != xi);
        if (end) {
            const double mean = run_sum / (double)run_len;
            if (gy) gy[a.base + i * a.es] = (T)mean;
            if (prev_end >= 0) {
                // boundary edge prev_end: sign of the jump from the previous run
                const double sgn = (xi > xprev_end_val) ? 1.0 : -1.0;
                const double d = sgn * (prev_mean - mean);
                if (gw && w_per_edge) gw[a.base + prev_end * a.es] = (T)d;
                wsum += d;
            }
            prev_mean = mean;
            prev_end = i;
            xprev_end_val = xi;
            run_sum = 0.0;
            run_len = 0;
        } else if (gw && w_per_edge) {
            gw[a.base + i * a.es] = (T)0;
        }
        xi = xn;
    }
    if (gw) {
        if (w_per_edge) gw[a.base + (n - 1) * a.es] = (T)0;
        else gw[c] = (T)wsum;
    }
    if (!gy) return;
    T cur = gy[a.base + (n - 1) * a.es];
    T xr = x[a.base + (n - 1) * a.es];
    for (int64_t i = n - 2; i >= 0; --i) {
        const int64_t o = a.base + i * a.es;
        const T xv = x[o];
        if (xv != xr) cur = gy[o];  // node i closes a run: its mean was stored here
        else gy[o] = cur;
        xr = xv;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_chain_prox(const ChainBatch &b, const T *y, const T *w, T w_scalar, T *x, void *workspace,
                             const SegPlan &plan, hipStream_t stream) {
    if (b.num_chains <= 0) return hipSuccess;
    SegWs<T> ws;
    seg_ws_layout<T, kRingSlots>(workspace, b.num_chains, b.n, plan.L, plan.H, plan.CK, &ws);
    if (w) {
        using Prob = PlainProb<T, true>;
        typename Prob::Params pp{y, w, w_scalar, x, b.es, b.cs, b.offsets};
        return seg_launch<T, Prob, kRingSlots, kTile>(ws, pp, stream);
    }
    using Prob = PlainProb<T, false>;
    typename Prob::Params pp{y, w, w_scalar, x, b.es, b.cs, b.offsets};
    return seg_launch<T, Prob, kRingSlots, kTile>(ws, pp, stream);
}

template <typename T>
hipError_t launch_chain_prox_multi(int nb, const ChainBatch *bs, const T *const *y, const T *const *w,
                                   const double *w_scalar, T *const *x, void *workspace, const SegPlan &plan,
                                   hipStream_t stream) {
    int64_t C = 0, n = 0;
    for (int b = 0; b < nb; ++b) {
        C += bs[b].num_chains;
        n = bs[b].n > n ? bs[b].n : n;
    }
    if (C <= 0) return hipSuccess;
    SegWs<T> ws;
    seg_ws_layout<T, kRingSlots>(workspace, C, n, plan.L, plan.H, plan.CK, &ws);
    auto fill = [&](auto &pp) {
        pp.nb = nb;
        int64_t c0 = 0;
        for (int b = 0; b < kMaxBatches; ++b) {
            const bool on = b < nb;
            pp.c0[b] = on ? c0 : C;
            pp.y[b] = on ? y[b] : nullptr;
            pp.w[b] = (on && w) ? w[b] : nullptr;
            pp.x[b] = on ? x[b] : nullptr;
            pp.ws[b] = on && !w ? (T)w_scalar[b] : (T)0;
            pp.n[b] = on ? bs[b].n : 0;
            pp.es[b] = on ? bs[b].es : 1;
            pp.cs[b] = on ? bs[b].cs : 0;
            if (on) c0 += bs[b].num_chains;
        }
    };
    if (w) {
        using Prob = MultiProb<T, true>;
        typename Prob::Params pp;
        fill(pp);
        return seg_launch<T, Prob, kRingSlots, kTile>(ws, pp, stream);
    }
    using Prob = MultiProb<T, false>;
    typename Prob::Params pp;
    fill(pp);
    return seg_launch<T, Prob, kRingSlots, kTile>(ws, pp, stream);
}

template <typename T>
size_t chain_prox_ws_bytes(const ChainBatch &b, const SegPlan &plan) {
    return seg_ws_layout<T, kRingSlots>(nullptr, b.num_chains, b.n, plan.L, plan.H, plan.CK, nullptr);
}

template <typename T>
hipError_t launch_chain_adjoint(const ChainBatch &b, const T *x, const T *g, T *gy, T *gw,
                                int w_per_edge, hipStream_t stream) {
    if (b.num_chains <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((b.num_chains + 63) / 64);
    hipLaunchKernelGGL((k_chain_adjoint<T>), dim3(blocks), dim3(64), 0, stream, b, x, g, gy, gw,
                       w_per_edge);
    return hipGetLastError();
}

template hipError_t launch_chain_prox<float>(const ChainBatch &, const float *, const float *, float,
                                             float *, void *, const SegPlan &, hipStream_t);
template hipError_t launch_chain_prox<double>(const ChainBatch &, const double *, const double *, double,
                                              double *, void *, const SegPlan &, hipStream_t);
template hipError_t launch_chain_prox_multi<float>(int, const ChainBatch *, const float *const *,
                                                   const float *const *, const double *, float *const *, void *,
                                                   const SegPlan &, hipStream_t);
template hipError_t launch_chain_prox_multi<double>(int, const ChainBatch *, const double *const *,
                                                    const double *const *, const double *, double *const *, void *,
                                                    const SegPlan &, hipStream_t);
template size_t chain_prox_ws_bytes<float>(const ChainBatch &, const SegPlan &);
template size_t chain_prox_ws_bytes<double>(const ChainBatch &, const SegPlan &);
template hipError_t launch_chain_adjoint<float>(const ChainBatch &, const float *, const float *,
                                                float *, float *, int, hipStream_t);
template hipError_t launch_chain_adjoint<double>(const ChainBatch &, const double *, const double *,
                                                 double *, double *, int, hipStream_t);

}  // namespace tvc
