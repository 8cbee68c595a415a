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
    using Tag = T;  // a_i = 1: integer tags in the working precision
    static constexpr bool kGen = false;
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
        bool vec;  // unit stride and element-aligned: load4 may be used
        __device__ __forceinline__ Src(const T *y_, const T *w_, T ws_, int64_t base_, int64_t es_)
            : y(y_), w(w_), ws(ws_), base(base_), es(es_),
              vec(es_ == 1 && elem_aligned(y_ + base_) && (!EDGE_W || elem_aligned(w_ + base_))) {}
        __device__ __forceinline__ Pre load(int64_t i) const { return load_off(base + i * es); }
        // element offset of node i, and the offset step between nodes
        __device__ __forceinline__ int64_t off(int64_t i) const { return base + i * es; }
        __device__ __forceinline__ int64_t step() const { return es; }
        __device__ __forceinline__ Pre load_off(int64_t o) const {
            Pre p;
            p.y = y[o];
            p.w = EDGE_W ? w[o] : ws;
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
        bool vec;  // unit stride and element-aligned: load4 / store4 may be used
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
    using Tag = T;  // a_i = 1: integer tags in the working precision
    static constexpr bool kGen = false;
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
// Adjoint for unit-stride chains (rows, CSR): one wave per chain.  The chain
// is processed in chunks of 64 * kAdjV nodes held in registers, lane l owning
// the kAdjV consecutive nodes [c0 + l kAdjV, c0 + (l + 1) kAdjV), so every
// load and store of the wave covers contiguous memory.  Per chunk:
//  - run ends: node i ends a run if i = n - 1 or x_i != x_{i+1};
//  - a segmented prefix sum (FP64) and count of g over the runs, lane-local
//    then across the wave, gives each run's total at its end, hence its mean;
//  - a reverse segmented scan hands every node the mean of its run (the first
//    run end at or after it);
//  - grad_y = run mean; grad_w = s_e (mean_left - mean_right) on run
//    boundaries e (s_e the sign of x_{e+1} - x_e), 0 inside runs.
// A run still open at the end of a chunk carries its sum, count and start
// into the next chunk; when it closes, its nodes in earlier chunks and the
// boundary edge before it are written then.  Every output element is
// written once.  Eight nodes per lane keep the kernel at 152 VGPRs, three
// waves per SIMD (sixteen took 240 VGPRs, two waves, and 10% longer).
// ---------------------------------------------------------------------------
constexpr int kAdjV = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_chain_adjoint_rows(ChainBatch b, const T *__restrict__ x,
                                                           const T *__restrict__ g, T *__restrict__ gy,
                                                           T *__restrict__ gw, int w_per_edge) {
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= b.num_chains) return;  // whole waves
    const ChainSpan a = PlainProb<T, false>::span(
        typename PlainProb<T, false>::Params{nullptr, nullptr, (T)0, nullptr, 1, b.cs, b.offsets}, c, b.n);
    const int64_t n = a.n;
    if (n <= 0) {
        if (gw && !w_per_edge && lane == 0) gw[c] = (T)0;
        return;
    }
    const T *__restrict__ xr = x + a.base;
    const T *__restrict__ gr = g + a.base;
    T *__restrict__ yr = gy ? gy + a.base : nullptr;
    T *__restrict__ wr = (gw && w_per_edge) ? gw + a.base : nullptr;
    const bool vec = elem_aligned(xr) && elem_aligned(gr) && (!yr || elem_aligned(yr)) && (!wr || elem_aligned(wr));
    constexpr int64_t CH = 64 * kAdjV;
    // run open at the start of the chunk (identical in every lane)
    double o_sum = 0.0;
    int64_t o_cnt = 0, o_start = 0;
    // boundary edge whose right-hand run is the open run
    int64_t p_edge = -1;
    double p_mean = 0.0, p_sgn = 0.0;
    double wsum = 0.0;  // this lane's part of the scalar-weight gradient
    for (int64_t c0 = 0; c0 < n; c0 += CH) {
        const int64_t i0 = c0 + lane * kAdjV;
        T xv[kAdjV], gv[kAdjV];
        const bool full = i0 + kAdjV <= n;
        if (vec && full) {
#pragma unroll
            for (int q = 0; q < kAdjV; q += 4) {
                T t[4], u[4];
                vload4(xr + i0 + q, t);
                vload4(gr + i0 + q, u);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    xv[q + m] = t[m];
                    gv[q + m] = u[m];
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kAdjV; ++k) {
                const int64_t i = i0 + k;
                xv[k] = i < n ? xr[i] : (T)0;
                gv[k] = i < n ? gr[i] : (T)0;
            }
        }
        T xnext_lane = __shfl_down(xv[0], 1, 64);
        if (lane == 63) xnext_lane = (c0 + CH < n) ? xr[c0 + CH] : (T)0;
        bool end[kAdjV];
        T xn[kAdjV];
#pragma unroll
        for (int k = 0; k < kAdjV; ++k) {
            const int64_t i = i0 + k;
            xn[k] = (k + 1 < kAdjV) ? xv[k + 1] : xnext_lane;
            end[k] = (i < n) && (i + 1 == n || xv[k] != xn[k]);
        }
        // lane-local segmented prefix sums and counts (reset after each end)
        double ps[kAdjV];
        int pc[kAdjV];
        double acc = 0.0;
        int cnt = 0;
        bool has_end = false;
#pragma unroll
        for (int k = 0; k < kAdjV; ++k) {
            if (i0 + k < n) {
                acc += (double)gv[k];
                ++cnt;
            }
            ps[k] = acc;
            pc[k] = cnt;
            if (end[k]) {
                acc = 0.0;
                cnt = 0;
                has_end = true;
            }
        }
        // across the wave: carry into each lane = sum / count since the last end
        // in an earlier lane (or the chunk's open run)
        double cs = acc;
        int cc = cnt;
        bool cf = has_end;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double s2 = __shfl_up(cs, off, 64);
            const int c2 = __shfl_up(cc, off, 64);
            const int f2 = __shfl_up((int)cf, off, 64);
            if (lane >= off && !cf) {
                cs = s2 + cs;
                cc = c2 + cc;
                cf = f2 != 0;
            }
        }
        double ex_s = __shfl_up(cs, 1, 64);
        int64_t ex_c = __shfl_up(cc, 1, 64);
        bool ex_f = __shfl_up((int)cf, 1, 64) != 0;
        if (lane == 0) {
            ex_s = 0.0;
            ex_c = 0;
            ex_f = false;
        }
        if (!ex_f) {
            ex_s = o_sum + ex_s;
            ex_c += o_cnt;
        }
        // run means at run ends
        double mean[kAdjV];
        bool first = true;
#pragma unroll
        for (int k = 0; k < kAdjV; ++k) {
            const double tot = first ? ex_s + ps[k] : ps[k];
            const int64_t tc = first ? ex_c + pc[k] : pc[k];
            mean[k] = end[k] ? tot / (double)tc : 0.0;
            if (end[k]) first = false;
        }
        // reverse: the first end at or after each node
        double val[kAdjV];
        bool known[kAdjV];
        {
            double cur = 0.0;
            bool kn = false;
#pragma unroll
            for (int k = kAdjV - 1; k >= 0; --k) {
                if (end[k]) {
                    cur = mean[k];
                    kn = true;
                }
                val[k] = cur;
                known[k] = kn;
            }
        }
        double rv = val[0];  // the lane's first-end mean
        bool rf = known[0];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double v2 = __shfl_down(rv, off, 64);
            const int f2 = __shfl_down((int)rf, off, 64);
            if (lane + off < 64 && !rf) {
                rv = v2;
                rf = f2 != 0;
            }
        }
        const double chunk_first_mean = __shfl(rv, 0, 64);  // mean of the chunk's first run end
        const bool chunk_has_end = __shfl((int)rf, 0, 64) != 0;
        double nx_v = __shfl_down(rv, 1, 64);
        bool nx_f = __shfl_down((int)rf, 1, 64) != 0;
        if (lane == 63) nx_f = false;
#pragma unroll
        for (int k = 0; k < kAdjV; ++k) {
            if (!known[k] && nx_f) {
                val[k] = nx_v;
                known[k] = true;
            }
        }
        // the run open before this chunk closes at the chunk's first end
        if ((o_cnt > 0 || p_edge >= 0) && chunk_has_end) {
            const T m = (T)chunk_first_mean;
            if (yr)
                for (int64_t i = o_start + lane; i < c0; i += 64) yr[i] = m;
            if (p_edge >= 0 && lane == 0) {
                const double d = p_sgn * (p_mean - chunk_first_mean);
                if (wr) wr[p_edge] = (T)d;
                wsum += d;
            }
            o_cnt = 0;
            p_edge = -1;
        }
        // grad_y of nodes whose run closes in this chunk
        if (yr) {
            bool all = full && vec;
#pragma unroll
            for (int k = 0; k < kAdjV; ++k) all = all && known[k];
            if (all) {
#pragma unroll
                for (int q = 0; q < kAdjV; q += 4) {
                    const T t[4] = {(T)val[q], (T)val[q + 1], (T)val[q + 2], (T)val[q + 3]};
                    vstore4(yr + i0 + q, t);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kAdjV; ++k)
                    if (i0 + k < n && known[k]) yr[i0 + k] = (T)val[k];
            }
        }
        // grad_w: the mean right of a boundary is the next node's value
        const double v0_next = __shfl_down(val[0], 1, 64);
        const bool k0_next = __shfl_down((int)known[0], 1, 64) != 0;
        double dw[kAdjV];
        bool dw_ok[kAdjV];
        int64_t pend_i = -1;
        double pend_m = 0.0, pend_s = 0.0;
#pragma unroll
        for (int k = 0; k < kAdjV; ++k) {
            const int64_t i = i0 + k;
            double vr;
            bool kr;
            if (k + 1 < kAdjV) {
                vr = val[k + 1];
                kr = known[k + 1];
            } else {
                vr = v0_next;
                kr = (lane < 63) && k0_next;
            }
            dw[k] = 0.0;
            dw_ok[k] = i < n;
            if (i < n && end[k] && i + 1 < n) {
                const double sg = (xn[k] > xv[k]) ? 1.0 : -1.0;
                if (kr) {
                    dw[k] = sg * (mean[k] - vr);
                } else {  // the right-hand run is still open
                    dw_ok[k] = false;
                    pend_i = i;
                    pend_m = mean[k];
                    pend_s = sg;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kAdjV; ++k)
            if (dw_ok[k]) wsum += dw[k];
        if (wr) {
            bool all = full && vec;
#pragma unroll
            for (int k = 0; k < kAdjV; ++k) all = all && dw_ok[k];
            if (all) {
#pragma unroll
                for (int q = 0; q < kAdjV; q += 4) {
                    const T t[4] = {(T)dw[q], (T)dw[q + 1], (T)dw[q + 2], (T)dw[q + 3]};
                    vstore4(wr + i0 + q, t);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kAdjV; ++k)
                    if (dw_ok[k]) wr[i0 + k] = (T)dw[k];
            }
        }
        // carry: the run open at the end of the chunk (never the chain's last run)
        const int64_t c1 = (c0 + CH < n) ? c0 + CH : n;
        if (c1 < n) {
            const double t_s = __shfl(cs, 63, 64);
            const int64_t t_c = __shfl(cc, 63, 64);
            const bool t_f = __shfl((int)cf, 63, 64) != 0;
            if (t_f) {  // the open run started in this chunk
                o_sum = t_s;
                o_cnt = t_c;
                o_start = c1 - t_c;
                // its left boundary edge, if it is pending, lives in some lane
                const unsigned long long bal = __ballot(pend_i >= 0);
                if (bal) {
                    const int src = 63 - __clzll(bal);  // the last lane with a pending edge
                    p_edge = __shfl(pend_i, src, 64);
                    p_mean = __shfl(pend_m, src, 64);
                    p_sgn = __shfl(pend_s, src, 64);
                }
            } else {  // no end in the whole chunk: the open run grows (or starts at c0)
                if (o_cnt == 0) o_start = c0;
                o_sum = o_sum + t_s;
                o_cnt += t_c;
            }
        }
    }
    if (gw && !w_per_edge) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, 64);
        if (lane == 0) gw[c] = (T)wsum;
    }
    if (wr && lane == 0) wr[n - 1] = (T)0;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_chain_prox(const ChainBatch &b, const T *y, const T *w, T w_scalar, T *x, void *workspace,
                             const SegPlan &plan, hipStream_t stream) {
    if (b.num_chains <= 0) return hipSuccess;
    if (w) {
        using Prob = PlainProb<T, true>;
        typename Prob::Params pp{y, w, w_scalar, x, b.es, b.cs, b.offsets};
        return seg_run<T, Prob, kTile>(workspace, b.num_chains, b.n, plan, pp, stream);
    }
    using Prob = PlainProb<T, false>;
    typename Prob::Params pp{y, w, w_scalar, x, b.es, b.cs, b.offsets};
    return seg_run<T, Prob, kTile>(workspace, b.num_chains, b.n, plan, pp, stream);
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
        return seg_run<T, Prob, kTile>(workspace, C, n, plan, pp, stream);
    }
    using Prob = MultiProb<T, false>;
    typename Prob::Params pp;
    fill(pp);
    return seg_run<T, Prob, kTile>(workspace, C, n, plan, pp, stream);
}

template <typename T>
size_t chain_prox_ws_bytes(const ChainBatch &b, const SegPlan &plan) {
    return seg_ws_bytes<T>(b.num_chains, b.n, plan);
}

// Autotuner candidates: segment lengths 32 .. 1024 and the whole chain (one
// segment per chain: no halo runs, for chains whose deques stay deeper than
// any halo recovers), halos 32, 64 and 128, rings of 16, 32, 64 or 128 slots
// (more than 16 only where segments are at least 4 times longer, to bound the
// saved deques; over 32 only for 8-byte entries), keeping only plans whose
// workspace stays within twice the default plan's (or the default's plus
// 64 MiB).  Segment lengths at or above the chain length are all the same
// plan, whose halo is never used; only one of them is kept.
template <typename T, typename G>
int seg_candidates(int64_t C, int64_t n, SegPlan *out, int max_out) {
    const SegPlan d = seg_default_plan(C, n);
    const size_t base = seg_ws_bytes<T, G>(C, n, d);
    const size_t cap = (2 * base > base + (size_t(64) << 20)) ? 2 * base : base + (size_t(64) << 20);
    int m = 0;
    if (m < max_out) out[m++] = d;
    bool whole = false;
    for (int64_t L = 32; !whole; L *= 2) {
        if (L > 1024) L = n;  // after 1024: the whole chain
        const int64_t Lr = (L >= n) ? ((n + kTile - 1) / kTile) * kTile : L;
        whole = L >= n;
        for (int K = 16; K <= 128; K *= 2) {
            if (K * 4 > Lr && K > 16) continue;
            if (K > ring_max<T, G>()) continue;
            for (int64_t H = 32; H <= (whole ? 32 : 128); H *= 2) {
                const SegPlan p{Lr, H, 16, K};
                if (seg_ws_bytes<T, G>(C, n, p) > cap) continue;
                bool dup = false;
                for (int j = 0; j < m; ++j)
                    dup = dup || (out[j].L == p.L && out[j].H == p.H && out[j].K == p.K);
                if (!dup && m < max_out) out[m++] = p;
            }
        }
    }
    return m;
}

template <typename T, typename G>
size_t seg_bytes_max(int64_t C, int64_t n, int kind) {
    SegPlan c[64];
    const int m = seg_candidates<T, G>(C, n, c, 64);
    size_t mx = 0;
    for (int j = 0; j < m; ++j) {
        const size_t b = seg_ws_bytes<T, G>(C, n, c[j]);
        mx = b > mx ? b : mx;
    }
    // a plan tuned for this shape earlier (or set by hand) must fit too
    const size_t t = seg_ws_bytes<T, G>(C, n, seg_plan(C, n, kind));
    return t > mx ? t : mx;
}

template <typename T, typename G>
size_t seg_ws_bytes_plan(int64_t C, int64_t n, const SegPlan &plan) {
    return seg_ws_bytes<T, G>(C, n, plan);
}
// Build parts: 1 the chain prox in FP32, 2 the multi-batch launch in FP32,
// 3 both in FP64, 4 the adjoint and the plan arithmetic.
#if TVC_IN_PART(4)
template size_t seg_ws_bytes_plan<float, float>(int64_t, int64_t, const SegPlan &);
template size_t seg_ws_bytes_plan<double, double>(int64_t, int64_t, const SegPlan &);
template size_t seg_ws_bytes_plan<float, double>(int64_t, int64_t, const SegPlan &);
template int seg_candidates<float, float>(int64_t, int64_t, SegPlan *, int);
template int seg_candidates<double, double>(int64_t, int64_t, SegPlan *, int);
template int seg_candidates<float, double>(int64_t, int64_t, SegPlan *, int);
template size_t seg_bytes_max<float, float>(int64_t, int64_t, int);
template size_t seg_bytes_max<double, double>(int64_t, int64_t, int);
template size_t seg_bytes_max<float, double>(int64_t, int64_t, int);
template size_t seg_ws_bytes_plan<float, TagJ<float>>(int64_t, int64_t, const SegPlan &);
template size_t seg_ws_bytes_plan<double, TagJ<double>>(int64_t, int64_t, const SegPlan &);
template int seg_candidates<float, TagJ<float>>(int64_t, int64_t, SegPlan *, int);
template int seg_candidates<double, TagJ<double>>(int64_t, int64_t, SegPlan *, int);
template size_t seg_bytes_max<float, TagJ<float>>(int64_t, int64_t, int);
template size_t seg_bytes_max<double, TagJ<double>>(int64_t, int64_t, int);
#endif

template <typename T>
hipError_t launch_chain_adjoint(const ChainBatch &b, const T *x, const T *g, T *gy, T *gw,
                                int w_per_edge, hipStream_t stream) {
    if (b.num_chains <= 0) return hipSuccess;
    if (b.offsets || b.es == 1) {  // unit-stride chains: one wave per chain, contiguous accesses
        const unsigned blocks = (unsigned)((b.num_chains + 3) / 4);
        hipLaunchKernelGGL((k_chain_adjoint_rows<T>), dim3(blocks), dim3(256), 0, stream, b, x, g, gy, gw,
                           w_per_edge);
        return hipGetLastError();
    }
    // strided chains (columns): one lane per chain, lanes read consecutive chains
    const unsigned blocks = (unsigned)((b.num_chains + 63) / 64);
    hipLaunchKernelGGL((k_chain_adjoint<T>), dim3(blocks), dim3(64), 0, stream, b, x, g, gy, gw,
                       w_per_edge);
    return hipGetLastError();
}

#if TVC_IN_PART(1)
template hipError_t launch_chain_prox<float>(const ChainBatch &, const float *, const float *, float,
                                             float *, void *, const SegPlan &, hipStream_t);
#endif
#if TVC_IN_PART(3)
template hipError_t launch_chain_prox<double>(const ChainBatch &, const double *, const double *, double,
                                              double *, void *, const SegPlan &, hipStream_t);
#endif
#if TVC_IN_PART(2)
template hipError_t launch_chain_prox_multi<float>(int, const ChainBatch *, const float *const *,
                                                   const float *const *, const double *, float *const *, void *,
                                                   const SegPlan &, hipStream_t);
#endif
#if TVC_IN_PART(3)
template hipError_t launch_chain_prox_multi<double>(int, const ChainBatch *, const double *const *,
                                                    const double *const *, const double *, double *const *, void *,
                                                    const SegPlan &, hipStream_t);
#endif
#if TVC_IN_PART(4)
template size_t chain_prox_ws_bytes<float>(const ChainBatch &, const SegPlan &);
template size_t chain_prox_ws_bytes<double>(const ChainBatch &, const SegPlan &);
template hipError_t launch_chain_adjoint<float>(const ChainBatch &, const float *, const float *,
                                                float *, float *, int, hipStream_t);
template hipError_t launch_chain_adjoint<double>(const ChainBatch &, const double *, const double *,
                                                 double *, double *, int, hipStream_t);
#endif

}  // namespace tvc
