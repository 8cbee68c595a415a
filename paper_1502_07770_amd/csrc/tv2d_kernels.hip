// tv2d_kernels.hip -- 2D ROF by Lagrangian decomposition into row and column
// chains (Sec. 5.1 of Kolmogorov, Pock, Rolinek, "Total variation on a tree").
//
//   min_x lambda (TV_h + TV_v)(x) + |x - f|^2 / 2,
//   saddle problem  min_x max_y <x, y> + lambda TV_h(x) + |x - f|^2/2 - (lambda TV_v)^*(y)
//   (eq. (rof-saddle)), solved by the accelerated primal-dual iteration eq. (pd):
//     column step: eta = y + sigma_k xbar;  y' = eta - prox_{lambda TV_v}(eta)
//                  (the dual prox through the Moreau identity, eq. (prox-tv-conj);
//                  the scale sigma drops out because TV is positively 1-homogeneous)
//     row step:    b = (tau_k f + x - tau_k y') / (1 + tau_k)
//                  x' = prox_{(lambda tau_k / (1 + tau_k)) TV_h}(b)
//                  (the primal prox with its quadratic weight 1 + 1/tau_k scaled to 1)
//                  xbar' = x' + theta_k (x' - x)
//   with theta_k = 1/sqrt(1 + 2 tau_k), tau_{k+1} = theta_k tau_k,
//   sigma_k = 1 / tau_k (G is 1-strongly convex, tau sigma = 1).
// Both steps are chain problems of eq. (1D-ROF) solved by the segmented exact
// DP (seg_kernels.h); the elementwise work is fused into the chain kernels'
// loads (data) and stores (epilogue).  x and y are double-buffered because the
// chain kernels re-read their inputs (halo and repair passes) after other
// segments have started writing outputs.
//
// Duality gap (FP64, every gap_every iterations).  Dual edge variables come
// from the two chain solves: down each column p_v,e = -sum_{k<=e} y'_k and
// along each row p_h,e = ((1 + tau)/tau) sum_{k<=e} (x'_k - b_k), both clipped
// to [-lambda, lambda] and rounded toward zero when stored in the iterate
// precision, so they are always feasible.  Then
//   P = lambda TV_h(x') + lambda TV_v(x') + |x' - f|^2 / 2,
//   D = |f|^2/2 - |f - D_h^T p_h - D_v^T p_v|^2 / 2,
// and P - D >= P(x') - min P >= 0 (weak duality).  The sums use a fixed block
// partition and tree reductions, so they are deterministic.
#include <math.h>

#include <vector>

#include "../../include/tvchain.h"
#include "kernels.h"
#include "seg_kernels.h"
#include "tv2d_common.h"

namespace tvc {

// Column step: chains are the W columns of the dense H x W state (es = W).
template <typename T>
struct ColProb {
    using Tag = T;  // a_i = 1: integer tags in the working precision
    static constexpr bool kGen = false;
    struct Params {
        const T *y_old;
        const T *xbar;
        T *y_new;
        const IterSched *sc;
        T lam;
        int64_t W;
    };
    struct Pre {
        T y, xb;
    };
    struct SinkPre {
        T y, xb;
    };
    struct Src {
        const T *__restrict__ y;
        const T *__restrict__ xb;
        T sigma, lam;
        int64_t c, W;
        __device__ __forceinline__ Pre load(int64_t i) const { return load_off(i * W + c); }
        __device__ __forceinline__ int64_t off(int64_t i) const { return i * W + c; }
        __device__ __forceinline__ int64_t step() const { return W; }
        __device__ __forceinline__ Pre load_off(int64_t o) const {
            Pre p;
            p.y = y[o];
            p.xb = xb[o];
            return p;
        }
        __device__ __forceinline__ T data(const Pre &p) const { return col_eta<T>(p.y, sigma, p.xb); }
        __device__ __forceinline__ T weight(const Pre &) const { return lam; }
        static constexpr bool vec = false;  // lanes of a wave already read consecutive columns
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const {
            for (int k = 0; k < 4; ++k) o[k] = load(i + k);
        }
    };
    struct Sink {
        const T *__restrict__ y;
        const T *__restrict__ xb;
        T *__restrict__ yn;
        T sigma;
        int64_t c, W;
        __device__ __forceinline__ SinkPre load(int64_t i) const {
            SinkPre p;
            p.y = y[i * W + c];
            p.xb = xb[i * W + c];
            return p;
        }
        __device__ __forceinline__ void store(int64_t i, T u, const SinkPre &p) const {
            yn[i * W + c] = col_dual<T>(p.y, sigma, p.xb, u);
        }
        static constexpr bool vec = false;
        __device__ __forceinline__ void load4(int64_t i, SinkPre *o) const {
            for (int k = 0; k < 4; ++k) o[k] = load(i + k);
        }
        __device__ __forceinline__ void store4(int64_t i, const T (&u)[4], const SinkPre (&p)[4]) const {
            for (int k = 0; k < 4; ++k) store(i + k, u[k], p[k]);
        }
    };
    static __device__ __forceinline__ ChainSpan span(const Params &, int64_t c, int64_t nmax) {
        return ChainSpan{c, 0, nmax, 0};
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) {
        return Src{p.y_old, p.xbar, (T)p.sc->sigma, p.lam, sp.base, p.W};
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{p.y_old, p.xbar, p.y_new, (T)p.sc->sigma, sp.base, p.W};
    }
};

// Row step: chains are the H rows (es = 1); f has its own leading dimension.
template <typename T>
struct RowProb {
    using Tag = T;  // a_i = 1: integer tags in the working precision
    static constexpr bool kGen = false;
    struct Params {
        const T *f;
        int64_t ldf;
        const T *x_old;
        const T *y;
        T *x_new;
        T *xbar;
        const IterSched *sc;
        double lam;
        int64_t W;
    };
    struct Pre {
        T f, x, y;
    };
    struct SinkPre {
        T x;
    };
    struct Src {
        const T *__restrict__ f;
        const T *__restrict__ x;
        const T *__restrict__ y;
        T tau, inv1p, w;
        int64_t r, ldf, W;
        bool vec;  // the row's three streams are element-aligned: load4 may be used
        __device__ __forceinline__ Src(const T *f_, const T *x_, const T *y_, T tau_, T inv1p_, T w_, int64_t r_,
                                       int64_t ldf_, int64_t W_)
            : f(f_), x(x_), y(y_), tau(tau_), inv1p(inv1p_), w(w_), r(r_), ldf(ldf_), W(W_),
              vec(elem_aligned(f_ + r_ * ldf_) && elem_aligned(x_ + r_ * W_) && elem_aligned(y_ + r_ * W_)) {}
        __device__ __forceinline__ Pre load(int64_t i) const {
            Pre p;
            p.f = f[r * ldf + i];
            p.x = x[r * W + i];
            p.y = y[r * W + i];
            return p;
        }
        __device__ __forceinline__ int64_t off(int64_t i) const { return i; }
        __device__ __forceinline__ int64_t step() const { return 1; }
        __device__ __forceinline__ Pre load_off(int64_t o) const { return load(o); }
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const {
            T a[4], b[4], c[4];
            vload4(f + r * ldf + i, a);
            vload4(x + r * W + i, b);
            vload4(y + r * W + i, c);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                o[k].f = a[k];
                o[k].x = b[k];
                o[k].y = c[k];
            }
        }
        __device__ __forceinline__ T data(const Pre &p) const { return row_data(p.f, p.x, p.y, tau, inv1p); }
        __device__ __forceinline__ T weight(const Pre &) const { return w; }
    };
    struct Sink {
        const T *__restrict__ x;
        T *__restrict__ xn;
        T *__restrict__ xb;
        T theta;
        int64_t r, W;
        bool vec;  // the row's streams are element-aligned: load4 / store4 may be used
        __device__ __forceinline__ Sink(const T *x_, T *xn_, T *xb_, T theta_, int64_t r_, int64_t W_)
            : x(x_), xn(xn_), xb(xb_), theta(theta_), r(r_), W(W_),
              vec(elem_aligned(x_ + r_ * W_) && elem_aligned(xn_ + r_ * W_) && elem_aligned(xb_ + r_ * W_)) {}
        __device__ __forceinline__ SinkPre load(int64_t i) const { return SinkPre{x[r * W + i]}; }
        __device__ __forceinline__ void load4(int64_t i, SinkPre *o) const {
            T v[4];
            vload4(x + r * W + i, v);
            for (int k = 0; k < 4; ++k) o[k].x = v[k];
        }
        __device__ __forceinline__ void store(int64_t i, T u, const SinkPre &p) const {
            xn[r * W + i] = u;
            xb[r * W + i] = row_xbar<T>(u, theta, p.x);
        }
        __device__ __forceinline__ void store4(int64_t i, const T (&u)[4], const SinkPre (&p)[4]) const {
            T b[4];
            for (int k = 0; k < 4; ++k) b[k] = row_xbar<T>(u[k], theta, p[k].x);
            vstore4(xn + r * W + i, u);
            vstore4(xb + r * W + i, b);
        }
    };
    static __device__ __forceinline__ ChainSpan span(const Params &, int64_t r, int64_t nmax) {
        return ChainSpan{r, 1, nmax, 0};
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) {
        const IterSched sc = *p.sc;
        return Src{p.f, p.x_old, p.y, (T)sc.tau, (T)sc.inv1p, (T)(p.lam * sc.tau * sc.inv1p), sp.base, p.ldf, p.W};
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{p.x_old, p.x_new, p.xbar, (T)p.sc->theta, sp.base, p.W};
    }
};

// ---------------------------------------------------------------------------
// Gap kernels.
// ---------------------------------------------------------------------------
// p_v down every column: p_v[r][c] = clip(-sum_{k<=r} y[k][c]), as a
// two-phase segmented scan over row blocks of kGapRows rows; lanes are
// consecutive columns, so every load is coalesced.

template <typename T>
__global__ __launch_bounds__(64) void k_gap_colsum(const T *__restrict__ y, double *__restrict__ colpart, int64_t H,
                                                   int64_t W, const int *__restrict__ stop) {
    if (*stop) return;
    const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t nseg = (H + kGapRows - 1) / kGapRows;
    if (g >= nseg * W) return;
    const int64_t c = g % W, sg = g / W;
    const int64_t r0 = sg * kGapRows, r1 = (r0 + kGapRows < H) ? r0 + kGapRows : H;
    double acc = 0.0;
#pragma unroll 8
    for (int64_t r = r0; r < r1; ++r) acc += (double)y[r * W + c];
    colpart[sg * W + c] = acc;
}

template <typename T>
__global__ __launch_bounds__(64) void k_gap_pv(const T *__restrict__ y, const double *__restrict__ colpart,
                                               T *__restrict__ pv, int64_t H, int64_t W, double lam,
                                               const int *__restrict__ stop) {
    if (*stop) return;
    const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t nseg = (H + kGapRows - 1) / kGapRows;
    if (g >= nseg * W) return;
    const int64_t c = g % W, sg = g / W;
    double cs = 0.0;
    for (int64_t j = 0; j < sg; ++j) cs += colpart[j * W + c];
    const int64_t r0 = sg * kGapRows, r1 = (r0 + kGapRows < H) ? r0 + kGapRows : H;
#pragma unroll 8
    for (int64_t r = r0; r < r1; ++r) {
        cs += (double)y[r * W + c];
        pv[r * W + c] = store_feasible<T>(clipd(-cs, lam));
    }
}

// One wave per row, 64 columns per pass: the row's residual x' - b is
// prefix-summed across the wave (FP64 shuffles) into p_h; every pixel adds its
// primal terms and its dual term 1/2 f^2 - 1/2 (f - z)^2 with
// z = (D_h^T p_h + D_v^T p_v) at that pixel.  Per-row sums go to part.

template <typename T>
__global__ __launch_bounds__(kGapBlock) void k_gap_rows(const T *__restrict__ f, int64_t ldf, const T *__restrict__ xn,
                                                        const T *__restrict__ xo, const T *__restrict__ y,
                                                        const T *__restrict__ pv, int64_t H, int64_t W, double lam,
                                                        const IterSched *__restrict__ sc, double *__restrict__ part,
                                                        const int *__restrict__ stop) {
    if (*stop) return;
    const T tau = (T)sc->tau, inv1p = (T)sc->inv1p;
    const double pscale = sc->pscale;
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (kGapBlock / 64) + (threadIdx.x >> 6);
    if (r >= H) return;  // whole waves exit together: no block barrier below
    double P = 0.0, D = 0.0, carry = 0.0, ph_last = 0.0;
    for (int64_t c0 = 0; c0 < W; c0 += 64) {
        const int64_t c = c0 + lane;
        const bool in = c < W;
        const int64_t k = r * W + c;
        T fv = 0, xv = 0, xo_v = 0, yv = 0, xr = 0, xd_ = 0, pvu = 0, pvd = 0;
        if (in) {
            fv = f[r * ldf + c];
            xv = xn[k];
            xo_v = xo[k];
            yv = y[k];
            if (c + 1 < W) xr = xn[k + 1];
            if (r + 1 < H) {
                xd_ = xn[k + W];
                pvd = pv[k];
            }
            if (r > 0) pvu = pv[k - W];
        }
        const T b = row_data<T>(fv, xo_v, yv, tau, inv1p);
        double res = (in && c + 1 < W) ? (double)xv - (double)b : 0.0;
        // inclusive prefix over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double t = __shfl_up(res, off, 64);
            if (lane >= off) res += t;
        }
        const double cs = carry + res;
        const double ph = (in && c + 1 < W) ? (double)store_feasible<T>(clipd(pscale * cs, lam)) : 0.0;
        double ph_left = __shfl_up(ph, 1, 64);
        if (lane == 0) ph_left = ph_last;
        if (in) {
            double z = ph_left - ph;
            if (r > 0) z += (double)pvu;
            if (r + 1 < H) z -= (double)pvd;
            const double fd = (double)fv, xd = (double)xv;
            P += 0.5 * (xd - fd) * (xd - fd);
            if (c + 1 < W) P += lam * fabs((double)xr - xd);
            if (r + 1 < H) P += lam * fabs((double)xd_ - xd);
            D += 0.5 * fd * fd - 0.5 * (fd - z) * (fd - z);
        }
        carry = __shfl(cs, 63, 64);
        ph_last = __shfl(ph, 63, 64);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        P += __shfl_down(P, off, 64);
        D += __shfl_down(D, off, 64);
    }
    if (lane == 0) {
        part[2 * r] = P;
        part[2 * r + 1] = D;
    }
}

struct Tv2dHeader {  // device-resident solver state header
    int64_t iters;   // iterations done (at the last gap evaluation)
    int64_t cur;     // which x / y buffer holds the current iterate
    double gap[3];   // P, D, gap_norm of the last evaluation
    SolveCtl ctl;    // schedule position and stop flag
};

// Final reduction (one block): the header gets {P, D, (P - D) / (H W)}, the
// iteration count and the buffer of the iterate (nxt); the gap history slot of
// this iteration is written; and the solve stops once the gap is at tol > 0,
// or is not finite.
static __global__ __launch_bounds__(kGapBlock) void k_gap_final(const double *__restrict__ part, int nparts, double HW,
                                                                Tv2dHeader *__restrict__ h, double *__restrict__ hist,
                                                                const IterSched *__restrict__ sc, double tol, int nxt) {
    if (*(volatile const int *)&h->ctl.stop) return;
    const int64_t hist_idx = sc->iter_after - 1;
    __shared__ double sP[kGapBlock], sD[kGapBlock];
    double P = 0.0, D = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kGapBlock) {
        P += part[2 * i];
        D += part[2 * i + 1];
    }
    sP[threadIdx.x] = P;
    sD[threadIdx.x] = D;
    __syncthreads();
    for (int st = kGapBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sP[threadIdx.x] += sP[threadIdx.x + st];
            sD[threadIdx.x] += sD[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double g = (sP[0] - sD[0]) / HW;
        h->gap[0] = sP[0];
        h->gap[1] = sD[0];
        h->gap[2] = g;
        h->iters = sc->iter_after;
        h->cur = nxt;
        if (hist) hist[hist_idx] = g;
        if (!isfinite(g)) ctl_stop(&h->ctl, TV_ERR_NONFINITE);
        else if (tol > 0.0 && g <= tol) ctl_stop(&h->ctl, TV_OK);
    }
}

// Copy of the iterate into the caller's x (ld >= W) and, from one thread, the
// stats of the solve.
template <typename T>
__global__ __launch_bounds__(256) void k_tv2d_finish(const Tv2dHeader *__restrict__ h, const T *__restrict__ x0,
                                                     const T *__restrict__ x1, T *__restrict__ out, int64_t ld,
                                                     int64_t H, int64_t W, tv2d_stats *__restrict__ stats, double tol,
                                                     double clk_khz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const T *src = h->cur ? x1 : x0;
    if (i < H * W) out[(i / W) * ld + i % W] = src[i];
    if (i == 0 && stats) {
        const double g = h->gap[2];
        int st = TV_OK;
        if (h->ctl.stop) st = h->ctl.status;
        else if (h->iters > 0 && !isfinite(g)) st = TV_ERR_NONFINITE;
        else if (tol > 0.0) st = TV_ERR_NOT_CONVERGED;
        stats->iters = (int)h->iters;
        stats->status = st;
        stats->gap_norm = g;
        stats->primal = h->gap[0];
        stats->dual = h->gap[1];
        stats->device_ms = ctl_ms(&h->ctl, clk_khz);
    }
}

// Fresh header: no iteration yet, tau0, the iterate in buffer 0.
static __global__ void k_tv2d_init_hdr(Tv2dHeader *h) {
    if (threadIdx.x != 0) return;
    h->iters = 0;
    h->cur = 0;
    h->gap[0] = h->gap[1] = h->gap[2] = __builtin_nan("");
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
template <typename T>
struct Tv2dWs {
    Tv2dHeader *hdr;
    T *x[2], *y[2], *xbar, *pv;
    IterSched *sched;  // [kSchedCap] per-iteration scalars of the current chunk
    double *part;
    double *colpart;
    void *seg;       // chain-prox workspace, shared by the row and column launches
    size_t seg_bytes;
};

template <typename T>
static size_t tv2d_layout(void *base, int64_t H, int64_t W, Tv2dWs<T> *out, bool l1 = false) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t N = (size_t)(H * W);
    // room for any plan the autotuner may choose for the row and column launches
    // (TV-l1 rows keep (lambda, tag, jump) sets)
    const size_t sr = l1 ? seg_bytes_max<double, TagJ<double>>(H, W, kPlan2dRowL1)  // FP64 set (WideL1)
                         : seg_bytes_max<T>(H, W, kPlan2dRow);
    const size_t scol = seg_bytes_max<T>(W, H, l1 ? kPlan2dColL1 : kPlan2dCol);
    const size_t nparts = (size_t)H;
    const size_t ncol = (size_t)(((H + kGapRows - 1) / kGapRows) * W);
    size_t off = 0;
    const size_t o_hdr = off; off += al(sizeof(Tv2dHeader));
    const size_t o_x0 = off;  off += al(sizeof(T) * N);
    const size_t o_x1 = off;  off += al(sizeof(T) * N);
    const size_t o_y0 = off;  off += al(sizeof(T) * N);
    const size_t o_y1 = off;  off += al(sizeof(T) * N);
    const size_t o_xb = off;  off += al(sizeof(T) * N);
    const size_t o_pv = off;  off += al(sizeof(T) * N);
    const size_t o_sc = off;  off += al(sizeof(IterSched) * kSchedCap);
    const size_t o_pt = off;  off += al(sizeof(double) * 2 * nparts);
    const size_t o_cp = off;  off += al(sizeof(double) * ncol);
    const size_t o_sg = off;  off += al(sr > scol ? sr : scol);
    if (base && out) {
        char *p = (char *)base;
        out->hdr = (Tv2dHeader *)(p + o_hdr);
        out->x[0] = (T *)(p + o_x0);
        out->x[1] = (T *)(p + o_x1);
        out->y[0] = (T *)(p + o_y0);
        out->y[1] = (T *)(p + o_y1);
        out->xbar = (T *)(p + o_xb);
        out->pv = (T *)(p + o_pv);
        out->sched = (IterSched *)(p + o_sc);
        out->part = (double *)(p + o_pt);
        out->colpart = (double *)(p + o_cp);
        out->seg = (void *)(p + o_sg);
        out->seg_bytes = sr > scol ? sr : scol;
    }
    return off;
}

// Column step: y[nxt] = eta - prox(eta), eta = y[cur] + sigma xbar.
template <typename T>
static hipError_t tv2d_col_step(const Tv2dWs<T> &ws, int64_t H, int64_t W, double lam, int cur, const IterSched *sc,
                                const SegPlan &pc, hipStream_t st, const int *stop = nullptr) {
    const int nxt = cur ^ 1;
    typename ColProb<T>::Params pp{ws.y[cur], ws.xbar, ws.y[nxt], sc, (T)lam, W};
    return seg_run<T, ColProb<T>, kTile>(ws.seg, W, H, pc, pp, st, stop);
}

// Row step: x[nxt] = prox(b), xbar = x[nxt] + theta (x[nxt] - x[cur]).
template <typename T>
static hipError_t tv2d_row_step(const Tv2dWs<T> &ws, const T *f, int64_t ldf, int64_t H, int64_t W, double lam,
                                int cur, const IterSched *sc, const SegPlan &pr, hipStream_t st,
                                const int *stop = nullptr) {
    const int nxt = cur ^ 1;
    typename RowProb<T>::Params pp{f, ldf, ws.x[cur], ws.y[nxt], ws.x[nxt], ws.xbar, sc, lam, W};
    return seg_run<T, RowProb<T>, kTile>(ws.seg, H, W, pr, pp, st, stop);
}

// `count` iterations from parity cur0, iteration j reading ws.sched[j]
// (generated on the device first); with `gap`, the gap evaluation and the
// stopping test follow the last one.  Launched directly or captured into a
// HIP graph: nothing here reads host memory.  Every kernel returns at once if
// the solve has stopped.
template <typename T>
static hipError_t tv2d_iters(const Tv2dWs<T> &ws, const T *f, int64_t ldf, int64_t H, int64_t W, double lam,
                             int cur0, int count, bool gap, double tol, double *hist, const SegPlan &pc,
                             const SegPlan &pr, hipStream_t st) {
    const int *stop = &ws.hdr->ctl.stop;
    hipLaunchKernelGGL(k_ctl_sched, dim3(1), dim3(64), 0, st, &ws.hdr->ctl, ws.sched, count);
    int cur = cur0;
    for (int j = 0; j < count; ++j) {
        const int nxt = cur ^ 1;
        const IterSched *sc = ws.sched + j;
        hipError_t e = tv2d_col_step<T>(ws, H, W, lam, cur, sc, pc, st, stop);
        if (e == hipSuccess) e = tv2d_row_step<T>(ws, f, ldf, H, W, lam, cur, sc, pr, st, stop);
        if (e != hipSuccess) return e;
        if (gap && j == count - 1) {
            const int64_t nseg = (H + kGapRows - 1) / kGapRows;
            const unsigned cb = (unsigned)((nseg * W + 63) / 64);
            hipLaunchKernelGGL((k_gap_colsum<T>), dim3(cb), dim3(64), 0, st, ws.y[nxt], ws.colpart, H, W, stop);
            hipLaunchKernelGGL((k_gap_pv<T>), dim3(cb), dim3(64), 0, st, ws.y[nxt], ws.colpart, ws.pv, H, W, lam,
                               stop);
            const unsigned rb = (unsigned)((H + kGapBlock / 64 - 1) / (kGapBlock / 64));
            hipLaunchKernelGGL((k_gap_rows<T>), dim3(rb), dim3(kGapBlock), 0, st, f, ldf, ws.x[nxt], ws.x[cur],
                               ws.y[nxt], ws.pv, H, W, lam, sc, ws.part, stop);
            hipLaunchKernelGGL(k_gap_final, dim3(1), dim3(kGapBlock), 0, st, ws.part, (int)H, (double)(H * W), ws.hdr,
                               hist, sc, tol, nxt);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur = nxt;
    }
    return hipSuccess;
}

// The solve is enqueued on st without waiting on the device (the stopping
// test runs on the device, see tv2d_iters), all of it, or with a lookahead
// the host keeps at most that many gap evaluations ahead and stops enqueuing
// once the device has stopped; a resume reads the header once to learn which
// buffer holds the iterate.
template <typename T>
static tv_status tv2d_solve_t(const T *f, int64_t H, int64_t W, int64_t ld, double lam, T *x,
                              const tv2d_options *opt, tv2d_stats *stats, void *workspace, hipStream_t st) {
    Tv2dWs<T> ws;
    tv2d_layout<T>(workspace, H, W, &ws);
    const unsigned nb = (unsigned)((H * W + 255) / 256);
    Lookahead la;
    const tv_status ls = la.begin(opt->lookahead, st);
    if (ls != TV_OK) return ls;
    int cur = 0;
    if (opt->resume) {
        int64_t c = 0;
        if (hipMemcpyAsync(&c, &ws.hdr->cur, sizeof(c), hipMemcpyDeviceToHost, st) != hipSuccess) return TV_ERR_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return TV_ERR_HIP;
        cur = (int)(c & 1);
        hipLaunchKernelGGL(k_ctl_resume, dim3(1), dim3(64), 0, st, &ws.hdr->ctl, la.dev_word(), la.seq);
    } else {
        // x^0 = xbar^0 = f, y^0 = 0
        hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, ld, ws.x[0], W, H, W);
        hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, ld, ws.xbar, W, H, W);
        hipLaunchKernelGGL((k_fill<T>), dim3(nb), dim3(256), 0, st, ws.y[0], H * W, (T)0);
        hipLaunchKernelGGL(k_tv2d_init_hdr, dim3(1), dim3(64), 0, st, ws.hdr);
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, &ws.hdr->ctl, opt->tau0, 1, la.dev_word(),
                           la.seq);
    }
    const int every = opt->gap_every > 0 ? opt->gap_every : 1;
    const SegPlan pc = seg_plan(W, H, kPlan2dCol), pr = seg_plan(H, W, kPlan2dRow);
    if (seg_ws_bytes_plan<T>(W, H, pc) > ws.seg_bytes || seg_ws_bytes_plan<T>(H, W, pr) > ws.seg_bytes)
        return TV_ERR_WORKSPACE;
    ChunkGraphs graphs;
    for (int done = 0; done < opt->max_iter;) {
        hipError_t le;
        if (la.stopped(&le)) break;
        if (le != hipSuccess) return TV_ERR_HIP;
        const int chunk = (opt->max_iter - done < every) ? opt->max_iter - done : every;
        for (int part = 0; part < chunk;) {
            const int piece = (chunk - part < kSchedCap) ? chunk - part : kSchedCap;
            const bool last = part + piece == chunk;
            const int c0 = cur;
            auto issue = [&](hipStream_t s2) {
                return tv2d_iters<T>(ws, f, ld, H, W, lam, c0, piece, last, opt->gap_tol, opt->gap_history, pc,
                                     pr, s2);
            };
            hipGraphExec_t ge = nullptr;
            if (opt->use_graph && last && piece == every && part == 0) ge = graphs.get(cur, issue);
            if (ge) {
                if (hipGraphLaunch(ge, st) != hipSuccess) return TV_ERR_HIP;
            } else if (issue(st) != hipSuccess) {
                return TV_ERR_HIP;
            }
            cur = (cur + piece) & 1;
            part += piece;
        }
        if (la.chunk_done(st) != hipSuccess) return TV_ERR_HIP;
        done += chunk;
    }
    hipLaunchKernelGGL((k_tv2d_finish<T>), dim3(nb), dim3(256), 0, st, ws.hdr, ws.x[0], ws.x[1], x, ld, H, W, stats,
                       opt->gap_tol, wall_clock_khz());
    if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
    // captured graphs live for this call only: wait for their replays
    if (graphs.exec[0] || graphs.exec[1]) return hipStreamSynchronize(st) == hipSuccess ? TV_OK : TV_ERR_HIP;
    return TV_OK;
}

// Autotune of the column and the row launch on the first iteration's data.
template <typename T>
static tv_status tv2d_autotune_t(const T *f, int64_t H, int64_t W, int64_t ld, double lam, double tau0,
                                 void *workspace, hipStream_t st, tv_tuning_result *col, tv_tuning_result *row) {
    Tv2dWs<T> ws;
    tv2d_layout<T>(workspace, H, W, &ws);
    const unsigned nb = (unsigned)((H * W + 255) / 256);
    hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, ld, ws.x[0], W, H, W);
    hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, ld, ws.xbar, W, H, W);
    hipLaunchKernelGGL((k_fill<T>), dim3(nb), dim3(256), 0, st, ws.y[0], H * W, (T)0);
    hipLaunchKernelGGL(k_tv2d_init_hdr, dim3(1), dim3(64), 0, st, ws.hdr);
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, &ws.hdr->ctl, tau0, 1, nullptr, 0u);
    // Run a few iterations first: the deques of the column and row chains
    // deepen as the dual variable builds up, and a plan timed on the first
    // iteration's data alone would pick a ring that overflows later on.
    if (tv2d_iters<T>(ws, f, ld, H, W, lam, 0, kTuneWarm, false, 0.0, nullptr, seg_plan(W, H, kPlan2dCol),
                      seg_plan(H, W, kPlan2dRow), st) != hipSuccess)
        return TV_ERR_HIP;
    // the timed steps read iteration kTuneWarm's scalars from the first slot
    hipLaunchKernelGGL(k_ctl_sched, dim3(1), dim3(64), 0, st, &ws.hdr->ctl, ws.sched, 1);
    SegPlan pc, pr;
    tv_status s = tune_launch<T>(
        W, H, ws.seg_bytes, [&](const SegPlan &p) { return tv2d_col_step<T>(ws, H, W, lam, 0, ws.sched, p, st); },
        st, &pc, col);
    if (s != TV_OK) return s;
    if (tv2d_col_step<T>(ws, H, W, lam, 0, ws.sched, pc, st) != hipSuccess) return TV_ERR_HIP;
    s = tune_launch<T>(
        H, W, ws.seg_bytes,
        [&](const SegPlan &p) { return tv2d_row_step<T>(ws, f, ld, H, W, lam, 0, ws.sched, p, st); }, st, &pr, row);
    if (s != TV_OK) return s;
    seg_set_tuned(kPlan2dCol, W, H, pc);
    seg_set_tuned(kPlan2dRow, H, W, pr);
    return hipStreamSynchronize(st) == hipSuccess ? TV_OK : TV_ERR_HIP;
}

// ---------------------------------------------------------------------------
// TV-l1 (Sec. 5.2): min_x lambda (TV_h + TV_v)(x) + |x - f|_1, eq. (pd) with
// constant steps (tau, sigma = 1 / tau, theta = 1).  The column step is the
// ROF one; the row step is the primal prox eq. (prox-pq) times tau, i.e. per
// row the TV-l1 chain prox argmin tau lambda TV + tau |x - f|_1 + |x - xi|^2/2
// with xi = x - tau y', formed in the loads; xbar in the stores.
// ---------------------------------------------------------------------------
template <typename T>
struct RowL1Prob {
    using Tag = TagJ<T>;
    static constexpr bool kGen = false;
    static constexpr bool kL1 = true;
    using Params = typename RowProb<T>::Params;
    using Pre = typename RowProb<T>::Pre;
    using SinkPre = typename RowProb<T>::SinkPre;
    using Sink = typename RowProb<T>::Sink;
    struct Src : RowProb<T>::Src {
        using Base = typename RowProb<T>::Src;
        __device__ __forceinline__ Src(const Base &b) : Base(b) {}
        __device__ __forceinline__ T data(const Pre &p) const { return l1_row_data<T>(p.x, this->tau, p.y); }
        __device__ __forceinline__ T dval(const Pre &p) const { return p.f; }
        __device__ __forceinline__ T cval(const Pre &) const { return this->tau; }
        __device__ __forceinline__ T weight(const Pre &) const { return this->w; }
    };
    static __device__ __forceinline__ ChainSpan span(const Params &p, int64_t r, int64_t nmax) {
        return RowProb<T>::span(p, r, nmax);
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) {
        const IterSched sc = *p.sc;
        // c = tau, w = tau lambda (inv1p slot unused)
        return Src(typename RowProb<T>::Src{p.f, p.x_old, p.y, (T)sc.tau, (T)0, (T)(p.lam * sc.tau), sp.base, p.ldf,
                                            p.W});
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return RowProb<T>::sink(p, sp);
    }
};

template <typename T>
static hipError_t tv2d_l1_row_step(const Tv2dWs<T> &ws, const T *f, int64_t ldf, int64_t H, int64_t W, double lam,
                                   int cur, const IterSched *sc, const SegPlan &pr, hipStream_t st) {
    const int nxt = cur ^ 1;
    using R = typename L1Run<RowL1Prob, T>::Prob;  // the set in FP64 (see WideL1)
    typename R::Params pp{f, ldf, ws.x[cur], ws.y[nxt], ws.x[nxt], ws.xbar, sc, lam, W};
    return seg_run<double, R, kTile>(ws.seg, H, W, pr, pp, st);
}

// TV-l1 energy lambda (TV_h + TV_v)(x) + |x - f|_1 in FP64: one wave per row
// (lanes over columns, butterfly sum), then one block over the rows in a fixed
// order.
template <typename T>
__global__ __launch_bounds__(kGapBlock) void k_l1_energy_rows(const T *__restrict__ x, const T *__restrict__ f,
                                                              int64_t ldf, int64_t H, int64_t W, double lam,
                                                              double *__restrict__ part) {
    const int64_t r = (int64_t)blockIdx.x * (kGapBlock / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (r >= H) return;
    double acc = 0.0;
    for (int64_t c = lane; c < W; c += 64) {
        const double v = (double)x[r * W + c];
        acc += fabs(v - (double)f[r * ldf + c]);
        if (c + 1 < W) acc += lam * fabs((double)x[r * W + c + 1] - v);
        if (r + 1 < H) acc += lam * fabs((double)x[(r + 1) * W + c] - v);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) part[r] = acc;
}

static __global__ __launch_bounds__(kGapBlock) void k_l1_energy_final(const double *__restrict__ part, int64_t H,
                                                               double *__restrict__ out, double *__restrict__ hist,
                                                               int64_t hist_at) {
    __shared__ double s[kGapBlock];
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < H; r += kGapBlock) acc += part[r];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kGapBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out = s[0];
        if (hist && hist_at >= 0) hist[hist_at] = s[0];
    }
}

template <typename T>
static hipError_t tv2d_l1_energy(const Tv2dWs<T> &ws, const T *x, const T *f, int64_t ldf, int64_t H, int64_t W,
                                 double lam, double *hist, int64_t hist_at, hipStream_t st) {
    const unsigned rb = (unsigned)((H + kGapBlock / 64 - 1) / (kGapBlock / 64));
    hipLaunchKernelGGL((k_l1_energy_rows<T>), dim3(rb), dim3(kGapBlock), 0, st, x, f, ldf, H, W, lam, ws.part);
    hipLaunchKernelGGL(k_l1_energy_final, dim3(1), dim3(kGapBlock), 0, st, ws.part, H, &ws.hdr->gap[0], hist,
                       hist_at);
    return hipGetLastError();
}

// Constant-step schedule: tau, sigma = 1/tau, theta = 1.
static __host__ __device__ IterSched l1_sched(double tau, int64_t k) {
    IterSched s;
    s.tau = tau;
    s.sigma = 1.0 / tau;
    s.theta = 1.0;
    s.inv1p = 0.0;
    s.pscale = 0.0;
    s.iter_after = k + 1;
    return s;
}

static __global__ void k_l1_sched_set(IterSched *sc, double tau) {
    if (threadIdx.x == 0) sc[0] = l1_sched(tau, 0);
}

template <typename T>
static tv_status tv2d_l1_init(const T *f, int64_t H, int64_t W, int64_t ld, double tau, const Tv2dWs<T> &ws,
                              hipStream_t st) {
    const unsigned nb = (unsigned)((H * W + 255) / 256);
    hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, ld, ws.x[0], W, H, W);
    hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, ld, ws.xbar, W, H, W);
    hipLaunchKernelGGL((k_fill<T>), dim3(nb), dim3(256), 0, st, ws.y[0], H * W, (T)0);
    // the same scalars every iteration
    hipLaunchKernelGGL(k_l1_sched_set, dim3(1), dim3(64), 0, st, ws.sched, tau);
    // the device clock starts here (no schedule: the count is 0)
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, &ws.hdr->ctl, tau, 1, nullptr, 0u);
    hipLaunchKernelGGL(k_ctl_sched, dim3(1), dim3(64), 0, st, &ws.hdr->ctl, ws.sched, 0);
    return hipGetLastError() == hipSuccess ? TV_OK : TV_ERR_HIP;
}

// Copy of the iterate into the caller's x and the stats of a TV-l1 solve (its
// energy in gap[0]; no duality gap).
template <typename T>
__global__ __launch_bounds__(256) void k_tv2d_l1_finish(const Tv2dHeader *__restrict__ h, const T *__restrict__ xc,
                                                        T *__restrict__ out, int64_t ld, int64_t H, int64_t W,
                                                        tv2d_stats *__restrict__ stats, int iters, double clk_khz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < H * W) out[(i / W) * ld + i % W] = xc[i];
    if (i == 0 && stats) {
        const double P = h->gap[0];
        stats->iters = iters;
        stats->status = isfinite(P) ? TV_OK : TV_ERR_NONFINITE;
        stats->primal = P;
        stats->dual = __builtin_nan("");
        stats->gap_norm = __builtin_nan("");
        stats->device_ms = ctl_ms(&h->ctl, clk_khz);
    }
}

template <typename T>
static tv_status tv2d_l1_solve_t(const T *f, int64_t H, int64_t W, int64_t ld, double lam, T *x,
                                 const tv2d_options *opt, tv2d_stats *stats, void *workspace, hipStream_t st) {
    Tv2dWs<T> ws;
    tv2d_layout<T>(workspace, H, W, &ws, true);
    tv_status s = tv2d_l1_init<T>(f, H, W, ld, opt->tau0, ws, st);
    if (s != TV_OK) return s;
    const SegPlan pc = seg_plan(W, H, kPlan2dColL1), pr = seg_plan(H, W, kPlan2dRowL1);
    if (seg_ws_bytes_plan<T>(W, H, pc) > ws.seg_bytes || seg_ws_bytes_plan<double, TagJ<double>>(H, W, pr) > ws.seg_bytes)
        return TV_ERR_WORKSPACE;
    const int every = opt->gap_every > 0 ? opt->gap_every : 1;
    int cur = 0;
    for (int k = 0; k < opt->max_iter; ++k) {
        if (tv2d_col_step<T>(ws, H, W, lam, cur, ws.sched, pc, st) != hipSuccess) return TV_ERR_HIP;
        if (tv2d_l1_row_step<T>(ws, f, ld, H, W, lam, cur, ws.sched, pr, st) != hipSuccess) return TV_ERR_HIP;
        cur ^= 1;
        if ((k + 1) % every == 0 || k + 1 == opt->max_iter) {
            if (tv2d_l1_energy<T>(ws, ws.x[cur], f, ld, H, W, lam, opt->gap_history, k, st) != hipSuccess)
                return TV_ERR_HIP;
        }
    }
    if (opt->max_iter == 0 && tv2d_l1_energy<T>(ws, ws.x[0], f, ld, H, W, lam, nullptr, -1, st) != hipSuccess)
        return TV_ERR_HIP;
    const unsigned nb = (unsigned)((H * W + 255) / 256);
    hipLaunchKernelGGL((k_tv2d_l1_finish<T>), dim3(nb), dim3(256), 0, st, ws.hdr, ws.x[cur], x, ld, H, W, stats,
                       opt->max_iter, wall_clock_khz());
    return hipGetLastError() == hipSuccess ? TV_OK : TV_ERR_HIP;
}

template <typename T>
static tv_status tv2d_l1_autotune_t(const T *f, int64_t H, int64_t W, int64_t ld, double lam, double tau0,
                                    void *workspace, hipStream_t st, tv_tuning_result *col, tv_tuning_result *row) {
    Tv2dWs<T> ws;
    tv2d_layout<T>(workspace, H, W, &ws, true);
    tv_status s = tv2d_l1_init<T>(f, H, W, ld, tau0, ws, st);
    if (s != TV_OK) return s;
    // a few iterations first, so the plans are timed on later-iteration data
    const SegPlan pc0 = seg_plan(W, H, kPlan2dColL1), pr0 = seg_plan(H, W, kPlan2dRowL1);
    for (int k = 0; k < kTuneWarm; ++k) {
        if (tv2d_col_step<T>(ws, H, W, lam, k & 1, ws.sched, pc0, st) != hipSuccess) return TV_ERR_HIP;
        if (tv2d_l1_row_step<T>(ws, f, ld, H, W, lam, k & 1, ws.sched, pr0, st) != hipSuccess) return TV_ERR_HIP;
    }
    SegPlan pc, pr;
    s = tune_launch<T>(
        W, H, ws.seg_bytes, [&](const SegPlan &p) { return tv2d_col_step<T>(ws, H, W, lam, 0, ws.sched, p, st); },
        st, &pc, col);
    if (s != TV_OK) return s;
    if (tv2d_col_step<T>(ws, H, W, lam, 0, ws.sched, pc, st) != hipSuccess) return TV_ERR_HIP;
    s = tune_launch<double, TagJ<double>>(
        H, W, ws.seg_bytes,
        [&](const SegPlan &p) { return tv2d_l1_row_step<T>(ws, f, ld, H, W, lam, 0, ws.sched, p, st); }, st, &pr,
        row);
    if (s != TV_OK) return s;
    seg_set_tuned(kPlan2dColL1, W, H, pc);
    seg_set_tuned(kPlan2dRowL1, H, W, pr);
    return hipStreamSynchronize(st) == hipSuccess ? TV_OK : TV_ERR_HIP;
}

// Entry points per solver and precision.  The build compiles this file in
// parts (1: ROF FP32, 2: ROF FP64, 3: TV-l1 FP32, 4: TV-l1 FP64 and the C
// ABI); each part defines its group and the ABI calls them through these
// declarations.
tv_status rof_solve_f32(const float *, int64_t, int64_t, int64_t, double, float *, const tv2d_options *,
                        tv2d_stats *, void *, hipStream_t);
tv_status rof_solve_f64(const double *, int64_t, int64_t, int64_t, double, double *, const tv2d_options *,
                        tv2d_stats *, void *, hipStream_t);
tv_status rof_autotune_f32(const float *, int64_t, int64_t, int64_t, double, double, void *, hipStream_t,
                           tv_tuning_result *, tv_tuning_result *);
tv_status rof_autotune_f64(const double *, int64_t, int64_t, int64_t, double, double, void *, hipStream_t,
                           tv_tuning_result *, tv_tuning_result *);
tv_status l1_solve_f32(const float *, int64_t, int64_t, int64_t, double, float *, const tv2d_options *,
                       tv2d_stats *, void *, hipStream_t);
tv_status l1_solve_f64(const double *, int64_t, int64_t, int64_t, double, double *, const tv2d_options *,
                       tv2d_stats *, void *, hipStream_t);
tv_status l1_autotune_f32(const float *, int64_t, int64_t, int64_t, double, double, void *, hipStream_t,
                          tv_tuning_result *, tv_tuning_result *);
tv_status l1_autotune_f64(const double *, int64_t, int64_t, int64_t, double, double, void *, hipStream_t,
                          tv_tuning_result *, tv_tuning_result *);

#if TVC_IN_PART(1)
tv_status rof_solve_f32(const float *f, int64_t H, int64_t W, int64_t ld, double lam, float *x,
                        const tv2d_options *o, tv2d_stats *st, void *ws, hipStream_t s) {
    return tv2d_solve_t<float>(f, H, W, ld, lam, x, o, st, ws, s);
}
tv_status rof_autotune_f32(const float *f, int64_t H, int64_t W, int64_t ld, double lam, double tau0, void *ws,
                           hipStream_t s, tv_tuning_result *col, tv_tuning_result *row) {
    return tv2d_autotune_t<float>(f, H, W, ld, lam, tau0, ws, s, col, row);
}
#endif
#if TVC_IN_PART(2)
tv_status rof_solve_f64(const double *f, int64_t H, int64_t W, int64_t ld, double lam, double *x,
                        const tv2d_options *o, tv2d_stats *st, void *ws, hipStream_t s) {
    return tv2d_solve_t<double>(f, H, W, ld, lam, x, o, st, ws, s);
}
tv_status rof_autotune_f64(const double *f, int64_t H, int64_t W, int64_t ld, double lam, double tau0, void *ws,
                           hipStream_t s, tv_tuning_result *col, tv_tuning_result *row) {
    return tv2d_autotune_t<double>(f, H, W, ld, lam, tau0, ws, s, col, row);
}
#endif
#if TVC_IN_PART(3)
tv_status l1_solve_f32(const float *f, int64_t H, int64_t W, int64_t ld, double lam, float *x,
                       const tv2d_options *o, tv2d_stats *st, void *ws, hipStream_t s) {
    return tv2d_l1_solve_t<float>(f, H, W, ld, lam, x, o, st, ws, s);
}
tv_status l1_autotune_f32(const float *f, int64_t H, int64_t W, int64_t ld, double lam, double tau0, void *ws,
                          hipStream_t s, tv_tuning_result *col, tv_tuning_result *row) {
    return tv2d_l1_autotune_t<float>(f, H, W, ld, lam, tau0, ws, s, col, row);
}
#endif
#if TVC_IN_PART(4)
tv_status l1_solve_f64(const double *f, int64_t H, int64_t W, int64_t ld, double lam, double *x,
                       const tv2d_options *o, tv2d_stats *st, void *ws, hipStream_t s) {
    return tv2d_l1_solve_t<double>(f, H, W, ld, lam, x, o, st, ws, s);
}
tv_status l1_autotune_f64(const double *f, int64_t H, int64_t W, int64_t ld, double lam, double tau0, void *ws,
                          hipStream_t s, tv_tuning_result *col, tv_tuning_result *row) {
    return tv2d_l1_autotune_t<double>(f, H, W, ld, lam, tau0, ws, s, col, row);
}
#endif

}  // namespace tvc

#if TVC_IN_PART(4)
using namespace tvc;

extern "C" {

size_t tv2d_workspace(int64_t H, int64_t W, tv_dtype dtype) {
    if (H < 1 || W < 1 || (dtype != TV_F32 && dtype != TV_F64)) return 0;
    return dtype == TV_F32 ? tv2d_layout<float>(nullptr, H, W, nullptr) : tv2d_layout<double>(nullptr, H, W, nullptr);
}

tv_status tv2d_solve(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda, void *x,
                     const tv2d_options *options, tv2d_stats *stats, void *workspace, size_t workspace_bytes,
                     hipStream_t stream) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (!f || !x || !options || H < 1 || W < 1 || ld < W) return TV_ERR_INVALID_ARG;
    if (!(isfinite(lambda) && lambda >= 0.0)) return TV_ERR_INVALID_ARG;
    if (options->max_iter < 0 || !(options->tau0 > 0.0) || !isfinite(options->tau0)) return TV_ERR_INVALID_ARG;
    if (options->lookahead < 0 || options->lookahead > kMaxLookahead) return TV_ERR_INVALID_ARG;
    const int64_t lim = (dtype == TV_F32) ? (int64_t(1) << 24) : (int64_t(1) << 31) - 8;
    if (H >= lim || W >= lim) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < tv2d_workspace(H, W, dtype)) return TV_ERR_WORKSPACE;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return TV_ERR_NO_DEVICE;
    if (dtype == TV_F32)
        return rof_solve_f32((const float *)f, H, W, ld, lambda, (float *)x, options, stats, workspace, stream);
    return rof_solve_f64((const double *)f, H, W, ld, lambda, (double *)x, options, stats, workspace, stream);
}

size_t tv2d_l1_workspace(int64_t H, int64_t W, tv_dtype dtype) {
    if (H < 1 || W < 1 || (dtype != TV_F32 && dtype != TV_F64)) return 0;
    return dtype == TV_F32 ? tv2d_layout<float>(nullptr, H, W, nullptr, true)
                           : tv2d_layout<double>(nullptr, H, W, nullptr, true);
}

static tv_status l1_args(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda, double tau0,
                         void *workspace, size_t workspace_bytes) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (!f || H < 1 || W < 1 || ld < W) return TV_ERR_INVALID_ARG;
    if (!(isfinite(lambda) && lambda >= 0.0) || !(tau0 > 0.0) || !isfinite(tau0)) return TV_ERR_INVALID_ARG;
    const int64_t lim = (dtype == TV_F32) ? (int64_t(1) << 24) : (int64_t(1) << 31) - 8;
    if (H >= lim || W >= lim) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < tv2d_l1_workspace(H, W, dtype)) return TV_ERR_WORKSPACE;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return TV_ERR_NO_DEVICE;
    return TV_OK;
}

tv_status tv2d_l1_solve(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda, void *x,
                        const tv2d_options *options, tv2d_stats *stats, void *workspace, size_t workspace_bytes,
                        hipStream_t stream) {
    if (!x || !options) return TV_ERR_INVALID_ARG;
    if (options->max_iter < 0 || options->resume || options->gap_tol > 0.0) return TV_ERR_INVALID_ARG;
    const tv_status s = l1_args(dtype, f, H, W, ld, lambda, options->tau0, workspace, workspace_bytes);
    if (s != TV_OK) return s;
    if (dtype == TV_F32)
        return l1_solve_f32((const float *)f, H, W, ld, lambda, (float *)x, options, stats, workspace, stream);
    return l1_solve_f64((const double *)f, H, W, ld, lambda, (double *)x, options, stats, workspace, stream);
}

tv_status tv2d_l1_autotune(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda,
                           double tau0, void *workspace, size_t workspace_bytes, hipStream_t stream,
                           tv_tuning_result *col, tv_tuning_result *row) {
    const tv_status s = l1_args(dtype, f, H, W, ld, lambda, tau0, workspace, workspace_bytes);
    if (s != TV_OK) return s;
    if (dtype == TV_F32)
        return l1_autotune_f32((const float *)f, H, W, ld, lambda, tau0, workspace, stream, col, row);
    return l1_autotune_f64((const double *)f, H, W, ld, lambda, tau0, workspace, stream, col, row);
}

tv_status tv2d_autotune(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda, double tau0,
                        void *workspace, size_t workspace_bytes, hipStream_t stream, tv_tuning_result *col,
                        tv_tuning_result *row) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (!f || H < 1 || W < 1 || ld < W) return TV_ERR_INVALID_ARG;
    if (!(isfinite(lambda) && lambda >= 0.0) || !(tau0 > 0.0) || !isfinite(tau0)) return TV_ERR_INVALID_ARG;
    const int64_t lim = (dtype == TV_F32) ? (int64_t(1) << 24) : (int64_t(1) << 31) - 8;
    if (H >= lim || W >= lim) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < tv2d_workspace(H, W, dtype)) return TV_ERR_WORKSPACE;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return TV_ERR_NO_DEVICE;
    if (dtype == TV_F32)
        return rof_autotune_f32((const float *)f, H, W, ld, lambda, tau0, workspace, stream, col, row);
    return rof_autotune_f64((const double *)f, H, W, ld, lambda, tau0, workspace, stream, col, row);
}

}  // extern "C"
#endif
