// tv2d_batched.hip -- many independent 2D ROF problems of different sizes in
// one solve (the Sec. 5.1 row/column decomposition of every image at once).
//
// Every image's column chains run in one segmented chain launch and every
// image's row chains in another.  Chains are listed longest first, so the 64
// lanes of a wave hold chains of (nearly) equal length; the chains of one image
// stay adjacent (its columns stay coalesced).  All images share the iteration
// counter and step schedule (tau_k, sigma_k = 1/tau_k, theta_k); each has its
// own lambda and its own FP64 duality gap, and an image whose gap reaches the
// tolerance is frozen on the device: its chains and gap terms are skipped from
// then on and its iterate stays in the buffer it was in.  Once every image is
// frozen the solve stops on the device (every later kernel returns at once),
// so the host enqueues all iterations without reading anything back.
#include <math.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/tvchain.h"
#include "kernels.h"
#include "seg_kernels.h"
#include "tv2d_common.h"

namespace tvc {

struct BChain {
    int64_t base;  // pixel of node 0 (packed image storage)
    int32_t n;     // nodes
    int32_t es;    // element stride (1 for rows, W_j for columns)
    int32_t img;
    int32_t pad;
};

template <typename T>
struct BColProb {
    using Tag = T;  // a_i = 1: integer tags in the working precision
    static constexpr bool kGen = false;
    struct Params {
        const BChain *desc;
        const T *y_old;
        const T *xbar;
        T *y_new;
        const IterSched *sc;
        const double *lam;
        const int *active;
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
        int64_t base, es;
        __device__ __forceinline__ Pre load(int64_t i) const { return load_off(base + i * es); }
        __device__ __forceinline__ int64_t off(int64_t i) const { return base + i * es; }
        __device__ __forceinline__ int64_t step() const { return es; }
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
        int64_t base, es;
        __device__ __forceinline__ SinkPre load(int64_t i) const {
            SinkPre p;
            p.y = y[base + i * es];
            p.xb = xb[base + i * es];
            return p;
        }
        __device__ __forceinline__ void store(int64_t i, T u, const SinkPre &p) const {
            yn[base + i * es] = col_dual<T>(p.y, sigma, p.xb, u);
        }
        static constexpr bool vec = false;
        __device__ __forceinline__ void load4(int64_t i, SinkPre *o) const {
            for (int k = 0; k < 4; ++k) o[k] = load(i + k);
        }
        __device__ __forceinline__ void store4(int64_t i, const T (&u)[4], const SinkPre (&p)[4]) const {
            for (int k = 0; k < 4; ++k) store(i + k, u[k], p[k]);
        }
    };
    static __device__ __forceinline__ ChainSpan span(const Params &p, int64_t c, int64_t) {
        const BChain d = p.desc[c];
        return ChainSpan{d.base, d.es, p.active[d.img] ? (int64_t)d.n : 0, d.img};
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) {
        return Src{p.y_old, p.xbar, (T)p.sc->sigma, (T)p.lam[sp.aux], sp.base, sp.es};
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{p.y_old, p.xbar, p.y_new, (T)p.sc->sigma, sp.base, sp.es};
    }
};

template <typename T>
struct BRowProb {
    using Tag = T;  // a_i = 1: integer tags in the working precision
    static constexpr bool kGen = false;
    struct Params {
        const BChain *desc;
        const T *f;
        const T *x_old;
        const T *y;
        T *x_new;
        T *xbar;
        const IterSched *sc;
        const double *lam;
        const int *active;
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
        int64_t base;
        bool vec;  // the row's three streams are element-aligned: load4 may be used
        __device__ __forceinline__ Src(const T *f_, const T *x_, const T *y_, T tau_, T inv1p_, T w_, int64_t base_)
            : f(f_), x(x_), y(y_), tau(tau_), inv1p(inv1p_), w(w_), base(base_),
              vec(elem_aligned(f_ + base_) && elem_aligned(x_ + base_) && elem_aligned(y_ + base_)) {}
        __device__ __forceinline__ Pre load(int64_t i) const {
            Pre p;
            p.f = f[base + i];
            p.x = x[base + i];
            p.y = y[base + i];
            return p;
        }
        __device__ __forceinline__ int64_t off(int64_t i) const { return i; }
        __device__ __forceinline__ int64_t step() const { return 1; }
        __device__ __forceinline__ Pre load_off(int64_t o) const { return load(o); }
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const {
            T a[4], b[4], c[4];
            vload4(f + base + i, a);
            vload4(x + base + i, b);
            vload4(y + base + i, c);
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
        int64_t base;
        bool vec;  // the row's streams are element-aligned: load4 / store4 may be used
        __device__ __forceinline__ Sink(const T *x_, T *xn_, T *xb_, T theta_, int64_t base_)
            : x(x_), xn(xn_), xb(xb_), theta(theta_), base(base_),
              vec(elem_aligned(x_ + base_) && elem_aligned(xn_ + base_) && elem_aligned(xb_ + base_)) {}
        __device__ __forceinline__ SinkPre load(int64_t i) const { return SinkPre{x[base + i]}; }
        __device__ __forceinline__ void load4(int64_t i, SinkPre *o) const {
            T v[4];
            vload4(x + base + i, v);
            for (int k = 0; k < 4; ++k) o[k].x = v[k];
        }
        __device__ __forceinline__ void store(int64_t i, T u, const SinkPre &p) const {
            xn[base + i] = u;
            xb[base + i] = row_xbar<T>(u, theta, p.x);
        }
        __device__ __forceinline__ void store4(int64_t i, const T (&u)[4], const SinkPre (&p)[4]) const {
            T b[4];
            for (int k = 0; k < 4; ++k) b[k] = row_xbar<T>(u[k], theta, p[k].x);
            vstore4(xn + base + i, u);
            vstore4(xb + base + i, b);
        }
    };
    static __device__ __forceinline__ ChainSpan span(const Params &p, int64_t c, int64_t) {
        const BChain d = p.desc[c];
        return ChainSpan{d.base, 1, p.active[d.img] ? (int64_t)d.n : 0, d.img};
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) {
        const IterSched sc = *p.sc;
        return Src{p.f, p.x_old, p.y, (T)sc.tau, (T)sc.inv1p, (T)(p.lam[sp.aux] * sc.tau * sc.inv1p), sp.base};
    }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) {
        return Sink{p.x_old, p.x_new, p.xbar, (T)p.sc->theta, sp.base};
    }
};

// Per-image geometry on the device.
struct BImg {
    int64_t off;       // first pixel
    int64_t H, W;
    int64_t row0;      // first row in the global row list
};

// p_v down every column of every active image (lane = column chain).
template <typename T>
__global__ __launch_bounds__(64) void k_bgap_pv(const BChain *__restrict__ cols, int64_t ncols,
                                                const T *__restrict__ y, T *__restrict__ pv,
                                                const double *__restrict__ lam, const int *__restrict__ active,
                                                const int *__restrict__ stop) {
    if (*stop) return;
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= ncols) return;
    const BChain d = cols[c];
    if (!active[d.img]) return;
    const double lm = lam[d.img];
    // same summation order as the single-image two-phase scan: the prefix of a
    // row is (sum of the earlier blocks' sums, each from zero) + the rows of its
    // own block in order
    double pre = 0.0;
    for (int64_t r0 = 0; r0 < d.n; r0 += kGapRows) {
        const int64_t r1 = (r0 + kGapRows < d.n) ? r0 + kGapRows : d.n;
        double cs = pre, bs = 0.0;
        for (int64_t r = r0; r < r1; ++r) {
            const int64_t k = d.base + r * d.es;
            const double v = (double)y[k];
            cs += v;
            bs += v;
            if (r + 1 < d.n) pv[k] = store_feasible<T>(clipd(-cs, lm));
        }
        pre += bs;
    }
}

// One wave per row of every active image; as k_gap_rows of the single-image
// solver, with the image's own geometry and lambda.
template <typename T>
__global__ __launch_bounds__(kGapBlock) void k_bgap_rows(const BImg *__restrict__ imgs, const int *__restrict__ rowimg,
                                                         int64_t nrows, const T *__restrict__ f,
                                                         const T *__restrict__ xn, const T *__restrict__ xo,
                                                         const T *__restrict__ y, const T *__restrict__ pv,
                                                         const double *__restrict__ lamv, const int *__restrict__ active,
                                                         const IterSched *__restrict__ sc, double *__restrict__ part,
                                                         const int *__restrict__ stop) {
    if (*stop) return;
    const T tau = (T)sc->tau, inv1p = (T)sc->inv1p;
    const double pscale = sc->pscale;
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * (kGapBlock / 64) + (threadIdx.x >> 6);
    if (t >= nrows) return;
    const int j = rowimg[t];
    if (!active[j]) return;
    const BImg im = imgs[j];
    const int64_t r = t - im.row0, H = im.H, W = im.W;
    const double lam = lamv[j];
    const T *fr = f + im.off, *xnr = xn + im.off, *xor_ = xo + im.off, *yr = y + im.off, *pvr = pv + im.off;
    double P = 0.0, D = 0.0, carry = 0.0, ph_last = 0.0;
    for (int64_t c0 = 0; c0 < W; c0 += 64) {
        const int64_t c = c0 + lane;
        const bool in = c < W;
        const int64_t k = r * W + c;
        T fv = 0, xv = 0, xo_v = 0, yv = 0, xr = 0, xd_ = 0, pvu = 0, pvd = 0;
        if (in) {
            fv = fr[k];
            xv = xnr[k];
            xo_v = xor_[k];
            yv = yr[k];
            if (c + 1 < W) xr = xnr[k + 1];
            if (r + 1 < H) {
                xd_ = xnr[k + W];
                pvd = pvr[k];
            }
            if (r > 0) pvu = pvr[k - W];
        }
        const T b = row_data<T>(fv, xo_v, yv, tau, inv1p);
        double res = (in && c + 1 < W) ? (double)xv - (double)b : 0.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double tt = __shfl_up(res, off, 64);
            if (lane >= off) res += tt;
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
        part[2 * t] = P;
        part[2 * t + 1] = D;
    }
}

// Per-image solver state on the device.
struct BState {
    int buf;        // buffer holding a frozen image's iterate
    int iters;      // iterations done at the image's last gap evaluation
    int status;     // a frozen image's status (TV_OK or TV_ERR_NONFINITE)
    double gap[3];  // P, D, gap_norm of the last evaluation
    uint64_t t1;    // device wall clock when the image froze
};

// One block per image: reduce the image's rows and record the gap.  An image
// whose gap is at tol > 0, or is not finite, is frozen (its iterate is in
// buffer `nxt`); the image that freezes last stops the solve.
static __global__ __launch_bounds__(kGapBlock) void k_bgap_final(const BImg *__restrict__ imgs, const double *__restrict__ part,
                                                          BState *__restrict__ bs, int *__restrict__ active,
                                                          SolveCtl *__restrict__ ctl, double tol, int nxt,
                                                          const IterSched *__restrict__ sc) {
    if (*(volatile const int *)&ctl->stop) return;
    const int j = blockIdx.x;
    if (!active[j]) return;  // uniform per block
    const int iter_after = (int)sc->iter_after;
    const BImg im = imgs[j];
    __shared__ double sP[kGapBlock], sD[kGapBlock];
    double P = 0.0, D = 0.0;
    for (int64_t r = threadIdx.x; r < im.H; r += kGapBlock) {
        P += part[2 * (im.row0 + r)];
        D += part[2 * (im.row0 + r) + 1];
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
        const double g = (sP[0] - sD[0]) / (double)(im.H * im.W);
        BState &b = bs[j];
        b.gap[0] = sP[0];
        b.gap[1] = sD[0];
        b.gap[2] = g;
        b.iters = iter_after;
        const bool bad = !isfinite(g);
        if (bad || (tol > 0.0 && g <= tol)) {
            b.status = bad ? TV_ERR_NONFINITE : TV_OK;
            b.buf = nxt;
            b.t1 = wall_clock64();
            active[j] = 0;
            // the image that freezes last stops the solve
            if (atomicSub(&ctl->n_active, 1) == 1) ctl_stop(ctl, TV_OK);
        }
    }
}

// Fresh per-image state: active, iterate in buffer 0, no gap yet.
static __global__ void k_binit(BState *__restrict__ bs, int *__restrict__ active, int nimg) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nimg) return;
    BState b;
    b.buf = 0;
    b.iters = 0;
    b.status = TV_OK;
    b.gap[0] = b.gap[1] = b.gap[2] = __builtin_nan("");
    b.t1 = 0;
    bs[j] = b;
    active[j] = 1;
}

// Stats of every image (one thread each).  An image still active after the
// last iteration has not reached tol > 0.
static __global__ void k_bstats(const BState *__restrict__ bs, const int *__restrict__ active,
                                const SolveCtl *__restrict__ ctl, int nimg, double tol, double clk_khz,
                                tv2d_stats *__restrict__ stats) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= nimg) return;
    const BState b = bs[j];
    const bool live = active[j] != 0;
    int st = TV_OK;
    if (!live) st = b.status;
    else if (tol > 0.0) st = TV_ERR_NOT_CONVERGED;
    double ms = 0.0;
    if (ctl->t0 != 0 && clk_khz > 0.0) {
        const uint64_t t1 = live ? (ctl->stop ? ctl->t1 : wall_clock64()) : b.t1;
        ms = (double)(t1 - ctl->t0) / clk_khz;
    }
    tv2d_stats o;
    o.iters = b.iters;
    o.status = st;
    o.gap_norm = b.gap[2];
    o.primal = b.gap[0];
    o.dual = b.gap[1];
    o.device_ms = ms;
    stats[j] = o;
}

// Copy each image's iterate (buffer buf[j], or `cur` if still active) out.
template <typename T>
__global__ __launch_bounds__(256) void k_bcopy_out(const BImg *__restrict__ imgs, int nimg, const int *__restrict__ active,
                                                   const BState *__restrict__ bs, int cur, const T *__restrict__ x0,
                                                   const T *__restrict__ x1, T *__restrict__ out, int64_t total) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    int lo = 0, hi = nimg - 1;  // image containing pixel i
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (imgs[mid].off <= i) lo = mid;
        else hi = mid - 1;
    }
    const int b = active[lo] ? cur : bs[lo].buf;
    out[i] = b ? x1[i] : x0[i];
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct BGeom {
    int nimg;
    int64_t total, nrows, ncols, maxH, maxW;
};

static bool batched_geom(int num_images, const int64_t *H, const int64_t *W, BGeom *g) {
    if (num_images < 1 || !H || !W) return false;
    g->nimg = num_images;
    g->total = g->nrows = g->ncols = g->maxH = g->maxW = 0;
    for (int j = 0; j < num_images; ++j) {
        if (H[j] < 1 || W[j] < 1) return false;
        g->total += H[j] * W[j];
        g->nrows += H[j];
        g->ncols += W[j];
        g->maxH = H[j] > g->maxH ? H[j] : g->maxH;
        g->maxW = W[j] > g->maxW ? W[j] : g->maxW;
    }
    return true;
}

template <typename T>
struct BWs {
    BImg *imgs;
    BChain *rows, *cols;
    int *rowimg, *active;  // active: 1 while an image iterates (read by the chain launches)
    BState *bs;
    SolveCtl *ctl;
    double *lam, *part;
    T *x[2], *y[2], *xbar, *pv;
    IterSched *sched;  // [kSchedCap] per-iteration scalars of the current chunk
    void *seg;
    size_t seg_bytes;
};

template <typename T>
static size_t batched_layout(void *base, const BGeom &g, BWs<T> *out) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    // room for any plan the autotuner may choose for the row and column launches
    const size_t sr = seg_bytes_max<T>(g.nrows, g.maxW, kPlanBatchRow);
    const size_t scol = seg_bytes_max<T>(g.ncols, g.maxH, kPlanBatchCol);
    const size_t N = (size_t)g.total;
    size_t off = 0;
    const size_t o_im = off;  off += al(sizeof(BImg) * g.nimg);
    const size_t o_rw = off;  off += al(sizeof(BChain) * (size_t)g.nrows);
    const size_t o_cl = off;  off += al(sizeof(BChain) * (size_t)g.ncols);
    const size_t o_ri = off;  off += al(sizeof(int) * (size_t)g.nrows);
    const size_t o_ac = off;  off += al(sizeof(int) * g.nimg);
    const size_t o_bs = off;  off += al(sizeof(BState) * g.nimg);
    const size_t o_ct = off;  off += al(sizeof(SolveCtl));
    const size_t o_lm = off;  off += al(sizeof(double) * g.nimg);
    const size_t o_pt = off;  off += al(sizeof(double) * 2 * (size_t)g.nrows);
    const size_t o_x0 = off;  off += al(sizeof(T) * N);
    const size_t o_x1 = off;  off += al(sizeof(T) * N);
    const size_t o_y0 = off;  off += al(sizeof(T) * N);
    const size_t o_y1 = off;  off += al(sizeof(T) * N);
    const size_t o_xb = off;  off += al(sizeof(T) * N);
    const size_t o_pv = off;  off += al(sizeof(T) * N);
    const size_t o_sc = off;  off += al(sizeof(IterSched) * kSchedCap);
    const size_t o_sg = off;  off += al(sr > scol ? sr : scol);
    if (base && out) {
        char *p = (char *)base;
        out->imgs = (BImg *)(p + o_im);
        out->rows = (BChain *)(p + o_rw);
        out->cols = (BChain *)(p + o_cl);
        out->rowimg = (int *)(p + o_ri);
        out->active = (int *)(p + o_ac);
        out->bs = (BState *)(p + o_bs);
        out->ctl = (SolveCtl *)(p + o_ct);
        out->lam = (double *)(p + o_lm);
        out->part = (double *)(p + o_pt);
        out->x[0] = (T *)(p + o_x0);
        out->x[1] = (T *)(p + o_x1);
        out->y[0] = (T *)(p + o_y0);
        out->y[1] = (T *)(p + o_y1);
        out->xbar = (T *)(p + o_xb);
        out->pv = (T *)(p + o_pv);
        out->sched = (IterSched *)(p + o_sc);
        out->seg = (void *)(p + o_sg);
        out->seg_bytes = sr > scol ? sr : scol;
    }
    return off;
}

// Uploads the geometry and chain lists (longest chains first; stable, so an
// image's chains stay adjacent and in order), sets x^0 = xbar^0 = f, y^0 = 0,
// and starts the device control at tau0 with every image active.  Waits once,
// for the uploads from host memory.
template <typename T>
static tv_status batched_setup(const BGeom &g, const int64_t *H, const int64_t *W, const int64_t *pix,
                               const double *lam, const T *f, double tau0, const BWs<T> &ws, hipStream_t st,
                               uint32_t *host_stop = nullptr, uint32_t seq = 0) {
    std::vector<BImg> imgs(g.nimg);
    std::vector<int> rowimg((size_t)g.nrows);
    std::vector<BChain> rows, cols;
    rows.reserve((size_t)g.nrows);
    cols.reserve((size_t)g.ncols);
    int64_t r0 = 0;
    for (int j = 0; j < g.nimg; ++j) {
        imgs[j] = BImg{pix[j], H[j], W[j], r0};
        for (int64_t r = 0; r < H[j]; ++r) {
            rowimg[(size_t)(r0 + r)] = j;
            rows.push_back(BChain{pix[j] + r * W[j], (int32_t)W[j], 1, j, 0});
        }
        for (int64_t c = 0; c < W[j]; ++c) cols.push_back(BChain{pix[j] + c, (int32_t)H[j], (int32_t)W[j], j, 0});
        r0 += H[j];
    }
    auto longer = [](const BChain &a, const BChain &b) { return a.n > b.n; };
    std::stable_sort(rows.begin(), rows.end(), longer);
    std::stable_sort(cols.begin(), cols.end(), longer);
    hipError_t e = hipSuccess;
    e = e ? e : hipMemcpyAsync(ws.imgs, imgs.data(), sizeof(BImg) * g.nimg, hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(ws.rows, rows.data(), sizeof(BChain) * rows.size(), hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(ws.cols, cols.data(), sizeof(BChain) * cols.size(), hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(ws.rowimg, rowimg.data(), sizeof(int) * rowimg.size(), hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(ws.lam, lam, sizeof(double) * g.nimg, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return TV_ERR_HIP;
    hipLaunchKernelGGL(k_binit, dim3((unsigned)((g.nimg + 255) / 256)), dim3(256), 0, st, ws.bs, ws.active, g.nimg);
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, ws.ctl, tau0, g.nimg, host_stop, seq);
    const unsigned nb = (unsigned)((g.total + 255) / 256);
    hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, g.total, ws.x[0], g.total, (int64_t)1, g.total);
    hipLaunchKernelGGL((k_copy2d<T>), dim3(nb), dim3(256), 0, st, f, g.total, ws.xbar, g.total, (int64_t)1, g.total);
    hipLaunchKernelGGL((k_fill<T>), dim3(nb), dim3(256), 0, st, ws.y[0], g.total, (T)0);
    // the host vectors above are read by the copies: wait before they go away
    return hipStreamSynchronize(st) == hipSuccess ? TV_OK : TV_ERR_HIP;
}

template <typename T>
static hipError_t batched_col_step(const BGeom &g, const BWs<T> &ws, int cur, const IterSched *sc, const SegPlan &pc,
                                   hipStream_t st, const int *stop = nullptr) {
    typename BColProb<T>::Params cp{ws.cols, ws.y[cur], ws.xbar, ws.y[cur ^ 1], sc, ws.lam, ws.active};
    return seg_run<T, BColProb<T>, kTile>(ws.seg, g.ncols, g.maxH, pc, cp, st, stop);
}

template <typename T>
static hipError_t batched_row_step(const BGeom &g, const BWs<T> &ws, const T *f, int cur, const IterSched *sc,
                                   const SegPlan &pr, hipStream_t st, const int *stop = nullptr) {
    typename BRowProb<T>::Params rp{ws.rows, f, ws.x[cur], ws.y[cur ^ 1], ws.x[cur ^ 1], ws.xbar, sc, ws.lam,
                                    ws.active};
    return seg_run<T, BRowProb<T>, kTile>(ws.seg, g.nrows, g.maxW, pr, rp, st, stop);
}

// Issues `count` iterations starting at parity cur0, iteration j reading
// ws.sched[j] (generated on the device first); with `gap`, the gap evaluation
// and the per-image stopping test follow the last one.  Nothing here reads host
// memory, so the same sequence is launched directly or captured into a HIP
// graph and replayed.  Every kernel returns at once once the solve has stopped.
template <typename T>
static hipError_t batched_iters(const BGeom &g, const BWs<T> &ws, const T *f, int cur0, int count, bool gap,
                                double gap_tol, const SegPlan &pc, const SegPlan &pr, hipStream_t st) {
    const int *stop = &ws.ctl->stop;
    hipLaunchKernelGGL(k_ctl_sched, dim3(1), dim3(64), 0, st, ws.ctl, ws.sched, count);
    int cur = cur0;
    for (int j = 0; j < count; ++j) {
        const int nxt = cur ^ 1;
        const IterSched *sc = ws.sched + j;
        hipError_t e = batched_col_step<T>(g, ws, cur, sc, pc, st, stop);
        if (e == hipSuccess) e = batched_row_step<T>(g, ws, f, cur, sc, pr, st, stop);
        if (e != hipSuccess) return e;
        if (gap && j == count - 1) {
            const unsigned cb = (unsigned)((g.ncols + 63) / 64);
            hipLaunchKernelGGL((k_bgap_pv<T>), dim3(cb), dim3(64), 0, st, ws.cols, g.ncols, ws.y[nxt], ws.pv, ws.lam,
                               ws.active, stop);
            const unsigned rb = (unsigned)((g.nrows + kGapBlock / 64 - 1) / (kGapBlock / 64));
            hipLaunchKernelGGL((k_bgap_rows<T>), dim3(rb), dim3(kGapBlock), 0, st, ws.imgs, ws.rowimg, g.nrows, f,
                               ws.x[nxt], ws.x[cur], ws.y[nxt], ws.pv, ws.lam, ws.active, sc, ws.part, stop);
            hipLaunchKernelGGL(k_bgap_final, dim3(g.nimg), dim3(kGapBlock), 0, st, ws.imgs, ws.part, ws.bs,
                               ws.active, ws.ctl, gap_tol, nxt, sc);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur = nxt;
    }
    return hipSuccess;
}

// The iterations are enqueued on st without waiting on the device (the
// stopping test runs on the device, see batched_iters), all of them, or with a
// lookahead at most that many gap evaluations ahead of the device (see
// Lookahead); the setup waits once for its uploads, and a solve that replays
// captured graphs waits for them before returning.
template <typename T>
static tv_status batched_solve_t(const BGeom &g, const int64_t *H, const int64_t *W, const int64_t *pix,
                                 const double *lam, const T *f, T *x, const tv2d_options *opt, tv2d_stats *stats,
                                 void *workspace, hipStream_t st) {
    BWs<T> ws;
    batched_layout<T>(workspace, g, &ws);
    Lookahead la;
    const tv_status ls = la.begin(opt->lookahead, st);
    if (ls != TV_OK) return ls;
    const tv_status s0 = batched_setup<T>(g, H, W, pix, lam, f, opt->tau0, ws, st, la.dev_word(), la.seq);
    if (s0 != TV_OK) return s0;
    const unsigned nb = (unsigned)((g.total + 255) / 256);
    const int every = opt->gap_every > 0 ? opt->gap_every : 1;
    const SegPlan pr = seg_plan(g.nrows, g.maxW, kPlanBatchRow), pc = seg_plan(g.ncols, g.maxH, kPlanBatchCol);
    if (seg_ws_bytes_plan<T>(g.nrows, g.maxW, pr) > ws.seg_bytes ||
        seg_ws_bytes_plan<T>(g.ncols, g.maxH, pc) > ws.seg_bytes)
        return TV_ERR_WORKSPACE;
    ChunkGraphs graphs;
    int cur = 0;
    for (int done = 0; done < opt->max_iter;) {
        hipError_t le;
        if (la.stopped(&le)) break;  // every image frozen: the copy-out reads each image's own buffer
        if (le != hipSuccess) return TV_ERR_HIP;
        const int chunk = (opt->max_iter - done < every) ? opt->max_iter - done : every;
        // pieces of at most kSchedCap iterations; the gap follows the chunk's last
        for (int part = 0; part < chunk;) {
            const int piece = (chunk - part < kSchedCap) ? chunk - part : kSchedCap;
            const bool last = part + piece == chunk;
            const int c0 = cur;
            auto issue = [&](hipStream_t s2) {
                return batched_iters<T>(g, ws, f, c0, piece, last, opt->gap_tol, pc, pr, s2);
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
    hipLaunchKernelGGL((k_bcopy_out<T>), dim3(nb), dim3(256), 0, st, ws.imgs, g.nimg, ws.active, ws.bs, cur, ws.x[0],
                       ws.x[1], x, g.total);
    if (stats)
        hipLaunchKernelGGL(k_bstats, dim3((unsigned)((g.nimg + 255) / 256)), dim3(256), 0, st, ws.bs, ws.active,
                           ws.ctl, g.nimg, opt->gap_tol, wall_clock_khz(), stats);
    if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
    // captured graphs live for this call only: wait for their replays
    if (graphs.exec[0] || graphs.exec[1]) return hipStreamSynchronize(st) == hipSuccess ? TV_OK : TV_ERR_HIP;
    return TV_OK;
}

// Autotune of the batched column and row launches on the first iteration's data.
template <typename T>
static tv_status batched_autotune_t(const BGeom &g, const int64_t *H, const int64_t *W, const int64_t *pix,
                                    const double *lam, const T *f, double tau0, void *workspace, hipStream_t st,
                                    tv_tuning_result *col, tv_tuning_result *row) {
    BWs<T> ws;
    batched_layout<T>(workspace, g, &ws);
    tv_status s = batched_setup<T>(g, H, W, pix, lam, f, tau0, ws, st);
    if (s != TV_OK) return s;
    // a few iterations first, so the plans are timed on deques as deep as the
    // solve's later iterations build (no gap evaluation: nothing stops)
    if (batched_iters<T>(g, ws, f, 0, kTuneWarm, false, 0.0, seg_plan(g.ncols, g.maxH, kPlanBatchCol),
                         seg_plan(g.nrows, g.maxW, kPlanBatchRow), st) != hipSuccess)
        return TV_ERR_HIP;
    // the timed steps read iteration kTuneWarm's scalars from the first slot
    hipLaunchKernelGGL(k_ctl_sched, dim3(1), dim3(64), 0, st, ws.ctl, ws.sched, 1);
    SegPlan pc, pr;
    s = tune_launch<T>(
        g.ncols, g.maxH, ws.seg_bytes,
        [&](const SegPlan &p) { return batched_col_step<T>(g, ws, 0, ws.sched, p, st); }, st, &pc, col);
    if (s != TV_OK) return s;
    if (batched_col_step<T>(g, ws, 0, ws.sched, pc, st) != hipSuccess) return TV_ERR_HIP;
    s = tune_launch<T>(
        g.nrows, g.maxW, ws.seg_bytes,
        [&](const SegPlan &p) { return batched_row_step<T>(g, ws, f, 0, ws.sched, p, st); }, st, &pr, row);
    if (s != TV_OK) return s;
    seg_set_tuned(kPlanBatchCol, g.ncols, g.maxH, pc);
    seg_set_tuned(kPlanBatchRow, g.nrows, g.maxW, pr);
    return hipStreamSynchronize(st) == hipSuccess ? TV_OK : TV_ERR_HIP;
}

// Entry points per precision.  The build compiles this file in two parts (1:
// FP32, 2: FP64 and the C ABI), each defining its group; the ABI calls them
// through these declarations.
tv_status batched_solve_f32(const BGeom &, const int64_t *, const int64_t *, const int64_t *, const double *,
                            const float *, float *, const tv2d_options *, tv2d_stats *, void *, hipStream_t);
tv_status batched_solve_f64(const BGeom &, const int64_t *, const int64_t *, const int64_t *, const double *,
                            const double *, double *, const tv2d_options *, tv2d_stats *, void *, hipStream_t);
tv_status batched_autotune_f32(const BGeom &, const int64_t *, const int64_t *, const int64_t *, const double *,
                               const float *, double, void *, hipStream_t, tv_tuning_result *, tv_tuning_result *);
tv_status batched_autotune_f64(const BGeom &, const int64_t *, const int64_t *, const int64_t *, const double *,
                               const double *, double, void *, hipStream_t, tv_tuning_result *, tv_tuning_result *);
#if TVC_IN_PART(1)
tv_status batched_solve_f32(const BGeom &g, const int64_t *H, const int64_t *W, const int64_t *pix, const double *lam,
                            const float *f, float *x, const tv2d_options *o, tv2d_stats *st, void *ws, hipStream_t s) {
    return batched_solve_t<float>(g, H, W, pix, lam, f, x, o, st, ws, s);
}
tv_status batched_autotune_f32(const BGeom &g, const int64_t *H, const int64_t *W, const int64_t *pix,
                               const double *lam, const float *f, double tau0, void *ws, hipStream_t s,
                               tv_tuning_result *col, tv_tuning_result *row) {
    return batched_autotune_t<float>(g, H, W, pix, lam, f, tau0, ws, s, col, row);
}
#endif
#if TVC_IN_PART(2)
tv_status batched_solve_f64(const BGeom &g, const int64_t *H, const int64_t *W, const int64_t *pix, const double *lam,
                            const double *f, double *x, const tv2d_options *o, tv2d_stats *st, void *ws,
                            hipStream_t s) {
    return batched_solve_t<double>(g, H, W, pix, lam, f, x, o, st, ws, s);
}
tv_status batched_autotune_f64(const BGeom &g, const int64_t *H, const int64_t *W, const int64_t *pix,
                               const double *lam, const double *f, double tau0, void *ws, hipStream_t s,
                               tv_tuning_result *col, tv_tuning_result *row) {
    return batched_autotune_t<double>(g, H, W, pix, lam, f, tau0, ws, s, col, row);
}
#endif

}  // namespace tvc

#if TVC_IN_PART(2)
using namespace tvc;

extern "C" {

size_t tv2d_batched_workspace(int num_images, const int64_t *H, const int64_t *W, tv_dtype dtype) {
    BGeom g;
    if ((dtype != TV_F32 && dtype != TV_F64) || !batched_geom(num_images, H, W, &g)) return 0;
    return dtype == TV_F32 ? batched_layout<float>(nullptr, g, nullptr) : batched_layout<double>(nullptr, g, nullptr);
}

// Host-side checks shared by the batched solve and its autotuner.
static tv_status batched_args(tv_dtype dtype, int num_images, const int64_t *H, const int64_t *W,
                              const int64_t *pixel_offsets, const double *lambda, const void *f, double tau0,
                              void *workspace, size_t workspace_bytes, BGeom *g) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (!batched_geom(num_images, H, W, g) || !pixel_offsets || !lambda || !f) return TV_ERR_INVALID_ARG;
    if (!(tau0 > 0.0) || !isfinite(tau0)) return TV_ERR_INVALID_ARG;
    const int64_t lim = (dtype == TV_F32) ? (int64_t(1) << 24) : (int64_t(1) << 31) - 8;
    if (g->maxH >= lim || g->maxW >= lim || g->nrows >= (int64_t(1) << 31) || g->ncols >= (int64_t(1) << 31))
        return TV_ERR_INVALID_ARG;
    // images must be packed back to back in order
    int64_t expect = 0;
    for (int j = 0; j < num_images; ++j) {
        if (pixel_offsets[j] != expect) return TV_ERR_INVALID_ARG;
        if (!(isfinite(lambda[j]) && lambda[j] >= 0.0)) return TV_ERR_INVALID_ARG;
        expect += H[j] * W[j];
    }
    if (!workspace || workspace_bytes < tv2d_batched_workspace(num_images, H, W, dtype)) return TV_ERR_WORKSPACE;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return TV_ERR_NO_DEVICE;
    return TV_OK;
}

tv_status tv2d_batched_autotune(tv_dtype dtype, int num_images, const int64_t *H, const int64_t *W,
                                const int64_t *pixel_offsets, const double *lambda, const void *f, double tau0,
                                void *workspace, size_t workspace_bytes, hipStream_t stream, tv_tuning_result *col,
                                tv_tuning_result *row) {
    BGeom g;
    tv_status s = batched_args(dtype, num_images, H, W, pixel_offsets, lambda, f, tau0, workspace, workspace_bytes, &g);
    if (s != TV_OK) return s;
    if (dtype == TV_F32)
        return batched_autotune_f32(g, H, W, pixel_offsets, lambda, (const float *)f, tau0, workspace, stream, col,
                                    row);
    return batched_autotune_f64(g, H, W, pixel_offsets, lambda, (const double *)f, tau0, workspace, stream, col,
                                row);
}

tv_status tv2d_solve_batched(tv_dtype dtype, int num_images, const int64_t *H, const int64_t *W,
                             const int64_t *pixel_offsets, const double *lambda, const void *f, void *x,
                             const tv2d_options *options, tv2d_stats *stats, void *workspace, size_t workspace_bytes,
                             hipStream_t stream) {
    BGeom g;
    if (!options || !x) return TV_ERR_INVALID_ARG;
    if (options->max_iter < 0 || options->resume) return TV_ERR_INVALID_ARG;
    if (options->lookahead < 0 || options->lookahead > kMaxLookahead) return TV_ERR_INVALID_ARG;
    tv_status s = batched_args(dtype, num_images, H, W, pixel_offsets, lambda, f, options->tau0, workspace,
                               workspace_bytes, &g);
    if (s != TV_OK) return s;
    if (dtype == TV_F32)
        return batched_solve_f32(g, H, W, pixel_offsets, lambda, (const float *)f, (float *)x, options, stats,
                                 workspace, stream);
    return batched_solve_f64(g, H, W, pixel_offsets, lambda, (const double *)f, (double *)x, options, stats,
                             workspace, stream);
}

}  // extern "C"
#endif
