// nc_chain.hip -- Sec. 3 (non-convex case) on a batch of chains:
//
//     x = argmin_x  sum_i f_i(x_i) + sum_e min(w_e |x_{e+1} - x_e|, C_e),
//
// f_i continuous piecewise-linear (breakpoints lambda_{i,1..t}, slopes
// s_{i,0..t}, bounded below), 0 < C_e <= +inf (+inf: plain TV).  One lane per
// chain (or, for messages of at most 256 breakpoints, a wave per chain with
// each pass spread over the lanes) runs the message passing of Sec. 3 exactly:
//   hat M_i = f_i + M_{i-1}                    Lemma 1 (breakpoint lists merged)
//   M_i = ((hat M_i (x) f^1) (x) f^2) (x) f^3  Lemma 2 via Prop. 2:
//     f^1 (w z on z >= 0): Algorithm 1, intervals Pi^1 mapping to their left end;
//     f^2 (w |z| on z <= 0): Algorithm 1 on the reversed function (Sec. 3's
//       reversal), scanned from the right, intervals Pi^2 mapping to their right end;
//     f^3 (C off zero): min(h, min h + C), Pi^3 = {h >= min h + C} mapping to the
//       first argmin breakpoint,
// then backward x_i = pi^1(pi^2(pi^3(x_{i+1}))) from an argmin of the last hat M.
// Messages are sequences (s_0, lambda_1, s_1, ..., lambda_t, s_t) in FP64, held
// in LDS (as many lanes per workgroup as fit in 160 KiB) or, for large
// msg_cap, in the chain's slice of the workspace; the interval lists are in
// the workspace.  A message
// longer than msg_cap, or more than map_cap intervals on a chain, stops that
// chain and the call returns TV_ERR_WORKSPACE; an invalid unary (no
// breakpoint, unsorted, unbounded below) returns TV_ERR_INVALID_ARG.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tvchain.h"

namespace tvc {
namespace {

constexpr int kNcFlagCapacity = 1;
constexpr int kNcFlagInvalid = 2;

// A message buffer: breakpoints l[0..t), slopes s[0..t] (s[k] left of l[k]).
struct NcBuf {
    double *l, *s;
    int64_t t, cap;
    __host__ __device__ __forceinline__ bool push(double lam, double right) {
        if (t >= cap) return false;
        l[t] = lam;
        s[t + 1] = right;
        ++t;
        return true;
    }
};

// Read access to a buffer as stored, or as its reversal phi^rev(z) = phi(-z).
struct NcFwd {
    const NcBuf *b;
    __host__ __device__ __forceinline__ int64_t t() const { return b->t; }
    __host__ __device__ __forceinline__ double l(int64_t k) const { return b->l[k]; }
    __host__ __device__ __forceinline__ double s(int64_t k) const { return b->s[k]; }
};
struct NcRev {
    const NcBuf *b;
    __host__ __device__ __forceinline__ int64_t t() const { return b->t; }
    __host__ __device__ __forceinline__ double l(int64_t k) const { return -b->l[b->t - 1 - k]; }
    __host__ __device__ __forceinline__ double s(int64_t k) const { return -b->s[b->t - k]; }
};

// The interval list of one chain (tree): interval k is [p[3k], p[3k+1]] and
// maps to p[3k+2], the three side by side so that a lane's appends and the
// backward scan each walk one stream.
struct NcMaps {
    double *p;
    int64_t n, cap;
    __host__ __device__ __forceinline__ void put(int64_t k, double lo, double hi, double target) const {
        p[3 * k] = lo;
        p[3 * k + 1] = hi;
        p[3 * k + 2] = target;
    }
    __host__ __device__ __forceinline__ bool add(double lo, double hi, double target) {
        if (n >= cap) return false;
        put(n, lo, hi, target);
        ++n;
        return true;
    }
};

// Lemma 1: out = unary + msg (equal positions merged into one breakpoint).
__host__ __device__ bool nc_sum(const double *ul, const double *us, int64_t tu, const NcBuf &m, NcBuf &out) {
    out.t = 0;
    out.s[0] = us[0] + m.s[0];
    int64_t i = 0, j = 0;
    while (i < tu || j < m.t) {
        double lam;
        if (j >= m.t || (i < tu && ul[i] < m.l[j])) {
            lam = ul[i++];
        } else if (i >= tu || m.l[j] < ul[i]) {
            lam = m.l[j++];
        } else {
            lam = ul[i];
            ++i;
            ++j;
        }
        if (!out.push(lam, us[i] + m.s[j])) return false;
    }
    return true;
}

// Algorithm 1 on h (forward or reversed view): out = h (x) f^1.  Each interval
// [lambda_p, lambda] found is reported through add(lo, hi) in h's coordinates.
template <class View, class Add>
__host__ __device__ bool nc_dt(const View &h, double w, NcBuf &out, Add add) {
    const int64_t t = h.t();
    out.t = 0;
    out.s[0] = h.s(0);
    int64_t p = 0;
    double vp = 0.0;  // h(l(p)), with h(l(0)) = 0
    while (p < t) {
        const double right = h.s(p + 1);
        if (!out.push(h.l(p), right < w ? right : w)) return false;
        if (right >= w) {
            // first breakpoint from p + 2 on where h lies below the line of slope
            // w through (l(p), vp); q = t stands for the unbounded right piece
            const double lp = h.l(p);
            int64_t q = p + 1;
            double vq = vp + h.s(p + 1) * (h.l(p + 1 < t ? p + 1 : p) - lp);  // h(l(p + 1))
            double vq1 = vq;                                                 // h(l(q - 1)) below
            bool found = false;
            for (q = p + 2; q < t; ++q) {
                vq1 = vq;
                vq = vq1 + h.s(q) * (h.l(q) - h.l(q - 1));
                if (vq < vp + w * (h.l(q) - lp)) {
                    found = true;
                    break;
                }
            }
            if (!found) {
                q = t;
                vq1 = vq;  // h(l(t - 1))
                if (p + 1 >= t) vq1 = vp;
                if (!(h.s(t) < w)) {  // h never falls below the line
                    if (!add(lp, HUGE_VAL)) return false;
                    return true;
                }
            }
            const double l0 = h.l(q - 1);
            double lam = l0 + (vp + w * (l0 - lp) - vq1) / (h.s(q) - w);
            if (lam < l0) lam = l0;
            if (q < t && lam > h.l(q)) lam = h.l(q);
            if (!out.push(lam, h.s(q))) return false;
            if (!add(lp, lam)) return false;
            p = q;
            vp = (q < t) ? vq : 0.0;
        } else {
            if (p + 1 < t) vp += h.s(p + 1) * (h.l(p + 1) - h.l(p));
            ++p;
        }
    }
    return true;
}

// min(h, min h + C) with Pi^3; h given through a view.
template <class View>
__host__ __device__ bool nc_trunc(const View &h, double C, NcBuf &out, NcMaps &mp) {
    const int64_t t = h.t();
    out.t = 0;
    if (t == 0) {
        out.s[0] = h.s(0);
        return true;
    }
    double v = 0.0, vmin = 0.0;
    int64_t pm = 0;
    for (int64_t k = 1; k < t; ++k) {
        v += h.s(k) * (h.l(k) - h.l(k - 1));
        if (v < vmin) {
            vmin = v;
            pm = k;
        }
    }
    const double cp = vmin + C, xm = h.l(pm);
    // Segments between consecutive kink candidates (breakpoints and crossings
    // of cp), each inside one piece of h; classified at their midpoints.
    // Emission lags one segment: a point is written once the slope right of it
    // is known.
    bool first = true, in_run = false;
    double prev = 0.0, run = 0.0, pend = 0.0;  // last point; run start; point awaiting its right slope
    bool has_pend = false;
    auto segment = [&](double lo, double hi, double slope, double vlo_at, double lo_ref) -> bool {
        // segment (lo, hi) of a piece with h(z) = vlo_at + slope (z - lo_ref)
        const double mid = (lo == -HUGE_VAL) ? hi - 1.0 : (hi == HUGE_VAL ? lo + 1.0 : 0.5 * (lo + hi));
        const bool above = vlo_at + slope * (mid - lo_ref) >= cp;
        const double sl = above ? 0.0 : slope;
        if (first) {
            out.s[0] = sl;
            first = false;
        } else if (has_pend) {
            if (sl != out.s[out.t] && !out.push(pend, sl)) return false;
            has_pend = false;
        }
        if (above && !in_run) {
            run = lo;
            in_run = true;
        } else if (!above && in_run) {
            if (!mp.add(run, lo, xm)) return false;
            in_run = false;
        }
        return true;
    };
    auto point = [&](double z) {
        pend = z;
        has_pend = true;
        prev = z;
    };
    v = 0.0;  // h(l(k - 1)) while walking piece k
    prev = -HUGE_VAL;
    for (int64_t k = 0; k <= t; ++k) {
        const double sk = h.s(k);
        // piece k: (l(k-1), l(k)) with h = vref + sk (z - lref)
        double lref, vref, hi;
        if (k == 0) {
            lref = h.l(0);
            vref = 0.0;
            hi = h.l(0);
        } else {
            lref = h.l(k - 1);
            vref = v;
            hi = (k < t) ? h.l(k) : HUGE_VAL;
        }
        const double vhi = (k < t) ? ((k == 0) ? 0.0 : v + sk * (h.l(k) - h.l(k - 1))) : 0.0;
        // a crossing of cp inside the piece
        bool cross = false;
        double zc = 0.0;
        if (k == 0) {
            cross = sk < 0.0 && 0.0 < cp;
            if (cross) zc = h.l(0) + cp / sk;
        } else if (k == t) {
            cross = sk > 0.0 && v < cp;
            if (cross) zc = h.l(t - 1) + (cp - v) / sk;
        } else {
            cross = (v < cp && vhi > cp) || (v > cp && vhi < cp);
            if (cross) zc = h.l(k - 1) + (cp - v) / sk;
        }
        if (cross) {
            if (!segment(prev, zc, sk, vref, lref)) return false;
            point(zc);
        }
        if (!segment(prev, hi, sk, vref, lref)) return false;
        if (k < t) {
            point(h.l(k));
            v = vhi;
        }
    }
    if (in_run && !mp.add(run, HUGE_VAL, xm)) return false;
    return true;
}

// pi(y) over intervals [lo, hi) of a list: the first interval containing y.
__host__ __device__ __forceinline__ double nc_apply(const NcMaps &mp, int64_t lo, int64_t hi, double y) {
    for (int64_t k = lo; k < hi; ++k)
        if (y >= mp.p[3 * k] && y <= mp.p[3 * k + 1]) return mp.p[3 * k + 2];
    return y;
}

struct NcArgs {
    int64_t num_chains, num_nodes;
    const int64_t *coff, *uoff;
    int64_t msg_cap, map_cap;
    double *bufs;     // per chain: 3 buffers of (msg_cap + msg_cap + 1) doubles
    double *maps;     // per chain: map_cap intervals of 3 doubles
    int64_t *eoff;    // per node: 3 offsets (Pi^1, Pi^2, Pi^3 of the edge leaving it)
    int *flag;
};

// One lane's chain c: the message passing and the backward pass with the
// three message buffers M, H, B given (each of msg_cap breakpoints); returns
// the flag bits to raise (0: x written).  Host-callable, so that its indexing
// can be run against exactly-sized buffers on a CPU.
template <typename T>
__host__ __device__ int nc_chain_lane(const NcArgs &A, const T *__restrict__ ulam, const T *__restrict__ uslope,
                                      const T *__restrict__ w, const T *__restrict__ C, T *__restrict__ x, int64_t c,
                                      NcBuf M, NcBuf H, NcBuf B) {
    const int64_t n0 = A.coff[c], n1 = A.coff[c + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) return kNcFlagInvalid;  // a range outside the nodes
    if (n1 == n0) return 0;
    double *mb = A.maps + c * 3 * A.map_cap;
    NcMaps mp{mb, 0, A.map_cap};
    M.t = 0;
    M.s[0] = 0.0;
    // unary slopes are read in FP64; a small staging copy of one unary
    int bad = 0;
    for (int64_t i = n0; i < n1; ++i) {
        const int64_t u0 = A.uoff[i], tu = A.uoff[i + 1] - u0;
        if (tu < 1 || tu > A.msg_cap) {
            bad = tu < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        // hat M = f_i + M into H (the unary is staged in B, which is free here)
        for (int64_t k = 0; k < tu; ++k) {
            B.l[k] = (double)ulam[u0 + k];
            if (k > 0 && !(B.l[k] >= B.l[k - 1])) bad = kNcFlagInvalid;
        }
        for (int64_t k = 0; k <= tu; ++k) B.s[k] = (double)uslope[u0 + i + k];
        if (!(B.s[0] <= 0.0) || !(B.s[tu] >= 0.0)) bad = kNcFlagInvalid;
        if (bad) break;
        if (!nc_sum(B.l, B.s, tu, M, H)) {
            bad = kNcFlagCapacity;
            break;
        }
        if (i == n1 - 1) break;
        const double wi = (double)w[i];
        const double ci = C ? (double)C[i] : HUGE_VAL;
        if (!(wi >= 0.0) || !(ci > 0.0)) {
            bad = kNcFlagInvalid;
            break;
        }
        int64_t *eo = A.eoff + 3 * i;
        // f^1: H -> B
        eo[0] = mp.n;
        if (!nc_dt(NcFwd{&H}, wi, B, [&](double lo, double hi) { return mp.add(lo, hi, lo); })) {
            bad = kNcFlagCapacity;
            break;
        }
        // f^2: reversed scan of B -> H (H holds the result reversed)
        eo[1] = mp.n;
        if (!nc_dt(NcRev{&B}, wi, H, [&](double lo, double hi) { return mp.add(-hi, -lo, -lo); })) {
            bad = kNcFlagCapacity;
            break;
        }
        // f^3 on rev(H) -> M, or M = rev(H)
        eo[2] = mp.n;
        if (ci < HUGE_VAL) {
            if (!nc_trunc(NcRev{&H}, ci, M, mp)) {
                bad = kNcFlagCapacity;
                break;
            }
        } else {
            const NcRev r{&H};
            M.t = r.t();
            for (int64_t k = 0; k < M.t; ++k) M.l[k] = r.l(k);
            for (int64_t k = 0; k <= M.t; ++k) M.s[k] = r.s(k);
        }
    }
    if (bad) return bad;
    // the last node: the first breakpoint attaining the minimum of hat M (in H)
    double v = 0.0, vmin = 0.0, y = H.t > 0 ? H.l[0] : 0.0;
    for (int64_t k = 1; k < H.t; ++k) {
        v += H.s[k] * (H.l[k] - H.l[k - 1]);
        if (v < vmin) {
            vmin = v;
            y = H.l[k];
        }
    }
    x[n1 - 1] = (T)y;
    for (int64_t i = n1 - 2; i >= n0; --i) {
        const int64_t *eo = A.eoff + 3 * i;
        const int64_t e3 = (i + 1 < n1 - 1) ? A.eoff[3 * (i + 1)] : mp.n;
        y = nc_apply(mp, eo[2], e3, y);
        y = nc_apply(mp, eo[1], eo[2], y);
        y = nc_apply(mp, eo[0], eo[1], y);
        x[i] = (T)y;
    }
    return 0;
}

// The three message buffers of a lane live in LDS when `lanes` lanes' worth
// fit in one workgroup (kLds; the rest of the wave idles), else in HBM.
template <typename T, bool kLds>
__global__ __launch_bounds__(64) void k_nc_chain(NcArgs A, const T *__restrict__ ulam, const T *__restrict__ uslope,
                                                 const T *__restrict__ w, const T *__restrict__ C, T *__restrict__ x,
                                                 int lanes) {
    extern __shared__ double s_nc[];
    if ((int)threadIdx.x >= lanes) return;
    const int64_t c = (int64_t)blockIdx.x * lanes + threadIdx.x;
    if (c >= A.num_chains) return;
    const int64_t bstride = 2 * A.msg_cap + 1;
    double *base = kLds ? s_nc + (int64_t)threadIdx.x * 3 * bstride : A.bufs + c * 3 * bstride;
    const int bad = nc_chain_lane<T>(A, ulam, uslope, w, C, x, c, NcBuf{base, base + A.msg_cap, 0, A.msg_cap},
                                     NcBuf{base + bstride, base + bstride + A.msg_cap, 0, A.msg_cap},
                                     NcBuf{base + 2 * bstride, base + 2 * bstride + A.msg_cap, 0, A.msg_cap});
    if (bad) atomicOr(A.flag, bad);
}

// ---------------------------------------------------------------------------
// A wave per chain.  The same message passing with each pass spread over the
// 64 lanes (element k of a message on lane k mod 64, the message in LDS):
//   Lemma 1: both sorted lists scattered by rank, equal positions merged, the
//     slope right of each point read from the two lists' counts;
//   f^1: h (x) f^1 (y) = w y + min_{x <= y} (h(x) - w x), so Algorithm 1 is a
//     prefix minimum of g = h - w x over the breakpoints plus, per piece, the
//     point where g comes back down to that minimum (the end of an interval of
//     Pi^1, which starts at the minimum's breakpoint);
//   f^2: the same on the reversed view; f^3: a wave minimum and per piece the
//     crossing of min h + C;
// each pass ends with a prefix count that places the points it emits.  The
// backward pass is one lane's.  Instantiated for messages of up to 128 and up
// to 256 breakpoints (16 and 32 KiB of LDS per wave), the smaller where
// msg_cap allows, so that more waves fit on a CU.
// ---------------------------------------------------------------------------
constexpr int kWaveMsg = 256;

__device__ __forceinline__ int wv_lane() { return (int)threadIdx.x; }

__device__ __forceinline__ double wv_scan_add(double x) {
    const int lane = wv_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ int wv_scan_int(int x) {
    const int lane = wv_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Inclusive prefix minimum; ties keep the earlier index.
__device__ __forceinline__ void wv_scan_min(double &v, int &i) {
    const int lane = wv_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double vo = __shfl_up(v, d, 64);
        const int io = __shfl_up(i, d, 64);
        if (lane >= d && (vo < v || (vo == v && io < i))) {
            v = vo;
            i = io;
        }
    }
}

// A message in LDS, read as stored or reversed (phi^rev(z) = phi(-z)).
struct WView {
    const double *L, *S;
    int t;
    bool rev;
    __device__ __forceinline__ double l(int k) const { return rev ? -L[t - 1 - k] : L[k]; }
    __device__ __forceinline__ double s(int k) const { return rev ? -S[t - k] : S[k]; }
};

// first index in a[0..n) with a[idx] >= v (strict = false: > v)
__device__ __forceinline__ int wv_lower(const double *a, int n, double v, bool strict) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool go = strict ? (a[mid] <= v) : (a[mid] < v);
        if (go) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Shared scratch of one wave.
struct WScratch {
    int tsize;     // entries of T
    double *T;     // [2 cap] merge staging
    int *CU, *CM;  // [2 kWaveMsg] unary / message breakpoints at or before each merged one
    double *V;     // [kWaveMsg] values at breakpoints
    double *PM;    // [kWaveMsg] prefix minimum
    int *PA;       // [kWaveMsg] its index
    double *PS, *PE;  // [kWaveMsg + 1] start / end slope of each piece
    int *Q0, *Q1;     // [kWaveMsg + 1] start / end status of each piece
};

// V[k] = h(l(k)) - h(l(0)).
__device__ void wv_values(const WView &h, double *V) {
    double carry = 0.0;
    for (int c = 0; c * 64 < h.t; ++c) {
        const int k = c * 64 + wv_lane();
        const double d = (k >= 1 && k < h.t) ? h.s(k) * (h.l(k) - h.l(k - 1)) : 0.0;
        const double inc = wv_scan_add(d) + carry;
        if (k < h.t) V[k] = inc;
        carry = __shfl(inc, 63, 64);
    }
    __syncthreads();
}

// Lemma 1: out = unary + M.  Returns the number of breakpoints, or -1 if more
// than cap.
__device__ int wv_sum(const double *ul, const double *us, int tu, const double *ml, const double *ms, int tm,
                      double *ol, double *os, int cap, const WScratch &W) {
    // scatter by rank (a unary breakpoint goes before equal message ones) and
    // record how many of each list lie at or before the element: for the last
    // element of a group of equal positions those are the counts of both lists
    // up to that position, which give the slope right of it
    for (int i = wv_lane(); i < tu; i += 64) {
        const int r = wv_lower(ml, tm, ul[i], false);
        W.T[i + r] = ul[i];
        W.CU[i + r] = i + 1;
        W.CM[i + r] = r;
    }
    for (int j = wv_lane(); j < tm; j += 64) {
        const int r = wv_lower(ul, tu, ml[j], true);
        W.T[j + r] = ml[j];
        W.CU[j + r] = r;
        W.CM[j + r] = j + 1;
    }
    __syncthreads();
    const int tot = tu + tm;
    int base = 0;
    for (int c = 0; c * 64 < tot; ++c) {
        const int k = c * 64 + wv_lane();
        const bool keep = k < tot && (k == 0 || W.T[k] != W.T[k - 1]);
        const int inc = wv_scan_int(keep ? 1 : 0);
        const int pos = base + inc - 1;
        if (keep && pos < cap) {
            const double lam = W.T[k];
            int last = k;
            while (last + 1 < tot && W.T[last + 1] == lam) ++last;
            ol[pos] = lam;
            os[pos + 1] = us[W.CU[last]] + ms[W.CM[last]];
        }
        base += __shfl(inc, 63, 64);
    }
    if (wv_lane() == 0) os[0] = us[0] + ms[0];
    __syncthreads();
    return base <= cap ? base : -1;
}

// h (x) f^1 (Algorithm 1 as a prefix minimum).  Intervals go to the chain's
// list at *nmap (rev: reported in the original coordinates).  Returns the
// number of breakpoints, -1 past cap, -2 past the interval capacity.
__device__ int wv_dt(const WView &h, double w, double *ol, double *os, int cap, const NcMaps &mp, int64_t &nmap,
                     const WScratch &W) {
    const int t = h.t;
    if (t == 0) {
        if (wv_lane() == 0) os[0] = h.s(0);
        __syncthreads();
        return 0;
    }
    wv_values(h, W.V);
    // prefix minimum of g_k = V_k - w l(k)
    double cv = HUGE_VAL;
    int ci = 0;
    for (int c = 0; c * 64 < t; ++c) {
        const int k = c * 64 + wv_lane();
        double v = (k < t) ? W.V[k] - w * h.l(k) : HUGE_VAL;
        int i = k;
        wv_scan_min(v, i);
        if (cv < v || (cv == v && ci < i)) {
            v = cv;
            i = ci;
        }
        if (k < t) {
            W.PM[k] = v;
            W.PA[k] = i;
        }
        cv = __shfl(v, 63, 64);
        ci = __shfl(i, 63, 64);
    }
    __syncthreads();
    // pieces k = 0..t: start / end slope of the result
    for (int k = wv_lane(); k <= t; k += 64) {
        double ps, pe;
        if (k == 0) {
            ps = pe = h.s(0);
        } else {
            const double sk = h.s(k), sig = sk - w;
            const double gl = W.V[k - 1] - w * h.l(k - 1), m = W.PM[k - 1];
            const bool on = gl <= m;
            if (on) {
                ps = pe = (sig < 0.0) ? sk : w;
            } else {
                const bool cross = (sig < 0.0) && (k == t || W.V[k] - w * h.l(k) <= m);
                ps = w;
                pe = cross ? sk : w;
            }
        }
        W.PS[k] = ps;
        W.PE[k] = pe;
    }
    __syncthreads();
    // emit, unit k = 1..t: breakpoint l(k-1) if the slope changes there, then
    // the crossing of piece k; close intervals at crossings (and an open end)
    int base = 0, ibase = 0;
    bool over = false;
    for (int c = 0; c * 64 < t; ++c) {
        const int k = 1 + c * 64 + wv_lane();
        const bool in = k <= t;
        bool e1 = false, e2 = false, close = false;
        double y = 0.0, ilo = 0.0, ihi = 0.0;
        if (in) {
            e1 = W.PE[k - 1] != W.PS[k];
            const double sk = h.s(k), sig = sk - w;
            const double gl = W.V[k - 1] - w * h.l(k - 1), m = W.PM[k - 1];
            const bool on = gl <= m;
            const double la = h.l(W.PA[k - 1]);
            if (!on && sig < 0.0 && (k == t || W.V[k] - w * h.l(k) <= m)) {
                y = h.l(k - 1) + (m - gl) / sig;
                if (y < h.l(k - 1)) y = h.l(k - 1);
                if (k < t && y > h.l(k)) y = h.l(k);
                e2 = true;
                close = true;
                ilo = la;
                ihi = y;
            } else if (k == t && sig >= 0.0) {  // flat to +inf
                close = true;
                ilo = on ? h.l(W.PA[k - 1]) : la;
                ihi = HUGE_VAL;
            }
        }
        const int cnt = (e1 ? 1 : 0) + (e2 ? 1 : 0);
        const int inc = wv_scan_int(cnt);
        int pos = base + inc - cnt;
        if (e1) {
            if (pos < cap) {
                ol[pos] = h.l(k - 1);
                os[pos + 1] = W.PS[k];
            }
            ++pos;
        }
        if (e2 && pos < cap) {
            ol[pos] = y;
            os[pos + 1] = W.PE[k];
        }
        base += __shfl(inc, 63, 64);
        const int iinc = wv_scan_int(close ? 1 : 0);
        const int64_t ipos = nmap + ibase + iinc - 1;
        if (close) {
            if (ipos < mp.cap) {
                mp.put(ipos, h.rev ? -ihi : ilo, h.rev ? -ilo : ihi, h.rev ? -ilo : ilo);
            } else {
                over = true;
            }
        }
        ibase += __shfl(iinc, 63, 64);
    }
    if (wv_lane() == 0) os[0] = W.PS[0];
    nmap += ibase;
    const bool any_over = __ballot(over) != 0;
    __syncthreads();
    if (any_over) return -2;
    return base <= cap ? base : -1;
}

// min(h, min h + C) with Pi^3 (h through a view).  Same returns as wv_dt.
__device__ int wv_trunc(const WView &h, double C, double *ol, double *os, int cap, const NcMaps &mp,
                        int64_t &nmap, const WScratch &W) {
    const int t = h.t;
    if (t == 0) {
        if (wv_lane() == 0) os[0] = h.s(0);
        __syncthreads();
        return 0;
    }
    wv_values(h, W.V);
    // minimum of V and its first index
    double mv = HUGE_VAL;
    int mi = 0;
    for (int c = 0; c * 64 < t; ++c) {
        const int k = c * 64 + wv_lane();
        double v = (k < t) ? W.V[k] : HUGE_VAL;
        int i = k;
        wv_scan_min(v, i);
        v = __shfl(v, 63, 64);
        i = __shfl(i, 63, 64);
        if (v < mv || (v == mv && i < mi)) {
            mv = v;
            mi = i;
        }
    }
    const double cp = mv + C, xm = h.l(mi);
    // per piece: crossing, and the status / slope of its first and last segment
    // (status decided at each segment's midpoint)
    auto hval = [&](int k, double z) { return (k == 0) ? W.V[0] + h.s(0) * (z - h.l(0)) : W.V[k - 1] + h.s(k) * (z - h.l(k - 1)); };
    auto crossing = [&](int k, double &z) -> bool {
        if (k == 0) {
            if (h.s(0) < 0.0 && W.V[0] < cp) {
                z = h.l(0) + (cp - W.V[0]) / h.s(0);
                return true;
            }
            return false;
        }
        if (k == t) {
            if (h.s(t) > 0.0 && W.V[t - 1] < cp) {
                z = h.l(t - 1) + (cp - W.V[t - 1]) / h.s(t);
                return true;
            }
            return false;
        }
        if ((W.V[k - 1] < cp && W.V[k] > cp) || (W.V[k - 1] > cp && W.V[k] < cp)) {
            z = h.l(k - 1) + (cp - W.V[k - 1]) / h.s(k);
            return true;
        }
        return false;
    };
    auto segstat = [&](int k, double lo, double hi) -> bool {
        const double mid = (lo == -HUGE_VAL) ? hi - 1.0 : (hi == HUGE_VAL ? lo + 1.0 : 0.5 * (lo + hi));
        return hval(k, mid) >= cp;
    };
    for (int k = wv_lane(); k <= t; k += 64) {
        const double lo = (k == 0) ? -HUGE_VAL : h.l(k - 1), hi = (k == t) ? HUGE_VAL : h.l(k);
        double z = 0.0;
        const bool cr = crossing(k, z);
        const bool s0 = segstat(k, lo, cr ? z : hi), s1 = cr ? segstat(k, z, hi) : s0;
        W.Q0[k] = s0 ? 1 : 0;
        W.Q1[k] = s1 ? 1 : 0;
        W.PS[k] = s0 ? 0.0 : h.s(k);
        W.PE[k] = s1 ? 0.0 : h.s(k);
    }
    __syncthreads();
    // emit: unit u = 0..t: breakpoint l(u-1) (u >= 1), then piece u's crossing;
    // status changes at those points start or end the runs of Pi^3
    int base = 0, sb = 0, eb = 0;
    bool over = false;
    for (int c = 0; c * 64 <= t; ++c) {
        const int u = c * 64 + wv_lane();
        const bool in = u <= t;
        bool e1 = false, e2 = false;
        int st1 = 0, en1 = 0, st2 = 0, en2 = 0;  // run start / end at the breakpoint, at the crossing
        double z = 0.0;
        bool cr = false;
        if (in) {
            cr = crossing(u, z);
            if (u >= 1) {
                e1 = W.PE[u - 1] != W.PS[u];
                st1 = (!W.Q1[u - 1] && W.Q0[u]) ? 1 : 0;
                en1 = (W.Q1[u - 1] && !W.Q0[u]) ? 1 : 0;
            } else {
                st1 = W.Q0[0] ? 1 : 0;  // a run from -inf
            }
            if (cr) {
                e2 = W.PS[u] != W.PE[u];
                st2 = (!W.Q0[u] && W.Q1[u]) ? 1 : 0;
                en2 = (W.Q0[u] && !W.Q1[u]) ? 1 : 0;
            }
        }
        const int cnt = (e1 ? 1 : 0) + (e2 ? 1 : 0);
        const int inc = wv_scan_int(cnt);
        int pos = base + inc - cnt;
        if (e1) {
            if (pos < cap) {
                ol[pos] = h.l(u - 1);
                os[pos + 1] = W.PS[u];
            }
            ++pos;
        }
        if (e2 && pos < cap) {
            ol[pos] = z;
            os[pos + 1] = W.PE[u];
        }
        base += __shfl(inc, 63, 64);
        // run starts and ends, in order; a run's interval is written at its
        // end (start positions kept in the T scratch)
        const double bpos = (u >= 1) ? h.l(u - 1) : -HUGE_VAL;
        const int scount = st1 + st2, ecount = en1 + en2;
        const int sinc = wv_scan_int(scount), einc = wv_scan_int(ecount);
        int sp = sb + sinc - scount;
        if (st1) {
            if (sp < W.tsize) W.T[sp] = bpos;
            ++sp;
        }
        if (st2 && sp < W.tsize) W.T[sp] = z;
        sb += __shfl(sinc, 63, 64);
        // ends are written after every start of this chunk is in T
        __syncthreads();
        int ep = eb + einc - ecount;
        auto put_end = [&](double e) {
            const int64_t ipos = nmap + ep;
            if (ipos < mp.cap && ep < W.tsize) {
                mp.put(ipos, W.T[ep], e, xm);
            } else {
                over = true;
            }
            ++ep;
        };
        if (en1) put_end(bpos);
        if (en2) put_end(z);
        eb += __shfl(einc, 63, 64);
        __syncthreads();
    }
    // a run still open at +inf
    if (sb > eb) {
        if (wv_lane() == 0) {
            const int64_t ipos = nmap + eb;
            if (ipos < mp.cap && eb < W.tsize) {
                mp.put(ipos, W.T[eb], HUGE_VAL, xm);
            } else {
                over = true;
            }
        }
        ++eb;
    }
    if (wv_lane() == 0) os[0] = W.PS[0];
    nmap += eb;
    const bool any_over = __ballot(over) != 0;
    __syncthreads();
    if (any_over) return -2;
    return base <= cap ? base : -1;
}

template <typename T, int kCap>
__global__ __launch_bounds__(64) void k_nc_wave(NcArgs A, const T *__restrict__ ulam, const T *__restrict__ uslope,
                                                const T *__restrict__ w, const T *__restrict__ C,
                                                T *__restrict__ x) {
    static_assert(kCap % 64 == 0 && kCap <= kWaveMsg, "wave message capacity");
    __shared__ double sU_l[kCap], sU_s[kCap + 1];
    __shared__ double sA_l[kCap], sA_s[kCap + 1];
    __shared__ double sB_l[kCap], sB_s[kCap + 1];
    __shared__ double sC_l[kCap], sC_s[kCap + 1];
    __shared__ double sT[2 * kCap], sV[kCap], sPM[kCap], sPS[kCap + 1], sPE[kCap + 1];
    __shared__ int sPA[kCap], sQ0[kCap + 1], sQ1[kCap + 1];
    // the merge's counts live only inside the sum, before V and PM are used:
    // they share those arrays (2 kCap ints in kCap doubles each)
    static_assert(2 * sizeof(int) == sizeof(double), "two counts per double");
    const WScratch W{2 * kCap, sT, (int *)sV, (int *)sPM, sV, sPM, sPA, sPS, sPE, sQ0, sQ1};
    const int64_t c = blockIdx.x;
    if (c >= A.num_chains) return;
    const int64_t n0 = A.coff[c], n1 = A.coff[c + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) {  // a range outside the nodes
        if (threadIdx.x == 0) atomicOr(A.flag, kNcFlagInvalid);
        return;
    }
    if (n1 == n0) return;
    const int lane = wv_lane();
    const int cap = (int)(A.msg_cap < kCap ? A.msg_cap : kCap);
    double *mb = A.maps + c * 3 * A.map_cap;
    const NcMaps mp{mb, 0, A.map_cap};
    int64_t nmap = 0;
    int tm = 0, th = 0, bad = 0;
    if (lane == 0) sA_s[0] = 0.0;
    // the next node's unary is loaded into registers while a node is processed
    constexpr int kPer = kCap / 64;
    double pl[kPer], ps[kPer + 1];
    auto fetch = [&](int64_t i) {
        const int64_t u0 = A.uoff[i], tu = A.uoff[i + 1] - u0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = lane + 64 * j;
            pl[j] = (k < tu && tu <= cap) ? (double)ulam[u0 + k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j <= kPer; ++j) {
            const int k = lane + 64 * j;
            ps[j] = (k <= tu && tu <= cap) ? (double)uslope[u0 + i + k] : 0.0;
        }
    };
    fetch(n0);
    __syncthreads();
    for (int64_t i = n0; i < n1; ++i) {
        const int64_t u0 = A.uoff[i], tu64 = A.uoff[i + 1] - u0;
        if (tu64 < 1 || tu64 > cap) {
            bad = tu64 < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        const int tu = (int)tu64;
        bool inval = false;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = lane + 64 * j;
            if (k < tu) sU_l[k] = pl[j];
        }
#pragma unroll
        for (int j = 0; j <= kPer; ++j) {
            const int k = lane + 64 * j;
            if (k <= tu) sU_s[k] = ps[j];
        }
        if (i + 1 < n1) fetch(i + 1);
        __syncthreads();
        for (int k = lane; k < tu; k += 64)
            if (k > 0 && !(sU_l[k] >= sU_l[k - 1])) inval = true;
        if (lane == 0 && (!(sU_s[0] <= 0.0) || !(sU_s[tu] >= 0.0))) inval = true;
        if (__ballot(inval) != 0) {
            bad = kNcFlagInvalid;
            break;
        }
        th = wv_sum(sU_l, sU_s, tu, sA_l, sA_s, tm, sB_l, sB_s, cap, W);
        if (th < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        if (i == n1 - 1) break;
        const double wi = (double)w[i];
        const double ci = C ? (double)C[i] : HUGE_VAL;
        if (!(wi >= 0.0) || !(ci > 0.0)) {
            bad = kNcFlagInvalid;
            break;
        }
        int64_t *eo = A.eoff + 3 * i;
        if (lane == 0) eo[0] = nmap;
        const int t1 = wv_dt(WView{sB_l, sB_s, th, false}, wi, sC_l, sC_s, cap, mp, nmap, W);
        if (t1 < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        if (lane == 0) eo[1] = nmap;
        const int t2 = wv_dt(WView{sC_l, sC_s, t1, true}, wi, sB_l, sB_s, cap, mp, nmap, W);
        if (t2 < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        if (lane == 0) eo[2] = nmap;
        const WView r{sB_l, sB_s, t2, true};
        if (ci < HUGE_VAL) {
            tm = wv_trunc(r, ci, sA_l, sA_s, cap, mp, nmap, W);
            if (tm < 0) {
                bad = kNcFlagCapacity;
                break;
            }
        } else {
            for (int k = lane; k < t2; k += 64) sA_l[k] = r.l(k);
            for (int k = lane; k <= t2; k += 64) sA_s[k] = r.s(k);
            tm = t2;
            __syncthreads();
        }
    }
    if (bad) {
        if (lane == 0) atomicOr(A.flag, bad);
        return;
    }
    if (lane != 0) return;
    // backward, one lane: the first minimum of the last hat M (in B), then pi
    double v = 0.0, vmin = 0.0, y = th > 0 ? sB_l[0] : 0.0;
    for (int k = 1; k < th; ++k) {
        v += sB_s[k] * (sB_l[k] - sB_l[k - 1]);
        if (v < vmin) {
            vmin = v;
            y = sB_l[k];
        }
    }
    x[n1 - 1] = (T)y;
    for (int64_t i = n1 - 2; i >= n0; --i) {
        const int64_t *eo = A.eoff + 3 * i;
        const int64_t e3 = (i + 1 < n1 - 1) ? A.eoff[3 * (i + 1)] : nmap;
        y = nc_apply(mp, eo[2], e3, y);
        y = nc_apply(mp, eo[1], eo[2], y);
        y = nc_apply(mp, eo[0], eo[1], y);
        x[i] = (T)y;
    }
}

// ---------------------------------------------------------------------------
// Sec. 3 on a batch of trees: one lane per tree, nodes in depth-first
// post-order (every subtree a contiguous range ending at its root), so the
// messages of a node's children are the top entries of a stack of finished,
// not yet consumed messages.  A node sums its unary and its children's
// messages (Lemma 1, one merge per child), then a non-root sends its
// min-convolved message (Algorithm 1, its reversal, the truncation) to the
// stack and a root takes its first argmin; backward, parents before children.
// The three working buffers, the stack and the interval lists live in the
// tree's slice of the workspace.
// ---------------------------------------------------------------------------
struct NcTreeArgs {
    int64_t num_trees, num_nodes;
    const int64_t *toff, *parent, *uoff;
    int64_t msg_cap, map_cap, stack_cap;
    double *bufs;      // per tree: 3 buffers of (2 msg_cap + 1) doubles
    double *stack;     // per tree: stack_cap doubles of pending messages (l then s)
    double *maps;      // per tree: map_cap intervals of 3 doubles
    int64_t *hstart;   // [N] pending message: start in the stack
    int64_t *hcount;   //     breakpoints
    int64_t *hparent;  //     node it is for
    int64_t *eoff;     // [N][6] start / end of the node's intervals in each list
    int *flag;
};

template <typename T>
__global__ __launch_bounds__(64) void k_nc_tree(NcTreeArgs A, const T *__restrict__ ulam,
                                                const T *__restrict__ uslope, const T *__restrict__ w,
                                                const T *__restrict__ C, T *__restrict__ x, int lanes) {
    if ((int)threadIdx.x >= lanes) return;
    const int64_t tr = (int64_t)blockIdx.x * lanes + threadIdx.x;
    if (tr >= A.num_trees) return;
    const int64_t n0 = A.toff[tr], n1 = A.toff[tr + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) {
        atomicOr(A.flag, kNcFlagInvalid);
        return;
    }
    if (n1 == n0) return;
    const int64_t bstride = 2 * A.msg_cap + 1;
    double *base = A.bufs + tr * 3 * bstride;
    NcBuf H{base, base + A.msg_cap, 0, A.msg_cap};
    NcBuf B{base + bstride, base + bstride + A.msg_cap, 0, A.msg_cap};
    NcBuf U{base + 2 * bstride, base + 2 * bstride + A.msg_cap, 0, A.msg_cap};  // the unary, staged
    double *stk = A.stack + tr * A.stack_cap;
    double *mb = A.maps + tr * 3 * A.map_cap;
    NcMaps mp{mb, 0, A.map_cap};
    int64_t top = 0;   // stack fill (doubles)
    int64_t sp = n0;   // header stack pointer
    int bad = 0;
    for (int64_t i = n0; i < n1 && !bad; ++i) {
        const int64_t p = A.parent[i];
        if (p != -1 && (p <= i || p >= n1)) {
            bad = kNcFlagInvalid;
            break;
        }
        // the unary, staged in U (validated)
        const int64_t u0 = A.uoff[i], tu = A.uoff[i + 1] - u0;
        if (tu < 1 || tu > A.msg_cap) {
            bad = tu < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        for (int64_t k = 0; k < tu; ++k) {
            U.l[k] = (double)ulam[u0 + k];
            if (k > 0 && !(U.l[k] >= U.l[k - 1])) bad = kNcFlagInvalid;
        }
        for (int64_t k = 0; k <= tu; ++k) U.s[k] = (double)uslope[u0 + i + k];
        if (!(U.s[0] <= 0.0) || !(U.s[tu] >= 0.0)) bad = kNcFlagInvalid;
        if (bad) break;
        // hat = f_i (+ 0), then + each child's message from the top of the stack
        B.t = 0;
        B.s[0] = 0.0;
        if (!nc_sum(U.l, U.s, tu, B, H)) {
            bad = kNcFlagCapacity;
            break;
        }
        while (sp > n0 && A.hparent[sp - 1] == i) {
            --sp;
            const int64_t cs = A.hstart[sp], ct = A.hcount[sp];
            if (cs < 0 || cs + 2 * ct + 1 != top) {  // not right below: not a post-order numbering
                bad = kNcFlagInvalid;
                break;
            }
            const NcBuf child{stk + cs, stk + cs + ct, ct, ct};
            if (!nc_sum(H.l, H.s, H.t, child, B)) {
                bad = kNcFlagCapacity;
                break;
            }
            const NcBuf t = H;
            H = B;
            B = t;
            top = cs;
        }
        if (bad) break;
        if (p < 0) {  // a root: the first breakpoint attaining the minimum
            double v = 0.0, vmin = 0.0, y = H.t > 0 ? H.l[0] : 0.0;
            for (int64_t k = 1; k < H.t; ++k) {
                v += H.s[k] * (H.l[k] - H.l[k - 1]);
                if (v < vmin) {
                    vmin = v;
                    y = H.l[k];
                }
            }
            x[i] = (T)y;
            continue;
        }
        const double wi = (double)w[i];
        const double ci = C ? (double)C[i] : HUGE_VAL;
        if (!(wi >= 0.0) || !(ci > 0.0)) {
            bad = kNcFlagInvalid;
            break;
        }
        int64_t *eo = A.eoff + 6 * i;
        eo[0] = mp.n;
        if (!nc_dt(NcFwd{&H}, wi, B, [&](double lo, double hi) { return mp.add(lo, hi, lo); })) {
            bad = kNcFlagCapacity;
            break;
        }
        eo[1] = mp.n;
        eo[2] = mp.n;
        if (!nc_dt(NcRev{&B}, wi, H, [&](double lo, double hi) { return mp.add(-hi, -lo, -lo); })) {
            bad = kNcFlagCapacity;
            break;
        }
        eo[3] = mp.n;
        eo[4] = mp.n;
        // the message (of rev(H), truncated or not) is written into U, then pushed
        if (ci < HUGE_VAL) {
            if (!nc_trunc(NcRev{&H}, ci, U, mp)) {
                bad = kNcFlagCapacity;
                break;
            }
        } else {
            const NcRev r{&H};
            U.t = r.t();
            for (int64_t k = 0; k < U.t; ++k) U.l[k] = r.l(k);
            for (int64_t k = 0; k <= U.t; ++k) U.s[k] = r.s(k);
        }
        eo[5] = mp.n;
        const int64_t need = 2 * U.t + 1;
        if (top + need > A.stack_cap) {
            bad = kNcFlagCapacity;
            break;
        }
        for (int64_t k = 0; k < U.t; ++k) stk[top + k] = U.l[k];
        for (int64_t k = 0; k <= U.t; ++k) stk[top + U.t + k] = U.s[k];
        A.hstart[sp] = top;
        A.hcount[sp] = U.t;
        A.hparent[sp] = p;
        ++sp;
        top += need;
    }
    if (!bad && sp != n0) bad = kNcFlagInvalid;  // messages left for parents outside the tree
    if (bad) {
        atomicOr(A.flag, bad);
        return;
    }
    for (int64_t i = n1 - 1; i >= n0; --i) {
        const int64_t p = A.parent[i];
        if (p < 0) continue;
        const int64_t *eo = A.eoff + 6 * i;
        double y = (double)x[p];
        y = nc_apply(mp, eo[4], eo[5], y);
        y = nc_apply(mp, eo[2], eo[3], y);
        y = nc_apply(mp, eo[0], eo[1], y);
        x[i] = (T)y;
    }
}

// A wave per tree, for batches with fewer trees than SIMDs: k_nc_tree's
// post-order walk with every pass spread over the wave (wv_sum for Lemma 1,
// reading each child's message straight from the tree's stack; wv_dt twice
// and wv_trunc for the edge), the working messages in LDS.  Every lane writes
// the stack headers (the same values), so each reads back its own writes; the
// pushed message itself is visible to the wave after the barrier.
template <typename T, int kCap>
__global__ __launch_bounds__(64) void k_nc_tree_wave(NcTreeArgs A, const T *__restrict__ ulam,
                                                     const T *__restrict__ uslope, const T *__restrict__ w,
                                                     const T *__restrict__ C, T *__restrict__ x) {
    static_assert(kCap % 64 == 0 && kCap <= kWaveMsg, "wave message capacity");
    __shared__ double sU_l[kCap], sU_s[kCap + 1];
    __shared__ double sA_l[kCap], sA_s[kCap + 1];
    __shared__ double sB_l[kCap], sB_s[kCap + 1];
    __shared__ double sC_l[kCap], sC_s[kCap + 1];
    __shared__ double sT[2 * kCap], sV[kCap], sPM[kCap], sPS[kCap + 1], sPE[kCap + 1];
    __shared__ int sPA[kCap], sQ0[kCap + 1], sQ1[kCap + 1];
    static_assert(2 * sizeof(int) == sizeof(double), "two counts per double");
    const WScratch W{2 * kCap, sT, (int *)sV, (int *)sPM, sV, sPM, sPA, sPS, sPE, sQ0, sQ1};
    const int64_t tr = blockIdx.x;
    if (tr >= A.num_trees) return;
    const int64_t n0 = A.toff[tr], n1 = A.toff[tr + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) {
        if (threadIdx.x == 0) atomicOr(A.flag, kNcFlagInvalid);
        return;
    }
    if (n1 == n0) return;
    const int lane = wv_lane();
    const int cap = (int)(A.msg_cap < kCap ? A.msg_cap : kCap);
    double *stk = A.stack + tr * A.stack_cap;
    double *mb = A.maps + tr * 3 * A.map_cap;
    const NcMaps mp{mb, 0, A.map_cap};
    int64_t nmap = 0, top = 0, sp = n0;
    int bad = 0;
    for (int64_t i = n0; i < n1; ++i) {
        const int64_t p = A.parent[i];
        if (p != -1 && (p <= i || p >= n1)) {
            bad = kNcFlagInvalid;
            break;
        }
        const int64_t u0 = A.uoff[i], tu64 = A.uoff[i + 1] - u0;
        if (tu64 < 1 || tu64 > cap) {
            bad = tu64 < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        const int tu = (int)tu64;
        for (int k = lane; k < tu; k += 64) sU_l[k] = (double)ulam[u0 + k];
        for (int k = lane; k <= tu; k += 64) sU_s[k] = (double)uslope[u0 + i + k];
        if (lane == 0) sA_s[0] = 0.0;  // an empty message
        __syncthreads();
        bool inval = false;
        for (int k = lane; k < tu; k += 64)
            if (k > 0 && !(sU_l[k] >= sU_l[k - 1])) inval = true;
        if (lane == 0 && (!(sU_s[0] <= 0.0) || !(sU_s[tu] >= 0.0))) inval = true;
        if (__ballot(inval) != 0) {
            bad = kNcFlagInvalid;
            break;
        }
        int th = wv_sum(sU_l, sU_s, tu, sA_l, sA_s, 0, sB_l, sB_s, cap, W);
        if (th < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        double *hl = sB_l, *hs = sB_s, *ol = sC_l, *os = sC_s;
        while (sp > n0 && A.hparent[sp - 1] == i) {
            --sp;
            const int64_t cs = A.hstart[sp], ct = A.hcount[sp];
            if (cs < 0 || ct < 0 || ct > cap || cs + 2 * ct + 1 != top) {
                bad = kNcFlagInvalid;
                break;
            }
            const int tn = wv_sum(hl, hs, th, stk + cs, stk + cs + ct, (int)ct, ol, os, cap, W);
            if (tn < 0) {
                bad = kNcFlagCapacity;
                break;
            }
            double *sw = hl;
            hl = ol;
            ol = sw;
            sw = hs;
            hs = os;
            os = sw;
            th = tn;
            top = cs;
        }
        if (bad) break;
        if (p < 0) {  // a root: the first breakpoint attaining the minimum
            if (lane == 0) {
                double v = 0.0, vmin = 0.0, y = th > 0 ? hl[0] : 0.0;
                for (int k = 1; k < th; ++k) {
                    v += hs[k] * (hl[k] - hl[k - 1]);
                    if (v < vmin) {
                        vmin = v;
                        y = hl[k];
                    }
                }
                x[i] = (T)y;
            }
            __syncthreads();
            continue;
        }
        const double wi = (double)w[i];
        const double ci = C ? (double)C[i] : HUGE_VAL;
        if (!(wi >= 0.0) || !(ci > 0.0)) {
            bad = kNcFlagInvalid;
            break;
        }
        int64_t *eo = A.eoff + 6 * i;
        if (lane == 0) eo[0] = nmap;
        const int t1 = wv_dt(WView{hl, hs, th, false}, wi, ol, os, cap, mp, nmap, W);
        if (t1 < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        if (lane == 0) eo[1] = eo[2] = nmap;
        const int t2 = wv_dt(WView{ol, os, t1, true}, wi, hl, hs, cap, mp, nmap, W);
        if (t2 < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        if (lane == 0) eo[3] = eo[4] = nmap;
        const WView r{hl, hs, t2, true};
        int tm;
        if (ci < HUGE_VAL) {
            tm = wv_trunc(r, ci, sA_l, sA_s, cap, mp, nmap, W);
            if (tm < 0) {
                bad = kNcFlagCapacity;
                break;
            }
        } else {
            for (int k = lane; k < t2; k += 64) sA_l[k] = r.l(k);
            for (int k = lane; k <= t2; k += 64) sA_s[k] = r.s(k);
            tm = t2;
            __syncthreads();
        }
        if (lane == 0) eo[5] = nmap;
        const int64_t need = 2 * (int64_t)tm + 1;
        if (top + need > A.stack_cap) {
            bad = kNcFlagCapacity;
            break;
        }
        for (int k = lane; k < tm; k += 64) stk[top + k] = sA_l[k];
        for (int k = lane; k <= tm; k += 64) stk[top + tm + k] = sA_s[k];
        A.hstart[sp] = top;
        A.hcount[sp] = tm;
        A.hparent[sp] = p;
        ++sp;
        top += need;
        __syncthreads();
    }
    if (!bad && sp != n0) bad = kNcFlagInvalid;
    if (bad) {
        if (lane == 0) atomicOr(A.flag, bad);
        return;
    }
    if (lane != 0) return;
    for (int64_t i = n1 - 1; i >= n0; --i) {
        const int64_t p = A.parent[i];
        if (p < 0) continue;
        const int64_t *eo = A.eoff + 6 * i;
        double y = (double)x[p];
        y = nc_apply(mp, eo[4], eo[5], y);
        y = nc_apply(mp, eo[2], eo[3], y);
        y = nc_apply(mp, eo[0], eo[1], y);
        x[i] = (T)y;
    }
}

size_t nc_tree_layout(int64_t num_trees, int64_t num_nodes, int64_t msg_cap, int64_t map_cap, int64_t stack_cap,
                      void *p, NcTreeArgs *A) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_b = off;  off += al(sizeof(double) * (size_t)(num_trees * 3 * (2 * msg_cap + 1)));
    const size_t o_s = off;  off += al(sizeof(double) * (size_t)(num_trees * stack_cap));
    const size_t o_m = off;  off += al(sizeof(double) * (size_t)(num_trees * 3 * map_cap));
    const size_t o_h = off;  off += al(sizeof(int64_t) * (size_t)(3 * num_nodes));
    const size_t o_e = off;  off += al(sizeof(int64_t) * (size_t)(6 * num_nodes));
    const size_t o_f = off;  off += al(sizeof(int));
    if (p && A) {
        char *c = (char *)p;
        A->bufs = (double *)(c + o_b);
        A->stack = (double *)(c + o_s);
        A->maps = (double *)(c + o_m);
        int64_t *h = (int64_t *)(c + o_h);
        A->hstart = h;
        A->hcount = h + num_nodes;
        A->hparent = h + 2 * num_nodes;
        A->eoff = (int64_t *)(c + o_e);
        A->flag = (int *)(c + o_f);
    }
    return off;
}

// Lanes per workgroup whose message buffers fit the LDS of one workgroup
// (160 KiB on gfx950); 0 if not even one lane's do.
constexpr size_t kNcLds = 160 * 1024;
int nc_lds_lanes(int64_t msg_cap) {
    const size_t per = sizeof(double) * 3 * (size_t)(2 * msg_cap + 1);
    const size_t k = kNcLds / per;
    return (int)(k > 64 ? 64 : k);
}

size_t nc_layout(int64_t num_chains, int64_t num_nodes, int64_t msg_cap, int64_t map_cap, void *p, NcArgs *A) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_b = off;
    // HBM message buffers only where they do not fit in LDS
    if (nc_lds_lanes(msg_cap) == 0) off += al(sizeof(double) * (size_t)(num_chains * 3 * (2 * msg_cap + 1)));
    const size_t o_m = off;
    off += al(sizeof(double) * (size_t)(num_chains * 3 * map_cap));
    const size_t o_e = off;
    off += al(sizeof(int64_t) * (size_t)(3 * num_nodes));
    const size_t o_f = off;
    off += al(sizeof(int));
    if (p && A) {
        char *c = (char *)p;
        A->bufs = (double *)(c + o_b);
        A->maps = (double *)(c + o_m);
        A->eoff = (int64_t *)(c + o_e);
        A->flag = (int *)(c + o_f);
    }
    return off;
}

// Launch check, then the device flag read back (synchronous).
// ---------------------------------------------------------------------------
// Sec. 3, Extensions (i): pairwise terms that are minima of one-sided linear
// pieces g(z) = alpha |z| + C on z > 0 or on z < 0 (g(0) = 0), applied one
// piece at a time (Prop. 2).  For a right-side piece and phi = h - alpha x,
//   (h (x) g)(y) = alpha y + min(phi(y), min_{x <= y} phi(x) + C).
// One sweep over the pieces of phi keeps its running minimum m and the first
// point a attaining it: the output follows h while phi <= m + C and is flat in
// phi's frame (slope alpha in h's) where phi rises above m + C; each such run
// maps to a, reported through add(lo, hi, a).  A left-side piece is the same
// sweep over the reversed view.
// ---------------------------------------------------------------------------
template <class View, class Add>
__host__ __device__ bool nc_side(const View &h, double alpha, double C, NcBuf &out, Add add) {
    const int64_t t = h.t();
    out.t = 0;
    out.s[0] = h.s(0);
    if (t == 0) return true;  // h constant: phi never rises above its running minimum
    double cur = h.s(0);      // the output's slope right of its last breakpoint
    auto emit = [&](double lam, double sl) -> bool {
        if (sl == cur) return true;
        if (out.t > 0 && out.l[out.t - 1] == lam) {  // a second slope at the same point
            out.s[out.t] = sl;
            if (out.s[out.t] == out.s[out.t - 1]) --out.t;
            cur = sl;
            return true;
        }
        cur = sl;
        return out.push(lam, sl);
    };
    // phi is non-increasing left of l(0) (s(0) <= 0 <= alpha): its minimum up to
    // l(0) is there; values relative to h(l(0)) = 0
    double phl = -alpha * h.l(0), m = phl, a = h.l(0), lo = 0.0;
    bool above = false;
    for (int64_t k = 1; k <= t; ++k) {
        const double L = h.l(k - 1), sk = h.s(k), sg = sk - alpha;
        const bool last = k == t;
        const double R = last ? HUGE_VAL : h.l(k);
        if (!above) {
            if (!emit(L, sk)) return false;
            if (sg > 0.0) {
                double y = L + (m + C - phl) / sg;  // phi climbs to m + C
                if (y < L) y = L;
                if (y < R) {
                    if (!emit(y, alpha)) return false;
                    above = true;
                    lo = y;
                }
            }
        } else if (sg < 0.0) {
            double y = L + (m + C - phl) / sg;  // phi comes back down to m + C
            if (y < L) y = L;
            if (y < R) {
                if (!add(lo, y, a)) return false;
                above = false;
                if (!emit(y, sk)) return false;
            }
        }
        if (last) break;
        const double phr = phl + sg * (R - L);
        if (!above && phr < m) {  // a new minimum (only where phi is not above m + C)
            m = phr;
            a = R;
        }
        phl = phr;
    }
    if (above && !add(lo, HUGE_VAL, a)) return false;
    return true;
}

struct NcgArgs {
    int64_t num_chains, num_nodes, num_pieces;
    const int64_t *coff, *uoff, *poff;
    int64_t msg_cap, map_cap;
    double *bufs;   // per chain: 3 buffers of (2 msg_cap + 1) doubles
    double *maps;   // per chain: map_cap intervals of 3 doubles
    int64_t *pmap;  // per piece: its interval range [pmap[2k], pmap[2k + 1])
    int *flag;
};

// One lane per chain (spread over at least 1024 waves), FP64 messages in the
// workspace.  Per node: hat = unary + incoming message (Lemma 1), then every
// piece of the edge to the next node in turn; backward, each node applies its
// edge's mappings, the last piece's first.
// One lane's chain c with its three message buffers given: X the incoming
// message, Y the other, U the staged unary (each of msg_cap breakpoints);
// returns the flag bits to raise (0: x written).  Host-callable, so that its
// indexing can be run against exactly-sized buffers on a CPU.
template <class T>
__host__ __device__ int ncg_chain_lane(const NcgArgs &A, const T *__restrict__ ulam, const T *__restrict__ uslope,
                                       const T *__restrict__ palpha, const T *__restrict__ pC,
                                       const int32_t *__restrict__ pside, T *__restrict__ x, int64_t c, NcBuf X,
                                       NcBuf Y, NcBuf U) {
    const int64_t n0 = A.coff[c], n1 = A.coff[c + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) return kNcFlagInvalid;
    if (n1 == n0) return 0;
    double *mb = A.maps + c * 3 * A.map_cap;
    NcMaps mp{mb, 0, A.map_cap};
    X.s[0] = 0.0;
    int bad = 0;
    for (int64_t i = n0; i < n1 && !bad; ++i) {
        const int64_t u0 = A.uoff[i], tu = A.uoff[i + 1] - u0;
        if (tu < 1 || tu > A.msg_cap) {
            bad = tu < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        for (int64_t k = 0; k < tu; ++k) {
            U.l[k] = (double)ulam[u0 + k];
            if (k > 0 && !(U.l[k] >= U.l[k - 1])) bad = kNcFlagInvalid;
        }
        for (int64_t k = 0; k <= tu; ++k) U.s[k] = (double)uslope[u0 + i + k];
        if (!(U.s[0] <= 0.0) || !(U.s[tu] >= 0.0)) bad = kNcFlagInvalid;
        if (bad) break;
        if (!nc_sum(U.l, U.s, tu, X, Y)) {  // hat in Y
            bad = kNcFlagCapacity;
            break;
        }
        if (i == n1 - 1) break;
        const int64_t k0 = A.poff[i], k1 = A.poff[i + 1];
        if (k0 < 0 || k1 < k0 || k1 > A.num_pieces) {
            bad = kNcFlagInvalid;
            break;
        }
        NcBuf *cur = &Y, *oth = &X;
        bool rev = false;  // cur holds the reversal of the message
        for (int64_t k = k0; k < k1; ++k) {
            const double al = (double)palpha[k], cc = (double)pC[k];
            const int sd = pside[k];
            if (!(al >= 0.0) || !(al < HUGE_VAL) || !(cc >= 0.0) || !(cc < HUGE_VAL) || (sd != 1 && sd != -1)) {
                bad = kNcFlagInvalid;
                break;
            }
            A.pmap[2 * k] = mp.n;
            bool ok;
            auto fwd = [&](double lo, double hi, double to) { return mp.add(lo, hi, to); };
            auto mir = [&](double lo, double hi, double to) { return mp.add(-hi, -lo, -to); };
            if (sd > 0) {
                ok = rev ? nc_side(NcRev{cur}, al, cc, *oth, fwd) : nc_side(NcFwd{cur}, al, cc, *oth, fwd);
                rev = false;
            } else {
                ok = rev ? nc_side(NcFwd{cur}, al, cc, *oth, mir) : nc_side(NcRev{cur}, al, cc, *oth, mir);
                rev = true;
            }
            A.pmap[2 * k + 1] = mp.n;
            if (!ok) {
                bad = kNcFlagCapacity;
                break;
            }
            NcBuf *sw = cur;
            cur = oth;
            oth = sw;
        }
        if (bad) break;
        if (rev) {  // store the message forward
            const NcRev r{cur};
            oth->t = r.t();
            for (int64_t k = 0; k < oth->t; ++k) oth->l[k] = r.l(k);
            for (int64_t k = 0; k <= oth->t; ++k) oth->s[k] = r.s(k);
            NcBuf *sw = cur;
            cur = oth;
            oth = sw;
        }
        if (cur != &X) {  // the message becomes X, the other buffer Y
            const NcBuf sw = X;
            X = Y;
            Y = sw;
        }
    }
    if (bad) return bad;
    // the last node: the first breakpoint attaining the minimum of its hat (Y)
    double v = 0.0, vmin = 0.0, y = Y.t > 0 ? Y.l[0] : 0.0;
    for (int64_t k = 1; k < Y.t; ++k) {
        v += Y.s[k] * (Y.l[k] - Y.l[k - 1]);
        if (v < vmin) {
            vmin = v;
            y = Y.l[k];
        }
    }
    x[n1 - 1] = (T)y;
    for (int64_t i = n1 - 2; i >= n0; --i) {
        for (int64_t k = A.poff[i + 1] - 1; k >= A.poff[i]; --k) y = nc_apply(mp, A.pmap[2 * k], A.pmap[2 * k + 1], y);
        x[i] = (T)y;
    }
    return 0;
}

template <class T>
__global__ __launch_bounds__(64) void k_nc_concave(NcgArgs A, const T *__restrict__ ulam,
                                                   const T *__restrict__ uslope, const T *__restrict__ palpha,
                                                   const T *__restrict__ pC, const int32_t *__restrict__ pside,
                                                   T *__restrict__ x, int lanes) {
    if ((int)threadIdx.x >= lanes) return;
    const int64_t c = (int64_t)blockIdx.x * lanes + threadIdx.x;
    if (c >= A.num_chains) return;
    const int64_t bstride = 2 * A.msg_cap + 1;
    double *base = A.bufs + c * 3 * bstride;
    const int bad = ncg_chain_lane<T>(A, ulam, uslope, palpha, pC, pside, x, c,
                                      NcBuf{base, base + A.msg_cap, 0, A.msg_cap},
                                      NcBuf{base + bstride, base + bstride + A.msg_cap, 0, A.msg_cap},
                                      NcBuf{base + 2 * bstride, base + 2 * bstride + A.msg_cap, 0, A.msg_cap});
    if (bad) atomicOr(A.flag, bad);
}

// nc_side spread over a wave: with g = h - alpha x, the prefix minimum m of g
// and its first argmin by a scan; per piece, whether g lies above m + C at its
// two ends, which puts at most one crossing in it (g is linear there and m is
// constant while g is above m + C); the output is flat in g's frame (slope
// alpha) over the runs above m + C, each run mapping to the argmin.  A run is
// closed at its down-crossing (or at +inf) and starts at the latest
// up-crossing, found by a running maximum.  `mirror`: the view is the
// reversal of the function, so intervals are reported mirrored.  Same
// returns as wv_dt.
__device__ int wv_side(const WView &h, double alpha, double C, bool mirror, double *ol, double *os, int cap,
                       const NcMaps &mp, int64_t &nmap, const WScratch &W) {
    const int t = h.t;
    if (t == 0) {
        if (wv_lane() == 0) os[0] = h.s(0);
        __syncthreads();
        return 0;
    }
    wv_values(h, W.V);
    double cv = HUGE_VAL;
    int ci = 0;
    for (int c = 0; c * 64 < t; ++c) {
        const int k = c * 64 + wv_lane();
        double v = (k < t) ? W.V[k] - alpha * h.l(k) : HUGE_VAL;
        int i = k;
        wv_scan_min(v, i);
        if (cv < v || (cv == v && ci < i)) {
            v = cv;
            i = ci;
        }
        if (k < t) {
            W.PM[k] = v;
            W.PA[k] = i;
        }
        cv = __shfl(v, 63, 64);
        ci = __shfl(i, 63, 64);
    }
    __syncthreads();
    // whether g lies above m + C at the start (end) of piece k >= 1
    auto above_l = [&](int k) { return W.V[k - 1] - alpha * h.l(k - 1) > W.PM[k - 1] + C; };
    auto above_r = [&](int k) {
        if (k < t) return W.V[k] - alpha * h.l(k) > W.PM[k - 1] + C;
        const double sg = h.s(t) - alpha;  // the unbounded right piece
        return above_l(k) ? sg >= 0.0 : sg > 0.0;
    };
    for (int k = wv_lane(); k <= t; k += 64) {
        double ps = h.s(0), pe = h.s(0);
        if (k > 0) {
            const double sk = h.s(k);
            ps = above_l(k) ? alpha : sk;
            pe = above_r(k) ? alpha : sk;
        }
        W.PS[k] = ps;
        W.PE[k] = pe;
    }
    __syncthreads();
    int base = 0, ibase = 0;
    bool over = false;
    double start = -HUGE_VAL;  // the latest up-crossing so far
    for (int c = 0; c * 64 < t; ++c) {
        const int k = 1 + c * 64 + wv_lane();
        const bool in = k <= t;
        bool e1 = false, e2 = false, up = false, close = false;
        double y = 0.0, ihi = 0.0, ito = 0.0;
        if (in) {
            e1 = W.PE[k - 1] != W.PS[k];
            const bool al = above_l(k), ar = above_r(k);
            const double L = h.l(k - 1), sg = h.s(k) - alpha;
            if (al != ar) {  // one crossing of m + C in the piece
                y = L + (W.PM[k - 1] + C - (W.V[k - 1] - alpha * L)) / sg;
                if (y < L) y = L;
                if (k < t && y > h.l(k)) y = h.l(k);
                e2 = true;
                up = ar;
                if (al) {
                    close = true;
                    ihi = y;
                } else if (k == t) {  // up in the unbounded piece: above to +inf
                    close = true;
                    ihi = HUGE_VAL;
                }
            } else if (k == t && ar) {
                close = true;  // above to +inf
                ihi = HUGE_VAL;
            }
            if (close) ito = h.l(W.PA[k - 1]);
        }
        double nv = up ? -y : HUGE_VAL;  // running maximum of the up-crossings
        int ni = k;
        wv_scan_min(nv, ni);
        double st = -nv;
        if (start > st) st = start;
        const int cnt = (e1 ? 1 : 0) + (e2 ? 1 : 0);
        const int inc = wv_scan_int(cnt);
        int pos = base + inc - cnt;
        if (e1) {
            if (pos < cap) {
                ol[pos] = h.l(k - 1);
                os[pos + 1] = W.PS[k];
            }
            ++pos;
        }
        if (e2 && pos < cap) {
            ol[pos] = y;
            os[pos + 1] = W.PE[k];
        }
        base += __shfl(inc, 63, 64);
        start = __shfl(st, 63, 64);
        const int iinc = wv_scan_int(close ? 1 : 0);
        const int64_t ipos = nmap + ibase + iinc - 1;
        if (close) {
            if (ipos < mp.cap) {
                if (mirror)
                    mp.put(ipos, -ihi, -st, -ito);
                else
                    mp.put(ipos, st, ihi, ito);
            } else {
                over = true;
            }
        }
        ibase += __shfl(iinc, 63, 64);
    }
    if (wv_lane() == 0) os[0] = W.PS[0];
    nmap += ibase;
    const bool any_over = __ballot(over) != 0;
    __syncthreads();
    if (any_over) return -2;
    return base <= cap ? base : -1;
}

// A wave per chain: k_nc_wave's node loop (Lemma 1 by wv_sum, the next unary
// prefetched into registers) with each edge's pieces applied by wv_side,
// ping-ponging between two LDS buffers; the message is stored forward for the
// next node.  Backward by one lane through every piece's mapping.
template <typename T, int kCap>
__global__ __launch_bounds__(64) void k_nc_wave_concave(NcgArgs A, const T *__restrict__ ulam,
                                                        const T *__restrict__ uslope, const T *__restrict__ palpha,
                                                        const T *__restrict__ pC,
                                                        const int32_t *__restrict__ pside, T *__restrict__ x) {
    static_assert(kCap % 64 == 0 && kCap <= kWaveMsg, "wave message capacity");
    __shared__ double sU_l[kCap], sU_s[kCap + 1];
    __shared__ double sA_l[kCap], sA_s[kCap + 1];
    __shared__ double sB_l[kCap], sB_s[kCap + 1];
    __shared__ double sC_l[kCap], sC_s[kCap + 1];
    __shared__ double sT[2 * kCap], sV[kCap], sPM[kCap], sPS[kCap + 1], sPE[kCap + 1];
    __shared__ int sPA[kCap], sQ0[kCap + 1], sQ1[kCap + 1];
    static_assert(2 * sizeof(int) == sizeof(double), "two counts per double");
    const WScratch W{2 * kCap, sT, (int *)sV, (int *)sPM, sV, sPM, sPA, sPS, sPE, sQ0, sQ1};
    const int64_t c = blockIdx.x;
    if (c >= A.num_chains) return;
    const int64_t n0 = A.coff[c], n1 = A.coff[c + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) {
        if (threadIdx.x == 0) atomicOr(A.flag, kNcFlagInvalid);
        return;
    }
    if (n1 == n0) return;
    const int lane = wv_lane();
    const int cap = (int)(A.msg_cap < kCap ? A.msg_cap : kCap);
    double *mb = A.maps + c * 3 * A.map_cap;
    const NcMaps mp{mb, 0, A.map_cap};
    int64_t nmap = 0;
    int tm = 0, th = 0, bad = 0;
    if (lane == 0) sA_s[0] = 0.0;
    constexpr int kPer = kCap / 64;
    double pl[kPer], ps[kPer + 1];
    auto fetch = [&](int64_t i) {
        const int64_t u0 = A.uoff[i], tu = A.uoff[i + 1] - u0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = lane + 64 * j;
            pl[j] = (k < tu && tu <= cap) ? (double)ulam[u0 + k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j <= kPer; ++j) {
            const int k = lane + 64 * j;
            ps[j] = (k <= tu && tu <= cap) ? (double)uslope[u0 + i + k] : 0.0;
        }
    };
    fetch(n0);
    __syncthreads();
    for (int64_t i = n0; i < n1; ++i) {
        const int64_t u0 = A.uoff[i], tu64 = A.uoff[i + 1] - u0;
        if (tu64 < 1 || tu64 > cap) {
            bad = tu64 < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        const int tu = (int)tu64;
        bool inval = false;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = lane + 64 * j;
            if (k < tu) sU_l[k] = pl[j];
        }
#pragma unroll
        for (int j = 0; j <= kPer; ++j) {
            const int k = lane + 64 * j;
            if (k <= tu) sU_s[k] = ps[j];
        }
        if (i + 1 < n1) fetch(i + 1);
        __syncthreads();
        for (int k = lane; k < tu; k += 64)
            if (k > 0 && !(sU_l[k] >= sU_l[k - 1])) inval = true;
        if (lane == 0 && (!(sU_s[0] <= 0.0) || !(sU_s[tu] >= 0.0))) inval = true;
        if (__ballot(inval) != 0) {
            bad = kNcFlagInvalid;
            break;
        }
        th = wv_sum(sU_l, sU_s, tu, sA_l, sA_s, tm, sB_l, sB_s, cap, W);
        if (th < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        if (i == n1 - 1) break;
        const int64_t k0 = A.poff[i], k1 = A.poff[i + 1];
        if (k0 < 0 || k1 < k0 || k1 > A.num_pieces) {
            bad = kNcFlagInvalid;
            break;
        }
        double *cl = sB_l, *cs = sB_s, *ol = sC_l, *os = sC_s;
        int tc = th;
        bool rev = false;  // the current buffer holds the reversal of the message
        for (int64_t k = k0; k < k1 && !bad; ++k) {
            const double al = (double)palpha[k], cc = (double)pC[k];
            const int sd = pside[k];
            if (!(al >= 0.0) || !(al < HUGE_VAL) || !(cc >= 0.0) || !(cc < HUGE_VAL) || (sd != 1 && sd != -1)) {
                bad = kNcFlagInvalid;
                break;
            }
            if (lane == 0) A.pmap[2 * k] = nmap;
            // right side: the function itself; left side: its reversal
            const bool want_rev = sd < 0;
            const int to = wv_side(WView{cl, cs, tc, rev != want_rev}, al, cc, want_rev, ol, os, cap, mp, nmap, W);
            if (lane == 0) A.pmap[2 * k + 1] = nmap;
            if (to < 0) {
                bad = kNcFlagCapacity;
                break;
            }
            rev = want_rev;
            tc = to;
            double *sw = cl;
            cl = ol;
            ol = sw;
            sw = cs;
            cs = os;
            os = sw;
        }
        if (bad) break;
        const WView fin{cl, cs, tc, rev};  // the message, stored forward in A
        for (int k = lane; k < tc; k += 64) sA_l[k] = fin.l(k);
        for (int k = lane; k <= tc; k += 64) sA_s[k] = fin.s(k);
        tm = tc;
        __syncthreads();
    }
    if (bad) {
        if (lane == 0) atomicOr(A.flag, bad);
        return;
    }
    if (lane != 0) return;
    double v = 0.0, vmin = 0.0, y = th > 0 ? sB_l[0] : 0.0;
    for (int k = 1; k < th; ++k) {
        v += sB_s[k] * (sB_l[k] - sB_l[k - 1]);
        if (v < vmin) {
            vmin = v;
            y = sB_l[k];
        }
    }
    x[n1 - 1] = (T)y;
    for (int64_t i = n1 - 2; i >= n0; --i) {
        for (int64_t k = A.poff[i + 1] - 1; k >= A.poff[i]; --k) y = nc_apply(mp, A.pmap[2 * k], A.pmap[2 * k + 1], y);
        x[i] = (T)y;
    }
}

size_t ncg_layout(int64_t num_chains, int64_t num_pieces, int64_t msg_cap, int64_t map_cap, void *p, NcgArgs *A) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_b = off;  off += al(sizeof(double) * (size_t)(num_chains * 3 * (2 * msg_cap + 1)));
    const size_t o_m = off;  off += al(sizeof(double) * (size_t)(num_chains * 3 * map_cap));
    const size_t o_p = off;  off += al(sizeof(int64_t) * (size_t)(2 * num_pieces));
    const size_t o_f = off;  off += al(sizeof(int));
    if (p && A) {
        char *c = (char *)p;
        A->bufs = (double *)(c + o_b);
        A->maps = (double *)(c + o_m);
        A->pmap = (int64_t *)(c + o_p);
        A->flag = (int *)(c + o_f);
    }
    return off;
}

// The concave pairwise terms on a batch of trees: k_nc_tree's post-order walk
// with its children's messages on a stack, each outgoing message taken through
// the pieces of the edge to the parent (z = x_parent - x_i) by nc_side, and
// pushed onto the stack from its forward or reversed view.
struct NcgTreeArgs {
    NcTreeArgs t;  // eoff unused
    int64_t num_pieces;
    const int64_t *poff;
    int64_t *pmap;  // per piece: its interval range [pmap[2k], pmap[2k + 1])
};

template <typename T>
__global__ __launch_bounds__(64) void k_nc_tree_concave(NcgTreeArgs G, const T *__restrict__ ulam,
                                                        const T *__restrict__ uslope, const T *__restrict__ palpha,
                                                        const T *__restrict__ pC,
                                                        const int32_t *__restrict__ pside, T *__restrict__ x,
                                                        int lanes) {
    const NcTreeArgs &A = G.t;
    if ((int)threadIdx.x >= lanes) return;
    const int64_t tr = (int64_t)blockIdx.x * lanes + threadIdx.x;
    if (tr >= A.num_trees) return;
    const int64_t n0 = A.toff[tr], n1 = A.toff[tr + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) {
        atomicOr(A.flag, kNcFlagInvalid);
        return;
    }
    if (n1 == n0) return;
    const int64_t bstride = 2 * A.msg_cap + 1;
    double *base = A.bufs + tr * 3 * bstride;
    NcBuf H{base, base + A.msg_cap, 0, A.msg_cap};
    NcBuf B{base + bstride, base + bstride + A.msg_cap, 0, A.msg_cap};
    NcBuf U{base + 2 * bstride, base + 2 * bstride + A.msg_cap, 0, A.msg_cap};  // the unary, staged
    double *stk = A.stack + tr * A.stack_cap;
    double *mb = A.maps + tr * 3 * A.map_cap;
    NcMaps mp{mb, 0, A.map_cap};
    int64_t top = 0, sp = n0;
    int bad = 0;
    for (int64_t i = n0; i < n1 && !bad; ++i) {
        const int64_t p = A.parent[i];
        if (p != -1 && (p <= i || p >= n1)) {
            bad = kNcFlagInvalid;
            break;
        }
        const int64_t u0 = A.uoff[i], tu = A.uoff[i + 1] - u0;
        if (tu < 1 || tu > A.msg_cap) {
            bad = tu < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        for (int64_t k = 0; k < tu; ++k) {
            U.l[k] = (double)ulam[u0 + k];
            if (k > 0 && !(U.l[k] >= U.l[k - 1])) bad = kNcFlagInvalid;
        }
        for (int64_t k = 0; k <= tu; ++k) U.s[k] = (double)uslope[u0 + i + k];
        if (!(U.s[0] <= 0.0) || !(U.s[tu] >= 0.0)) bad = kNcFlagInvalid;
        if (bad) break;
        // hat = f_i (+ 0), then + each child's message from the top of the stack
        B.t = 0;
        B.s[0] = 0.0;
        if (!nc_sum(U.l, U.s, tu, B, H)) {
            bad = kNcFlagCapacity;
            break;
        }
        while (sp > n0 && A.hparent[sp - 1] == i) {
            --sp;
            const int64_t cs = A.hstart[sp], ct = A.hcount[sp];
            if (cs < 0 || cs + 2 * ct + 1 != top) {  // not right below: not a post-order numbering
                bad = kNcFlagInvalid;
                break;
            }
            const NcBuf child{stk + cs, stk + cs + ct, ct, ct};
            if (!nc_sum(H.l, H.s, H.t, child, B)) {
                bad = kNcFlagCapacity;
                break;
            }
            const NcBuf t = H;
            H = B;
            B = t;
            top = cs;
        }
        if (bad) break;
        if (p < 0) {  // a root: the first breakpoint attaining the minimum
            double v = 0.0, vmin = 0.0, y = H.t > 0 ? H.l[0] : 0.0;
            for (int64_t k = 1; k < H.t; ++k) {
                v += H.s[k] * (H.l[k] - H.l[k - 1]);
                if (v < vmin) {
                    vmin = v;
                    y = H.l[k];
                }
            }
            x[i] = (T)y;
            continue;
        }
        const int64_t k0 = G.poff[i], k1 = G.poff[i + 1];
        if (k0 < 0 || k1 < k0 || k1 > G.num_pieces) {
            bad = kNcFlagInvalid;
            break;
        }
        NcBuf *cur = &H, *oth = &B;
        bool rev = false;  // cur holds the reversal of the message
        for (int64_t k = k0; k < k1; ++k) {
            const double al = (double)palpha[k], cc = (double)pC[k];
            const int sd = pside[k];
            if (!(al >= 0.0) || !(al < HUGE_VAL) || !(cc >= 0.0) || !(cc < HUGE_VAL) || (sd != 1 && sd != -1)) {
                bad = kNcFlagInvalid;
                break;
            }
            G.pmap[2 * k] = mp.n;
            bool ok;
            auto fwd = [&](double lo, double hi, double to) { return mp.add(lo, hi, to); };
            auto mir = [&](double lo, double hi, double to) { return mp.add(-hi, -lo, -to); };
            if (sd > 0) {
                ok = rev ? nc_side(NcRev{cur}, al, cc, *oth, fwd) : nc_side(NcFwd{cur}, al, cc, *oth, fwd);
                rev = false;
            } else {
                ok = rev ? nc_side(NcFwd{cur}, al, cc, *oth, mir) : nc_side(NcRev{cur}, al, cc, *oth, mir);
                rev = true;
            }
            G.pmap[2 * k + 1] = mp.n;
            if (!ok) {
                bad = kNcFlagCapacity;
                break;
            }
            NcBuf *sw = cur;
            cur = oth;
            oth = sw;
        }
        if (bad) break;
        // push the message (forward) onto the stack: l then s, 2t + 1 doubles
        const int64_t tm = cur->t, need = 2 * tm + 1;
        if (top + need > A.stack_cap) {
            bad = kNcFlagCapacity;
            break;
        }
        if (rev) {
            const NcRev r{cur};
            for (int64_t k = 0; k < tm; ++k) stk[top + k] = r.l(k);
            for (int64_t k = 0; k <= tm; ++k) stk[top + tm + k] = r.s(k);
        } else {
            for (int64_t k = 0; k < tm; ++k) stk[top + k] = cur->l[k];
            for (int64_t k = 0; k <= tm; ++k) stk[top + tm + k] = cur->s[k];
        }
        A.hstart[sp] = top;
        A.hcount[sp] = tm;
        A.hparent[sp] = p;
        ++sp;
        top += need;
    }
    if (!bad && sp != n0) bad = kNcFlagInvalid;  // messages left for parents outside the tree
    if (bad) {
        atomicOr(A.flag, bad);
        return;
    }
    for (int64_t i = n1 - 1; i >= n0; --i) {
        const int64_t p = A.parent[i];
        if (p < 0) continue;
        double y = (double)x[p];
        for (int64_t k = G.poff[i + 1] - 1; k >= G.poff[i]; --k) y = nc_apply(mp, G.pmap[2 * k], G.pmap[2 * k + 1], y);
        x[i] = (T)y;
    }
}

// A wave per tree for the concave pairwise terms (fewer trees than SIMDs):
// k_nc_tree_wave's walk with each edge's pieces applied by wv_side, as in
// k_nc_wave_concave, and the message pushed onto the stack forward.
template <typename T, int kCap>
__global__ __launch_bounds__(64) void k_nc_tree_wave_concave(NcgTreeArgs G, const T *__restrict__ ulam,
                                                             const T *__restrict__ uslope,
                                                             const T *__restrict__ palpha, const T *__restrict__ pC,
                                                             const int32_t *__restrict__ pside, T *__restrict__ x) {
    static_assert(kCap % 64 == 0 && kCap <= kWaveMsg, "wave message capacity");
    __shared__ double sU_l[kCap], sU_s[kCap + 1];
    __shared__ double sA_l[kCap], sA_s[kCap + 1];
    __shared__ double sB_l[kCap], sB_s[kCap + 1];
    __shared__ double sC_l[kCap], sC_s[kCap + 1];
    __shared__ double sT[2 * kCap], sV[kCap], sPM[kCap], sPS[kCap + 1], sPE[kCap + 1];
    __shared__ int sPA[kCap], sQ0[kCap + 1], sQ1[kCap + 1];
    static_assert(2 * sizeof(int) == sizeof(double), "two counts per double");
    const WScratch W{2 * kCap, sT, (int *)sV, (int *)sPM, sV, sPM, sPA, sPS, sPE, sQ0, sQ1};
    const NcTreeArgs &A = G.t;
    const int64_t tr = blockIdx.x;
    if (tr >= A.num_trees) return;
    const int64_t n0 = A.toff[tr], n1 = A.toff[tr + 1];
    if (n0 < 0 || n1 > A.num_nodes || n1 < n0) {
        if (threadIdx.x == 0) atomicOr(A.flag, kNcFlagInvalid);
        return;
    }
    if (n1 == n0) return;
    const int lane = wv_lane();
    const int cap = (int)(A.msg_cap < kCap ? A.msg_cap : kCap);
    double *stk = A.stack + tr * A.stack_cap;
    double *mb = A.maps + tr * 3 * A.map_cap;
    const NcMaps mp{mb, 0, A.map_cap};
    int64_t nmap = 0, top = 0, sp = n0;
    int bad = 0;
    for (int64_t i = n0; i < n1; ++i) {
        const int64_t p = A.parent[i];
        if (p != -1 && (p <= i || p >= n1)) {
            bad = kNcFlagInvalid;
            break;
        }
        const int64_t u0 = A.uoff[i], tu64 = A.uoff[i + 1] - u0;
        if (tu64 < 1 || tu64 > cap) {
            bad = tu64 < 1 ? kNcFlagInvalid : kNcFlagCapacity;
            break;
        }
        const int tu = (int)tu64;
        for (int k = lane; k < tu; k += 64) sU_l[k] = (double)ulam[u0 + k];
        for (int k = lane; k <= tu; k += 64) sU_s[k] = (double)uslope[u0 + i + k];
        if (lane == 0) sA_s[0] = 0.0;  // an empty message
        __syncthreads();
        bool inval = false;
        for (int k = lane; k < tu; k += 64)
            if (k > 0 && !(sU_l[k] >= sU_l[k - 1])) inval = true;
        if (lane == 0 && (!(sU_s[0] <= 0.0) || !(sU_s[tu] >= 0.0))) inval = true;
        if (__ballot(inval) != 0) {
            bad = kNcFlagInvalid;
            break;
        }
        int th = wv_sum(sU_l, sU_s, tu, sA_l, sA_s, 0, sB_l, sB_s, cap, W);
        if (th < 0) {
            bad = kNcFlagCapacity;
            break;
        }
        double *cl = sB_l, *cs = sB_s, *ol = sC_l, *os = sC_s;
        while (sp > n0 && A.hparent[sp - 1] == i) {
            --sp;
            const int64_t hs0 = A.hstart[sp], ct = A.hcount[sp];
            if (hs0 < 0 || ct < 0 || ct > cap || hs0 + 2 * ct + 1 != top) {
                bad = kNcFlagInvalid;
                break;
            }
            const int tn = wv_sum(cl, cs, th, stk + hs0, stk + hs0 + ct, (int)ct, ol, os, cap, W);
            if (tn < 0) {
                bad = kNcFlagCapacity;
                break;
            }
            double *sw = cl;
            cl = ol;
            ol = sw;
            sw = cs;
            cs = os;
            os = sw;
            th = tn;
            top = hs0;
        }
        if (bad) break;
        if (p < 0) {  // a root: the first breakpoint attaining the minimum
            if (lane == 0) {
                double v = 0.0, vmin = 0.0, y = th > 0 ? cl[0] : 0.0;
                for (int k = 1; k < th; ++k) {
                    v += cs[k] * (cl[k] - cl[k - 1]);
                    if (v < vmin) {
                        vmin = v;
                        y = cl[k];
                    }
                }
                x[i] = (T)y;
            }
            __syncthreads();
            continue;
        }
        const int64_t k0 = G.poff[i], k1 = G.poff[i + 1];
        if (k0 < 0 || k1 < k0 || k1 > G.num_pieces) {
            bad = kNcFlagInvalid;
            break;
        }
        int tc = th;
        bool rev = false;  // the current buffer holds the reversal of the message
        for (int64_t k = k0; k < k1 && !bad; ++k) {
            const double al = (double)palpha[k], cc = (double)pC[k];
            const int sd = pside[k];
            if (!(al >= 0.0) || !(al < HUGE_VAL) || !(cc >= 0.0) || !(cc < HUGE_VAL) || (sd != 1 && sd != -1)) {
                bad = kNcFlagInvalid;
                break;
            }
            if (lane == 0) G.pmap[2 * k] = nmap;
            const bool want_rev = sd < 0;
            const int to = wv_side(WView{cl, cs, tc, rev != want_rev}, al, cc, want_rev, ol, os, cap, mp, nmap, W);
            if (lane == 0) G.pmap[2 * k + 1] = nmap;
            if (to < 0) {
                bad = kNcFlagCapacity;
                break;
            }
            rev = want_rev;
            tc = to;
            double *sw = cl;
            cl = ol;
            ol = sw;
            sw = cs;
            cs = os;
            os = sw;
        }
        if (bad) break;
        const int64_t need = 2 * (int64_t)tc + 1;
        if (top + need > A.stack_cap) {
            bad = kNcFlagCapacity;
            break;
        }
        const WView fin{cl, cs, tc, rev};  // pushed forward
        for (int k = lane; k < tc; k += 64) stk[top + k] = fin.l(k);
        for (int k = lane; k <= tc; k += 64) stk[top + tc + k] = fin.s(k);
        A.hstart[sp] = top;
        A.hcount[sp] = tc;
        A.hparent[sp] = p;
        ++sp;
        top += need;
        __syncthreads();
    }
    if (!bad && sp != n0) bad = kNcFlagInvalid;
    if (bad) {
        if (lane == 0) atomicOr(A.flag, bad);
        return;
    }
    if (lane != 0) return;
    for (int64_t i = n1 - 1; i >= n0; --i) {
        const int64_t p = A.parent[i];
        if (p < 0) continue;
        double y = (double)x[p];
        for (int64_t k = G.poff[i + 1] - 1; k >= G.poff[i]; --k) y = nc_apply(mp, G.pmap[2 * k], G.pmap[2 * k + 1], y);
        x[i] = (T)y;
    }
}

size_t ncg_tree_layout(int64_t num_trees, int64_t num_nodes, int64_t num_pieces, int64_t msg_cap, int64_t map_cap,
                       int64_t stack_cap, void *p, NcgTreeArgs *G) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_b = off;  off += al(sizeof(double) * (size_t)(num_trees * 3 * (2 * msg_cap + 1)));
    const size_t o_s = off;  off += al(sizeof(double) * (size_t)(num_trees * stack_cap));
    const size_t o_m = off;  off += al(sizeof(double) * (size_t)(num_trees * 3 * map_cap));
    const size_t o_h = off;  off += al(sizeof(int64_t) * (size_t)(3 * num_nodes));
    const size_t o_p = off;  off += al(sizeof(int64_t) * (size_t)(2 * num_pieces));
    const size_t o_f = off;  off += al(sizeof(int));
    if (p && G) {
        char *c = (char *)p;
        G->t.bufs = (double *)(c + o_b);
        G->t.stack = (double *)(c + o_s);
        G->t.maps = (double *)(c + o_m);
        int64_t *h = (int64_t *)(c + o_h);
        G->t.hstart = h;
        G->t.hcount = h + num_nodes;
        G->t.hparent = h + 2 * num_nodes;
        G->t.eoff = nullptr;
        G->pmap = (int64_t *)(c + o_p);
        G->t.flag = (int *)(c + o_f);
    }
    return off;
}

tv_status nc_finish(int *dflag, hipStream_t stream) {
    if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
    int flag = 0;
    if (hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess) return TV_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return TV_ERR_HIP;
    if (flag & kNcFlagInvalid) return TV_ERR_INVALID_ARG;
    if (flag & kNcFlagCapacity) return TV_ERR_WORKSPACE;
    return TV_OK;
}

}  // namespace
}  // namespace tvc

using namespace tvc;

extern "C" {

size_t tv_chain_nc_workspace(int64_t num_chains, int64_t num_nodes, int64_t msg_cap, int64_t map_cap) {
    if (num_chains < 0 || num_nodes < 0 || msg_cap < 1 || map_cap < 1) return 0;
    if (msg_cap > (int64_t(1) << 24) || map_cap > (int64_t(1) << 30)) return 0;
    return nc_layout(num_chains, num_nodes, msg_cap, map_cap, nullptr, nullptr);
}

tv_status tv_chain_nc(tv_dtype dtype, int64_t num_chains, int64_t num_nodes, const int64_t *chain_offsets,
                      const int64_t *unary_offsets, const void *ulam, const void *uslope, const void *w,
                      const void *C, void *x, int64_t msg_cap, int64_t map_cap, void *workspace,
                      size_t workspace_bytes, hipStream_t stream) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (num_chains < 0 || num_nodes < 0) return TV_ERR_INVALID_ARG;
    if (num_chains >= (int64_t(1) << 31)) return TV_ERR_INVALID_ARG;  // one workgroup per chain at most
    if (num_chains == 0) return TV_OK;
    if (!chain_offsets || !unary_offsets || !ulam || !uslope || !w || !x) return TV_ERR_INVALID_ARG;
    const size_t need = tv_chain_nc_workspace(num_chains, num_nodes, msg_cap, map_cap);
    if (need == 0) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return TV_ERR_WORKSPACE;
    NcArgs A;
    A.num_chains = num_chains;
    A.num_nodes = num_nodes;
    A.coff = chain_offsets;
    A.uoff = unary_offsets;
    A.msg_cap = msg_cap;
    A.map_cap = map_cap;
    nc_layout(num_chains, num_nodes, msg_cap, map_cap, workspace, &A);
    if (hipMemsetAsync(A.flag, 0, sizeof(int), stream) != hipSuccess) return TV_ERR_HIP;
    if (msg_cap <= kWaveMsg) {  // a wave per chain
        const dim3 gw((unsigned)num_chains);
        if (dtype == TV_F32) {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_wave<float, 128>), gw, dim3(64), 0, stream, A, (const float *)ulam,
                                   (const float *)uslope, (const float *)w, (const float *)C, (float *)x);
            else
                hipLaunchKernelGGL((k_nc_wave<float, kWaveMsg>), gw, dim3(64), 0, stream, A, (const float *)ulam,
                                   (const float *)uslope, (const float *)w, (const float *)C, (float *)x);
        } else {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_wave<double, 128>), gw, dim3(64), 0, stream, A, (const double *)ulam,
                                   (const double *)uslope, (const double *)w, (const double *)C, (double *)x);
            else
                hipLaunchKernelGGL((k_nc_wave<double, kWaveMsg>), gw, dim3(64), 0, stream, A, (const double *)ulam,
                                   (const double *)uslope, (const double *)w, (const double *)C, (double *)x);
        }
        return nc_finish(A.flag, stream);
    }
    int ll = nc_lds_lanes(msg_cap);
    if (ll > 0) {  // allow the kernel more than the default 64 KiB of dynamic LDS
        const int bytes = (int)(sizeof(double) * 3 * (size_t)(2 * msg_cap + 1) * (size_t)ll);
        const hipError_t e = (dtype == TV_F32)
                                 ? hipFuncSetAttribute((const void *)k_nc_chain<float, true>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
                                 : hipFuncSetAttribute((const void *)k_nc_chain<double, true>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ll = 0;
        }
    }
    if (ll == 0 && nc_lds_lanes(msg_cap) > 0) return TV_ERR_HIP;  // the workspace holds no HBM buffers
    // Spread the chains over the 1024 SIMDs before packing them into waves: a
    // lane's work is a serial, branchy walk, so lanes sharing a wave mostly wait
    // for each other.
    const int64_t spread = (num_chains + 1023) / 1024;
    int lanes = ll > 0 ? ll : 64;
    if (spread < lanes) lanes = (int)(spread < 1 ? 1 : spread);
    const dim3 grid((unsigned)((num_chains + lanes - 1) / lanes));
    const size_t lds = ll > 0 ? sizeof(double) * 3 * (size_t)(2 * msg_cap + 1) * (size_t)lanes : 0;
    if (dtype == TV_F32) {
        if (ll > 0)
            hipLaunchKernelGGL((k_nc_chain<float, true>), grid, dim3(64), lds, stream, A, (const float *)ulam,
                               (const float *)uslope, (const float *)w, (const float *)C, (float *)x, lanes);
        else
            hipLaunchKernelGGL((k_nc_chain<float, false>), grid, dim3(64), 0, stream, A, (const float *)ulam,
                               (const float *)uslope, (const float *)w, (const float *)C, (float *)x, lanes);
    } else {
        if (ll > 0)
            hipLaunchKernelGGL((k_nc_chain<double, true>), grid, dim3(64), lds, stream, A, (const double *)ulam,
                               (const double *)uslope, (const double *)w, (const double *)C, (double *)x, lanes);
        else
            hipLaunchKernelGGL((k_nc_chain<double, false>), grid, dim3(64), 0, stream, A, (const double *)ulam,
                               (const double *)uslope, (const double *)w, (const double *)C, (double *)x, lanes);
    }
    return nc_finish(A.flag, stream);
}

}  // extern "C"

extern "C" {

size_t tv_tree_nc_workspace(int64_t num_trees, int64_t num_nodes, int64_t msg_cap, int64_t map_cap,
                            int64_t stack_cap) {
    if (num_trees < 0 || num_nodes < 0 || msg_cap < 1 || map_cap < 1 || stack_cap < 1) return 0;
    if (msg_cap > (int64_t(1) << 24) || map_cap > (int64_t(1) << 30) || stack_cap > (int64_t(1) << 34)) return 0;
    return nc_tree_layout(num_trees, num_nodes, msg_cap, map_cap, stack_cap, nullptr, nullptr);
}

tv_status tv_tree_nc(tv_dtype dtype, int64_t num_trees, int64_t num_nodes, const int64_t *tree_offsets,
                     const int64_t *parent, const int64_t *unary_offsets, const void *ulam, const void *uslope,
                     const void *w, const void *C, void *x, int64_t msg_cap, int64_t map_cap, int64_t stack_cap,
                     void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (num_trees < 0 || num_nodes < 0 || num_trees >= (int64_t(1) << 31)) return TV_ERR_INVALID_ARG;
    if (num_trees == 0) return TV_OK;
    if (!tree_offsets || !parent || !unary_offsets || !ulam || !uslope || !w || !x) return TV_ERR_INVALID_ARG;
    const size_t need = tv_tree_nc_workspace(num_trees, num_nodes, msg_cap, map_cap, stack_cap);
    if (need == 0) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return TV_ERR_WORKSPACE;
    NcTreeArgs A;
    A.num_trees = num_trees;
    A.num_nodes = num_nodes;
    A.toff = tree_offsets;
    A.parent = parent;
    A.uoff = unary_offsets;
    A.msg_cap = msg_cap;
    A.map_cap = map_cap;
    A.stack_cap = stack_cap;
    nc_tree_layout(num_trees, num_nodes, msg_cap, map_cap, stack_cap, workspace, &A);
    if (hipMemsetAsync(A.flag, 0, sizeof(int), stream) != hipSuccess) return TV_ERR_HIP;
    if (num_trees < 1024 && msg_cap <= kWaveMsg) {  // fewer trees than SIMDs: a wave per tree
        const dim3 gw((unsigned)num_trees);
        if (dtype == TV_F32) {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_tree_wave<float, 128>), gw, dim3(64), 0, stream, A, (const float *)ulam,
                                   (const float *)uslope, (const float *)w, (const float *)C, (float *)x);
            else
                hipLaunchKernelGGL((k_nc_tree_wave<float, kWaveMsg>), gw, dim3(64), 0, stream, A,
                                   (const float *)ulam, (const float *)uslope, (const float *)w, (const float *)C,
                                   (float *)x);
        } else {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_tree_wave<double, 128>), gw, dim3(64), 0, stream, A,
                                   (const double *)ulam, (const double *)uslope, (const double *)w,
                                   (const double *)C, (double *)x);
            else
                hipLaunchKernelGGL((k_nc_tree_wave<double, kWaveMsg>), gw, dim3(64), 0, stream, A,
                                   (const double *)ulam, (const double *)uslope, (const double *)w,
                                   (const double *)C, (double *)x);
        }
        return nc_finish(A.flag, stream);
    }
    // Each lane walks its tree serially, so spread the trees over at least
    // 1024 waves (one per SIMD) before packing 64 into a wave.
    const int64_t spread = (num_trees + 1023) / 1024;
    const int lanes = spread < 64 ? (int)spread : 64;
    const dim3 grid((unsigned)((num_trees + lanes - 1) / lanes));
    if (dtype == TV_F32)
        hipLaunchKernelGGL((k_nc_tree<float>), grid, dim3(64), 0, stream, A, (const float *)ulam,
                           (const float *)uslope, (const float *)w, (const float *)C, (float *)x, lanes);
    else
        hipLaunchKernelGGL((k_nc_tree<double>), grid, dim3(64), 0, stream, A, (const double *)ulam,
                           (const double *)uslope, (const double *)w, (const double *)C, (double *)x, lanes);
    return nc_finish(A.flag, stream);
}

size_t tv_chain_nc_concave_workspace(int64_t num_chains, int64_t num_nodes, int64_t num_pieces, int64_t msg_cap,
                                     int64_t map_cap) {
    if (num_chains < 0 || num_nodes < 0 || num_pieces < 0 || msg_cap < 1 || map_cap < 1) return 0;
    if (msg_cap > (int64_t(1) << 24) || map_cap > (int64_t(1) << 30)) return 0;
    return ncg_layout(num_chains, num_pieces, msg_cap, map_cap, nullptr, nullptr);
}

tv_status tv_chain_nc_concave(tv_dtype dtype, int64_t num_chains, int64_t num_nodes, int64_t num_pieces,
                              const int64_t *chain_offsets, const int64_t *unary_offsets, const void *ulam,
                              const void *uslope, const int64_t *piece_offsets, const void *piece_alpha,
                              const void *piece_C, const int32_t *piece_side, void *x, int64_t msg_cap,
                              int64_t map_cap, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (num_chains < 0 || num_nodes < 0 || num_pieces < 0 || num_chains >= (int64_t(1) << 31))
        return TV_ERR_INVALID_ARG;
    if (num_chains == 0) return TV_OK;
    if (!chain_offsets || !unary_offsets || !ulam || !uslope || !piece_offsets || !x) return TV_ERR_INVALID_ARG;
    if (num_pieces > 0 && (!piece_alpha || !piece_C || !piece_side)) return TV_ERR_INVALID_ARG;
    const size_t need = tv_chain_nc_concave_workspace(num_chains, num_nodes, num_pieces, msg_cap, map_cap);
    if (need == 0) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return TV_ERR_WORKSPACE;
    NcgArgs A;
    A.num_chains = num_chains;
    A.num_nodes = num_nodes;
    A.num_pieces = num_pieces;
    A.coff = chain_offsets;
    A.uoff = unary_offsets;
    A.poff = piece_offsets;
    A.msg_cap = msg_cap;
    A.map_cap = map_cap;
    ncg_layout(num_chains, num_pieces, msg_cap, map_cap, workspace, &A);
    if (hipMemsetAsync(A.flag, 0, sizeof(int), stream) != hipSuccess) return TV_ERR_HIP;
    if (msg_cap <= kWaveMsg) {  // a wave per chain, messages in LDS
        const dim3 gw((unsigned)num_chains);
        if (dtype == TV_F32) {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_wave_concave<float, 128>), gw, dim3(64), 0, stream, A, (const float *)ulam,
                                   (const float *)uslope, (const float *)piece_alpha, (const float *)piece_C,
                                   piece_side, (float *)x);
            else
                hipLaunchKernelGGL((k_nc_wave_concave<float, kWaveMsg>), gw, dim3(64), 0, stream, A,
                                   (const float *)ulam, (const float *)uslope, (const float *)piece_alpha,
                                   (const float *)piece_C, piece_side, (float *)x);
        } else {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_wave_concave<double, 128>), gw, dim3(64), 0, stream, A,
                                   (const double *)ulam, (const double *)uslope, (const double *)piece_alpha,
                                   (const double *)piece_C, piece_side, (double *)x);
            else
                hipLaunchKernelGGL((k_nc_wave_concave<double, kWaveMsg>), gw, dim3(64), 0, stream, A,
                                   (const double *)ulam, (const double *)uslope, (const double *)piece_alpha,
                                   (const double *)piece_C, piece_side, (double *)x);
        }
        return nc_finish(A.flag, stream);
    }
    const int64_t spread = (num_chains + 1023) / 1024;
    const int lanes = spread < 64 ? (int)spread : 64;
    const dim3 grid((unsigned)((num_chains + lanes - 1) / lanes));
    if (dtype == TV_F32)
        hipLaunchKernelGGL((k_nc_concave<float>), grid, dim3(64), 0, stream, A, (const float *)ulam,
                           (const float *)uslope, (const float *)piece_alpha, (const float *)piece_C, piece_side,
                           (float *)x, lanes);
    else
        hipLaunchKernelGGL((k_nc_concave<double>), grid, dim3(64), 0, stream, A, (const double *)ulam,
                           (const double *)uslope, (const double *)piece_alpha, (const double *)piece_C, piece_side,
                           (double *)x, lanes);
    return nc_finish(A.flag, stream);
}

size_t tv_tree_nc_concave_workspace(int64_t num_trees, int64_t num_nodes, int64_t num_pieces, int64_t msg_cap,
                                    int64_t map_cap, int64_t stack_cap) {
    if (num_trees < 0 || num_nodes < 0 || num_pieces < 0 || msg_cap < 1 || map_cap < 1 || stack_cap < 1) return 0;
    if (msg_cap > (int64_t(1) << 24) || map_cap > (int64_t(1) << 30) || stack_cap > (int64_t(1) << 34)) return 0;
    return ncg_tree_layout(num_trees, num_nodes, num_pieces, msg_cap, map_cap, stack_cap, nullptr, nullptr);
}

tv_status tv_tree_nc_concave(tv_dtype dtype, int64_t num_trees, int64_t num_nodes, int64_t num_pieces,
                             const int64_t *tree_offsets, const int64_t *parent, const int64_t *unary_offsets,
                             const void *ulam, const void *uslope, const int64_t *piece_offsets,
                             const void *piece_alpha, const void *piece_C, const int32_t *piece_side, void *x,
                             int64_t msg_cap, int64_t map_cap, int64_t stack_cap, void *workspace,
                             size_t workspace_bytes, hipStream_t stream) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (num_trees < 0 || num_nodes < 0 || num_pieces < 0 || num_trees >= (int64_t(1) << 31))
        return TV_ERR_INVALID_ARG;
    if (num_trees == 0) return TV_OK;
    if (!tree_offsets || !parent || !unary_offsets || !ulam || !uslope || !piece_offsets || !x)
        return TV_ERR_INVALID_ARG;
    if (num_pieces > 0 && (!piece_alpha || !piece_C || !piece_side)) return TV_ERR_INVALID_ARG;
    const size_t need = tv_tree_nc_concave_workspace(num_trees, num_nodes, num_pieces, msg_cap, map_cap, stack_cap);
    if (need == 0) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return TV_ERR_WORKSPACE;
    NcgTreeArgs G;
    G.t.num_trees = num_trees;
    G.t.num_nodes = num_nodes;
    G.t.toff = tree_offsets;
    G.t.parent = parent;
    G.t.uoff = unary_offsets;
    G.t.msg_cap = msg_cap;
    G.t.map_cap = map_cap;
    G.t.stack_cap = stack_cap;
    G.num_pieces = num_pieces;
    G.poff = piece_offsets;
    ncg_tree_layout(num_trees, num_nodes, num_pieces, msg_cap, map_cap, stack_cap, workspace, &G);
    if (hipMemsetAsync(G.t.flag, 0, sizeof(int), stream) != hipSuccess) return TV_ERR_HIP;
    if (num_trees < 1024 && msg_cap <= kWaveMsg) {  // fewer trees than SIMDs: a wave per tree
        const dim3 gw((unsigned)num_trees);
        if (dtype == TV_F32) {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_tree_wave_concave<float, 128>), gw, dim3(64), 0, stream, G,
                                   (const float *)ulam, (const float *)uslope, (const float *)piece_alpha,
                                   (const float *)piece_C, piece_side, (float *)x);
            else
                hipLaunchKernelGGL((k_nc_tree_wave_concave<float, kWaveMsg>), gw, dim3(64), 0, stream, G,
                                   (const float *)ulam, (const float *)uslope, (const float *)piece_alpha,
                                   (const float *)piece_C, piece_side, (float *)x);
        } else {
            if (msg_cap <= 128)
                hipLaunchKernelGGL((k_nc_tree_wave_concave<double, 128>), gw, dim3(64), 0, stream, G,
                                   (const double *)ulam, (const double *)uslope, (const double *)piece_alpha,
                                   (const double *)piece_C, piece_side, (double *)x);
            else
                hipLaunchKernelGGL((k_nc_tree_wave_concave<double, kWaveMsg>), gw, dim3(64), 0, stream, G,
                                   (const double *)ulam, (const double *)uslope, (const double *)piece_alpha,
                                   (const double *)piece_C, piece_side, (double *)x);
        }
        return nc_finish(G.t.flag, stream);
    }
    const int64_t spread = (num_trees + 1023) / 1024;
    const int lanes = spread < 64 ? (int)spread : 64;
    const dim3 grid((unsigned)((num_trees + lanes - 1) / lanes));
    if (dtype == TV_F32)
        hipLaunchKernelGGL((k_nc_tree_concave<float>), grid, dim3(64), 0, stream, G, (const float *)ulam,
                           (const float *)uslope, (const float *)piece_alpha, (const float *)piece_C, piece_side,
                           (float *)x, lanes);
    else
        hipLaunchKernelGGL((k_nc_tree_concave<double>), grid, dim3(64), 0, stream, G, (const double *)ulam,
                           (const double *)uslope, (const double *)piece_alpha, (const double *)piece_C, piece_side,
                           (double *)x, lanes);
    return nc_finish(G.t.flag, stream);
}

}  // extern "C"
