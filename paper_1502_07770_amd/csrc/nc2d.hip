// nc2d.hip -- Sec. 5.3: truncated TV with non-convex piecewise-linear unaries
// on an H x W grid,
//
//     min_x  sum_{horizontal (i,j)} min(w_ij |x_i - x_j|, C) + sum_{vertical} ... + sum_i f_i(x_i),
//
// f_i piecewise-linear through the costs cost[i][k] at the levels d0 + k dd
// (slopes -steep / +steep outside), by the Lagrangian splitting
// Psi_h(x_h) + Psi_v(x_v) + <x_h - x_v, y>, Psi = TV^C + f / 2, and the
// primal-dual iteration
//     x_h <- prox_{tau Psi_h}(x_h - tau ybar),  x_v <- prox_{tau Psi_v}(x_v + tau ybar),
//     y <- y + sigma (x_h - x_v),  ybar <- 2 y_new - y_old,
// tau_k = tau0 / k, sigma_k = 1 / (2 tau_k) (L^2 = 2), theta = 1.  Each prox is
// the exact minimiser over every row (column) chain of Psi plus the
// piecewise-linear interpolant of |x - z|^2 / (2 tau) on the cost levels: a
// kernel forms those unaries (FP64) and one tv_chain_nc launch solves the H
// row and W column chains together (both prox steps read only the previous
// iterate).  Nodes 0..N-1 are the rows (row-major), N..2N-1 the columns
// (column-major, x_v kept in that order), so every chain is contiguous.  Starts
// from the per-pixel minimiser of f with y = 0.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tvchain.h"

namespace tvc {
namespace {

struct Nc2dWs {
    double *xh, *xv, *y, *ybar;  // [N]; xv column-major, right after xh (the chains' output)
    double *ulam, *uslope;       // [2N D], [2N (D + 1)]
    double *wr, *wc, *cc;        // [N] row, [N] column edge weights (adjacent), [2N] C
    int64_t *coff, *uoff;        // [H + W + 1] chain ranges, [2N + 1]
    void *chain_ws;
    size_t chain_bytes;
};

template <typename T>
__global__ __launch_bounds__(256) void k_nc2d_setup(Nc2dWs ws, const T *__restrict__ cost, int64_t H, int64_t W,
                                                    int64_t D, double d0, double dd, const T *__restrict__ w_h,
                                                    double whs, const T *__restrict__ w_v, double wvs, double C) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t N = H * W;
    if (i <= H) ws.coff[i] = i * W;
    if (i >= 1 && i <= W) ws.coff[H + i] = N + i * H;
    if (i > 2 * N) return;
    ws.uoff[i] = i * D;
    if (i >= N) return;
    const int64_t r = i / W, c = i % W;
    const T *cr = cost + i * D;
    int64_t kb = 0;
    double vb = (double)cr[0];
    for (int64_t k = 1; k < D; ++k) {
        const double v = (double)cr[k];
        if (v < vb) {
            vb = v;
            kb = k;
        }
    }
    const double x0 = d0 + (double)kb * dd;
    ws.xh[i] = x0;
    ws.xv[c * H + r] = x0;
    ws.y[i] = 0.0;
    ws.ybar[i] = 0.0;
    ws.wr[i] = (c + 1 < W) ? (w_h ? (double)w_h[r * (W - 1) + c] : whs) : 0.0;
    ws.wc[c * H + r] = (r + 1 < H) ? (w_v ? (double)w_v[r * W + c] : wvs) : 0.0;
    ws.cc[i] = C;
    ws.cc[N + i] = C;
}

// Unaries of the prox steps: f / 2 plus the interpolant of |x - z|^2 / (2 tau)
// on the levels; z = x_h - tau ybar for the row nodes (0..N-1, row-major),
// z = x_v + tau ybar for the column nodes (N..2N-1, column-major).  One thread
// per slope (node, k), so the slope array is written contiguously.
template <typename T>
__global__ __launch_bounds__(256) void k_nc2d_unary(Nc2dWs ws, const T *__restrict__ cost, int64_t H, int64_t W,
                                                    int64_t D, double d0, double dd, double steep, double tau) {
    const int64_t N = H * W;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= 2 * N * (D + 1)) return;
    const int64_t node = j / (D + 1), k = j % (D + 1);
    const bool horizontal = node < N;
    const int64_t q = horizontal ? node : node - N;
    int64_t r, c;
    if (horizontal) {
        r = q / W;
        c = q % W;
    } else {
        c = q / H;
        r = q % H;
    }
    const int64_t i = r * W + c;
    const double xs = horizontal ? ws.xh[i] : ws.xv[q];
    const double z = xs + (horizontal ? -tau : tau) * ws.ybar[i];
    double v;
    if (k == 0) {
        v = -0.5 * steep + (d0 - z) / tau;
        v = v < 0.0 ? v : 0.0;
    } else if (k == D) {
        v = 0.5 * steep + (d0 + (double)(D - 1) * dd - z) / tau;
        v = v > 0.0 ? v : 0.0;
    } else {
        const T *cr = cost + i * D;
        const double la = d0 + (double)(k - 1) * dd, lb = d0 + (double)k * dd;
        v = 0.5 * ((double)cr[k] - (double)cr[k - 1]) / dd + (la + lb - 2.0 * z) / (2.0 * tau);
    }
    ws.uslope[j] = v;
}

// The levels of every node (the same for rows and columns), one thread per entry.
__global__ __launch_bounds__(256) void k_nc2d_levels(double *ulam, int64_t total, int64_t D, double d0, double dd) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < total) ulam[j] = d0 + (double)(j % D) * dd;
}

__global__ __launch_bounds__(256) void k_nc2d_update(Nc2dWs ws, int64_t H, int64_t W, double sigma) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= H * W) return;
    const int64_t r = i / W, c = i % W;
    const double yo = ws.y[i];
    const double yn = yo + sigma * (ws.xh[i] - ws.xv[c * H + r]);
    ws.ybar[i] = 2.0 * yn - yo;
    ws.y[i] = yn;
}

template <typename T>
__global__ __launch_bounds__(256) void k_nc2d_out(const double *__restrict__ xh, T *__restrict__ x, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < N) x[i] = (T)xh[i];
}

size_t nc2d_layout(int64_t H, int64_t W, int64_t D, int64_t msg_cap, int64_t map_cap, void *p, Nc2dWs *out) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t N = H * W;
    const size_t cw = tv_chain_nc_workspace(H + W, 2 * N, msg_cap, map_cap);
    if (cw == 0) return 0;
    size_t off = 0;
    const size_t o_x = off;   off += al(sizeof(double) * (size_t)(4 * N));
    const size_t o_l = off;   off += al(sizeof(double) * (size_t)(2 * N * D));
    const size_t o_s = off;   off += al(sizeof(double) * (size_t)(2 * N * (D + 1)));
    const size_t o_w = off;   off += al(sizeof(double) * (size_t)(4 * N));
    const size_t o_o = off;   off += al(sizeof(int64_t) * (size_t)(H + W + 1 + 2 * N + 1));
    const size_t o_c = off;   off += al(cw);
    if (p && out) {
        char *b = (char *)p;
        double *x = (double *)(b + o_x);
        out->xh = x;
        out->xv = x + N;
        out->y = x + 2 * N;
        out->ybar = x + 3 * N;
        out->ulam = (double *)(b + o_l);
        out->uslope = (double *)(b + o_s);
        double *w = (double *)(b + o_w);
        out->wr = w;
        out->wc = w + N;
        out->cc = w + 2 * N;
        int64_t *o = (int64_t *)(b + o_o);
        out->coff = o;
        out->uoff = o + H + W + 1;
        out->chain_ws = b + o_c;
        out->chain_bytes = cw;
    }
    return off;
}

}  // namespace
}  // namespace tvc

using namespace tvc;

extern "C" {

size_t tv2d_nc_workspace(int64_t H, int64_t W, int64_t D, int64_t msg_cap, int64_t map_cap) {
    if (H < 1 || W < 1 || D < 2 || msg_cap < D || map_cap < 1) return 0;
    if (H > (int64_t(1) << 20) || W > (int64_t(1) << 20) || D > (int64_t(1) << 16)) return 0;
    return nc2d_layout(H, W, D, msg_cap, map_cap, nullptr, nullptr);
}

tv_status tv2d_nc_solve(tv_dtype dtype, const void *cost, int64_t H, int64_t W, int64_t D, double d0, double dd,
                        double steep, const void *w_h, double w_h_scalar, const void *w_v, double w_v_scalar,
                        double C, double tau0, int iters, void *x, int64_t msg_cap, int64_t map_cap,
                        void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (!cost || !x || iters < 0) return TV_ERR_INVALID_ARG;
    if (!(dd > 0.0) || !std::isfinite(dd) || !std::isfinite(d0) || !(steep > 0.0) || !std::isfinite(steep))
        return TV_ERR_INVALID_ARG;
    if (!(tau0 > 0.0) || !std::isfinite(tau0) || !(C > 0.0)) return TV_ERR_INVALID_ARG;
    if (!w_h && !(w_h_scalar >= 0.0 && std::isfinite(w_h_scalar))) return TV_ERR_INVALID_ARG;
    if (!w_v && !(w_v_scalar >= 0.0 && std::isfinite(w_v_scalar))) return TV_ERR_INVALID_ARG;
    const size_t need = tv2d_nc_workspace(H, W, D, msg_cap, map_cap);
    if (need == 0) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return TV_ERR_WORKSPACE;
    Nc2dWs ws;
    nc2d_layout(H, W, D, msg_cap, map_cap, workspace, &ws);
    const int64_t N = H * W;
    const dim3 blk(256);
    const dim3 g1((unsigned)((2 * N + 1 + 255) / 256 + ((H > W ? H : W) + 256) / 256));
    const dim3 gN((unsigned)((N + 255) / 256));
    if (dtype == TV_F32)
        hipLaunchKernelGGL((k_nc2d_setup<float>), g1, blk, 0, stream, ws, (const float *)cost, H, W, D, d0, dd,
                           (const float *)w_h, w_h_scalar, (const float *)w_v, w_v_scalar, C);
    else
        hipLaunchKernelGGL((k_nc2d_setup<double>), g1, blk, 0, stream, ws, (const double *)cost, H, W, D, d0, dd,
                           (const double *)w_h, w_h_scalar, (const double *)w_v, w_v_scalar, C);
    if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
    hipLaunchKernelGGL(k_nc2d_levels, dim3((unsigned)((2 * N * D + 255) / 256)), blk, 0, stream, ws.ulam,
                       2 * N * D, D, d0, dd);
    if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
    const dim3 gS((unsigned)((2 * N * (D + 1) + 255) / 256));
    const double *cc = std::isfinite(C) ? ws.cc : nullptr;
    for (int k = 1; k <= iters; ++k) {
        const double tau = tau0 / k, sigma = 1.0 / (2.0 * tau);
        if (dtype == TV_F32)
            hipLaunchKernelGGL((k_nc2d_unary<float>), gS, blk, 0, stream, ws, (const float *)cost, H, W, D, d0, dd,
                               steep, tau);
        else
            hipLaunchKernelGGL((k_nc2d_unary<double>), gS, blk, 0, stream, ws, (const double *)cost, H, W, D, d0,
                               dd, steep, tau);
        if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
        // rows and columns in one launch; x_h then x_v (column-major) are the
        // output.  Messages of at most 128 breakpoints let twice as many waves
        // share a CU: that capacity first, the caller's if a message outgrows it
        // (the chain workspace does not depend on it for msg_cap <= 256).
        const int64_t first = msg_cap > 128 && msg_cap <= 256 ? 128 : msg_cap;
        tv_status st = tv_chain_nc(TV_F64, H + W, 2 * N, ws.coff, ws.uoff, ws.ulam, ws.uslope, ws.wr, cc, ws.xh,
                                   first, map_cap, ws.chain_ws, ws.chain_bytes, stream);
        if (st == TV_ERR_WORKSPACE && first < msg_cap)
            st = tv_chain_nc(TV_F64, H + W, 2 * N, ws.coff, ws.uoff, ws.ulam, ws.uslope, ws.wr, cc, ws.xh, msg_cap,
                             map_cap, ws.chain_ws, ws.chain_bytes, stream);
        if (st != TV_OK) return st;
        hipLaunchKernelGGL(k_nc2d_update, gN, blk, 0, stream, ws, H, W, sigma);
        if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
    }
    if (dtype == TV_F32)
        hipLaunchKernelGGL((k_nc2d_out<float>), gN, blk, 0, stream, ws.xh, (float *)x, N);
    else
        hipLaunchKernelGGL((k_nc2d_out<double>), gN, blk, 0, stream, ws.xh, (double *)x, N);
    if (hipGetLastError() != hipSuccess) return TV_ERR_HIP;
    return hipStreamSynchronize(stream) == hipSuccess ? TV_OK : TV_ERR_HIP;
}

}  // extern "C"
