/*
 * tv_oracle.c -- plain FP64 CPU oracle for "Total variation on a tree"
 * (Kolmogorov, Pock, Rolinek, arXiv 1502.07770).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Contents (each function cites the passage it follows):
 *   orc_chain_dp        -- Sec. 4.1 O(n) chain algorithm (Algorithm 2 specialised
 *                          to strictly convex quadratic unaries), general a_i > 0
 *                          and asymmetric pairwise slopes w^-_i <= w^+_i.
 *   orc_chain_prox_tv   -- the TV-l2 chain prox, eq. (1D-ROF): a_i = 1, b_i = y_i,
 *                          w^-_i = -w_i, w^+_i = +w_i; batched over strided chains.
 *   orc_chain_brute     -- brute force over all 3^(n-1) edge sign patterns for
 *                          tiny chains (n <= 12); independent of the DP.
 *   orc_tv2d            -- Sec. 5.1 ROF by Lagrangian decomposition, the
 *                          accelerated primal-dual iteration eq. (pd) with the
 *                          primal prox on rows and the dual prox (Moreau identity,
 *                          eq. (prox-tv-conj)) on columns, plus an FP64 duality gap.
 *   orc_chain_adjoint   -- gradient of <g, x(y,w)> for the chain prox, from the
 *                          optimality conditions of eq. (1D-ROF) and the clip
 *                          structure of the backward pass of Algorithm 2.
 *   orc_chain_pq        -- Sec. 4.2, piecewise-quadratic unaries
 *                          a_i x^2/2 - b_i x + c_i |x - d_i| on a chain (the
 *                          unaries of the TV-l1 primal prox, eq. (prox-pq)), with
 *                          the breakpoint multiset kept as a sorted array.
 *   orc_chain_pq_brute  -- brute force for the same objective on tiny chains
 *                          (n <= 6): every edge and node state, independent of
 *                          the DP.
 *   orc_chain_prox_l1   -- the TV-l1 chain prox x = argmin sum w|dx| + sum
 *                          (x - y)^2/2 + sum c |x - d|, batched over chains.
 *   orc_tree_pq         -- Algorithm 2 on a forest (nodes numbered children
 *                          before parents) with the Sec. 4.2 unaries: each
 *                          node's message is the sum of its children's clipped
 *                          messages (the union of their breakpoint sets, the
 *                          "Extension to trees" of Sec. 4.2) plus its unary.
 *   orc_tree_pq_brute   -- brute force over edge and node states, n <= 6.
 *   orc_nc_chain        -- Sec. 3, non-convex case on a chain: piecewise-linear
 *                          unaries and truncated TV min(w|z|, C), messages as
 *                          slope/breakpoint sequences, Lemma 1 (sum), Lemma 2 via
 *                          Prop. 2 (Algorithm 1, its reversal, the truncation)
 *                          and the backward pass through the mappings pi.
 *   orc_nc_brute        -- exact minimum of the same energy on tiny chains
 *                          (n <= 5) by a Viterbi pass over vertex candidates.
 *   orc_ncg_chain       -- Sec. 3, Extensions (i): the same chain with every
 *                          pairwise term a minimum of one-sided linear pieces
 *                          g(z) = alpha|z| + C on z > 0 or on z < 0 (concave,
 *                          non-decreasing in |z| on each side, 0 at z = 0),
 *                          applied one piece at a time by Prop. 2 with
 *                          h (x) g = (h^alpha (x) g^alpha)^-alpha.
 *   orc_ncg_brute       -- exact minimum of that energy on tiny chains (n <= 6)
 *                          by a Viterbi pass over the unary breakpoints.
 *   orc_ncg_tree        -- the same pairwise terms on a forest (Sec. 3 on trees:
 *                          children's messages summed by Lemma 1), with
 *                          orc_ncg_tree_brute its min-sum check on n <= 6.
 *   orc_tv2d_l1         -- Sec. 5.2 TV-l1 by the same decomposition: the
 *                          primal-dual iteration eq. (pd) with the dual prox of
 *                          lambda TV_v on the columns (as for ROF) and the primal
 *                          prox eq. (prox-pq) on the rows (orc_chain_prox_l1),
 *                          constant steps tau sigma = 1, theta = 1.
 *
 * Conventions: node indices are 0-based here (the paper's node i is index i-1);
 * edge e joins nodes e and e+1, so a chain of n nodes has n-1 edge weights.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t pushes;          /* breakpoints added (2 per non-root node)          */
    int64_t pops;            /* breakpoints removed at either end                */
    int64_t max_breakpoints; /* largest number t of breakpoints held at once     */
} orc_counts;

/* ------------------------------------------------------------------------ */
/* Sec. 4.1: O(n) DP for f_i(x) = a_i x^2 / 2 - b_i x on a chain, pairwise    */
/* f_e(z) = w^-_e z (z < 0), w^+_e z (z >= 0) on edge (e, e+1).               */
/* ------------------------------------------------------------------------ */
/*
 * The current message (either \hat m_i or m_ij) is the sequence
 * (s_0, lam_1, s_1, ..., lam_t, s_t) held contiguously in seq[h..e]
 * (s_p at h + 2p, lam_p at h + 2p - 1).  The true slope of segment p is
 * s_p + Abar_i with Abar_i = a_1 + ... + a_i (implicit-slope representation),
 * so adding g_i(z) = a_i z - b_i only advances Abar.  The array has 4n + O(1)
 * entries and the sequence starts in its middle, growing both ways.
 *
 * lam_lo[i], lam_hi[i] receive lambda^-_{i,i+1}, lambda^+_{i,i+1}; x receives
 * the minimiser.  seq must hold 4n + 9 doubles.  Returns 0, or -1 on n < 1.
 */
int orc_chain_dp(int64_t n, const double *a, const double *b,
                 const double *wm, const double *wp,
                 double *x, double *lam_lo, double *lam_hi,
                 double *seq, orc_counts *cnt)
{
    if (n < 1) return -1;
    int64_t h = 2 * n + 4, e = h;  /* sequence = (s_0) only               */
    double Abar = 0.0;
    seq[h] = 0.0;                  /* s_0 = -Abar_0 = 0                  */
    double wm_prev = 0.0, wp_prev = 0.0;
    if (cnt) { cnt->pushes = 0; cnt->pops = 0; cnt->max_breakpoints = 0; }

    for (int64_t i = 0; i < n; ++i) {
        const int root = (i == n - 1);
        /* Algorithm 2 gives the root a virtual parent edge with
           w^- = w^+ = 0, so its interval collapses to the zero of \hat m. */
        const double lo = root ? 0.0 : wm[i];
        const double hi = root ? 0.0 : wp[i];
        const double ai = a[i], bi = b[i];
        Abar += ai;                 /* transformation (a): \hat m_i = m_ki + g_i */
        const int64_t t = (e - h) / 2;
        double lm, lp;
        int64_t ell = 0, r = 1;

        if (t == 0) {
            /* First node: no incoming message, \hat m_1(z) = a_1 z - b_1. */
            lm = (lo + bi) / ai;
            lp = (hi + bi) / ai;
            ell = 0;
            r = 1;
        } else {
#define LAM(p) seq[h + 2 * (p) - 1]
#define SLP(p) seq[h + 2 * (p)]
            /* Left end: largest ell with \hat m_i(lam_ell) < w^-, values by the
               recursion \hat m(lam_1) = w^-_ki + a_i lam_1 - b_i,
               \hat m(lam_{p+1}) = \hat m(lam_p) + (s_p + Abar)(lam_{p+1} - lam_p). */
            double v = wm_prev + ai * LAM(1) - bi;
            double v_ell = v;
            if (!(v < lo)) {
                ell = 0;
                /* zero on the left end segment (true slope s_0 + Abar = a_i) */
                lm = LAM(1) - (v - lo) / (SLP(0) + Abar);
            } else {
                ell = 1;
                while (ell < t) {
                    double vn = v_ell + (SLP(ell) + Abar) * (LAM(ell + 1) - LAM(ell));
                    if (!(vn < lo)) break;
                    ++ell;
                    v_ell = vn;
                }
                /* zero on segment ell, which starts at lam_ell */
                lm = LAM(ell) + (lo - v_ell) / (SLP(ell) + Abar);
                /* rounding guard: stay inside the bracketing segment */
                if (lm < LAM(ell)) lm = LAM(ell);
                if (ell < t && lm > LAM(ell + 1)) lm = LAM(ell + 1);
            }

            if (root) {
                x[i] = lm;
                if (cnt) cnt->pops += ell;
                break;
            }

            /* Right end: smallest r >= ell + 1 with \hat m_i(lam_r) > w^+
               (r = t + 1 if none), values by the recursion from
               \hat m(lam_t) = w^+_ki + a_i lam_t - b_i downward. */
            if (ell == t) {
                /* every old breakpoint left of the zero of w^-: the segment
                   right of lam^- is the old right end, true slope a_i */
                r = t + 1;
                lp = lm + (hi - lo) / (SLP(t) + Abar);
            } else {
                double vr = wp_prev + ai * LAM(t) - bi;
                if (!(vr > hi)) {
                    r = t + 1;
                    lp = LAM(t) + (hi - vr) / (SLP(t) + Abar);
                } else {
                    r = t;
                    double v_r = vr;
                    while (r - 1 >= ell + 1) {
                        double vp = v_r - (SLP(r - 1) + Abar) * (LAM(r) - LAM(r - 1));
                        if (!(vp > hi)) break;
                        --r;
                        v_r = vp;
                    }
                    /* zero on the segment ending at lam_r; its slope is
                       s_{r-1}, which is s_ell when that segment starts at lam^- */
                    lp = LAM(r) - (v_r - hi) / (SLP(r - 1) + Abar);
                    if (lp > LAM(r)) lp = LAM(r);
                    if (r - 1 >= ell + 1 && lp < LAM(r - 1)) lp = LAM(r - 1);
                }
            }
            if (lp < lm) lp = lm;   /* rounding guard: lam^- <= lam^+ */
#undef LAM
#undef SLP
        }

        if (root) {             /* only reached for n == 1 */
            x[i] = lm;
            break;
        }
        lam_lo[i] = lm;
        lam_hi[i] = lp;
        if (cnt) {
            cnt->pushes += 2;
            cnt->pops += ell + (t - r + 1);
        }
        /* New sequence (-Abar, lam^-, s_ell, lam_{ell+1}, ..., s_{r-1}, lam^+, -Abar):
           keep s_ell at h + 2 ell and s_{r-1} at h + 2(r-1); write around them. */
        {
            const int64_t h_old = h;
            seq[h_old + 2 * ell - 1] = lm;
            seq[h_old + 2 * ell - 2] = -Abar;
            seq[h_old + 2 * r - 1] = lp;
            seq[h_old + 2 * r] = -Abar;
            h = h_old + 2 * ell - 2;
            e = h_old + 2 * r;
        }
        if (cnt) {
            int64_t tn = (e - h) / 2;
            if (tn > cnt->max_breakpoints) cnt->max_breakpoints = tn;
        }
        wm_prev = lo;
        wp_prev = hi;
    }

    /* Backward pass of Algorithm 2: x_i = clip(x_{i+1}, lam^-_i, lam^+_i). */
    for (int64_t i = n - 2; i >= 0; --i) {
        double v = x[i + 1];
        if (v < lam_lo[i]) v = lam_lo[i];
        if (v > lam_hi[i]) v = lam_hi[i];
        x[i] = v;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* eq. (1D-ROF): min_x sum_e w_e |x_{e+1} - x_e| + 1/2 sum_i (x_i - y_i)^2,   */
/* batched over chains read with arbitrary strides.                          */
/* ------------------------------------------------------------------------ */
/*
 * Chain c, node i lives at y[c * chain_stride + i * elem_stride].  The edge
 * weight of edge (i, i+1) is w[c * chain_stride + i * elem_stride] when w is
 * non-NULL (the slot of the last node is ignored), else w_scalar.
 * counts (optional) receives per-chain counters.  threads <= 0 means all.
 * Returns 0, or -1 on invalid arguments.
 */
int orc_chain_prox_tv(int64_t num_chains, int64_t n, int64_t elem_stride, int64_t chain_stride,
                      const double *y, const double *w, double w_scalar, double *x,
                      orc_counts *counts, int threads)
{
    if (num_chains < 0 || n < 1) return -1;
    if (!w && !(w_scalar >= 0.0)) return -1;
    int bad = 0;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel num_threads(threads) reduction(|:bad)
#endif
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(4 * n + 9 + 8 * n));
        double *seq = buf;
        double *a = buf + 4 * n + 9;
        double *b = a + n;
        double *wm = b + n;
        double *wp = wm + n;
        double *xc = wp + n;
        double *llo = xc + n;
        double *lhi = llo + n;
        for (int64_t i = 0; i < n; ++i) a[i] = 1.0;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 8)
#endif
        for (int64_t c = 0; c < num_chains; ++c) {
            const double *yc = y + c * chain_stride;
            for (int64_t i = 0; i < n; ++i) b[i] = yc[i * elem_stride];
            for (int64_t i = 0; i + 1 < n; ++i) {
                double we = w ? w[c * chain_stride + i * elem_stride] : w_scalar;
                if (!(we >= 0.0)) bad = 1;
                wm[i] = -we;
                wp[i] = we;
            }
            orc_chain_dp(n, a, b, wm, wp, xc, llo, lhi, seq, counts ? counts + c : NULL);
            double *xo = x + c * chain_stride;
            for (int64_t i = 0; i < n; ++i) xo[i * elem_stride] = xc[i];
        }
        free(buf);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Brute force for tiny chains: enumerate every sign pattern of the n-1      */
/* edges (fused, up, down).  For each, solve the equality-constrained        */
/* stationarity system (runs of fused nodes share one value), evaluate the  */
/* TRUE objective at that point, and keep the best.  The optimum's own sign */
/* pattern reproduces it, and every candidate is a feasible point, so the   */
/* minimum over candidates is the global minimum of the strictly convex     */
/* objective of Sec. 4.1 (quadratic unaries, slopes w^- <= w^+).            */
/* ------------------------------------------------------------------------ */
static double objective_general(int64_t n, const double *a, const double *b,
                                const double *wm, const double *wp, const double *x)
{
    double f = 0.0;
    for (int64_t i = 0; i < n; ++i) f += 0.5 * a[i] * x[i] * x[i] - b[i] * x[i];
    for (int64_t e = 0; e + 1 < n; ++e) {
        double z = x[e + 1] - x[e];
        f += (z < 0.0) ? wm[e] * z : wp[e] * z;
    }
    return f;
}

int orc_chain_brute(int64_t n, const double *a, const double *b,
                    const double *wm, const double *wp, double *x_best)
{
    if (n < 1 || n > 12) return -1;
    int64_t m = n - 1, total = 1;
    for (int64_t e = 0; e < m; ++e) total *= 3;
    double best = INFINITY;
    double x[12];
    int state[12];
    for (int64_t code = 0; code < total; ++code) {
        int64_t c = code;
        for (int64_t e = 0; e < m; ++e) { state[e] = (int)(c % 3); c /= 3; }
        /* q_e: the pairwise subgradient used on a non-fused edge
           (state 1: x_{e+1} > x_e -> w^+_e; state 2: x_{e+1} < x_e -> w^-_e). */
        int64_t start = 0;
        while (start < n) {
            int64_t end = start;
            while (end < m && state[end] == 0) ++end;   /* run [start..end] */
            double qin = 0.0, qout = 0.0, sa = 0.0, sb = 0.0;
            if (start > 0) qin = (state[start - 1] == 1) ? wp[start - 1] : wm[start - 1];
            if (end < m) qout = (state[end] == 1) ? wp[end] : wm[end];
            for (int64_t k = start; k <= end; ++k) { sa += a[k]; sb += b[k]; }
            /* stationarity of the run: sum_k (a_k c - b_k) = qout - qin */
            double cval = (sb + qout - qin) / sa;
            for (int64_t k = start; k <= end; ++k) x[k] = cval;
            start = end + 1;
        }
        double f = objective_general(n, a, b, wm, wp, x);
        if (f < best) {
            best = f;
            for (int64_t k = 0; k < n; ++k) x_best[k] = x[k];
        }
    }
    return 0;
}

/* Objective of eq. (1D-ROF) for one chain (unit stride). */
double orc_rof1d_objective(int64_t n, const double *y, const double *w, double w_scalar,
                           const double *x)
{
    double f = 0.0;
    for (int64_t i = 0; i < n; ++i) f += 0.5 * (x[i] - y[i]) * (x[i] - y[i]);
    for (int64_t e = 0; e + 1 < n; ++e) f += (w ? w[e] : w_scalar) * fabs(x[e + 1] - x[e]);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the chain prox.                                               */
/* ------------------------------------------------------------------------ */
/*
 * On a run R = [s..t] of equal x (maximal, by exact equality of consecutive
 * values) the optimality conditions of eq. (1D-ROF) give
 *   x_R = (sum_R y + w_t s_t - w_{s-1} s_{s-1}) / |R|,
 * where s_e = sign(x_{e+1} - x_e) on the boundary edges (and no term at the
 * chain ends).  Hence for L = <g, x>:
 *   dL/dy_i = mean of g over the run containing i,
 *   dL/dw_e = s_e (mean_g(left run) - mean_g(right run)) on a run boundary e,
 *   dL/dw_e = 0 inside a run.
 * dw (length n, slot n-1 unused and set to 0) may be NULL.  With
 * dw_scalar non-NULL the sum over all edges is written there (scalar w).
 */
int orc_chain_adjoint(int64_t num_chains, int64_t n, int64_t elem_stride, int64_t chain_stride,
                      const double *x, const double *g, double *dy, double *dw,
                      double *dw_scalar, int threads)
{
    if (num_chains < 0 || n < 1) return -1;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(threads)
#endif
    for (int64_t c = 0; c < num_chains; ++c) {
        const double *xc = x + c * chain_stride;
        const double *gc = g + c * chain_stride;
        double *dyc = dy + c * chain_stride;
        double *dwc = dw ? dw + c * chain_stride : NULL;
        double prev_mean = 0.0, wsum = 0.0;
        int64_t s = 0;
        while (s < n) {
            int64_t t = s;
            while (t + 1 < n && xc[(t + 1) * elem_stride] == xc[t * elem_stride]) ++t;
            double sg = 0.0;
            for (int64_t k = s; k <= t; ++k) sg += gc[k * elem_stride];
            double mean = sg / (double)(t - s + 1);
            for (int64_t k = s; k <= t; ++k) {
                dyc[k * elem_stride] = mean;
                if (dwc) dwc[k * elem_stride] = 0.0;
            }
            if (s > 0) {
                int64_t eb = s - 1;   /* boundary edge between the runs */
                double sign = (xc[s * elem_stride] > xc[eb * elem_stride]) ? 1.0 : -1.0;
                double d = sign * (prev_mean - mean);
                if (dwc) dwc[eb * elem_stride] = d;
                wsum += d;
            }
            prev_mean = mean;
            s = t + 1;
        }
        if (dw_scalar) dw_scalar[c] = wsum;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 5.1: ROF by Lagrangian decomposition and accelerated primal-dual.   */
/* ------------------------------------------------------------------------ */
/*
 * Image f is H x W, row-major (pixel (r, c) at r * W + c).  Horizontal edges
 * join (r, c)-(r, c+1) and form the H row chains; vertical edges join
 * (r, c)-(r+1, c) and form the W column chains; every edge has weight lambda.
 *
 * Iteration (eq. (pd), K = identity, G = lambda TV_h + |.-f|^2/2 which is
 * 1-strongly convex, F = lambda TV_v):
 *   eta    = y + sigma_k xbar
 *   y      = eta - prox_{lambda TV_v}(eta)            (column chains; Moreau
 *            identity, eq. (prox-tv-conj), with TV 1-homogeneous)
 *   b      = (tau_k f + x - tau_k y) / (1 + tau_k)
 *   x_new  = prox_{(lambda tau_k/(1+tau_k)) TV_h}(b) (row chains; the primal prox
 *            rescaled to unit quadratic weight)
 *   theta  = 1/sqrt(1 + 2 tau_k); tau_{k+1} = theta tau_k; sigma_{k+1} = sigma_k/theta
 *   xbar   = x_new + theta (x_new - x)
 * with x^0 = xbar^0 = f, y^0 = 0, sigma_0 = 1/tau_0.
 *
 * Duality gap (FP64) after each iteration, at x_new and the dual edge
 * variables recovered from the two chain solves:
 *   p_v,e = clip(-sum_{k<=e} y_k, +-lambda) down each column,
 *   p_h,e = clip(((1+tau)/tau) sum_{k<=e} (x_new_k - b_k), +-lambda) along each row,
 *   P = lambda TV_h(x) + lambda TV_v(x) + |x - f|^2/2,
 *   D = |f|^2/2 - |f - D_h^T p_h - D_v^T p_v|^2/2,
 * (D^T p)_0 = -p_0, (D^T p)_i = p_{i-1} - p_i, (D^T p)_{n-1} = p_{n-2}.
 * Any |p| <= lambda gives D <= min P (weak duality), so P - D >= 0 bounds the
 * suboptimality of x.  gap_hist[k] = (P - D) / (H W) after iteration k+1.
 *
 * The iteration stops after max_iter iterations, or after the first one whose
 * normalised gap is <= gap_tol (gap_tol <= 0 disables).  Returns the number
 * of iterations run, or -1 on bad arguments.  x (H*W) receives the iterate;
 * out3 (optional) receives {P, D, gap_norm} of the last iteration.
 */
static void tv2d_gap(int64_t H, int64_t W, double lambda, double tau, const double *f,
                     const double *x, const double *bb, const double *y,
                     double *ph, double *pv, double *out3)
{
    /* p_v down each column, p_h along each row */
    for (int64_t c = 0; c < W; ++c) {
        double cs = 0.0;
        for (int64_t r = 0; r + 1 < H; ++r) {
            cs += y[r * W + c];
            double p = -cs;
            if (p > lambda) p = lambda;
            if (p < -lambda) p = -lambda;
            pv[r * W + c] = p;
        }
    }
    const double scale = (1.0 + tau) / tau;
    for (int64_t r = 0; r < H; ++r) {
        double cs = 0.0;
        for (int64_t c = 0; c + 1 < W; ++c) {
            cs += x[r * W + c] - bb[r * W + c];
            double p = scale * cs;
            if (p > lambda) p = lambda;
            if (p < -lambda) p = -lambda;
            ph[r * W + c] = p;
        }
    }
    double P = 0.0, D = 0.0;
    for (int64_t r = 0; r < H; ++r) {
        for (int64_t c = 0; c < W; ++c) {
            const int64_t k = r * W + c;
            double xv = x[k], fv = f[k];
            P += 0.5 * (xv - fv) * (xv - fv);
            if (c + 1 < W) P += lambda * fabs(x[k + 1] - xv);
            if (r + 1 < H) P += lambda * fabs(x[k + W] - xv);
            double z = 0.0;
            if (c > 0) z += ph[k - 1];
            if (c + 1 < W) z -= ph[k];
            if (r > 0) z += pv[k - W];
            if (r + 1 < H) z -= pv[k];
            D += 0.5 * fv * fv - 0.5 * (fv - z) * (fv - z);
        }
    }
    out3[0] = P;
    out3[1] = D;
    out3[2] = (P - D) / (double)(H * W);
}

int64_t orc_tv2d(int64_t H, int64_t W, const double *f, double lambda, double tau0,
                 int64_t max_iter, double gap_tol, double *x, double *gap_hist,
                 double *out3, int threads)
{
    if (H < 1 || W < 1 || !(lambda >= 0.0) || !(tau0 > 0.0) || max_iter < 0) return -1;
    const int64_t N = H * W;
    double *y = (double *)calloc((size_t)N, sizeof(double));
    double *xbar = (double *)malloc(sizeof(double) * (size_t)N);
    double *eta = (double *)malloc(sizeof(double) * (size_t)N);
    double *u = (double *)malloc(sizeof(double) * (size_t)N);
    double *bb = (double *)malloc(sizeof(double) * (size_t)N);
    double *xn = (double *)malloc(sizeof(double) * (size_t)N);
    double *ph = (double *)malloc(sizeof(double) * (size_t)N);
    double *pv = (double *)malloc(sizeof(double) * (size_t)N);
    memcpy(x, f, sizeof(double) * (size_t)N);
    memcpy(xbar, f, sizeof(double) * (size_t)N);
    double tau = tau0, sigma = 1.0 / tau0;
    double last[3] = {0.0, 0.0, 0.0};
    int64_t k = 0;
    for (k = 0; k < max_iter; ++k) {
        /* dual step on the column chains */
        for (int64_t i = 0; i < N; ++i) eta[i] = y[i] + sigma * xbar[i];
        orc_chain_prox_tv(W, H, W, 1, eta, NULL, lambda, u, NULL, threads);
        for (int64_t i = 0; i < N; ++i) y[i] = eta[i] - u[i];
        /* primal step on the row chains */
        for (int64_t i = 0; i < N; ++i) bb[i] = (tau * f[i] + x[i] - tau * y[i]) / (1.0 + tau);
        orc_chain_prox_tv(H, W, 1, W, bb, NULL, lambda * tau / (1.0 + tau), xn, NULL, threads);
        /* gap at (x_new, p) */
        tv2d_gap(H, W, lambda, tau, f, xn, bb, y, ph, pv, last);
        if (gap_hist) gap_hist[k] = last[2];
        /* acceleration */
        const double theta = 1.0 / sqrt(1.0 + 2.0 * tau);
        for (int64_t i = 0; i < N; ++i) {
            xbar[i] = xn[i] + theta * (xn[i] - x[i]);
            x[i] = xn[i];
        }
        tau *= theta;
        sigma /= theta;
        if (gap_tol > 0.0 && last[2] <= gap_tol) { ++k; break; }
    }
    if (out3) { out3[0] = last[0]; out3[1] = last[1]; out3[2] = last[2]; }
    free(y); free(xbar); free(eta); free(u); free(bb); free(xn); free(ph); free(pv);
    return k;
}

/* Primal ROF objective lambda (TV_h + TV_v)(x) + |x - f|^2 / 2. */
double orc_rof2d_objective(int64_t H, int64_t W, const double *f, double lambda, const double *x)
{
    double P = 0.0;
    for (int64_t r = 0; r < H; ++r)
        for (int64_t c = 0; c < W; ++c) {
            const int64_t k = r * W + c;
            P += 0.5 * (x[k] - f[k]) * (x[k] - f[k]);
            if (c + 1 < W) P += lambda * fabs(x[k + 1] - x[k]);
            if (r + 1 < H) P += lambda * fabs(x[k + W] - x[k]);
        }
    return P;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.2: piecewise-quadratic unaries on a chain.                         */
/*   f_i(x) = a_i x^2 / 2 - b_i x + c_i |x - d_i|   (a_i > 0, c_i >= 0)       */
/*   f_e(z) = w^-_e z (z < 0), w^+_e z (z >= 0), z = x_{e+1} - x_e.           */
/* The derivative h of the current message is non-decreasing and piecewise   */
/* linear with jumps; it is kept as its left end (al, bl) (h(z) = al z + bl  */
/* as z -> -inf), its right end (ar, br), and the multiset S of breakpoints  */
/* (lam, da, db) sorted by lam: right of lam the linear piece changes by     */
/* (da, db).  h is left-continuous: h(z) uses the breakpoints with lam < z.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *lam, *da, *db;
    int64_t t;
} pq_set;

static void pq_insert(pq_set *S, int64_t pos, double lam, double da, double db)
{
    memmove(S->lam + pos + 1, S->lam + pos, sizeof(double) * (size_t)(S->t - pos));
    memmove(S->da + pos + 1, S->da + pos, sizeof(double) * (size_t)(S->t - pos));
    memmove(S->db + pos + 1, S->db + pos, sizeof(double) * (size_t)(S->t - pos));
    S->lam[pos] = lam;
    S->da[pos] = da;
    S->db[pos] = db;
    S->t++;
}

static void pq_erase_front(pq_set *S, int64_t k)
{
    if (k <= 0) return;
    memmove(S->lam, S->lam + k, sizeof(double) * (size_t)(S->t - k));
    memmove(S->da, S->da + k, sizeof(double) * (size_t)(S->t - k));
    memmove(S->db, S->db + k, sizeof(double) * (size_t)(S->t - k));
    S->t -= k;
}

/* The point where h crosses level v from below: the z with h(z) <= v <= h(z+)
   (unique: every linear piece between the ends has slope > 0).  Scans from
   the left; returns the number of breakpoints passed (they lie left of the
   crossing), the linear piece (pa, pb) in force just left of the crossing,
   and in *jump whether the crossing is the jump of breakpoint `passed`. */
static double pq_cross_left(const pq_set *S, double al, double bl, double v, int64_t *passed,
                            double *pa, double *pb, int *jump)
{
    double A = al, B = bl;
    int64_t j = 0;
    double z;
    *jump = 0;
    for (;;) {
        if (j == S->t) { z = (v - B) / A; break; }
        const double l = S->lam[j];
        const double vl = A * l + B;            /* h just left of lam_j */
        if (vl >= v) {                           /* inside the piece left of lam_j */
            z = (v - B) / A;
            if (z > l) z = l;
            if (j > 0 && z < S->lam[j - 1]) z = S->lam[j - 1];
            break;
        }
        const double vr = vl + S->da[j] * l + S->db[j];   /* h just right of lam_j */
        if (vr >= v) { z = l; *jump = 1; break; }  /* the jump at lam_j crosses v */
        A += S->da[j];
        B += S->db[j];
        ++j;
    }
    *passed = j;
    *pa = A;
    *pb = B;
    return z;
}

/* Mirror image from the right: the z with h(z) <= v <= h(z+), scanning from
   the right end (ar, br); returns the breakpoints passed (right of z), the
   piece just right of the crossing, and whether it is the jump of breakpoint
   t - 1 - passed. */
static double pq_cross_right(const pq_set *S, double ar, double br, double v, int64_t *passed,
                             double *pa, double *pb, int *jump)
{
    double A = ar, B = br;
    int64_t j = S->t - 1, k = 0;
    double z;
    *jump = 0;
    for (;;) {
        if (j < 0) { z = (v - B) / A; break; }
        const double l = S->lam[j];
        const double vr = A * l + B;            /* h just right of lam_j */
        if (vr <= v) {                           /* inside the piece right of lam_j */
            z = (v - B) / A;
            if (z < l) z = l;
            if (j + 1 < S->t && z > S->lam[j + 1]) z = S->lam[j + 1];
            break;
        }
        const double vl = vr - (S->da[j] * l + S->db[j]);  /* h just left of lam_j */
        if (vl <= v) { z = l; *jump = 1; break; }
        A -= S->da[j];
        B -= S->db[j];
        --j;
        ++k;
    }
    *passed = k;
    *pa = A;
    *pb = B;
    return z;
}

/* lam_lo / lam_hi receive lambda^-_{i,i+1} / lambda^+_{i,i+1}; x the
   minimiser; buf holds 3 (3n + 4) doubles.  Returns 0, or -1 on n < 1. */
int orc_chain_pq(int64_t n, const double *a, const double *b, const double *c, const double *d,
                 const double *wm, const double *wp, double *x, double *lam_lo, double *lam_hi,
                 double *buf, orc_counts *cnt)
{
    if (n < 1) return -1;
    const int64_t cap = 3 * n + 4;
    pq_set S = {buf, buf + cap, buf + 2 * cap, 0};
    double al = 0.0, bl = 0.0, ar = 0.0, br = 0.0;  /* the zero message into node 0 */
    if (cnt) { cnt->pushes = 0; cnt->pops = 0; cnt->max_breakpoints = 0; }
    for (int64_t i = 0; i < n; ++i) {
        /* transformation (a): add g_i = a_i z - b_i + c_i sign(z - d_i) */
        al += a[i];
        bl += -b[i] - c[i];
        ar += a[i];
        br += -b[i] + c[i];
        if (c[i] > 0.0) {
            int64_t pos = S.t;  /* after every breakpoint with lam <= d_i */
            int64_t lo_i = 0, hi_i = S.t;
            while (lo_i < hi_i) {
                const int64_t mid = (lo_i + hi_i) / 2;
                if (S.lam[mid] <= d[i]) lo_i = mid + 1; else hi_i = mid;
            }
            pos = lo_i;
            pq_insert(&S, pos, d[i], 0.0, 2.0 * c[i]);
            if (cnt) cnt->pushes++;
        }
        if (i == n - 1) {  /* root: the zero of h */
            int64_t k;
            double pa, pb;
            int jump;
            x[i] = pq_cross_left(&S, al, bl, 0.0, &k, &pa, &pb, &jump);
            break;
        }
        /* transformation (b): clip to [w^-_i, w^+_i].  Left: h becomes flat at
           lo left of lm.  Where lm is the jump of a breakpoint, that
           breakpoint's increment is updated (merged with the new one), so
           every breakpoint keeps a non-negative jump in value. */
        const double lo = wm[i], hi = wp[i];
        int64_t k;
        double pa, pb;
        int jump;
        const double lm = pq_cross_left(&S, al, bl, lo, &k, &pa, &pb, &jump);
        double nda = pa, ndb = pb - lo;
        if (jump) {
            nda += S.da[k];
            ndb += S.db[k];
        }
        pq_erase_front(&S, k + jump);
        if (cnt) cnt->pops += k;
        pq_insert(&S, 0, lm, nda, ndb);
        al = 0.0;
        bl = lo;
        /* right: flat at hi right of lp */
        const double lp = pq_cross_right(&S, ar, br, hi, &k, &pa, &pb, &jump);
        nda = -pa;
        ndb = hi - pb;
        if (jump) {
            nda += S.da[S.t - 1 - k];
            ndb += S.db[S.t - 1 - k];
        }
        S.t -= k + jump;
        pq_insert(&S, S.t, lp, nda, ndb);
        ar = 0.0;
        br = hi;
        lam_lo[i] = lm;
        lam_hi[i] = lp < lm ? lm : lp;
        if (cnt) {
            cnt->pushes += 2;
            cnt->pops += k;
            if (S.t > cnt->max_breakpoints) cnt->max_breakpoints = S.t;
        }
    }
    /* backward pass of Algorithm 2 */
    for (int64_t i = n - 2; i >= 0; --i) {
        double v = x[i + 1];
        if (v < lam_lo[i]) v = lam_lo[i];
        if (v > lam_hi[i]) v = lam_hi[i];
        x[i] = v;
    }
    return 0;
}

double orc_pq_objective(int64_t n, const double *a, const double *b, const double *c, const double *d,
                        const double *wm, const double *wp, const double *x)
{
    double f = 0.0;
    for (int64_t i = 0; i < n; ++i) f += 0.5 * a[i] * x[i] * x[i] - b[i] * x[i] + c[i] * fabs(x[i] - d[i]);
    for (int64_t e = 0; e + 1 < n; ++e) {
        const double z = x[e + 1] - x[e];
        f += (z < 0.0) ? wm[e] * z : wp[e] * z;
    }
    return f;
}

/* Brute force over every edge state (fused / up / down) and node state
   (below d_i / at d_i / above d_i) for n <= 6.  For each pattern the runs of
   fused nodes take one value: d of the first node of the run that is "at d",
   else the stationary point sum(b - c s - q_in + q_out) / sum(a) of the run
   (s = -1 below, +1 above; q the edge slopes entering / leaving the run).
   Every candidate is a feasible point and the optimum's own pattern
   reproduces it, so the best true objective over all candidates is the
   minimum. */
int orc_chain_pq_brute(int64_t n, const double *a, const double *b, const double *c, const double *d,
                       const double *wm, const double *wp, double *x_best)
{
    if (n < 1 || n > 6) return -1;
    const int64_t m = n - 1;
    int64_t ne = 1, nn = 1;
    for (int64_t e = 0; e < m; ++e) ne *= 3;
    for (int64_t i = 0; i < n; ++i) nn *= 3;
    double best = INFINITY, xc[6];
    int es[6], ns[6];
    for (int64_t ce = 0; ce < ne; ++ce) {
        int64_t t = ce;
        for (int64_t e = 0; e < m; ++e) { es[e] = (int)(t % 3); t /= 3; }
        for (int64_t cn = 0; cn < nn; ++cn) {
            int64_t u = cn;
            for (int64_t i = 0; i < n; ++i) { ns[i] = (int)(u % 3); u /= 3; }
            int64_t start = 0;
            while (start < n) {
                int64_t end = start;
                while (end < m && es[end] == 0) ++end;   /* run [start..end] */
                double qin = 0.0, qout = 0.0;
                if (start > 0) qin = (es[start - 1] == 1) ? wp[start - 1] : wm[start - 1];
                if (end < m) qout = (es[end] == 1) ? wp[end] : wm[end];
                double A = 0.0, B = 0.0, val = NAN;
                for (int64_t i = start; i <= end; ++i) {
                    if (ns[i] == 1 && isnan(val)) val = d[i];
                    A += a[i];
                    B += b[i] - c[i] * (ns[i] == 0 ? -1.0 : 1.0);
                }
                if (isnan(val)) val = (B - qin + qout) / A;
                for (int64_t i = start; i <= end; ++i) xc[i] = val;
                start = end + 1;
            }
            const double f = orc_pq_objective(n, a, b, c, d, wm, wp, xc);
            if (f < best) {
                best = f;
                for (int64_t i = 0; i < n; ++i) x_best[i] = xc[i];
            }
        }
    }
    return 0;
}

/* TV-l1 chain prox x = argmin sum_e w_e |x_{e+1} - x_e| + sum_i (x_i - y_i)^2 / 2
   + sum_i c_i |x_i - d_i| (orc_chain_pq with a = 1, b = y, w^- = -w, w^+ = w),
   batched over strided chains.  w and c are per-node arrays in y's layout or
   NULL (use w_scalar / c_scalar).  Returns 0, or -1 on a bad argument. */
int orc_chain_prox_l1(int64_t num_chains, int64_t n, int64_t elem_stride, int64_t chain_stride,
                      const double *y, const double *d, const double *w, double w_scalar,
                      const double *c, double c_scalar, double *x, orc_counts *counts, int threads)
{
    if (n < 1 || num_chains < 0) return -1;
    if (!w && !(w_scalar >= 0.0)) return -1;
    if (!c && !(c_scalar >= 0.0)) return -1;
    int bad = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
#endif
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(9 * n + 12 + 10 * n));
        if (!buf) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            bad = 1;
        } else {
            double *a = buf + 9 * n + 12, *b = a + n, *cc = b + n, *dd = cc + n, *wm = dd + n, *wp = wm + n;
            double *xc = wp + n, *llo = xc + n, *lhi = llo + n;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
            for (int64_t ch = 0; ch < num_chains; ++ch) {
                const int64_t base = ch * chain_stride;
                for (int64_t i = 0; i < n; ++i) {
                    const int64_t o = base + i * elem_stride;
                    a[i] = 1.0;
                    b[i] = y[o];
                    dd[i] = d[o];
                    cc[i] = c ? c[o] : c_scalar;
                    const double we = (i + 1 < n) ? (w ? w[o] : w_scalar) : 0.0;
                    wm[i] = -we;
                    wp[i] = we;
                }
                orc_chain_pq(n, a, b, cc, dd, wm, wp, xc, llo, lhi, buf, counts ? counts + ch : NULL);
                for (int64_t i = 0; i < n; ++i) x[base + i * elem_stride] = xc[i];
            }
            free(buf);
        }
    }
    return bad ? -1 : 0;
}

/* TV-l1 objective lambda (TV_h + TV_v)(x) + sum |x - f|. */
double orc_tvl1_2d_objective(int64_t H, int64_t W, const double *f, double lambda, const double *x)
{
    double P = 0.0;
    for (int64_t r = 0; r < H; ++r)
        for (int64_t c = 0; c < W; ++c) {
            const int64_t k = r * W + c;
            P += fabs(x[k] - f[k]);
            if (c + 1 < W) P += lambda * fabs(x[k + 1] - x[k]);
            if (r + 1 < H) P += lambda * fabs(x[k + W] - x[k]);
        }
    return P;
}

/* Sec. 5.2: min_x lambda (TV_h + TV_v)(x) + |x - f|_1 through the saddle
   problem min_x max_y <x, y> + lambda TV_h(x) + |x - f|_1 - (lambda TV_v)^*(y)
   and eq. (pd) with constant steps (tau, sigma = 1 / tau, theta = 1):
     column step: eta = y + sigma xbar, y' = eta - prox_{lambda TV_v}(eta)
                  (the dual prox through the Moreau identity, as for ROF);
     row step:    x' = prox_{tau (lambda TV_h + |. - f|_1)}(x - tau y'), i.e. per
                  row argmin tau lambda TV + tau |x - f|_1 + |x - xi|^2 / 2
                  (eq. (prox-pq) times tau), the Sec. 4.2 chain problem;
     xbar' = 2 x' - x.
   x^0 = xbar^0 = f, y^0 = 0.  energy_hist[k] = objective after iteration k+1.
   Returns the iterations run, or -1 on a bad argument. */
int64_t orc_tv2d_l1(int64_t H, int64_t W, const double *f, double lambda, double tau,
                    int64_t max_iter, double *x, double *energy_hist, int threads)
{
    if (H < 1 || W < 1 || !(lambda >= 0.0) || !(tau > 0.0) || max_iter < 0) return -1;
    const int64_t N = H * W;
    double *y = (double *)calloc((size_t)N, sizeof(double));
    double *xbar = (double *)malloc(sizeof(double) * (size_t)N);
    double *eta = (double *)malloc(sizeof(double) * (size_t)N);
    double *u = (double *)malloc(sizeof(double) * (size_t)N);
    double *xi = (double *)malloc(sizeof(double) * (size_t)N);
    double *xn = (double *)malloc(sizeof(double) * (size_t)N);
    memcpy(x, f, sizeof(double) * (size_t)N);
    memcpy(xbar, f, sizeof(double) * (size_t)N);
    const double sigma = 1.0 / tau;
    int64_t k;
    for (k = 0; k < max_iter; ++k) {
        for (int64_t i = 0; i < N; ++i) eta[i] = y[i] + sigma * xbar[i];
        orc_chain_prox_tv(W, H, W, 1, eta, NULL, lambda, u, NULL, threads);
        for (int64_t i = 0; i < N; ++i) y[i] = eta[i] - u[i];
        for (int64_t i = 0; i < N; ++i) xi[i] = x[i] - tau * y[i];
        orc_chain_prox_l1(H, W, 1, W, xi, f, NULL, tau * lambda, NULL, tau, xn, NULL, threads);
        for (int64_t i = 0; i < N; ++i) {
            xbar[i] = 2.0 * xn[i] - x[i];
            x[i] = xn[i];
        }
        if (energy_hist) energy_hist[k] = orc_tvl1_2d_objective(H, W, f, lambda, x);
    }
    free(y); free(xbar); free(eta); free(u); free(xi); free(xn);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 on a forest.  parent[i] > i for every non-root node (children  */
/* numbered before their parents), parent[i] = -1 for roots.  Edge i joins    */
/* node i to parent[i]: f_i(z) = w^-_i z (z < 0), w^+_i z (z >= 0) with       */
/* z = x_parent - x_i (the chain convention with parent = i + 1).  Unaries as */
/* in orc_chain_pq.  Each node accumulates the derivative of the sum of its   */
/* children's clipped messages (ends added, breakpoint multisets merged in    */
/* order), adds its unary, and is clipped (Algorithm 2, lines 2-4) or, at a   */
/* root, solved for its zero; the backward pass clips each node to its        */
/* parent's value.  Returns 0, or -1 on a bad argument or allocation failure. */
/* ------------------------------------------------------------------------ */
typedef struct {
    double al, bl, ar, br;
    pq_set S;
    int64_t cap;
} pq_msg;

static int pq_msg_reserve(pq_msg *m, int64_t need)
{
    if (need <= m->cap) return 0;
    int64_t cap = m->cap > 0 ? m->cap : 8;
    while (cap < need) cap *= 2;
    double *buf = (double *)malloc(sizeof(double) * (size_t)(3 * cap));
    if (!buf) return -1;
    if (m->S.t > 0) {
        memcpy(buf, m->S.lam, sizeof(double) * (size_t)m->S.t);
        memcpy(buf + cap, m->S.da, sizeof(double) * (size_t)m->S.t);
        memcpy(buf + 2 * cap, m->S.db, sizeof(double) * (size_t)m->S.t);
    }
    free(m->S.lam);
    m->S.lam = buf;
    m->S.da = buf + cap;
    m->S.db = buf + 2 * cap;
    m->cap = cap;
    return 0;
}

int orc_tree_pq(int64_t n, const int64_t *parent, const double *a, const double *b, const double *c,
                const double *d, const double *wm, const double *wp, double *x, double *lam_lo,
                double *lam_hi)
{
    if (n < 1) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (parent[i] != -1 && (parent[i] <= i || parent[i] >= n)) return -1;
    pq_msg *acc = (pq_msg *)calloc((size_t)n, sizeof(pq_msg));
    if (!acc) return -1;
    int rc = 0;
    for (int64_t i = 0; i < n && rc == 0; ++i) {
        pq_msg *m = &acc[i];
        /* add g_i */
        m->al += a[i];
        m->bl += -b[i] - c[i];
        m->ar += a[i];
        m->br += -b[i] + c[i];
        if (c[i] > 0.0) {
            if (pq_msg_reserve(m, m->S.t + 1)) { rc = -1; break; }
            int64_t lo_i = 0, hi_i = m->S.t;
            while (lo_i < hi_i) {
                const int64_t mid = (lo_i + hi_i) / 2;
                if (m->S.lam[mid] <= d[i]) lo_i = mid + 1; else hi_i = mid;
            }
            pq_insert(&m->S, lo_i, d[i], 0.0, 2.0 * c[i]);
        }
        int64_t k;
        double pa, pb;
        int jump;
        if (parent[i] < 0) {  /* root */
            x[i] = pq_cross_left(&m->S, m->al, m->bl, 0.0, &k, &pa, &pb, &jump);
            lam_lo[i] = lam_hi[i] = x[i];
            free(m->S.lam);
            continue;
        }
        /* clip to [w^-_i, w^+_i] as in orc_chain_pq */
        const double lo = wm[i], hi = wp[i];
        if (pq_msg_reserve(m, m->S.t + 2)) { rc = -1; break; }
        const double lm = pq_cross_left(&m->S, m->al, m->bl, lo, &k, &pa, &pb, &jump);
        double nda = pa, ndb = pb - lo;
        if (jump) { nda += m->S.da[k]; ndb += m->S.db[k]; }
        pq_erase_front(&m->S, k + jump);
        pq_insert(&m->S, 0, lm, nda, ndb);
        const double lp = pq_cross_right(&m->S, m->ar, m->br, hi, &k, &pa, &pb, &jump);
        nda = -pa;
        ndb = hi - pb;
        if (jump) { nda += m->S.da[m->S.t - 1 - k]; ndb += m->S.db[m->S.t - 1 - k]; }
        m->S.t -= k + jump;
        pq_insert(&m->S, m->S.t, lp, nda, ndb);
        lam_lo[i] = lm;
        lam_hi[i] = lp < lm ? lm : lp;
        /* merge the clipped message (ends (0, lo), (0, hi)) into the parent's sum */
        pq_msg *q = &acc[parent[i]];
        q->al += 0.0;
        q->bl += lo;
        q->ar += 0.0;
        q->br += hi;
        if (pq_msg_reserve(q, q->S.t + m->S.t)) { rc = -1; break; }
        int64_t u = q->S.t - 1, v = m->S.t - 1, w = q->S.t + m->S.t - 1;
        while (v >= 0) {  /* merge from the back, in place in q */
            if (u >= 0 && q->S.lam[u] > m->S.lam[v]) {
                q->S.lam[w] = q->S.lam[u]; q->S.da[w] = q->S.da[u]; q->S.db[w] = q->S.db[u]; --u;
            } else {
                q->S.lam[w] = m->S.lam[v]; q->S.da[w] = m->S.da[v]; q->S.db[w] = m->S.db[v]; --v;
            }
            --w;
        }
        q->S.t += m->S.t;
        free(m->S.lam);
        m->S.lam = NULL;
    }
    if (rc != 0) {
        for (int64_t i = 0; i < n; ++i) free(acc[i].S.lam);
    }
    free(acc);
    if (rc != 0) return rc;
    /* backward pass: parents before children */
    for (int64_t i = n - 1; i >= 0; --i) {
        if (parent[i] < 0) continue;
        double v = x[parent[i]];
        if (v < lam_lo[i]) v = lam_lo[i];
        if (v > lam_hi[i]) v = lam_hi[i];
        x[i] = v;
    }
    return 0;
}

double orc_tree_pq_objective(int64_t n, const int64_t *parent, const double *a, const double *b, const double *c,
                             const double *d, const double *wm, const double *wp, const double *x)
{
    double f = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        f += 0.5 * a[i] * x[i] * x[i] - b[i] * x[i] + c[i] * fabs(x[i] - d[i]);
        if (parent[i] >= 0) {
            const double z = x[parent[i]] - x[i];
            f += (z < 0.0) ? wm[i] * z : wp[i] * z;
        }
    }
    return f;
}

/* Brute force for n <= 6 as orc_chain_pq_brute, on the forest's edges: the
   components of fused edges take d of their first "at d" node or their
   stationary point sum(b - c s + q_in - q_out)... with q the slopes of the
   edges leaving the component toward a parent (q_out) or entering it from a
   child (q_in). */
int orc_tree_pq_brute(int64_t n, const int64_t *parent, const double *a, const double *b, const double *c,
                      const double *d, const double *wm, const double *wp, double *x_best)
{
    if (n < 1 || n > 6) return -1;
    int64_t ne = 1, nn = 1;
    for (int64_t i = 0; i < n; ++i) { ne *= 3; nn *= 3; }
    double best = INFINITY, xc[6];
    int es[6], ns[6], comp[6];
    for (int64_t ce = 0; ce < ne; ++ce) {
        int64_t t = ce;
        int skip = 0;
        for (int64_t i = 0; i < n; ++i) {
            es[i] = (int)(t % 3);
            t /= 3;
            if (parent[i] < 0 && es[i] != 0) skip = 1;  /* roots have no edge */
        }
        if (skip) continue;
        /* components of fused edges: label by the topmost node (parents have larger indices) */
        for (int64_t i = n - 1; i >= 0; --i) comp[i] = (parent[i] >= 0 && es[i] == 0) ? comp[parent[i]] : (int)i;
        for (int64_t cn = 0; cn < nn; ++cn) {
            int64_t u = cn;
            for (int64_t i = 0; i < n; ++i) { ns[i] = (int)(u % 3); u /= 3; }
            for (int64_t r = 0; r < n; ++r) {
                if (comp[r] != r) continue;
                double A = 0.0, B = 0.0, val = NAN;
                for (int64_t i = 0; i < n; ++i) {
                    if (comp[i] != r) continue;
                    if (ns[i] == 1 && isnan(val)) val = d[i];
                    A += a[i];
                    B += b[i] - c[i] * (ns[i] == 0 ? -1.0 : 1.0);
                    /* edge i (to its parent) leaves the component when not fused */
                    if (parent[i] >= 0 && es[i] != 0) B += (es[i] == 1) ? wp[i] : wm[i];
                }
                for (int64_t i = 0; i < n; ++i)  /* edges from a child outside into the component */
                    if (parent[i] >= 0 && es[i] != 0 && comp[parent[i]] == r) B -= (es[i] == 1) ? wp[i] : wm[i];
                if (isnan(val)) val = B / A;
                for (int64_t i = 0; i < n; ++i)
                    if (comp[i] == r) xc[i] = val;
            }
            const double f = orc_tree_pq_objective(n, parent, a, b, c, d, wm, wp, xc);
            if (f < best) {
                best = f;
                for (int64_t i = 0; i < n; ++i) x_best[i] = xc[i];
            }
        }
    }
    return 0;
}

/* ======================================================================== *
 * Sec. 3: non-convex case on a chain.  Unaries f_i are continuous
 * piecewise-linear (breakpoints lam_{i,1..t_i}, slopes s_{i,0..t_i}, fixed by
 * f_i(lam_{i,1}) = 0); pairwise terms are the truncated TV f_e(z) = min(w_e |z|,
 * C_e) with w_e >= 0 and 0 < C_e <= +inf, z = x_{e+1} - x_e.
 *
 * Messages are kept as in Sec. 3: the sequence (s_0, lam_1, s_1, ..., lam_t,
 * s_t), defined up to an additive constant.  Per edge:
 *   hat M_i = f_i + M_{i-1}                       (Lemma 1: breakpoints merged,
 *                                                  slopes added)
 *   M_i = ((hat M_i (x) f^1) (x) f^2) (x) f^3     (Lemma 2 via the consecutive
 *                                                  min-convolutions of Prop. 2)
 * with f^1 = w z on z >= 0 (+inf below), f^2 = w|z| on z <= 0 (+inf above),
 * f^3 = C off zero (0 at zero).  h (x) f^1 follows Algorithm 1 and records the
 * intervals Pi^1 on which the minimiser is the interval's left end; h (x) f^2
 * is the reversal of rev(h) (x) f^1; h (x) f^3 = min(h, min h + C) with Pi^3 the
 * set where h >= min h + C (minimiser: the argmin breakpoint).  Backward: the
 * last node takes an argmin of its hat M, then x_i = pi^1(pi^2(pi^3(x_{i+1}))).
 * ======================================================================== */
typedef struct {
    int64_t t, cap;
    double *l, *s; /* l[0..t-1], s[0..t]: s[k] is the slope left of l[k] */
} nc_plf;

typedef struct {
    int64_t n, cap;
    double *a, *b, *to; /* interval [a, b] maps to `to` */
} nc_ivs;

static int nc_reserve(nc_plf *h, int64_t t)
{
    if (t <= h->cap) return 0;
    int64_t c = h->cap ? h->cap : 16;
    while (c < t) c *= 2;
    double *l = (double *)realloc(h->l, sizeof(double) * (size_t)c);
    if (!l) return -2;
    h->l = l;
    double *s = (double *)realloc(h->s, sizeof(double) * (size_t)(c + 1));
    if (!s) return -2;
    h->s = s;
    h->cap = c;
    return 0;
}

static void nc_free(nc_plf *h)
{
    free(h->l);
    free(h->s);
    h->l = h->s = NULL;
    h->t = h->cap = 0;
}

static int nc_iv_add(nc_ivs *v, double a, double b, double to)
{
    if (v->n == v->cap) {
        int64_t c = v->cap ? 2 * v->cap : 64;
        double *na = (double *)realloc(v->a, sizeof(double) * (size_t)c);
        if (!na) return -2;
        v->a = na;
        double *nb = (double *)realloc(v->b, sizeof(double) * (size_t)c);
        if (!nb) return -2;
        v->b = nb;
        double *nt = (double *)realloc(v->to, sizeof(double) * (size_t)c);
        if (!nt) return -2;
        v->to = nt;
        v->cap = c;
    }
    v->a[v->n] = a;
    v->b[v->n] = b;
    v->to[v->n] = to;
    v->n++;
    return 0;
}

/* Append breakpoint lam with slope `right` to its right. */
static int nc_push(nc_plf *h, double lam, double right)
{
    if (nc_reserve(h, h->t + 1)) return -2;
    h->l[h->t] = lam;
    h->s[h->t + 1] = right;
    h->t++;
    return 0;
}

/* Values v[p] = h(l[p]) relative to v[0] = 0, accumulated along the slopes. */
static void nc_values(const nc_plf *h, double *v)
{
    if (h->t == 0) return;
    v[0] = 0.0;
    for (int64_t p = 1; p < h->t; ++p) v[p] = v[p - 1] + h->s[p] * (h->l[p] - h->l[p - 1]);
}

/* Lemma 1: out = a + b (breakpoint lists merged; equal positions become one). */
static int nc_add(const nc_plf *a, const nc_plf *b, nc_plf *out)
{
    out->t = 0;
    if (nc_reserve(out, a->t + b->t)) return -2;
    int64_t i = 0, j = 0;
    out->s[0] = a->s[0] + b->s[0];
    while (i < a->t || j < b->t) {
        double lam;
        if (j >= b->t || (i < a->t && a->l[i] < b->l[j])) {
            lam = a->l[i++];
        } else if (i >= a->t || b->l[j] < a->l[i]) {
            lam = b->l[j++];
        } else {
            lam = a->l[i];
            ++i;
            ++j;
        }
        /* slope right of lam: each function's slope after its breakpoints <= lam */
        out->l[out->t] = lam;
        out->s[out->t + 1] = a->s[i] + b->s[j];
        out->t++;
    }
    return 0;
}

/* Algorithm 1: out = h (x) f^1 (f^1(z) = w z for z >= 0), Pi^1 appended to iv
 * (each interval maps to its left end).  h must have s[0] <= 0. */
static int nc_dt_f1(const nc_plf *h, double w, nc_plf *out, nc_ivs *iv)
{
    const int64_t t = h->t;
    double *v = (double *)malloc(sizeof(double) * (size_t)(t > 0 ? t : 1));
    if (!v) return -2;
    nc_values(h, v);
    out->t = 0;
    if (nc_reserve(out, t)) {
        free(v);
        return -2;
    }
    out->s[0] = h->s[0];
    int64_t p = 0;
    int rc = 0;
    while (p < t && rc == 0) {
        const double right = h->s[p + 1];
        rc = nc_push(out, h->l[p], right < w ? right : w);
        if (rc) break;
        if (right >= w) {
            /* the line of slope w through (l[p], v[p]); first later breakpoint
             * (skipping p + 1, which lies on or above it) where h is below it */
            const double lp = h->l[p], vp = v[p];
            int64_t q = p + 2 < t ? p + 2 : t;  /* q = t: the unbounded right piece */
            while (q < t && !(v[q] < vp + w * (h->l[q] - lp))) ++q;
            if (q == t && !(h->s[t] < w)) {  /* h never drops below the line */
                rc = nc_iv_add(iv, lp, INFINITY, lp);
                break;
            }
            /* crossing on the piece left of breakpoint q (slope s[q] < w) */
            const double l0 = h->l[q - 1], v0 = v[q - 1];
            double lam = l0 + (vp + w * (l0 - lp) - v0) / (h->s[q] - w);
            if (lam < l0) lam = l0;
            if (q < t && lam > h->l[q]) lam = h->l[q];
            rc = nc_push(out, lam, h->s[q]);
            if (rc == 0) rc = nc_iv_add(iv, lp, lam, lp);
            p = q;
        } else {
            ++p;
        }
    }
    free(v);
    return rc;
}

/* phi^rev(z) = phi(-z): sequence reversed, every component negated. */
static int nc_rev(const nc_plf *h, nc_plf *out)
{
    out->t = 0;
    if (nc_reserve(out, h->t)) return -2;
    out->t = h->t;
    for (int64_t k = 0; k < h->t; ++k) out->l[k] = -h->l[h->t - 1 - k];
    for (int64_t k = 0; k <= h->t; ++k) out->s[k] = -h->s[h->t - k];
    return 0;
}

/* h (x) f^2 = (rev(h) (x) f^1)^rev; each interval maps to its right end. */
static int nc_dt_f2(const nc_plf *h, double w, nc_plf *out, nc_ivs *iv, nc_plf *tmp1, nc_plf *tmp2)
{
    nc_ivs r = {0, 0, NULL, NULL, NULL};
    int rc = nc_rev(h, tmp1);
    if (rc == 0) rc = nc_dt_f1(tmp1, w, tmp2, &r);
    if (rc == 0) rc = nc_rev(tmp2, out);
    for (int64_t k = 0; rc == 0 && k < r.n; ++k) rc = nc_iv_add(iv, -r.b[k], -r.a[k], -r.to[k]);
    free(r.a);
    free(r.b);
    free(r.to);
    return rc;
}

/* h at z, from the values v at the breakpoints (t >= 1). */
static double nc_eval(const nc_plf *h, const double *v, double z)
{
    const int64_t t = h->t;
    if (z <= h->l[0]) return v[0] + h->s[0] * (z - h->l[0]);
    for (int64_t k = 1; k < t; ++k)
        if (z <= h->l[k]) return v[k - 1] + h->s[k] * (z - h->l[k - 1]);
    return v[t - 1] + h->s[t] * (z - h->l[t - 1]);
}

/* slope of h at z (z inside a piece) */
static double nc_slope_at(const nc_plf *h, double z)
{
    int64_t k = 0;
    while (k < h->t && z > h->l[k]) ++k;
    return h->s[k];
}

/* h (x) f^3 = min(h, C'), C' = min h + C.  The points where the result may
 * kink are h's breakpoints and, in each piece, where h crosses C'; between
 * consecutive points the result is h (below C') or flat (at or above C',
 * decided at the segment's midpoint).  Pi^3 = the flat runs, each mapped to
 * the first argmin breakpoint. */
static int nc_trunc(const nc_plf *h, double C, nc_plf *out, nc_ivs *iv)
{
    const int64_t t = h->t;
    out->t = 0;
    if (nc_reserve(out, 2 * t + 2)) return -2;
    if (t == 0) {  /* bounded below and linear: constant, never above C' */
        out->s[0] = h->s[0];
        return 0;
    }
    /* v: t values; pts: up to 2t + 1 points; sl: up to 2t + 2 segment slopes */
    double *v = (double *)malloc(sizeof(double) * (size_t)(5 * t + 3));
    if (!v) return -2;
    double *pts = v + t, *sl = v + 3 * t + 1;
    nc_values(h, v);
    int64_t pm = 0;
    for (int64_t p = 1; p < t; ++p)
        if (v[p] < v[pm]) pm = p;
    const double cp = v[pm] + C, xm = h->l[pm];
    int64_t m = 0;
    for (int64_t k = 0; k <= t; ++k) {
        /* crossing of C' inside piece k (left of l[k]; piece 0 and t unbounded) */
        if (k == 0) {
            if (h->s[0] < 0.0 && v[0] < cp) pts[m++] = h->l[0] + (cp - v[0]) / h->s[0];
        } else if (k == t) {
            if (h->s[t] > 0.0 && v[t - 1] < cp) pts[m++] = h->l[t - 1] + (cp - v[t - 1]) / h->s[t];
        } else if ((v[k - 1] < cp && v[k] > cp) || (v[k - 1] > cp && v[k] < cp)) {
            pts[m++] = h->l[k - 1] + (cp - v[k - 1]) / h->s[k];
        }
        if (k < t) pts[m++] = h->l[k];
    }
    /* segment j in 0..m spans (pts[j-1], pts[j]) with pts[-1] = -inf, pts[m] = +inf */
    int rc = 0;
    double run = 0.0;
    int in_run = 0;
    for (int64_t j = 0; j <= m; ++j) {
        const double mid = (j == 0) ? pts[0] - 1.0 : (j == m ? pts[m - 1] + 1.0 : 0.5 * (pts[j - 1] + pts[j]));
        const int above = nc_eval(h, v, mid) >= cp;
        sl[j] = above ? 0.0 : nc_slope_at(h, mid);
        if (above && !in_run) {
            run = (j == 0) ? -INFINITY : pts[j - 1];
            in_run = 1;
        } else if (!above && in_run) {
            rc = nc_iv_add(iv, run, pts[j - 1], xm);
            in_run = 0;
        }
        if (rc) break;
    }
    if (rc == 0 && in_run) rc = nc_iv_add(iv, run, INFINITY, xm);
    if (rc == 0) {
        out->s[0] = sl[0];
        for (int64_t j = 0; j < m && rc == 0; ++j)
            if (sl[j + 1] != out->s[out->t]) rc = nc_push(out, pts[j], sl[j + 1]);
    }
    free(v);
    return rc;
}

/* pi(y) for a set of intervals: the first interval containing y, else y. */
static double nc_apply(const nc_ivs *iv, int64_t lo, int64_t hi, double y)
{
    for (int64_t k = lo; k < hi; ++k)
        if (y >= iv->a[k] && y <= iv->b[k]) return iv->to[k];
    return y;
}

static int nc_unary(int64_t i, const int64_t *uoff, const double *ulam, const double *uslope, nc_plf *f)
{
    const int64_t t = uoff[i + 1] - uoff[i];
    if (t < 1) return -1;
    f->t = 0;
    if (nc_reserve(f, t)) return -2;
    f->t = t;
    const double *l = ulam + uoff[i], *s = uslope + uoff[i] + i;
    for (int64_t k = 0; k < t; ++k) {
        if (k > 0 && !(l[k] >= l[k - 1])) return -1;
        f->l[k] = l[k];
    }
    for (int64_t k = 0; k <= t; ++k) f->s[k] = s[k];
    if (!(f->s[0] <= 0.0) || !(f->s[t] >= 0.0)) return -1;  /* bounded below */
    return 0;
}

/* The chain: nodes 0..n-1; node i has t_i = uoff[i+1] - uoff[i] >= 1
 * breakpoints ulam[uoff[i] ..] and t_i + 1 slopes uslope[uoff[i] + i ..];
 * edge e (nodes e, e+1) has w[e] >= 0 and C[e] > 0 (INFINITY: plain TV).
 * max_bp (optional) receives the largest number of breakpoints of any
 * message.  Returns 0, -1 for invalid input, -2 if out of memory. */
int orc_nc_chain(int64_t n, const int64_t *uoff, const double *ulam, const double *uslope, const double *w,
                 const double *C, double *x, int64_t *max_bp)
{
    if (n < 1) return -1;
    nc_plf hat = {0, 0, NULL, NULL}, f = {0, 0, NULL, NULL}, m1 = {0, 0, NULL, NULL}, m2 = {0, 0, NULL, NULL},
           t1 = {0, 0, NULL, NULL}, t2 = {0, 0, NULL, NULL}, msg = {0, 0, NULL, NULL};
    nc_ivs iv1 = {0, 0, NULL, NULL, NULL}, iv2 = {0, 0, NULL, NULL, NULL}, iv3 = {0, 0, NULL, NULL, NULL};
    int64_t *o1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(3 * n + 3));
    int rc = o1 ? 0 : -2;
    int64_t *o2 = o1 ? o1 + (n + 1) : NULL, *o3 = o1 ? o1 + 2 * (n + 1) : NULL;
    int64_t mb = 0;
    if (rc == 0) rc = nc_reserve(&msg, 1);
    msg.t = 0;
    if (rc == 0) msg.s[0] = 0.0;
    for (int64_t i = 0; i < n && rc == 0; ++i) {
        rc = nc_unary(i, uoff, ulam, uslope, &f);
        if (rc == 0) rc = nc_add(&f, &msg, &hat);
        if (rc) break;
        mb = hat.t > mb ? hat.t : mb;
        if (i == n - 1) break;
        if (!(w[i] >= 0.0) || !(C[i] > 0.0)) {
            rc = -1;
            break;
        }
        o1[i] = iv1.n;
        o2[i] = iv2.n;
        o3[i] = iv3.n;
        rc = nc_dt_f1(&hat, w[i], &m1, &iv1);
        if (rc == 0) rc = nc_dt_f2(&m1, w[i], &m2, &iv2, &t1, &t2);
        if (rc == 0 && isfinite(C[i])) {
            rc = nc_trunc(&m2, C[i], &msg, &iv3);
        } else if (rc == 0) {
            rc = nc_reserve(&msg, m2.t);
            if (rc == 0) {
                msg.t = m2.t;
                memcpy(msg.l, m2.l, sizeof(double) * (size_t)m2.t);
                memcpy(msg.s, m2.s, sizeof(double) * (size_t)(m2.t + 1));
            }
        }
        o1[i + 1] = iv1.n;
        o2[i + 1] = iv2.n;
        o3[i + 1] = iv3.n;
        if (rc == 0) mb = msg.t > mb ? msg.t : mb;
    }
    if (rc == 0) {
        /* the last node: an argmin of hat M (a breakpoint, the function being
         * bounded below with slopes s_0 <= 0 <= s_t) */
        double *v = (double *)malloc(sizeof(double) * (size_t)(hat.t > 0 ? hat.t : 1));
        if (!v) {
            rc = -2;
        } else {
            nc_values(&hat, v);
            int64_t pm = 0;
            for (int64_t p = 1; p < hat.t; ++p)
                if (v[p] < v[pm]) pm = p;
            double y = hat.t > 0 ? hat.l[pm] : 0.0;
            x[n - 1] = y;
            for (int64_t i = n - 2; i >= 0; --i) {
                y = nc_apply(&iv3, o3[i], o3[i + 1], y);
                y = nc_apply(&iv2, o2[i], o2[i + 1], y);
                y = nc_apply(&iv1, o1[i], o1[i + 1], y);
                x[i] = y;
            }
            free(v);
        }
    }
    if (max_bp) *max_bp = mb;
    nc_free(&hat);
    nc_free(&f);
    nc_free(&m1);
    nc_free(&m2);
    nc_free(&t1);
    nc_free(&t2);
    nc_free(&msg);
    free(iv1.a); free(iv1.b); free(iv1.to);
    free(iv2.a); free(iv2.b); free(iv2.to);
    free(iv3.a); free(iv3.b); free(iv3.to);
    free(o1);
    return rc;
}

/* f_i(z) with f_i(lam_{i,1}) = 0. */
static double nc_unary_val(int64_t i, const int64_t *uoff, const double *ulam, const double *uslope, double z)
{
    const int64_t t = uoff[i + 1] - uoff[i];
    const double *l = ulam + uoff[i], *s = uslope + uoff[i] + i;
    if (z <= l[0]) return s[0] * (z - l[0]);
    double v = 0.0;
    for (int64_t k = 1; k < t; ++k) {
        if (z <= l[k]) return v + s[k] * (z - l[k - 1]);
        v += s[k] * (l[k] - l[k - 1]);
    }
    return v + s[t] * (z - l[t - 1]);
}

double orc_nc_energy(int64_t n, const int64_t *uoff, const double *ulam, const double *uslope, const double *w,
                     const double *C, const double *x)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) e += nc_unary_val(i, uoff, ulam, uslope, x[i]);
    for (int64_t i = 0; i + 1 < n; ++i) {
        const double d = w[i] * fabs(x[i + 1] - x[i]);
        e += (isfinite(C[i]) && C[i] < d) ? C[i] : d;
    }
    return e;
}

/* Brute force for tiny chains (n <= 5), independent of the message passing: a
 * minimiser of a coercive piecewise-linear energy lies at a vertex, where every
 * x_i equals some unary breakpoint b plus a sum of offsets in {0, +-C_e/w_e}
 * over the edges between i and b's node.  An exact Viterbi over those
 * candidates gives the minimum energy (and a minimiser). */
int orc_nc_brute(int64_t n, const int64_t *uoff, const double *ulam, const double *uslope, const double *w,
                 const double *C, double *xbest, double *emin)
{
    if (n < 1 || n > 5) return -1;
    int64_t nb = uoff[n] - uoff[0];
    /* offsets reachable over up to n-1 consecutive edges */
    enum { MAXC = 8192 };
    static double cand[MAXC];
    int64_t nc = 0;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t k = uoff[j]; k < uoff[j + 1]; ++k) {
            /* paths from node j to every node i: offsets of the edges between */
            for (int64_t i = 0; i < n; ++i) {
                const int64_t lo = i < j ? i : j, hi = i < j ? j : i;  /* edges lo .. hi-1 */
                const int64_t m = hi - lo;
                int64_t combos = 1;
                for (int64_t q = 0; q < m; ++q) combos *= 3;
                for (int64_t cmb = 0; cmb < combos; ++cmb) {
                    double z = ulam[k];
                    int64_t r = cmb;
                    int ok = 1;
                    for (int64_t q = 0; q < m; ++q) {
                        const int d = (int)(r % 3) - 1;
                        r /= 3;
                        if (d != 0) {
                            const double e = lo + q, c = C[(int64_t)e];
                            if (!isfinite(c) || !(w[(int64_t)e] > 0.0)) {
                                ok = 0;
                                break;
                            }
                            z += d * c / w[(int64_t)e];
                        }
                    }
                    if (ok && nc < MAXC) cand[nc++] = z;
                }
            }
        }
    }
    (void)nb;
    /* Viterbi over the candidate set (every node takes any candidate) */
    double *cost = (double *)malloc(sizeof(double) * (size_t)(nc * n));
    int64_t *arg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc * n));
    if (!cost || !arg) {
        free(cost);
        free(arg);
        return -2;
    }
    for (int64_t a = 0; a < nc; ++a) {
        cost[a] = nc_unary_val(0, uoff, ulam, uslope, cand[a]);
        arg[a] = -1;
    }
    for (int64_t i = 1; i < n; ++i) {
        for (int64_t b = 0; b < nc; ++b) {
            double best = INFINITY;
            int64_t ab = 0;
            for (int64_t a = 0; a < nc; ++a) {
                double d = w[i - 1] * fabs(cand[b] - cand[a]);
                if (isfinite(C[i - 1]) && C[i - 1] < d) d = C[i - 1];
                const double v = cost[(i - 1) * nc + a] + d;
                if (v < best) {
                    best = v;
                    ab = a;
                }
            }
            cost[i * nc + b] = best + nc_unary_val(i, uoff, ulam, uslope, cand[b]);
            arg[i * nc + b] = ab;
        }
    }
    int64_t bb = 0;
    for (int64_t b = 1; b < nc; ++b)
        if (cost[(n - 1) * nc + b] < cost[(n - 1) * nc + bb]) bb = b;
    *emin = cost[(n - 1) * nc + bb];
    for (int64_t i = n - 1; i >= 0; --i) {
        xbest[i] = cand[bb];
        bb = arg[i * nc + bb];
    }
    free(cost);
    free(arg);
    return 0;
}

/* ------------------------------------------------------------------------ *
 * Sec. 3 on a forest: nodes numbered children before parents (parent[i] > i,
 * -1 at roots); edge i joins node i to parent[i] with w[i] >= 0 and C[i] > 0.
 * A node's message hat M_i = f_i + sum over its children of M_c (Lemma 1, the
 * children's lists merged one after another); a non-root then sends
 * M_i = ((hat M_i (x) f^1) (x) f^2) (x) f^3 to its parent, recording the
 * mappings pi of its edge; a root takes the first argmin of hat M_i.  Backward
 * (parents before children): x_i = pi^1(pi^2(pi^3(x_parent))).
 * ------------------------------------------------------------------------ */
int orc_nc_tree(int64_t n, const int64_t *parent, const int64_t *uoff, const double *ulam, const double *uslope,
                const double *w, const double *C, double *x, int64_t *max_bp)
{
    if (n < 1) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (parent[i] != -1 && (parent[i] <= i || parent[i] >= n)) return -1;
    nc_plf *msg = (nc_plf *)calloc((size_t)n, sizeof(nc_plf));
    /* per node: start and end of its intervals in each of the three lists */
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(6 * n));
    /* children lists (CSR) */
    int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *kid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    nc_plf hat = {0, 0, NULL, NULL}, tmp = {0, 0, NULL, NULL}, f = {0, 0, NULL, NULL}, m1 = {0, 0, NULL, NULL},
           m2 = {0, 0, NULL, NULL}, t1 = {0, 0, NULL, NULL}, t2 = {0, 0, NULL, NULL};
    nc_ivs iv1 = {0, 0, NULL, NULL, NULL}, iv2 = {0, 0, NULL, NULL, NULL}, iv3 = {0, 0, NULL, NULL, NULL};
    int rc = (msg && off && cnt && kid) ? 0 : -2;
    int64_t mb = 0;
    if (rc == 0) {
        for (int64_t i = 0; i < n; ++i)
            if (parent[i] >= 0) cnt[parent[i] + 1]++;
        for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
        int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        if (!fill) rc = -2;
        for (int64_t i = 0; rc == 0 && i < n; ++i)
            if (parent[i] >= 0) kid[cnt[parent[i]] + fill[parent[i]]++] = i;
        free(fill);
    }
    for (int64_t i = 0; i < n && rc == 0; ++i) {
        rc = nc_unary(i, uoff, ulam, uslope, &f);
        if (rc) break;
        /* hat = f + the children's messages */
        rc = nc_reserve(&hat, f.t);
        if (rc) break;
        hat.t = f.t;
        memcpy(hat.l, f.l, sizeof(double) * (size_t)f.t);
        memcpy(hat.s, f.s, sizeof(double) * (size_t)(f.t + 1));
        for (int64_t k = cnt[i]; k < cnt[i + 1] && rc == 0; ++k) {
            const int64_t c = kid[k];
            rc = nc_add(&hat, &msg[c], &tmp);
            nc_free(&msg[c]);
            if (rc == 0) {
                nc_plf sw = hat;
                hat = tmp;
                tmp = sw;
            }
        }
        if (rc) break;
        mb = hat.t > mb ? hat.t : mb;
        if (parent[i] < 0) {
            double *v = (double *)malloc(sizeof(double) * (size_t)(hat.t > 0 ? hat.t : 1));
            if (!v) {
                rc = -2;
                break;
            }
            nc_values(&hat, v);
            int64_t pm = 0;
            for (int64_t p = 1; p < hat.t; ++p)
                if (v[p] < v[pm]) pm = p;
            x[i] = hat.t > 0 ? hat.l[pm] : 0.0;
            free(v);
            continue;
        }
        if (!(w[i] >= 0.0) || !(C[i] > 0.0)) {
            rc = -1;
            break;
        }
        off[6 * i] = iv1.n;
        rc = nc_dt_f1(&hat, w[i], &m1, &iv1);
        off[6 * i + 1] = iv1.n;
        off[6 * i + 2] = iv2.n;
        if (rc == 0) rc = nc_dt_f2(&m1, w[i], &m2, &iv2, &t1, &t2);
        off[6 * i + 3] = iv2.n;
        off[6 * i + 4] = iv3.n;
        if (rc == 0 && isfinite(C[i])) {
            rc = nc_trunc(&m2, C[i], &msg[i], &iv3);
        } else if (rc == 0) {
            rc = nc_reserve(&msg[i], m2.t);
            if (rc == 0) {
                msg[i].t = m2.t;
                memcpy(msg[i].l, m2.l, sizeof(double) * (size_t)m2.t);
                memcpy(msg[i].s, m2.s, sizeof(double) * (size_t)(m2.t + 1));
            }
        }
        off[6 * i + 5] = iv3.n;
        if (rc == 0) mb = msg[i].t > mb ? msg[i].t : mb;
    }
    if (rc == 0) {
        for (int64_t i = n - 1; i >= 0; --i) {
            if (parent[i] < 0) continue;
            double y = x[parent[i]];
            y = nc_apply(&iv3, off[6 * i + 4], off[6 * i + 5], y);
            y = nc_apply(&iv2, off[6 * i + 2], off[6 * i + 3], y);
            y = nc_apply(&iv1, off[6 * i], off[6 * i + 1], y);
            x[i] = y;
        }
    }
    if (max_bp) *max_bp = mb;
    for (int64_t i = 0; msg && i < n; ++i) nc_free(&msg[i]);
    free(msg);
    free(off);
    free(cnt);
    free(kid);
    nc_free(&hat);
    nc_free(&tmp);
    nc_free(&f);
    nc_free(&m1);
    nc_free(&m2);
    nc_free(&t1);
    nc_free(&t2);
    free(iv1.a); free(iv1.b); free(iv1.to);
    free(iv2.a); free(iv2.b); free(iv2.to);
    free(iv3.a); free(iv3.b); free(iv3.to);
    return rc;
}

double orc_nc_tree_energy(int64_t n, const int64_t *parent, const int64_t *uoff, const double *ulam,
                          const double *uslope, const double *w, const double *C, const double *x)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        e += nc_unary_val(i, uoff, ulam, uslope, x[i]);
        if (parent[i] >= 0) {
            const double d = w[i] * fabs(x[parent[i]] - x[i]);
            e += (isfinite(C[i]) && C[i] < d) ? C[i] : d;
        }
    }
    return e;
}

/* Brute force for tiny forests (n <= 5), independent of the message passing:
 * vertex candidates b + sum of offsets in {0, +-C_e/w_e} over the edges of the
 * tree path between a breakpoint's node and each node, then an exact min-sum
 * pass over the candidates, children before parents. */
int orc_nc_tree_brute(int64_t n, const int64_t *parent, const int64_t *uoff, const double *ulam,
                      const double *uslope, const double *w, const double *C, double *emin)
{
    if (n < 1 || n > 5) return -1;
    enum { MAXC = 16384 };
    static double cand[MAXC];
    int64_t nc = 0;
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t k = uoff[j]; k < uoff[j + 1]; ++k) {
            for (int64_t i = 0; i < n; ++i) {
                /* edges on the path i .. j: climb both to the common ancestor */
                int64_t path[8], m = 0, a = i, b = j;
                int ok = 1;
                while (a != b) {
                    if (a < b) {  /* the lower index is deeper (children before parents) */
                        if (parent[a] < 0) { ok = 0; break; }
                        path[m++] = a;
                        a = parent[a];
                    } else {
                        if (parent[b] < 0) { ok = 0; break; }
                        path[m++] = b;
                        b = parent[b];
                    }
                }
                if (!ok) continue;  /* different trees */
                int64_t combos = 1;
                for (int64_t q = 0; q < m; ++q) combos *= 3;
                for (int64_t cmb = 0; cmb < combos; ++cmb) {
                    double z = ulam[k];
                    int64_t r = cmb;
                    int fine = 1;
                    for (int64_t q = 0; q < m; ++q) {
                        const int d = (int)(r % 3) - 1;
                        r /= 3;
                        if (d != 0) {
                            const int64_t e = path[q];
                            if (!isfinite(C[e]) || !(w[e] > 0.0)) {
                                fine = 0;
                                break;
                            }
                            z += d * C[e] / w[e];
                        }
                    }
                    if (fine && nc < MAXC) cand[nc++] = z;
                }
            }
        }
    }
    double *cost = (double *)malloc(sizeof(double) * (size_t)(nc * n));
    if (!cost) return -2;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t a = 0; a < nc; ++a) cost[i * nc + a] = nc_unary_val(i, uoff, ulam, uslope, cand[a]);
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) {  /* children are complete before their parent */
        if (parent[i] < 0) {
            double best = INFINITY;
            for (int64_t a = 0; a < nc; ++a) best = cost[i * nc + a] < best ? cost[i * nc + a] : best;
            total += best;
            continue;
        }
        const int64_t p = parent[i];
        for (int64_t a = 0; a < nc; ++a) {
            double best = INFINITY;
            for (int64_t b = 0; b < nc; ++b) {
                double d = w[i] * fabs(cand[a] - cand[b]);
                if (isfinite(C[i]) && C[i] < d) d = C[i];
                const double v = cost[i * nc + b] + d;
                best = v < best ? v : best;
            }
            cost[p * nc + a] += best;
        }
    }
    free(cost);
    *emin = total;
    return 0;
}


/* ========================================================================
 * Sec. 3, Extensions (i): pairwise terms f_e(z) of z = x_{e+1} - x_e that are
 * piecewise-linear, non-increasing and concave for z < 0, non-decreasing and
 * concave for z > 0, with f_e(0) = 0.  Such an f_e is the minimum of pieces
 * g(z) = alpha z + C on z > 0 (+inf on z < 0) and g(z) = alpha (-z) + C on
 * z < 0 (+inf on z > 0), alpha >= 0, C >= 0, each with g(0) = 0 (truncated TV:
 * (w, 0) and (0, C) on both sides; Potts: (0, C) on both sides).  f_e
 * satisfies the triangle inequality, so by Prop. 2 the message is the
 * consecutive min-convolution with the pieces in any order, and the mapping
 * of the edge is the composition of the pieces' mappings.  A side without
 * pieces makes f_e infinite there (a hard order constraint; no pieces at all:
 * x_{e+1} = x_e).
 *
 * One right-side piece: with phi(x) = h(x) - alpha x (every slope minus
 * alpha),
 *   (h (x) g)(y) = alpha y + min( phi(y), min_{x <= y} phi(x) + C ),
 * the minimiser being y where the first term is not larger and otherwise the
 * first argmin of phi on (-inf, y] (min over x < y equals min over x <= y for
 * continuous phi).  C = 0 gives Algorithm 1.  A left-side piece is the
 * reversal of the right-side piece applied to the reversed function.
 * ======================================================================== */

/* One right-side piece (alpha, C) applied to h; its intervals go to iv.  At a
 * point z of piece k (between l[k-1] and l[k], k >= 1) phi is linear, so the
 * running minimum there is min(mn[k-1], phi(z)). */
static int ncg_side(const nc_plf *h, double alpha, double C, nc_plf *out, nc_ivs *iv)
{
    const int64_t t = h->t;
    out->t = 0;
    if (nc_reserve(out, 2 * t + 2)) return -2;
    out->s[0] = h->s[0];
    if (t == 0) return 0; /* h constant (bounded below): phi non-increasing, no change */
    double *ph = (double *)malloc(sizeof(double) * (size_t)t);
    double *mn = (double *)malloc(sizeof(double) * (size_t)t);
    double *am = (double *)malloc(sizeof(double) * (size_t)t);
    double *cp = (double *)malloc(sizeof(double) * (size_t)(2 * t + 1));
    if (!ph || !mn || !am || !cp) {
        free(ph); free(mn); free(am); free(cp);
        return -2;
    }
    const double *l = h->l, *sl = h->s;
    /* phi at the breakpoints (h(l[0]) = 0), running minimum and first argmin;
     * on the left piece phi is non-increasing (s[0] <= 0 <= alpha), so the
     * minimum up to l[0] is phi(l[0]) */
    ph[0] = -alpha * l[0];
    mn[0] = ph[0];
    am[0] = l[0];
    for (int64_t p = 1; p < t; ++p) {
        ph[p] = ph[p - 1] + (sl[p] - alpha) * (l[p] - l[p - 1]);
        mn[p] = mn[p - 1];
        am[p] = am[p - 1];
        if (ph[p] < mn[p]) {
            mn[p] = ph[p];
            am[p] = l[p];
        }
    }
    /* kink candidates in order: the breakpoints, and in each piece k >= 1 the
     * point where phi meets mn[k-1] + C */
    int64_t nc = 0;
    for (int64_t k = 1; k <= t; ++k) {
        cp[nc++] = l[k - 1];
        const double sg = sl[k] - alpha, L = l[k - 1];
        const double R = k < t ? l[k] : INFINITY;
        if (sg != 0.0) {
            const double y1 = L + (mn[k - 1] + C - ph[k - 1]) / sg;
            if (y1 > L && y1 < R) cp[nc++] = y1;
        }
    }
    /* classify each segment between consecutive candidates at its midpoint
     * (the last one, unbounded, one unit to the right of its start) */
    double prev_slope = sl[0];
    int in_run = 0;
    double run_lo = 0.0, run_to = 0.0;
    int rc = 0;
    for (int64_t c = 0; c < nc && rc == 0; ++c) {
        const double a = cp[c], b = c + 1 < nc ? cp[c + 1] : INFINITY;
        if (!(b > a)) continue; /* empty segment */
        const double z = isfinite(b) ? 0.5 * (a + b) : a + 1.0;
        int64_t k = 1; /* the piece holding z */
        while (k < t && z > l[k]) ++k;
        const double sg = sl[k] - alpha;
        const double phz = ph[k - 1] + sg * (z - l[k - 1]);
        const double mz = phz < mn[k - 1] ? phz : mn[k - 1];
        const int above = phz > mz + C;
        const double slope = above ? alpha : sl[k];
        if (slope != prev_slope) {
            rc = nc_push(out, a, slope);
            prev_slope = slope;
        }
        if (above && !in_run) {
            in_run = 1;
            run_lo = a;
            run_to = am[k - 1];
        } else if (!above && in_run) {
            in_run = 0;
            if (rc == 0) rc = nc_iv_add(iv, run_lo, a, run_to);
        }
    }
    if (rc == 0 && in_run) rc = nc_iv_add(iv, run_lo, INFINITY, run_to);
    free(ph); free(mn); free(am); free(cp);
    return rc;
}

/* One piece on either side; a left-side piece through two reversals, its
 * intervals mirrored back. */
static int ncg_piece(const nc_plf *h, double alpha, double C, int side, nc_plf *out, nc_ivs *iv, nc_plf *t1,
                     nc_plf *t2)
{
    if (side > 0) return ncg_side(h, alpha, C, out, iv);
    const int64_t n0 = iv->n;
    int rc = nc_rev(h, t1);
    if (rc == 0) rc = ncg_side(t1, alpha, C, t2, iv);
    if (rc == 0) rc = nc_rev(t2, out);
    for (int64_t k = n0; rc == 0 && k < iv->n; ++k) {
        const double a = iv->a[k];
        iv->a[k] = -iv->b[k];
        iv->b[k] = -a;
        iv->to[k] = -iv->to[k];
    }
    return rc;
}

static int ncg_check_pieces(int64_t n, const int64_t *poff, const double *alpha, const double *C, const int32_t *side)
{
    if (poff[0] != 0) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (poff[i + 1] < poff[i]) return -1;
    for (int64_t k = 0; k < poff[n]; ++k)
        if (!(alpha[k] >= 0.0) || !isfinite(alpha[k]) || !(C[k] >= 0.0) || !isfinite(C[k]) ||
            (side[k] != 1 && side[k] != -1))
            return -1;
    return 0;
}

/* The chain: unaries as for orc_nc_chain; the pieces of edge e (nodes e and
 * e+1) are alpha, C, side [poff[e], poff[e+1]) (poff has n + 1 entries; the
 * last node's pieces are ignored).  Returns 0, -1 for invalid input, -2 if out
 * of memory; max_bp (optional) as for orc_nc_chain. */
int orc_ncg_chain(int64_t n, const int64_t *uoff, const double *ulam, const double *uslope, const int64_t *poff,
                  const double *alpha, const double *C, const int32_t *side, double *x, int64_t *max_bp)
{
    if (n < 1 || ncg_check_pieces(n, poff, alpha, C, side)) return -1;
    nc_plf hat = {0, 0, NULL, NULL}, f = {0, 0, NULL, NULL}, a = {0, 0, NULL, NULL}, b = {0, 0, NULL, NULL},
           t1 = {0, 0, NULL, NULL}, t2 = {0, 0, NULL, NULL};
    nc_ivs iv = {0, 0, NULL, NULL, NULL};
    const int64_t np = poff[n];
    int64_t *pr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * np + 2)); /* per piece: its intervals */
    int rc = pr ? 0 : -2;
    int64_t mb = 0;
    if (rc == 0) rc = nc_reserve(&a, 1);
    a.t = 0;
    if (rc == 0) a.s[0] = 0.0; /* the incoming message of node 0: zero */
    for (int64_t i = 0; i < n && rc == 0; ++i) {
        rc = nc_unary(i, uoff, ulam, uslope, &f);
        if (rc == 0) rc = nc_add(&f, &a, &hat);
        if (rc) break;
        mb = hat.t > mb ? hat.t : mb;
        if (i == n - 1) break;
        /* the message: hat, then each piece in turn */
        rc = nc_reserve(&a, hat.t);
        if (rc) break;
        a.t = hat.t;
        memcpy(a.l, hat.l, sizeof(double) * (size_t)hat.t);
        memcpy(a.s, hat.s, sizeof(double) * (size_t)(hat.t + 1));
        for (int64_t k = poff[i]; k < poff[i + 1] && rc == 0; ++k) {
            pr[2 * k] = iv.n;
            rc = ncg_piece(&a, alpha[k], C[k], side[k], &b, &iv, &t1, &t2);
            pr[2 * k + 1] = iv.n;
            if (rc == 0) {
                nc_plf sw = a;
                a = b;
                b = sw;
                mb = a.t > mb ? a.t : mb;
            }
        }
    }
    if (rc == 0) {
        double *v = (double *)malloc(sizeof(double) * (size_t)(hat.t > 0 ? hat.t : 1));
        if (!v) {
            rc = -2;
        } else {
            nc_values(&hat, v);
            int64_t pm = 0;
            for (int64_t p = 1; p < hat.t; ++p)
                if (v[p] < v[pm]) pm = p;
            double y = hat.t > 0 ? hat.l[pm] : 0.0;
            x[n - 1] = y;
            for (int64_t i = n - 2; i >= 0; --i) {
                /* pi = pi^1 o ... o pi^m: the last piece's mapping first */
                for (int64_t k = poff[i + 1] - 1; k >= poff[i]; --k) y = nc_apply(&iv, pr[2 * k], pr[2 * k + 1], y);
                x[i] = y;
            }
            free(v);
        }
    }
    if (max_bp) *max_bp = mb;
    nc_free(&hat);
    nc_free(&f);
    nc_free(&a);
    nc_free(&b);
    nc_free(&t1);
    nc_free(&t2);
    free(iv.a); free(iv.b); free(iv.to);
    free(pr);
    return rc;
}

/* f_e(z): 0 at z = 0, else the least piece on z's side (+inf without one). */
static double ncg_pair(const int64_t *poff, const double *alpha, const double *C, const int32_t *side, int64_t e,
                       double z)
{
    if (z == 0.0) return 0.0;
    const int sd = z > 0.0 ? 1 : -1;
    double best = INFINITY;
    for (int64_t k = poff[e]; k < poff[e + 1]; ++k)
        if (side[k] == sd) {
            const double v = alpha[k] * fabs(z) + C[k];
            if (v < best) best = v;
        }
    return best;
}

double orc_ncg_energy(int64_t n, const int64_t *uoff, const double *ulam, const double *uslope, const int64_t *poff,
                      const double *alpha, const double *C, const int32_t *side, const double *x)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        e += nc_unary_val(i, uoff, ulam, uslope, x[i]);
        if (i + 1 < n) e += ncg_pair(poff, alpha, C, side, i, x[i + 1] - x[i]);
    }
    return e;
}

/* Exact minimum for n <= 6.  Fixing, per edge, "equal", one right-side piece
 * or one left-side piece (with its closed sign constraint), and per node one
 * linear piece of its unary, leaves a linear program whose feasible set has
 * vertices (every coordinate is bounded on at least one side); at a vertex
 * each run of equal values holds a unary breakpoint.  The energy is the
 * minimum over these choices and never exceeds any of them, so the minimum
 * over x with every x_i a unary breakpoint is exact. */
int orc_ncg_brute(int64_t n, const int64_t *uoff, const double *ulam, const double *uslope, const int64_t *poff,
                  const double *alpha, const double *C, const int32_t *side, double *xbest, double *emin)
{
    if (n < 1 || n > 6 || ncg_check_pieces(n, poff, alpha, C, side)) return -1;
    const int64_t nc = uoff[n] - uoff[0];
    const double *cand = ulam + uoff[0];
    double *cost = (double *)malloc(sizeof(double) * (size_t)(nc * n));
    int64_t *arg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc * n));
    if (!cost || !arg) {
        free(cost);
        free(arg);
        return -2;
    }
    for (int64_t a = 0; a < nc; ++a) {
        cost[a] = nc_unary_val(0, uoff, ulam, uslope, cand[a]);
        arg[a] = -1;
    }
    for (int64_t i = 1; i < n; ++i) {
        for (int64_t b = 0; b < nc; ++b) {
            double best = INFINITY;
            int64_t ab = 0;
            for (int64_t a = 0; a < nc; ++a) {
                const double v = cost[(i - 1) * nc + a] + ncg_pair(poff, alpha, C, side, i - 1, cand[b] - cand[a]);
                if (v < best) {
                    best = v;
                    ab = a;
                }
            }
            cost[i * nc + b] = best + nc_unary_val(i, uoff, ulam, uslope, cand[b]);
            arg[i * nc + b] = ab;
        }
    }
    int64_t bb = 0;
    for (int64_t b = 1; b < nc; ++b)
        if (cost[(n - 1) * nc + b] < cost[(n - 1) * nc + bb]) bb = b;
    *emin = cost[(n - 1) * nc + bb];
    for (int64_t i = n - 1; i >= 0; --i) {
        xbest[i] = cand[bb];
        bb = arg[i * nc + bb];
    }
    free(cost);
    free(arg);
    return 0;
}


/* Forests (parent[i] > i, -1 at roots) with the pairwise terms above: the
 * pieces [poff[i], poff[i+1]) belong to the edge from i to its parent, with
 * z = x_parent - x_i (a chain numbered as a tree, parent = i + 1, is the chain
 * case); a root's pieces are ignored.  hat M_i = f_i + the children's
 * messages (Lemma 1), each message hat M_i through the pieces in turn, a root
 * at the first breakpoint attaining the minimum of its hat M, and backward
 * x_i = the composed mappings of its edge applied to x_parent. */
int orc_ncg_tree(int64_t n, const int64_t *parent, const int64_t *uoff, const double *ulam, const double *uslope,
                 const int64_t *poff, const double *alpha, const double *C, const int32_t *side, double *x,
                 int64_t *max_bp)
{
    if (n < 1 || ncg_check_pieces(n, poff, alpha, C, side)) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (parent[i] != -1 && (parent[i] <= i || parent[i] >= n)) return -1;
    nc_plf *msg = (nc_plf *)calloc((size_t)n, sizeof(nc_plf));
    const int64_t np = poff[n];
    int64_t *pr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * np + 2));
    int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *kid = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    nc_plf hat = {0, 0, NULL, NULL}, tmp = {0, 0, NULL, NULL}, f = {0, 0, NULL, NULL}, a = {0, 0, NULL, NULL},
           b = {0, 0, NULL, NULL}, t1 = {0, 0, NULL, NULL}, t2 = {0, 0, NULL, NULL};
    nc_ivs iv = {0, 0, NULL, NULL, NULL};
    int rc = (msg && pr && cnt && kid) ? 0 : -2;
    int64_t mb = 0;
    if (rc == 0) { /* children lists */
        for (int64_t i = 0; i < n; ++i)
            if (parent[i] >= 0) cnt[parent[i] + 1]++;
        for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
        int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        if (!fill) rc = -2;
        for (int64_t i = 0; rc == 0 && i < n; ++i)
            if (parent[i] >= 0) kid[cnt[parent[i]] + fill[parent[i]]++] = i;
        free(fill);
    }
    for (int64_t i = 0; i < n && rc == 0; ++i) {
        rc = nc_unary(i, uoff, ulam, uslope, &f);
        if (rc == 0) rc = nc_reserve(&hat, f.t);
        if (rc) break;
        hat.t = f.t;
        memcpy(hat.l, f.l, sizeof(double) * (size_t)f.t);
        memcpy(hat.s, f.s, sizeof(double) * (size_t)(f.t + 1));
        for (int64_t k = cnt[i]; k < cnt[i + 1] && rc == 0; ++k) {
            rc = nc_add(&hat, &msg[kid[k]], &tmp);
            nc_free(&msg[kid[k]]);
            if (rc == 0) {
                nc_plf sw = hat;
                hat = tmp;
                tmp = sw;
            }
        }
        if (rc) break;
        mb = hat.t > mb ? hat.t : mb;
        if (parent[i] < 0) {
            double *v = (double *)malloc(sizeof(double) * (size_t)(hat.t > 0 ? hat.t : 1));
            if (!v) {
                rc = -2;
                break;
            }
            nc_values(&hat, v);
            int64_t pm = 0;
            for (int64_t p = 1; p < hat.t; ++p)
                if (v[p] < v[pm]) pm = p;
            x[i] = hat.t > 0 ? hat.l[pm] : 0.0;
            free(v);
            continue;
        }
        rc = nc_reserve(&a, hat.t);
        if (rc) break;
        a.t = hat.t;
        memcpy(a.l, hat.l, sizeof(double) * (size_t)hat.t);
        memcpy(a.s, hat.s, sizeof(double) * (size_t)(hat.t + 1));
        for (int64_t k = poff[i]; k < poff[i + 1] && rc == 0; ++k) {
            pr[2 * k] = iv.n;
            rc = ncg_piece(&a, alpha[k], C[k], side[k], &b, &iv, &t1, &t2);
            pr[2 * k + 1] = iv.n;
            if (rc == 0) {
                nc_plf sw = a;
                a = b;
                b = sw;
                mb = a.t > mb ? a.t : mb;
            }
        }
        if (rc) break;
        /* the message moves to msg[i]; a gets fresh storage */
        msg[i] = a;
        a.t = a.cap = 0;
        a.l = a.s = NULL;
    }
    if (rc == 0) {
        for (int64_t i = n - 1; i >= 0; --i) {
            if (parent[i] < 0) continue;
            double y = x[parent[i]];
            for (int64_t k = poff[i + 1] - 1; k >= poff[i]; --k) y = nc_apply(&iv, pr[2 * k], pr[2 * k + 1], y);
            x[i] = y;
        }
    }
    if (max_bp) *max_bp = mb;
    for (int64_t i = 0; msg && i < n; ++i) nc_free(&msg[i]);
    free(msg);
    free(pr);
    free(cnt);
    free(kid);
    nc_free(&hat);
    nc_free(&tmp);
    nc_free(&f);
    nc_free(&a);
    nc_free(&b);
    nc_free(&t1);
    nc_free(&t2);
    free(iv.a); free(iv.b); free(iv.to);
    return rc;
}

double orc_ncg_tree_energy(int64_t n, const int64_t *parent, const int64_t *uoff, const double *ulam,
                           const double *uslope, const int64_t *poff, const double *alpha, const double *C,
                           const int32_t *side, const double *x)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        e += nc_unary_val(i, uoff, ulam, uslope, x[i]);
        if (parent[i] >= 0) e += ncg_pair(poff, alpha, C, side, i, x[parent[i]] - x[i]);
    }
    return e;
}

/* Exact minimum for n <= 6 by min-sum over the unary breakpoints (the same
 * vertex argument as orc_ncg_brute: every run of equal values, here a
 * connected set of nodes, holds a unary breakpoint at an optimal vertex). */
int orc_ncg_tree_brute(int64_t n, const int64_t *parent, const int64_t *uoff, const double *ulam,
                       const double *uslope, const int64_t *poff, const double *alpha, const double *C,
                       const int32_t *side, double *emin)
{
    if (n < 1 || n > 6 || ncg_check_pieces(n, poff, alpha, C, side)) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (parent[i] != -1 && (parent[i] <= i || parent[i] >= n)) return -1;
    const int64_t nc = uoff[n] - uoff[0];
    const double *cand = ulam + uoff[0];
    double *cost = (double *)malloc(sizeof(double) * (size_t)(nc * n));
    if (!cost) return -2;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t a = 0; a < nc; ++a) cost[i * nc + a] = nc_unary_val(i, uoff, ulam, uslope, cand[a]);
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) { /* children are complete before their parent */
        if (parent[i] < 0) {
            double best = INFINITY;
            for (int64_t a = 0; a < nc; ++a) best = cost[i * nc + a] < best ? cost[i * nc + a] : best;
            total += best;
            continue;
        }
        const int64_t p = parent[i];
        for (int64_t a = 0; a < nc; ++a) {  /* x_parent = cand[a] */
            double best = INFINITY;
            for (int64_t b = 0; b < nc; ++b) {
                const double v = cost[i * nc + b] + ncg_pair(poff, alpha, C, side, i, cand[a] - cand[b]);
                best = v < best ? v : best;
            }
            cost[p * nc + a] += best;
        }
    }
    free(cost);
    *emin = total;
    return 0;
}
