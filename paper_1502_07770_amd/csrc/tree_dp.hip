// tree_dp.hip -- Algorithm 2 on a batch of trees with the Sec. 4.2 unaries
//
//     x = argmin_x  sum_i ( a_i x_i^2 / 2 - b_i x_i + c_i |x_i - d_i| ) + sum_{i != root} f_i(x_parent(i) - x_i),
//     f_i(z) = wm_i z (z < 0), wp_i z (z >= 0),
//
// (the chain is the tree with parent(i) = i + 1).  One lane per tree.  The
// derivative of each message is kept as in Sec. 4.2: its left end (al, bl),
// right end (ar, br) and the multiset of breakpoints (lambda, da, db) sorted
// by lambda (right of lambda the linear piece changes by (da, db)).  A node's
// message is its unary plus the sum of its children's clipped messages, i.e.
// the union of their breakpoint sets with the ends added (the "Extension to
// trees" of Sec. 4.2); clipping it to [wm_i, wp_i] pops the breakpoints past
// each crossing and pushes the crossing point, updating a crossed
// breakpoint's increment in place at a jump.  All arithmetic is FP64.
//
// Trees are numbered in depth-first post-order (every subtree is a contiguous
// range ending at its root), so the clipped messages of a node's children are
// the top entries of a stack of pending messages: each tree has an arena in
// the workspace holding that stack (at most 3 breakpoints per node of the
// finished subtrees) and a merge buffer.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "chain_core.h"

namespace tvc {

struct TreeBatch {
    int64_t num_trees;
    const int64_t *offsets;  // [num_trees + 1] node ranges
    const int64_t *parent;   // [N] global parent index, -1 at each tree's root
};

// A breakpoint: lambda and the changes (da, db) of the linear piece to its
// right.  Each record is one 32-byte block, so a lane's access to it is one
// pair of 16-byte loads from a single cache line.
struct alignas(32) TBp {
    double l, a, b, pad;
};
// A pending message: its run [start, start + count) inside the region that
// starts at reg, the node it is for, and its clip levels (flat ends).
struct alignas(16) THdr {
    int64_t start, count, reg, parent;
    double lo, hi;
};
// lambda^-, lambda^+ of a node's edge (root: x_root twice).
struct alignas(16) TLam {
    double lo, hi;
};

struct TreeWs {
    TBp *ent;   // arena [6 N + 16 T] (entries of tree t from 6 off[t] + 16 t)
    THdr *hdr;  // pending-message stack [N]
    TLam *lam;  // [N]
    int *bad;   // set if a tree is not numbered in post-order
};

__device__ __forceinline__ TBp tb_get(const TreeWs &W, int64_t i) { return W.ent[i]; }
__device__ __forceinline__ void tb_put(const TreeWs &W, int64_t i, const TBp &e) { W.ent[i] = e; }

// Moves cnt breakpoints from src to dst (overlap allowed), eight at a time with
// every load of a group issued before its stores, so a group costs one memory
// latency rather than eight.
constexpr int kMoveGroup = 8;
__device__ __forceinline__ void arena_move_n(const TreeWs &W, int64_t dst, int64_t src, int64_t cnt) {
    if (cnt <= 0 || dst == src) return;
    TBp r[kMoveGroup];
    if (dst > src) {  // from the top down
        for (int64_t hi = cnt; hi > 0; hi -= kMoveGroup) {
            const int64_t lo = hi > kMoveGroup ? hi - kMoveGroup : 0;
#pragma unroll
            for (int g = 0; g < kMoveGroup; ++g)
                if (lo + g < hi) r[g] = tb_get(W, src + lo + g);
#pragma unroll
            for (int g = 0; g < kMoveGroup; ++g)
                if (lo + g < hi) tb_put(W, dst + lo + g, r[g]);
        }
    } else {  // from the bottom up
        for (int64_t lo = 0; lo < cnt; lo += kMoveGroup) {
            const int64_t hi = lo + kMoveGroup < cnt ? lo + kMoveGroup : cnt;
#pragma unroll
            for (int g = 0; g < kMoveGroup; ++g)
                if (lo + g < hi) r[g] = tb_get(W, src + lo + g);
#pragma unroll
            for (int g = 0; g < kMoveGroup; ++g)
                if (lo + g < hi) tb_put(W, dst + lo + g, r[g]);
        }
    }
}

// h(z) <= v <= h(z+) scanning from the left over entries [s, s + t) of the
// arena; returns z, the entries passed, the piece left of z and whether z is
// the jump of entry s + passed.  The next entry is loaded one step ahead.
__device__ double tree_cross_left(const TreeWs &W, int64_t s, int64_t t, double A, double B, double v,
                                  int64_t *passed, double *pa, double *pb, bool *jump) {
    int64_t j = 0;
    double z;
    *jump = false;
    TBp e{0.0, 0.0, 0.0}, nx{0.0, 0.0, 0.0};
    if (t > 0) e = tb_get(W, s);
    double lprev = 0.0;
    for (;;) {
        if (j == t) {
            z = (v - B) / A;
            break;
        }
        if (j + 1 < t) nx = tb_get(W, s + j + 1);
        const double l = e.l;
        const double vl = A * l + B;
        if (vl >= v) {
            z = (v - B) / A;
            z = z > l ? l : z;
            if (j > 0 && z < lprev) z = lprev;
            break;
        }
        const double vr = vl + e.a * l + e.b;
        if (vr >= v) {
            z = l;
            *jump = true;
            break;
        }
        A += e.a;
        B += e.b;
        lprev = l;
        e = nx;
        ++j;
    }
    *passed = j;
    *pa = A;
    *pb = B;
    return z;
}

__device__ double tree_cross_right(const TreeWs &W, int64_t s, int64_t t, double A, double B, double v,
                                   int64_t *passed, double *pa, double *pb, bool *jump) {
    int64_t j = t - 1, k = 0;
    double z;
    *jump = false;
    TBp e{0.0, 0.0, 0.0}, nx{0.0, 0.0, 0.0};
    if (j >= 0) e = tb_get(W, s + j);
    double lnext = 0.0;
    for (;;) {
        if (j < 0) {
            z = (v - B) / A;
            break;
        }
        if (j > 0) nx = tb_get(W, s + j - 1);
        const double l = e.l;
        const double vr = A * l + B;
        if (vr <= v) {
            z = (v - B) / A;
            z = z < l ? l : z;
            if (j + 1 < t && z > lnext) z = lnext;
            break;
        }
        const double vl = vr - (e.a * l + e.b);
        if (vl <= v) {
            z = l;
            *jump = true;
            break;
        }
        A -= e.a;
        B -= e.b;
        lnext = l;
        e = nx;
        --j;
        ++k;
    }
    *passed = k;
    *pa = A;
    *pb = B;
    return z;
}

// tree_cross_left / tree_cross_right on a run of at most kRankMerge entries:
// the run is loaded at once and scanned in registers with the same
// arithmetic, in the same order, so the results are the same bits; the
// crossed entry's increments come back in ja, jb when z is its jump.
template <int N>
__device__ __forceinline__ double tree_cross_left_short(const TreeWs &W, int64_t s, int64_t t, double A, double B,
                                                        double v, int64_t *passed, double *pa, double *pb,
                                                        bool *jump, double *ja, double *jb) {
    TBp E[N];
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (j < t) E[j] = tb_get(W, s + j);
    bool done = false;
    double z = 0.0, lprev = 0.0;
    int64_t k = t;
    *jump = false;
    *ja = 0.0;
    *jb = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (!done && j < t) {
            const double l = E[j].l;
            const double vl = A * l + B;
            if (vl >= v) {
                z = (v - B) / A;
                z = z > l ? l : z;
                if (j > 0 && z < lprev) z = lprev;
                k = j;
                done = true;
            } else {
                const double vr = vl + E[j].a * l + E[j].b;
                if (vr >= v) {
                    z = l;
                    *jump = true;
                    *ja = E[j].a;
                    *jb = E[j].b;
                    k = j;
                    done = true;
                } else {
                    A += E[j].a;
                    B += E[j].b;
                    lprev = l;
                }
            }
        }
    }
    if (!done) z = (v - B) / A;
    *passed = k;
    *pa = A;
    *pb = B;
    return z;
}

template <int N>
__device__ __forceinline__ double tree_cross_right_short(const TreeWs &W, int64_t s, int64_t t, double A, double B,
                                                         double v, int64_t *passed, double *pa, double *pb,
                                                         bool *jump, double *ja, double *jb) {
    TBp E[N];  // E[m]: entry t - 1 - m of the run
#pragma unroll
    for (int m = 0; m < N; ++m)
        if (m < t) E[m] = tb_get(W, s + t - 1 - m);
    bool done = false;
    double z = 0.0, lnext = 0.0;
    int64_t k = t;
    *jump = false;
    *ja = 0.0;
    *jb = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        if (!done && m < t) {
            const double l = E[m].l;
            const double vr = A * l + B;
            if (vr <= v) {
                z = (v - B) / A;
                z = z < l ? l : z;
                if (m > 0 && z > lnext) z = lnext;
                k = m;
                done = true;
            } else {
                const double vl = vr - (E[m].a * l + E[m].b);
                if (vl <= v) {
                    z = l;
                    *jump = true;
                    *ja = E[m].a;
                    *jb = E[m].b;
                    k = m;
                    done = true;
                } else {
                    A -= E[m].a;
                    B -= E[m].b;
                    lnext = l;
                }
            }
        }
    }
    if (!done) z = (v - B) / A;
    *passed = k;
    *pa = A;
    *pb = B;
    return z;
}

// A node's inputs in FP64 and its parent.
struct TIn {
    double a, b, c, d, lo, hi;
    int64_t p;
};

// Runs of at most this many breakpoints are merged by rank: both are loaded
// at once and every entry goes straight to its place (an entry of the first
// run after the second run's entries with a smaller lambda, one of the second
// run after the first run's entries with a lambda at most its own, as the
// sequential merge orders them), so a merge costs one memory latency rather
// than one per entry.  The same bound selects the unary's insertion point
// from parallel loads.
constexpr int kRankMerge = 8;

// Merge runs [cs, cs + ct) and [s, s + t) (1 <= ct, t <= kRankMerge) into
// [dst, dst + ct + t); every load precedes every store, so dst may overlap
// both runs.
__device__ __forceinline__ void tree_rank_merge(const TreeWs &W, int64_t cs, int64_t ct, int64_t s, int64_t t,
                                                int64_t dst) {
    TBp U[kRankMerge], V[kRankMerge];
#pragma unroll
    for (int k = 0; k < kRankMerge; ++k)
        if (k < ct) U[k] = tb_get(W, cs + k);
#pragma unroll
    for (int m = 0; m < kRankMerge; ++m)
        if (m < t) V[m] = tb_get(W, s + m);
    int64_t pu[kRankMerge], pv[kRankMerge];
#pragma unroll
    for (int k = 0; k < kRankMerge; ++k) {
        int64_t pos = k;
#pragma unroll
        for (int m = 0; m < kRankMerge; ++m) pos += (k < ct && m < t && V[m].l < U[k].l) ? 1 : 0;
        pu[k] = pos;
    }
#pragma unroll
    for (int m = 0; m < kRankMerge; ++m) {
        int64_t pos = m;
#pragma unroll
        for (int k = 0; k < kRankMerge; ++k) pos += (k < ct && m < t && U[k].l <= V[m].l) ? 1 : 0;
        pv[m] = pos;
    }
#pragma unroll
    for (int k = 0; k < kRankMerge; ++k)
        if (k < ct) tb_put(W, dst + pu[k], U[k]);
#pragma unroll
    for (int m = 0; m < kRankMerge; ++m)
        if (m < t) tb_put(W, dst + pv[m], V[m]);
}

// The working message of a node is the run [s, s + t) of its region [r, s + t)
// (the front may float inside the region, so front pops and pushes move
// nothing); the region ends at top = s + t, and the regions of pending
// messages are stacked contiguously below it.
// Lanes (trees) per 64-wide wave.  Each lane's work is a chain of dependent
// memory accesses, so waves that are partly empty trade issue slots for more
// waves per SIMD to hide that latency.
constexpr int kTreeLanes = 64;

template <typename T>
__global__ __launch_bounds__(64) void k_tree_dp(TreeBatch tb, TreeWs W, const T *__restrict__ a,
                                                const T *__restrict__ b, const T *__restrict__ c,
                                                const T *__restrict__ d, const T *__restrict__ wm,
                                                const T *__restrict__ wp, T *__restrict__ x, int lanes) {
    if ((int)threadIdx.x >= lanes) return;
    const int64_t tr = (int64_t)blockIdx.x * lanes + threadIdx.x;
    if (tr >= tb.num_trees) return;
    const int64_t n0 = tb.offsets[tr], n1 = tb.offsets[tr + 1];
    if (n1 <= n0) return;
    const int64_t abase = 6 * n0 + 16 * tr;     // this tree's arena
    const int64_t aend = abase + 6 * (n1 - n0) + 16;
    int64_t top = abase;                          // end of the pending stack's regions
    int64_t sp = n0;                              // header stack pointer
    bool ok = true;
    // a node's inputs are loaded while the node before it is processed
    auto load_in = [&](int64_t i) {
        TIn q;
        q.a = a ? (double)a[i] : 1.0;
        q.b = (double)b[i];
        q.c = c ? (double)c[i] : 0.0;
        q.d = d ? (double)d[i] : 0.0;
        q.lo = (double)wm[i];
        q.hi = (double)wp[i];
        q.p = tb.parent[i];
        return q;
    };
    TIn nx = load_in(n0);
    for (int64_t i = n0; i < n1 && ok; ++i) {
        const TIn in = nx;
        if (i + 1 < n1) nx = load_in(i + 1);
        // (a) the children's messages: the top headers whose node is i, their
        // regions stacked right below the working one; the first is adopted in
        // place, each further one merged with it via the buffer at top
        double al = 0.0, bl = 0.0, ar = 0.0, br = 0.0;
        int64_t r = top, s = top, t = 0;
        while (sp > n0) {
            const THdr hd = W.hdr[sp - 1];
            if (hd.parent != i) break;
            --sp;
            const int64_t cs = hd.start, ct = hd.count, cr = hd.reg;
            if (cr < abase || cs < cr || cs + ct != r || top + ct + t > aend) {
                ok = false;
                break;
            }
            bl += hd.lo;
            br += hd.hi;
            if (t == 0) {
                r = cr;
                s = cs;
                t = ct;
                continue;
            }
            if (ct <= kRankMerge && t <= kRankMerge) {
                tree_rank_merge(W, cs, ct, s, t, cr);
                r = cr;
                s = cr;
                t += ct;
                top = s + t;
                continue;
            }
            // merge run [cs, cs + ct) with run [s, s + t) into [top, top + ct + t)
            int64_t u = cs, v = s, w = top;
            const int64_t ue = cs + ct, ve = s + t;
            TBp eu{0.0, 0.0, 0.0}, ev{0.0, 0.0, 0.0};
            if (u < ue) eu = tb_get(W, u);
            if (v < ve) ev = tb_get(W, v);
            while (u < ue && v < ve) {
                if (eu.l <= ev.l) {
                    tb_put(W, w++, eu);
                    if (++u < ue) eu = tb_get(W, u);
                } else {
                    tb_put(W, w++, ev);
                    if (++v < ve) ev = tb_get(W, v);
                }
            }
            arena_move_n(W, w, u, ue - u);
            w += ue - u;
            arena_move_n(W, w, v, ve - v);
            arena_move_n(W, cr, top, ct + t);  // back to the bottom of the merged regions
            r = cr;
            s = cr;
            t += ct;
            top = s + t;
        }
        if (!ok) break;
        top = s + t;
        // (b) add the unary
        const double ai = in.a, bi = in.b, ci = in.c, di = in.d;
        al += ai;
        bl += -bi - ci;
        ar += ai;
        br += -bi + ci;
        if (ci > 0.0) {
            // insertion point: after every breakpoint <= d_i; the shorter side moves
            int64_t q = t;
            if (t <= kRankMerge) {
                double l[kRankMerge];
#pragma unroll
                for (int j = 0; j < kRankMerge; ++j) l[j] = j < t ? W.ent[s + j].l : 0.0;
                q = 0;
#pragma unroll
                for (int j = 0; j < kRankMerge; ++j) q += (j < t && l[j] <= di) ? 1 : 0;
            } else {
                while (q > 0 && W.ent[s + q - 1].l > di) --q;
            }
            if (s > r && q < t - q) {
                arena_move_n(W, s - 1, s, q);
                --s;
            } else {
                if (top + 1 > aend) {
                    ok = false;
                    break;
                }
                arena_move_n(W, s + q + 1, s + q, t - q);
            }
            tb_put(W, s + q, TBp{di, 0.0, 2.0 * ci, 0.0});
            ++t;
            top = s + t;
        }
        const int64_t p = in.p;
        int64_t k;
        double pa, pb;
        bool jump;
        if (p < 0) {  // root: the zero of h
            const double xr = tree_cross_left(W, s, t, al, bl, 0.0, &k, &pa, &pb, &jump);
            W.lam[i] = TLam{xr, xr};
            top = r;  // nothing stays pending for this root
            continue;
        }
        if (p <= i || p >= n1) {
            ok = false;
            break;
        }
        // (c) clip to [wm_i, wp_i]
        const double lo = in.lo, hi = in.hi;
        if (top + 2 > aend) {
            ok = false;
            break;
        }
        double ja, jb;
        double lm;
        if (t <= kRankMerge) {
            lm = tree_cross_left_short<kRankMerge>(W, s, t, al, bl, lo, &k, &pa, &pb, &jump, &ja, &jb);
        } else {
            lm = tree_cross_left(W, s, t, al, bl, lo, &k, &pa, &pb, &jump);
            if (jump) {
                const TBp e = tb_get(W, s + k);
                ja = e.a;
                jb = e.b;
            }
        }
        double nda = pa, ndb = pb - lo;
        if (jump) {
            nda += ja;
            ndb += jb;
        }
        const int64_t drop = k + (jump ? 1 : 0);
        if (drop == 0) {  // a new front: room in the region, else shift right by one
            if (s > r) {
                --s;
            } else {
                arena_move_n(W, s + 1, s, t);
            }
            ++t;
        } else {  // the new front takes the last dropped slot
            s += drop - 1;
            t -= drop - 1;
        }
        tb_put(W, s, TBp{lm, nda, ndb});
        double lp;
        if (t <= kRankMerge) {
            lp = tree_cross_right_short<kRankMerge>(W, s, t, ar, br, hi, &k, &pa, &pb, &jump, &ja, &jb);
        } else {
            lp = tree_cross_right(W, s, t, ar, br, hi, &k, &pa, &pb, &jump);
            if (jump) {
                const TBp e = tb_get(W, s + t - 1 - k);
                ja = e.a;
                jb = e.b;
            }
        }
        nda = -pa;
        ndb = hi - pb;
        if (jump) {
            nda += ja;
            ndb += jb;
        }
        t -= k + (jump ? 1 : 0);
        tb_put(W, s + t, TBp{lp, nda, ndb});
        ++t;
        top = s + t;
        W.lam[i] = TLam{lm, lp < lm ? lm : lp};
        // push the clipped message for the parent
        W.hdr[sp] = THdr{s, t, r, p, lo, hi};
        ++sp;
    }
    if (!ok || sp != n0) {  // not a post-order numbering (or a tree left children pending)
        *W.bad = 1;
        return;
    }
    // backward pass: parents (higher indices) before children
    for (int64_t i = n1 - 1; i >= n0; --i) {
        const int64_t p = tb.parent[i];
        double v;
        const TLam L = W.lam[i];
        if (p < 0) {
            v = L.lo;
        } else {
            v = (double)x[p];
            v = v < L.lo ? L.lo : (v > L.hi ? L.hi : v);
        }
        x[i] = (T)v;
    }
}

// Workspace: arena of 6 N + 16 T breakpoint records, the header stack and the
// lambda pairs (one record per node each), flag.
static size_t tree_layout(void *p, int64_t T, int64_t N, TreeWs *out) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t A = (size_t)(6 * N + 16 * T);
    size_t off = 0;
    const size_t o_e = off;  off += al(sizeof(TBp) * A);
    const size_t o_h = off;  off += al(sizeof(THdr) * (size_t)N);
    const size_t o_l = off;  off += al(sizeof(TLam) * (size_t)N);
    const size_t o_bd = off; off += al(sizeof(int));
    if (p && out) {
        char *c = (char *)p;
        out->ent = (TBp *)(c + o_e);
        out->hdr = (THdr *)(c + o_h);
        out->lam = (TLam *)(c + o_l);
        out->bad = (int *)(c + o_bd);
    }
    return off;
}

size_t tree_dp_ws_bytes(int64_t num_trees, int64_t num_nodes) {
    return tree_layout(nullptr, num_trees, num_nodes, nullptr);
}

template <typename T>
hipError_t launch_tree_dp_lanes(int64_t num_trees, int64_t num_nodes, const int64_t *offsets, const int64_t *parent,
                                const T *a, const T *b, const T *c, const T *d, const T *wm, const T *wp, T *x,
                                void *workspace, int *bad_host, hipStream_t stream, int lanes) {
    TreeWs W;
    tree_layout(workspace, num_trees, num_nodes, &W);
    hipError_t e = hipMemsetAsync(W.bad, 0, sizeof(int), stream);
    if (e != hipSuccess) return e;
    const TreeBatch tb{num_trees, offsets, parent};
    hipLaunchKernelGGL((k_tree_dp<T>), dim3((unsigned)((num_trees + lanes - 1) / lanes)), dim3(64), 0, stream, tb, W,
                       a, b, c, d, wm, wp, x, lanes);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(bad_host, W.bad, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
}

template <typename T>
hipError_t launch_tree_dp(int64_t num_trees, int64_t num_nodes, const int64_t *offsets, const int64_t *parent,
                          const T *a, const T *b, const T *c, const T *d, const T *wm, const T *wp, T *x,
                          void *workspace, int *bad_host, hipStream_t stream) {
    return launch_tree_dp_lanes<T>(num_trees, num_nodes, offsets, parent, a, b, c, d, wm, wp, x, workspace, bad_host,
                                   stream, kTreeLanes);
}

template hipError_t launch_tree_dp<float>(int64_t, int64_t, const int64_t *, const int64_t *, const float *,
                                          const float *, const float *, const float *, const float *, const float *,
                                          float *, void *, int *, hipStream_t);
template hipError_t launch_tree_dp<double>(int64_t, int64_t, const int64_t *, const int64_t *, const double *,
                                           const double *, const double *, const double *, const double *,
                                           const double *, double *, void *, int *, hipStream_t);

}  // namespace tvc
