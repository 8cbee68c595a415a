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

struct TreeWs {
    double *lam, *da, *db;  // arena [6 N + 16 T] (entries of tree t from 6 off[t] + 16 t)
    int64_t *hstart;        // pending-message stack [N]: start of its breakpoints in the arena
    int64_t *hcount;        //   number of breakpoints
    int64_t *hparent;       //   node the message is for
    double *hlo, *hhi;      //   clip levels (the message's flat ends)
    double *llo, *lhi;      // [N] lambda^-, lambda^+ of each node's edge (root: x_root twice)
    int *bad;               // set if a tree is not numbered in post-order
};

// h(z) <= v <= h(z+) scanning from the left over entries [s, s + t) of the
// arena; returns z, the entries passed, the piece left of z and whether z is
// the jump of entry s + passed.
__device__ double tree_cross_left(const TreeWs &W, int64_t s, int64_t t, double A, double B, double v,
                                  int64_t *passed, double *pa, double *pb, bool *jump) {
    int64_t j = 0;
    double z;
    *jump = false;
    for (;;) {
        if (j == t) {
            z = (v - B) / A;
            break;
        }
        const double l = W.lam[s + j];
        const double vl = A * l + B;
        if (vl >= v) {
            z = (v - B) / A;
            z = z > l ? l : z;
            if (j > 0 && z < W.lam[s + j - 1]) z = W.lam[s + j - 1];
            break;
        }
        const double vr = vl + W.da[s + j] * l + W.db[s + j];
        if (vr >= v) {
            z = l;
            *jump = true;
            break;
        }
        A += W.da[s + j];
        B += W.db[s + j];
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
    for (;;) {
        if (j < 0) {
            z = (v - B) / A;
            break;
        }
        const double l = W.lam[s + j];
        const double vr = A * l + B;
        if (vr <= v) {
            z = (v - B) / A;
            z = z < l ? l : z;
            if (j + 1 < t && z > W.lam[s + j + 1]) z = W.lam[s + j + 1];
            break;
        }
        const double vl = vr - (W.da[s + j] * l + W.db[s + j]);
        if (vl <= v) {
            z = l;
            *jump = true;
            break;
        }
        A -= W.da[s + j];
        B -= W.db[s + j];
        --j;
        ++k;
    }
    *passed = k;
    *pa = A;
    *pb = B;
    return z;
}

__device__ __forceinline__ void arena_move(const TreeWs &W, int64_t to, int64_t from) {
    W.lam[to] = W.lam[from];
    W.da[to] = W.da[from];
    W.db[to] = W.db[from];
}

template <typename T>
__global__ __launch_bounds__(64) void k_tree_dp(TreeBatch tb, TreeWs W, const T *__restrict__ a,
                                                const T *__restrict__ b, const T *__restrict__ c,
                                                const T *__restrict__ d, const T *__restrict__ wm,
                                                const T *__restrict__ wp, T *__restrict__ x) {
    const int64_t tr = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (tr >= tb.num_trees) return;
    const int64_t n0 = tb.offsets[tr], n1 = tb.offsets[tr + 1];
    if (n1 <= n0) return;
    const int64_t abase = 6 * n0 + 16 * tr;     // this tree's arena
    const int64_t acap = 6 * (n1 - n0) + 16;
    int64_t top = abase;                          // arena end of the pending stack
    int64_t sp = n0;                              // header stack pointer
    bool ok = true;
    for (int64_t i = n0; i < n1 && ok; ++i) {
        // (a) the children's messages: the top headers whose node is i (contiguous
        // in the arena); merge them pairwise from the top into one sorted run
        double al = 0.0, bl = 0.0, ar = 0.0, br = 0.0;
        int64_t s = top, t = 0;
        while (sp > n0 && W.hparent[sp - 1] == i) {
            --sp;
            const int64_t cs = W.hstart[sp], ct = W.hcount[sp];
            // a child's run must lie right below the merged run, and the merge
            // buffer above it must fit the arena
            if (cs < abase || cs + ct != s || top + ct + t > abase + acap) {
                ok = false;
                break;
            }
            bl += W.hlo[sp];
            br += W.hhi[sp];
            // merge run [cs, cs + ct) with run [s, s + t) (which follows it) via the buffer at top
            int64_t u = cs, v = s, w = top;
            while (u < cs + ct || v < s + t) {
                if (v >= s + t || (u < cs + ct && W.lam[u] <= W.lam[v])) arena_move(W, w++, u++);
                else arena_move(W, w++, v++);
            }
            for (int64_t q = 0; q < ct + t; ++q) arena_move(W, cs + q, top + q);
            s = cs;
            t += ct;
            top = s + t;
        }
        if (!ok) break;
        // (b) add the unary
        const double ai = a ? (double)a[i] : 1.0;
        const double bi = (double)b[i];
        const double ci = c ? (double)c[i] : 0.0;
        const double di = d ? (double)d[i] : 0.0;
        al += ai;
        bl += -bi - ci;
        ar += ai;
        br += -bi + ci;
        if (ci > 0.0) {
            if (top + 2 - abase > acap) {
                ok = false;
                break;
            }
            int64_t q = t;
            while (q > 0 && W.lam[s + q - 1] > di) {
                arena_move(W, s + q, s + q - 1);
                --q;
            }
            W.lam[s + q] = di;
            W.da[s + q] = 0.0;
            W.db[s + q] = 2.0 * ci;
            ++t;
            top = s + t;
        }
        const int64_t p = tb.parent[i];
        int64_t k;
        double pa, pb;
        bool jump;
        if (p < 0) {  // root: the zero of h
            const double xr = tree_cross_left(W, s, t, al, bl, 0.0, &k, &pa, &pb, &jump);
            W.llo[i] = W.lhi[i] = xr;
            top = s;  // nothing stays pending for this root
            continue;
        }
        if (p <= i || p >= n1) {
            ok = false;
            break;
        }
        // (c) clip to [wm_i, wp_i]
        const double lo = (double)wm[i], hi = (double)wp[i];
        if (top + 2 - abase > acap) {
            ok = false;
            break;
        }
        const double lm = tree_cross_left(W, s, t, al, bl, lo, &k, &pa, &pb, &jump);
        double nda = pa, ndb = pb - lo;
        if (jump) {
            nda += W.da[s + k];
            ndb += W.db[s + k];
        }
        const int64_t drop = k + (jump ? 1 : 0);
        // new front at s + drop - 1 (the dropped entries' last slot), shifting nothing
        const int64_t f = s + drop - 1;
        if (drop == 0) {  // room at the front: shift the run right by one
            for (int64_t q = t; q > 0; --q) arena_move(W, s + q, s + q - 1);
            W.lam[s] = lm;
            W.da[s] = nda;
            W.db[s] = ndb;
            ++t;
        } else {
            W.lam[f] = lm;
            W.da[f] = nda;
            W.db[f] = ndb;
            t -= drop - 1;
            // keep the run starting at s (the stack stays contiguous)
            for (int64_t q = 0; q < t; ++q) arena_move(W, s + q, f + q);
        }
        const double lp = tree_cross_right(W, s, t, ar, br, hi, &k, &pa, &pb, &jump);
        nda = -pa;
        ndb = hi - pb;
        if (jump) {
            nda += W.da[s + t - 1 - k];
            ndb += W.db[s + t - 1 - k];
        }
        t -= k + (jump ? 1 : 0);
        W.lam[s + t] = lp;
        W.da[s + t] = nda;
        W.db[s + t] = ndb;
        ++t;
        top = s + t;
        W.llo[i] = lm;
        W.lhi[i] = lp < lm ? lm : lp;
        // push the clipped message for the parent
        W.hstart[sp] = s;
        W.hcount[sp] = t;
        W.hparent[sp] = p;
        W.hlo[sp] = lo;
        W.hhi[sp] = hi;
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
        if (p < 0) {
            v = W.llo[i];
        } else {
            v = (double)x[p];
            v = v < W.llo[i] ? W.llo[i] : (v > W.lhi[i] ? W.lhi[i] : v);
        }
        x[i] = (T)v;
    }
}

// Workspace: arena 3 x (6 N + 16 T) doubles, headers 3 x N int64 + 2 x N
// doubles, lambdas 2 x N doubles, flag.
static size_t tree_layout(void *p, int64_t T, int64_t N, TreeWs *out) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t A = (size_t)(6 * N + 16 * T);
    size_t off = 0;
    const size_t o_l = off;  off += al(sizeof(double) * A);
    const size_t o_a = off;  off += al(sizeof(double) * A);
    const size_t o_b = off;  off += al(sizeof(double) * A);
    const size_t o_hs = off; off += al(sizeof(int64_t) * (size_t)N);
    const size_t o_hc = off; off += al(sizeof(int64_t) * (size_t)N);
    const size_t o_hp = off; off += al(sizeof(int64_t) * (size_t)N);
    const size_t o_hl = off; off += al(sizeof(double) * (size_t)N);
    const size_t o_hh = off; off += al(sizeof(double) * (size_t)N);
    const size_t o_ll = off; off += al(sizeof(double) * (size_t)N);
    const size_t o_lh = off; off += al(sizeof(double) * (size_t)N);
    const size_t o_bd = off; off += al(sizeof(int));
    if (p && out) {
        char *c = (char *)p;
        out->lam = (double *)(c + o_l);
        out->da = (double *)(c + o_a);
        out->db = (double *)(c + o_b);
        out->hstart = (int64_t *)(c + o_hs);
        out->hcount = (int64_t *)(c + o_hc);
        out->hparent = (int64_t *)(c + o_hp);
        out->hlo = (double *)(c + o_hl);
        out->hhi = (double *)(c + o_hh);
        out->llo = (double *)(c + o_ll);
        out->lhi = (double *)(c + o_lh);
        out->bad = (int *)(c + o_bd);
    }
    return off;
}

size_t tree_dp_ws_bytes(int64_t num_trees, int64_t num_nodes) {
    return tree_layout(nullptr, num_trees, num_nodes, nullptr);
}

template <typename T>
hipError_t launch_tree_dp(int64_t num_trees, int64_t num_nodes, const int64_t *offsets, const int64_t *parent,
                          const T *a, const T *b, const T *c, const T *d, const T *wm, const T *wp, T *x,
                          void *workspace, int *bad_host, hipStream_t stream) {
    TreeWs W;
    tree_layout(workspace, num_trees, num_nodes, &W);
    hipError_t e = hipMemsetAsync(W.bad, 0, sizeof(int), stream);
    if (e != hipSuccess) return e;
    const TreeBatch tb{num_trees, offsets, parent};
    hipLaunchKernelGGL((k_tree_dp<T>), dim3((unsigned)((num_trees + 63) / 64)), dim3(64), 0, stream, tb, W, a, b, c,
                       d, wm, wp, x);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(bad_host, W.bad, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(stream);
}

template hipError_t launch_tree_dp<float>(int64_t, int64_t, const int64_t *, const int64_t *, const float *,
                                          const float *, const float *, const float *, const float *, const float *,
                                          float *, void *, int *, hipStream_t);
template hipError_t launch_tree_dp<double>(int64_t, int64_t, const int64_t *, const int64_t *, const double *,
                                           const double *, const double *, const double *, const double *,
                                           const double *, double *, void *, int *, hipStream_t);

}  // namespace tvc
