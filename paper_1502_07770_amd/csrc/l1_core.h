// l1_core.h -- one step of the TV-l1 chain prox (Sec. 4.2, piecewise-quadratic
// unaries), on any sorted breakpoint store:
//
//     x = argmin_x  sum_e w_e |x_{e+1} - x_e| + sum_i (x_i - y_i)^2 / 2 + sum_i c_i |x_i - d_i| .
//
// The derivative h of the message is non-decreasing, piecewise linear and may
// jump.  With unit quadratic weights every linear piece has an integer slope
// s - k (s = i + 1 unaries added so far; k the step at which the piece was a
// flat end), so a breakpoint holds its position lam, the tag k of the piece to
// its right and the jump of h at lam (>= 0).  The pieces beyond either end
// have slope 1 once the current unary is added; the left end's value is the
// previous clip level w^- plus the unary's left part, the right end's
// likewise.  The back breakpoint's right piece is the right end: its tag is
// kept at 0 (a canonical value, so equal sets compare equal entry by entry).
//
// Adding the unary g_i = z - y_i + c_i sign(z - d_i) inserts a breakpoint at
// d_i with jump 2 c_i; the clip to [-w_i, w_i] scans each end, pops the
// breakpoints it passes and pushes the crossing point.  A crossing at a jump
// replaces that breakpoint with the part of its jump inside the clip range
// (the update of FindMin's increment in Sec. 4.2), so every stored jump stays
// >= 0.
//
// A store provides: size, ovf (set when a push finds it full; the run is then
// discarded), get(j) / put(j, e) on logical positions, pop_front / pop_back,
// push_front / push_back and insert(q, e) keeping the order.
#pragma once
#include "chain_core.h"

namespace tvc {

// Every rounded operation of the DP is the one written: no multiply-add
// contraction (FMAs are explicit), so each step rounds the same in every
// kernel that inlines it and in every build, which the bit-for-bit comparison
// of segment states and the segmented = sequential results rely on.
#pragma clang fp contract(off)


// Slope tag and value jump of a TV-l1 breakpoint.
template <typename T>
struct TagJ {
    T k, j;
};
template <typename T>
__device__ __forceinline__ bool operator==(const TagJ<T> &a, const TagJ<T> &b) {
    return a.k == b.k && a.j == b.j;
}

template <typename T>
struct L1E {
    T l, k, j;  // position, tag of the piece to the right, jump at l
};

// The set in a plain per-lane array in HBM (the fallback), starting in its
// middle: at most one front push per node, and at most three pushes per node.
template <typename T>
struct L1ArrayStore {
    T *lam;
    TagJ<T> *tj;
    int64_t head, size, cap;
    bool ovf;
    __device__ __forceinline__ void init(T *l, TagJ<T> *t, int64_t capacity, int64_t front_room) {
        lam = l;
        tj = t;
        cap = capacity;
        head = front_room;
        size = 0;
        ovf = false;
    }
    __device__ __forceinline__ L1E<T> get(int64_t j) const {
        const TagJ<T> t = tj[head + j];
        return L1E<T>{lam[head + j], t.k, t.j};
    }
    __device__ __forceinline__ void put(int64_t j, const L1E<T> &e) const {
        lam[head + j] = e.l;
        tj[head + j] = TagJ<T>{e.k, e.j};
    }
    __device__ __forceinline__ void pop_front(int64_t k) {
        head += k;
        size -= k;
    }
    __device__ __forceinline__ void pop_back(int64_t k) { size -= k; }
    __device__ __forceinline__ void push_front(const L1E<T> &e) {
        if (head <= 0) {
            ovf = true;
            return;
        }
        --head;
        ++size;
        put(0, e);
    }
    __device__ __forceinline__ void push_back(const L1E<T> &e) {
        if (head + size >= cap) {
            ovf = true;
            return;
        }
        ++size;
        put(size - 1, e);
    }
    __device__ __forceinline__ void insert(int64_t q, const L1E<T> &e) {
        if (head + size >= cap) {
            ovf = true;
            return;
        }
        for (int64_t j = size; j > q; --j) put(j, get(j - 1));
        ++size;
        put(q, e);
    }
};

// The point where h crosses level v from below, scanning from the left:
// h(z) <= v <= h(z+), with h(z) = z + base on the left end piece.  Returns z
// and sets p (breakpoints passed), jump (the crossing is the jump of
// breakpoint p; vj is then h just right of it) and the tag of the piece the
// crossing lies in.
template <typename T, class St>
__device__ __forceinline__ T l1_cross_left(const St &S, T s, T base, T v, int &p, bool &jump, T &vj, T &tagc) {
    const int t = (int)S.size;
    jump = false;
    vj = (T)0;
    if (t == 0) {
        p = 0;
        tagc = s - (T)1;
        return v - base;  // slope 1
    }
    L1E<T> e = S.get(0);
    T vl = e.l + base;  // h just left of the first breakpoint
    if (vl >= v) {
        p = 0;
        tagc = s - (T)1;
        return e.l - (vl - v);
    }
    int j = 0;
    for (;;) {
        const T vr = vl + e.j;
        if (vr >= v) {
            p = j;
            jump = true;
            vj = vr;
            tagc = e.k;
            return e.l;
        }
        if (j + 1 == t) {  // right end piece, slope 1
            p = t;
            tagc = s - (T)1;
            return e.l + (v - vr);
        }
        const L1E<T> nx = S.get(j + 1);
        const T sl = s - e.k;
        const T vn = vr + sl * (nx.l - e.l);  // h just left of the next breakpoint
        if (vn >= v) {
            p = j + 1;
            tagc = e.k;
            return clampv(e.l + (v - vr) * recip(sl), e.l, nx.l);
        }
        vl = vn;
        e = nx;
        ++j;
    }
}

// One forward step at node i (s = i + 1); lop / hip are the clip levels of the
// previous edge, lo / hi those of the leaving edge.  An empty store (the first
// node of a chain, or the start of a run from an assumed zero message) has no
// previous clip: lop = hip = 0 there.  At the root only lm (the zero of h) is
// computed.
template <typename T, class St>
__device__ __forceinline__ void l1_step(St &S, T s, T yi, T di, T ci, T lop, T hip, T lo, T hi, bool root, T &lm,
                                        T &lp) {
    if (S.size == 0) {
        lop = (T)0;
        hip = (T)0;
    }
    // (a) add the unary: the data breakpoint at d_i with jump 2 c_i
    if (ci > (T)0) {
        const int t = (int)S.size;
        int q = 0;
        while (q < t && S.get(q).l <= di) ++q;
        // the new breakpoint splits a piece and inherits its tag; the end pieces
        // have slope 1 (tag s - 1); beyond the back, the old back's right piece
        // becomes interior (slope 1) and the new breakpoint is the back (tag 0)
        T g;
        if (q == t) {
            if (t > 0) {
                L1E<T> b = S.get(t - 1);
                b.k = s - (T)1;
                S.put(t - 1, b);
            }
            g = (T)0;
        } else {
            g = (q == 0) ? s - (T)1 : S.get(q - 1).k;
        }
        S.insert(q, L1E<T>{di, g, (T)2 * ci});
        if (S.ovf) {  // the run is discarded; keep every access in bounds
            lm = lp = (T)0;
            return;
        }
    }
    const T basel = lop - yi - ci;  // left end: h(z) = z + basel
    const T baser = hip - yi + ci;  // right end: h(z) = z + baser
    int p;
    bool jump;
    T vj, tagc;
    lm = l1_cross_left<T>(S, s, basel, root ? (T)0 : lo, p, jump, vj, tagc);
    if (root) return;
    // (b) left clip: flat at lo left of lm; a crossed jump keeps its part above lo
    const int t0 = (int)S.size;
    const bool all = !jump && p == t0;  // lm lies on the right end piece
    if (jump) {
        const T jm = vj - lo;
        S.pop_front(p + 1);
        S.push_front(L1E<T>{lm, (p + 1 == t0) ? (T)0 : tagc, jm < (T)0 ? (T)0 : jm});
    } else {
        S.pop_front(p);
        S.push_front(L1E<T>{lm, all ? (T)0 : tagc, (T)0});
    }
    if (S.ovf) {
        lp = lm;
        return;
    }
    // (c) right clip: flat at hi right of lp; never passes the front entry
    const int t = (int)S.size;
    int j = t - 1;
    L1E<T> e = S.get(j);
    T ur = e.l + baser;  // h just right of the back breakpoint (right end piece)
    if (ur <= hi) {
        lp = e.l + (hi - ur);  // slope 1
        e.k = s - (T)1;         // its right piece is now interior, slope 1
        S.put(j, e);
        S.push_back(L1E<T>{lp, (T)0, (T)0});
    } else {
        for (;;) {
            const T ul = ur - e.j;
            if (ul <= hi || j == 0) {  // crossing at the jump of lam_j
                lp = e.l;
                const T jm = hi - ul;
                S.pop_back(t - j);
                S.push_back(L1E<T>{e.l, (T)0, jm < (T)0 ? (T)0 : jm});
                break;
            }
            const L1E<T> q = S.get(j - 1);
            const T sl = s - q.k;
            const T uq = ul - sl * (e.l - q.l);  // h just right of lam_{j-1}
            if (uq <= hi) {  // inside the piece (lam_{j-1}, lam_j)
                lp = clampv(e.l - (ul - hi) * recip(sl), q.l, e.l);
                S.pop_back(t - j);
                S.push_back(L1E<T>{lp, (T)0, (T)0});
                break;
            }
            ur = uq;
            e = q;
            --j;
        }
    }
    lp = lp < lm ? lm : lp;
}

#pragma clang fp contract(fast)
}  // namespace tvc
