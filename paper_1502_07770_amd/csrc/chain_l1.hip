// chain_l1.hip -- TV-l1 chain prox (Sec. 4.2, piecewise-quadratic unaries):
//
//     x = argmin_x  sum_e w_e |x_{e+1} - x_e| + sum_i (x_i - y_i)^2 / 2 + sum_i c_i |x_i - d_i|,
//
// the row subproblem of the TV-l1 primal-dual iteration (eq. (prox-pq), with
// the quadratic weight normalised to 1).  One lane per chain.
//
// Message representation.  The derivative h of the message is non-decreasing,
// piecewise linear and may jump.  With unit quadratic weights every linear
// piece has an integer slope s - k (s = i + 1 unaries added so far; k the step
// at which the piece was a flat end), so each breakpoint stores its position
// lam, the tag k of the piece to its right, and the jump of h at lam (>= 0).
// The pieces beyond either end have slope 1 once the current unary is added;
// the left end's value is the previous clip level w^- plus the unary's left
// part, the right end's likewise.  Adding the unary g_i = z - y_i +
// c_i sign(z - d_i) inserts a breakpoint at d_i with jump 2 c_i into the
// sorted set; the clip to [-w_i, w_i] scans each end, pops the breakpoints it
// passes and pushes the crossing point.  A crossing at a jump replaces that
// breakpoint with the part of its jump inside the clip range (the update of
// FindMin's increment in Sec. 4.2), so every stored jump stays >= 0.
//
// The set lives in a per-lane ring of K slots in LDS (structure of arrays,
// lane-interleaved); a chain whose set outgrows it is redone by k_l1_ovf with
// the set in HBM.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "seg_kernels.h"

namespace tvc {

constexpr int kL1Ring = 16;
constexpr int kL1Lanes = 1024;  // lanes of the HBM fallback pool

// Sorted breakpoint set in a ring of K slots (LDS) or in a plain array
// (HBM, capacity cap, starting in its middle).
template <typename T, int K>
struct L1RingStore {
    T *lam, *tag, *jmp;  // this lane's columns (slot m at [m * 64])
    int head, size;
    bool ovf;
    __device__ __forceinline__ void init(T *l, T *g, T *j, int lane) {
        lam = l + lane;
        tag = g + lane;
        jmp = j + lane;
        head = 0;
        size = 0;
        ovf = false;
    }
    __device__ __forceinline__ int at(int j) const { return ((head + j) & (K - 1)) * 64; }
    __device__ __forceinline__ T L(int j) const { return lam[at(j)]; }
    __device__ __forceinline__ T G(int j) const { return tag[at(j)]; }
    __device__ __forceinline__ T J(int j) const { return jmp[at(j)]; }
    __device__ __forceinline__ void put(int j, T l, T g, T m) const {
        const int o = at(j);
        lam[o] = l;
        tag[o] = g;
        jmp[o] = m;
    }
    __device__ __forceinline__ bool room() { return size < K ? true : (ovf = true, false); }
    __device__ __forceinline__ void pop_front(int k) {
        head = (head + k) & (K - 1);
        size -= k;
    }
    __device__ __forceinline__ void pop_back(int k) { size -= k; }
    __device__ __forceinline__ void push_front(T l, T g, T m) {
        if (!room()) return;
        head = (head + K - 1) & (K - 1);
        ++size;
        put(0, l, g, m);
    }
    __device__ __forceinline__ void push_back(T l, T g, T m) {
        if (!room()) return;
        ++size;
        put(size - 1, l, g, m);
    }
    // insert at logical position q (0 <= q <= size), shifting the shorter side
    __device__ __forceinline__ void insert(int q, T l, T g, T m) {
        if (!room()) return;
        if (q < size - q) {
            head = (head + K - 1) & (K - 1);
            for (int j = 0; j < q; ++j) put(j, L(j + 1), G(j + 1), J(j + 1));
        } else {
            for (int j = size; j > q; --j) put(j, L(j - 1), G(j - 1), J(j - 1));
        }
        ++size;
        put(q, l, g, m);
    }
};

template <typename T>
struct L1ArrayStore {
    T *lam, *tag, *jmp;
    int64_t head, size, cap;
    bool ovf;
    __device__ __forceinline__ void init(T *l, T *g, T *j, int64_t capacity, int64_t front_room) {
        lam = l;
        tag = g;
        jmp = j;
        cap = capacity;
        head = front_room;
        size = 0;
        ovf = false;
    }
    __device__ __forceinline__ T L(int64_t j) const { return lam[head + j]; }
    __device__ __forceinline__ T G(int64_t j) const { return tag[head + j]; }
    __device__ __forceinline__ T J(int64_t j) const { return jmp[head + j]; }
    __device__ __forceinline__ void put(int64_t j, T l, T g, T m) const {
        lam[head + j] = l;
        tag[head + j] = g;
        jmp[head + j] = m;
    }
    __device__ __forceinline__ void pop_front(int64_t k) {
        head += k;
        size -= k;
    }
    __device__ __forceinline__ void pop_back(int64_t k) { size -= k; }
    __device__ __forceinline__ void push_front(T l, T g, T m) {
        if (head <= 0) {
            ovf = true;
            return;
        }
        --head;
        ++size;
        put(0, l, g, m);
    }
    __device__ __forceinline__ void push_back(T l, T g, T m) {
        if (head + size >= cap) {
            ovf = true;
            return;
        }
        ++size;
        put(size - 1, l, g, m);
    }
    __device__ __forceinline__ void insert(int64_t q, T l, T g, T m) {
        if (head + size >= cap) {
            ovf = true;
            return;
        }
        for (int64_t j = size; j > q; --j) put(j, L(j - 1), G(j - 1), J(j - 1));
        ++size;
        put(q, l, g, m);
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
    T lj = S.L(0);
    T vl = lj + base;  // h just left of the first breakpoint
    if (vl >= v) {
        p = 0;
        tagc = s - (T)1;
        return lj - (vl - v);
    }
    int j = 0;
    for (;;) {
        const T vr = vl + S.J(j);
        if (vr >= v) {
            p = j;
            jump = true;
            vj = vr;
            tagc = S.G(j);
            return lj;
        }
        if (j + 1 == t) {  // right end piece, slope 1
            p = t;
            tagc = s - (T)1;
            return lj + (v - vr);
        }
        const T g = S.G(j);
        const T ln = S.L(j + 1);
        const T sl = s - g;
        const T vn = vr + sl * (ln - lj);  // h just left of the next breakpoint
        if (vn >= v) {
            p = j + 1;
            tagc = g;
            return clampv(lj + (v - vr) * recip(sl), lj, ln);
        }
        vl = vn;
        lj = ln;
        ++j;
    }
}

// One forward step at node i (s = i + 1); lop / hip are the clip levels of the
// previous edge (0 at the first node), lo / hi those of the leaving edge.  At
// the root only lm (the zero of h) is computed.
template <typename T, class St>
__device__ __forceinline__ void l1_step(St &S, T s, T yi, T di, T ci, T lop, T hip, T lo, T hi, bool root, T &lm,
                                        T &lp) {
    // (a) add the unary: the data breakpoint at d_i with jump 2 c_i
    if (ci > (T)0) {
        const int t = (int)S.size;
        int q = 0;
        while (q < t && S.L(q) <= di) ++q;
        // the new breakpoint splits a piece and inherits its tag; the end pieces
        // have slope 1 (tag s - 1), and the old back's right piece becomes
        // interior when d_i lies beyond it (the back entry's tag is never read)
        if (q == t && t > 0) S.put(t - 1, S.L(t - 1), s - (T)1, S.J(t - 1));
        const T g = (q == 0 || q == t) ? s - (T)1 : S.G(q - 1);
        S.insert(q, di, g, (T)2 * ci);
    }
    const T basel = lop - yi - ci;  // left end: h(z) = z + basel
    const T baser = hip - yi + ci;  // right end: h(z) = z + baser
    int p;
    bool jump;
    T vj, tagc;
    lm = l1_cross_left<T>(S, s, basel, root ? (T)0 : lo, p, jump, vj, tagc);
    if (root) return;
    // (b) left clip: flat at lo left of lm; a crossed jump keeps its part above lo
    if (jump) {
        const T jm = vj - lo;
        S.pop_front(p + 1);
        S.push_front(lm, tagc, jm < (T)0 ? (T)0 : jm);
    } else {
        S.pop_front(p);
        S.push_front(lm, tagc, (T)0);
    }
    // (c) right clip: flat at hi right of lp; never passes the front entry
    {
        const int t = (int)S.size;
        int j = t - 1;
        T lj = S.L(j);
        T ur = lj + baser;  // h just right of the back breakpoint (right end piece)
        if (ur <= hi) {
            lp = lj + (hi - ur);  // slope 1
            S.put(j, lj, s - (T)1, S.J(j));  // its right piece is now interior, slope 1
            S.push_back(lp, (T)0, (T)0);
        } else {
            for (;;) {
                const T ul = ur - S.J(j);
                if (ul <= hi || j == 0) {  // crossing at the jump of lam_j
                    lp = lj;
                    T jm = hi - ul;
                    jm = jm < (T)0 ? (T)0 : jm;
                    const T g = S.G(j);
                    S.pop_back(t - j);
                    S.push_back(lj, g, jm);
                    break;
                }
                const T lq = S.L(j - 1);
                const T sl = s - S.G(j - 1);
                const T uq = ul - sl * (lj - lq);  // h just right of lam_{j-1}
                if (uq <= hi) {  // inside the piece (lam_{j-1}, lam_j)
                    lp = clampv(lj - (ul - hi) * recip(sl), lq, lj);
                    S.pop_back(t - j);
                    S.push_back(lp, (T)0, (T)0);
                    break;
                }
                ur = uq;
                lj = lq;
                --j;
            }
        }
    }
    lp = lp < lm ? lm : lp;
}

struct L1Params {
    int64_t C, n, es, cs;
    const int64_t *offsets;
};

template <typename T>
struct L1Ws {
    LamPair<T> *lam;    // [n][C]
    uint8_t *ovf;       // [C]
    int *ovf_count;
    int *ovf_list;      // [C]
    T *fb;              // [lanes][3][cap] HBM sets of the fallback
    int64_t fb_cap, fb_lanes;
};

__device__ __forceinline__ void l1_extent(const L1Params &g, int64_t c, int64_t *base, int64_t *es, int64_t *len) {
    if (g.offsets) {
        const int64_t o0 = g.offsets[c], l = g.offsets[c + 1] - o0;
        *base = o0;
        *es = 1;
        *len = l < 0 ? 0 : (l < g.n ? l : g.n);
    } else {
        *base = c * g.cs;
        *es = g.es;
        *len = g.n;
    }
}

// Forward pass of one chain into the lambda stream; false on overflow.
template <typename T, class St>
__device__ bool l1_forward(St &S, const L1Params &g, const L1Ws<T> &ws, int64_t c, const T *__restrict__ y,
                           const T *__restrict__ d, const T *__restrict__ w, T w_scalar, const T *__restrict__ cw,
                           T c_scalar, T *xroot) {
    int64_t base, es, n;
    l1_extent(g, c, &base, &es, &n);
    T wprev = (T)0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t o = base + i * es;
        const T yi = y[o], di = d[o];
        const T ci = cw ? cw[o] : c_scalar;
        const T wi = w ? w[o] : w_scalar;
        const bool root = (i == n - 1);
        T lm, lp;
        l1_step<T>(S, (T)(int)(i + 1), yi, di, ci, -wprev, wprev, -wi, wi, root, lm, lp);
        if (S.ovf) return false;
        if (root) {
            *xroot = lm;
        } else {
            LamPair<T> pr;
            pr.lo = lm;
            pr.hi = lp;
            ws.lam[i * g.C + c] = pr;
        }
        wprev = wi;
    }
    return true;
}

template <typename T>
__device__ void l1_backward(const L1Params &g, const L1Ws<T> &ws, int64_t c, T xroot, T *__restrict__ x) {
    int64_t base, es, n;
    l1_extent(g, c, &base, &es, &n);
    if (n <= 0) return;
    T v = xroot;
    x[base + (n - 1) * es] = v;
    for (int64_t i = n - 2; i >= 0; --i) {
        const LamPair<T> p = ws.lam[i * g.C + c];
        v = clampv(v, p.lo, p.hi);
        x[base + i * es] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_l1_chain(L1Params g, L1Ws<T> ws, const T *__restrict__ y,
                                                 const T *__restrict__ d, const T *__restrict__ w, T w_scalar,
                                                 const T *__restrict__ cw, T c_scalar, T *__restrict__ x) {
    __shared__ T s_lam[kL1Ring * 64], s_tag[kL1Ring * 64], s_jmp[kL1Ring * 64];
    const int lane = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * 64 + lane;
    if (c == 0) *ws.ovf_count = 0;  // consumed by k_l1_ovf after this kernel
    if (c >= g.C) return;
    L1RingStore<T, kL1Ring> S;
    S.init(s_lam, s_tag, s_jmp, lane);
    T xr = (T)0;
    const bool ok = l1_forward<T>(S, g, ws, c, y, d, w, w_scalar, cw, c_scalar, &xr);
    ws.ovf[c] = ok ? 0 : 1;
    if (ok) l1_backward<T>(g, ws, c, xr, x);
}

// Chains whose set outgrew the ring: a pool of lanes redoes them with the set
// in HBM (lane l owns set storage l).
template <typename T>
__global__ __launch_bounds__(64) void k_l1_collect(L1Params g, L1Ws<T> ws) {
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= g.C || !ws.ovf[c]) return;
    ws.ovf_list[atomicAdd(ws.ovf_count, 1)] = (int)c;
}

template <typename T>
__global__ __launch_bounds__(64) void k_l1_ovf(L1Params g, L1Ws<T> ws, const T *__restrict__ y,
                                               const T *__restrict__ d, const T *__restrict__ w, T w_scalar,
                                               const T *__restrict__ cw, T c_scalar, T *__restrict__ x) {
    const int64_t l = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t cnt = *ws.ovf_count;
    for (int64_t j = l; j < cnt; j += ws.fb_lanes) {
        const int64_t c = ws.ovf_list[j];
        T *base = ws.fb + l * 3 * ws.fb_cap;
        L1ArrayStore<T> S;
        S.init(base, base + ws.fb_cap, base + 2 * ws.fb_cap, ws.fb_cap, g.n + 4);
        T xr = (T)0;
        if (l1_forward<T>(S, g, ws, c, y, d, w, w_scalar, cw, c_scalar, &xr)) l1_backward<T>(g, ws, c, xr, x);
    }
}

// Workspace: [lambda stream n x C][ovf flags C][count][list C][fallback sets].
template <typename T>
size_t l1_ws_layout(void *p, int64_t C, int64_t n, L1Ws<T> *out) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t lanes = C < kL1Lanes ? (C + 63) / 64 * 64 : kL1Lanes;
    // at most one front push per node, and at most three pushes per node in all
    const int64_t cap = 4 * n + 8;
    size_t off = 0;
    const size_t o_lam = off;  off += al(sizeof(LamPair<T>) * (size_t)(n * C));
    const size_t o_ovf = off;  off += al((size_t)C);
    const size_t o_cnt = off;  off += al(sizeof(int));
    const size_t o_lst = off;  off += al(sizeof(int) * (size_t)C);
    const size_t o_fb = off;   off += al(sizeof(T) * (size_t)(lanes * 3 * cap));
    if (p && out) {
        char *b = (char *)p;
        out->lam = (LamPair<T> *)(b + o_lam);
        out->ovf = (uint8_t *)(b + o_ovf);
        out->ovf_count = (int *)(b + o_cnt);
        out->ovf_list = (int *)(b + o_lst);
        out->fb = (T *)(b + o_fb);
        out->fb_cap = cap;
        out->fb_lanes = lanes;
    }
    return off;
}

template <typename T>
size_t chain_l1_ws_bytes(int64_t C, int64_t n) {
    return l1_ws_layout<T>(nullptr, C, n, nullptr);
}

template <typename T>
hipError_t launch_chain_l1(const ChainBatch &bt, const T *y, const T *d, const T *w, T w_scalar, const T *c,
                           T c_scalar, T *x, void *workspace, hipStream_t stream) {
    if (bt.num_chains <= 0) return hipSuccess;
    L1Ws<T> ws;
    l1_ws_layout<T>(workspace, bt.num_chains, bt.n, &ws);
    const L1Params g{bt.num_chains, bt.n, bt.es, bt.cs, bt.offsets};
    const unsigned blocks = (unsigned)((bt.num_chains + 63) / 64);
    hipLaunchKernelGGL((k_l1_chain<T>), dim3(blocks), dim3(64), 0, stream, g, ws, y, d, w, w_scalar, c, c_scalar, x);
    hipLaunchKernelGGL((k_l1_collect<T>), dim3(blocks), dim3(64), 0, stream, g, ws);
    hipLaunchKernelGGL((k_l1_ovf<T>), dim3((unsigned)(ws.fb_lanes / 64)), dim3(64), 0, stream, g, ws, y, d, w,
                       w_scalar, c, c_scalar, x);
    return hipGetLastError();
}

template size_t chain_l1_ws_bytes<float>(int64_t, int64_t);
template size_t chain_l1_ws_bytes<double>(int64_t, int64_t);
template hipError_t launch_chain_l1<float>(const ChainBatch &, const float *, const float *, const float *, float,
                                           const float *, float, float *, void *, hipStream_t);
template hipError_t launch_chain_l1<double>(const ChainBatch &, const double *, const double *, const double *,
                                            double, const double *, double, double *, void *, hipStream_t);

}  // namespace tvc
