// seg_kernels.h -- segment-parallel exact chain TV prox (gfx950).
//
// A chain of n nodes is cut into segments of L nodes; lane (s, c) owns segment
// s of chain c, and consecutive lanes own the same segment of consecutive
// chains (coalesced for column layouts and for the lambda stream).
//
// Why segments can be solved independently and still exactly.  The deque of
// the Sec. 4.1 dynamic program forgets its history: a run started at node
// a - H from an empty deque (an assumed zero incoming message) ends up holding
// bit-for-bit the same breakpoints as the true run after a few dozen nodes on
// the workloads here (median 14, 99th percentile 66 on the 4096^2 image).  From
// the first node where the two deques are equal every later step computes the
// same values.  So:
//  k_seg_main   runs its segment's DP from an empty deque starting H nodes
//               early (the halo, which stores nothing), streams lambda^-/
//               lambda^+ for its own nodes, and saves its deque after the halo
//               (HS), at checkpoints a + 16, 32, 64, 128 inside the segment and
//               at its end (ES).  It then runs the backward clip pass of
//               Algorithm 2 over its own nodes: composing x_i = clip(x_{i+1},
//               lam^-_i, lam^+_i) from the right, the composed map is a clip onto
//               an interval, and once that interval is a single point every node
//               left of it is determined and written; the sweep's state at
//               the checkpoints is recorded for the repair.
//  k_seg_repair compares the saved end state of segment s-1 with the halo state
//               of segment s (hash, then exact comparison of breakpoints and
//               tags); where they differ it reruns the segment from that end
//               state until the deque meets a first-pass checkpoint (or the
//               segment end) and redoes the backward pass left of it.
//  k_seg_fix    one lane per chain: redoes, sequentially, the rare segments
//               whose repair started from a state that was not yet the true one;
//               then composes the value entering each segment from the root.
//               Chains whose deque outgrew the ring go to k_seg_ovf.
//  k_seg_ovf    a pool of lanes solves the overflowed chains with the deque in
//               HBM.
//  k_seg_tail   finishes each segment's un-collapsed right tail from the value at
//               the segment's right end.
// The output is bit-identical to running the DP sequentially per chain.
//
// The deque is a ring of packed (lambda, tag) entries in LDS whose first
// kRingCopies slots are also stored past its end, so the first kRingCopies
// entries lie at fixed offsets from the head: a step reads them in one window
// (the whole deque, almost always) and scans it branch-free (dp_step_ring).
// Loads of node data run P nodes ahead into registers (four per 16-byte load
// on unit-stride chains), so each memory wait covers requests issued a tile
// earlier.
#pragma once
#include <type_traits>

#include "chain_core.h"
#include "l1_core.h"

namespace tvc {

// Every rounded operation of the DP is the one written: no multiply-add
// contraction (FMAs are explicit), so each step rounds the same in every
// kernel that inlines it and in every build, which the bit-for-bit comparison
// of segment states and the segmented = sequential results rely on.
#pragma clang fp contract(off)


template <typename T>
struct alignas(2 * sizeof(T)) LamPair {
    T lo, hi;
};

// A deque entry: breakpoint lambda and the tag k of the segment to its right.
// With a_i = 1 the tag is the birth step, kept as a floating-point integer in
// the working precision (exact below 2^24 for float) so the slope s - k is one
// exact subtraction; with general a_i it is the FP64 prefix sum Abar_k; for
// TV-l1 sets it is the birth step and the jump of h at lambda (TagJ).  Every
// step leaves the back entry's tag at a value fixed by the node (the step's
// own index in the Sec. 4.1 deque, 0 in a TV-l1 set), so saved states compare
// entry by entry, tags included.
constexpr size_t ent_align(size_t b) { return b <= 8 ? 8 : (b <= 16 ? 16 : 32); }
template <typename T, typename G = T>
struct alignas(ent_align(sizeof(T) + sizeof(G))) Ent {
    T l;
    G k;
};

template <typename T, typename G> __device__ __forceinline__ Ent<T, G> mk_ent(T l, G k) {
    Ent<T, G> e;
    e.l = l;
    e.k = k;
    return e;
}

// Segment geometry: halo H and checkpoint spacing CK (both multiples of the
// tile) and the saved-state slots per segment.
constexpr int kCheckpoints = 4;  // first-pass deques saved at a + CK, 2 CK, 4 CK, 8 CK in a segment
constexpr int kSaves = 3 + kCheckpoints;  // HS, CK..., ES, ES2
// Ring slots stored twice (slot m < kRingCopies also at m + K): the step reads
// the first kRingCopies entries of a deque at fixed offsets from its head.
// The rings of the TV deque (tags in the working precision) copy twice as
// many, so that a window twice as wide needs no wrap either: the 2D
// iterations' deques often hold 8 to 15 breakpoints.  The general DP's FP32
// rings (FP64 prefix-sum tags, 16-byte entries, shallow deques) and the TV-l1
// sets (TagJ entries, which no window reads) keep kRingCopies.
constexpr int kRingCopies = 8;
template <typename T, typename G> constexpr int ring_copies() {
    return std::is_same<T, G>::value ? 2 * kRingCopies : kRingCopies;
}
// Nodes the backward sweep loads ahead of their use.
constexpr int kSweepTile = 16;
// Lanes (each with a 2n + 4 entry HBM deque) for chains that overflow the ring.
constexpr int64_t kOverflowLanes = 1024;
// Nodes per register tile of the overflow kernel's forward runs.
constexpr int kTileOvf = 8;
constexpr int kSaveHalo = 0, kSaveCk = 1, kSaveEnd = 1 + kCheckpoints, kSaveEnd2 = 2 + kCheckpoints;

template <typename T, typename G = T>
struct SegWs {
    int64_t C;          // chains
    int64_t n;          // maximum chain length
    int64_t L;          // segment length
    int64_t S;          // segments per chain of length n
    int64_t H;          // halo
    int64_t CK;         // checkpoint spacing
    LamPair<T> *lam;    // [n][C]
    Ent<T, G> *st;      // saved deques [S][kSaves][K][C] (ES2: the repair's end state)
    int *st_size;       // [S][kSaves][C]
    uint32_t *st_hash;  // [S][kSaves][C]
    uint8_t *ovf;       // [C][S] ring overflow
    uint8_t *mis;       // [C][S] halo state != end state of the previous segment
    uint8_t *clean;     // [C][S] the repair met a first-pass checkpoint
    int *rep_stop;      // [S][C] node where the repair stopped
    T *seg_lo;          // [S][C] composed backward clip of the segment
    T *seg_hi;
    int *seg_unc;       // [S][C] first node of the un-collapsed tail
    T *seg_xb;          // [S][C] x at the first node after the segment
    int *ovf_count;     // chains appended to ovf_list (zeroed by k_seg_main)
    int *ovf_list;      // [C] chains whose deque outgrew the LDS ring
    LamPair<T> *sw_cp;  // [kCheckpoints][S][C] first-pass backward-sweep state at the checkpoints
    T *fb_lam;          // [fb_lanes][2n+4] HBM deques of the overflow kernel
    G *fb_tag;
    int64_t fb_cap;
    int64_t fb_lanes;
    const int *stop;    // device flag (or null): when set, every kernel of the launch returns at once
};

// The launch's stop flag is set (a 2D solve that already met its stopping test).
template <typename T, typename G>
__device__ __forceinline__ bool seg_stopped(const SegWs<T, G> &ws) {
    return ws.stop && *(volatile const int *)ws.stop;
}

struct ChainSpan {
    int64_t base;  // element of node 0
    int64_t es;    // element stride
    int64_t n;     // nodes
    int64_t aux;   // problem-specific tag (e.g. the image of a batched chain)
};

template <typename T> __device__ __forceinline__ T pos_inf();
template <> __device__ __forceinline__ float pos_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double pos_inf<double>() { return __builtin_huge_val(); }

template <int K> __device__ __forceinline__ int clamp_size(int v) { return v < 0 ? 0 : (v > K ? K : v); }

__device__ __forceinline__ uint32_t bits32(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t bits32(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return (uint32_t)b ^ (uint32_t)(b >> 32) * 0x9E3779B1u;
}

// State comparison of two deque entries (bit for bit: two runs whose states
// hold the same bits compute the same values from then on; == would also take
// -0 for +0), and the entry's share of the state hash.
__device__ __forceinline__ bool same_bits(float a, float b) { return __float_as_uint(a) == __float_as_uint(b); }
__device__ __forceinline__ bool same_bits(double a, double b) {
    return __double_as_longlong(a) == __double_as_longlong(b);
}
template <typename T, typename G> __device__ __forceinline__ bool ent_same(T la, const G &ka, T lb, const G &kb) {
    return same_bits(la, lb) && same_bits(ka, kb);
}
template <typename T>
__device__ __forceinline__ bool ent_same(T la, const TagJ<T> &ka, T lb, const TagJ<T> &kb) {
    return same_bits(la, lb) && same_bits(ka.k, kb.k) && same_bits(ka.j, kb.j);
}
template <typename T, typename G> __device__ __forceinline__ uint32_t ent_hash(uint32_t h, T l, const G &k, bool tag) {
    h = (h ^ bits32(l)) * 0x01000193u;
    return tag ? (h ^ bits32(k)) * 0x01000193u : h;
}
template <typename T>
__device__ __forceinline__ uint32_t ent_hash(uint32_t h, T l, const TagJ<T> &k, bool tag) {
    h = (h ^ bits32(l)) * 0x01000193u;
    h = (h ^ bits32(k.j)) * 0x01000193u;
    return tag ? (h ^ bits32(k.k)) * 0x01000193u : h;
}

template <typename T, int K, typename G = T> struct CRing;

// Entry-by-entry comparison of a ring with a saved state of the same size,
// loading the saved entries in independent batches of eight.
template <typename T, int K, typename G>
__device__ __forceinline__ bool saved_equal(const CRing<T, K, G> &R, const Ent<T, G> *src, int64_t stride);

// ---------------------------------------------------------------------------
// LDS ring of K entries per lane.  The first kRingCopies slots are stored
// twice, at slot m and at slot m + K, so the first kRingCopies entries of the
// deque lie at fixed offsets from the head slot (logical j at physical
// head + j < K + kRingCopies): the step's window needs no per-read index
// arithmetic and never wraps, and a lane needs K + kRingCopies slots rather
// than 2K.  Slots are lane-interleaved (slot m of lane l at m * 64 + l), so the
// 64 lanes of a wave hit distinct banks.
// ---------------------------------------------------------------------------
template <typename T, int K, typename G>
struct CRing {
    static_assert((K & (K - 1)) == 0, "ring size must be a power of two");
    using E = Ent<T, G>;
    // Small rings of 8-byte entries copy every slot (2K rows: a copy is one
    // more store at a fixed offset, no address select); others only the first
    // kCopies.
    static constexpr bool kAll = (K <= 16 && sizeof(E) <= 8);
    static constexpr int kCopies = kAll ? K : ring_copies<T, G>();
    static_assert(kCopies <= K, "the copied slots are ring slots");
    // slot rows of the per-wave LDS array (64 entries each)
    static constexpr int kRows = kAll ? 2 * K : K + kCopies;
    E *col;  // this lane's column: slot m at col[m * 64], its copy at col[(m + K) * 64]
    int head, size;

    __device__ __forceinline__ void init(E *base, int lane) {
        col = base + lane;
        head = 0;
        size = 0;
        seal();
    }
    __device__ __forceinline__ E ld(int j) const { return col[((head + j) & (K - 1)) * 64]; }
    __device__ __forceinline__ void put_slot(int m, const E &e) const {
        col[m * 64] = e;
        if constexpr (kAll)
            col[(m + K) * 64] = e;
        else
            col[(m < kCopies ? m + K : m) * 64] = e;  // other slots: the same slot again
    }
    // The slot after the back holds a +inf breakpoint (dp_step_ring's
    // sentinel; the TV-l1 sets never read it).  A full ring has no such slot.
    __device__ __forceinline__ void seal() const {
        if (size < K) put_slot((head + size) & (K - 1), mk_ent<T, G>(pos_inf<T>(), G{}));
    }
    __device__ __forceinline__ void set(int j, const E &e) const { put_slot((head + j) & (K - 1), e); }
    // Order-sensitive 32-bit hash of the breakpoints and tags (the back tag is
    // excluded; see ent_hash); a filter only: equality is always confirmed
    // entry by entry.
    __device__ __forceinline__ uint32_t hash() const {
        uint32_t h = 0x811C9DC5u ^ (uint32_t)size;
        for (int j = 0; j < size; ++j) {
            const E e = ld(j);
            h = ent_hash<T>(h, e.l, e.k, j + 1 < size);
        }
        return h;
    }
    __device__ __forceinline__ void save(E *dst, int *szdst, uint32_t *hdst, int64_t stride) const {
        *szdst = size;
        *hdst = hash();
        for (int j = 0; j < size; ++j) dst[j * stride] = ld(j);
    }
    __device__ __forceinline__ void load(const E *src, const int *szsrc, int64_t stride) {
        head = 0;
        size = clamp_size<K>(*szsrc);
        for (int j = 0; j < size; ++j) put_slot(j, src[j * stride]);
        seal();
    }
    // Same breakpoints and tags (the back entry's tag is never read).  Size
    // and hash reject most unequal states with two loads; the exact check
    // loads the saved entries eight at a time.
    __device__ __forceinline__ bool equals(const E *src, const int *szsrc, const uint32_t *hsrc,
                                           int64_t stride) const {
        if (*szsrc != size || *hsrc != hash()) return false;
        return saved_equal<T, K, G>(*this, src, stride);
    }
};

template <typename T, int K, typename G>
__device__ __forceinline__ bool saved_equal(const CRing<T, K, G> &R, const Ent<T, G> *src, int64_t stride) {
    const int n = R.size;
    bool eq = true;
    for (int j0 = 0; j0 < n && eq; j0 += 8) {
        Ent<T, G> e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = src[(j0 + j < n ? j0 + j : n - 1) * stride];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int jj = j0 + j;
            if (jj < n) {
                const Ent<T, G> m = R.ld(jj);
                eq = eq && ent_same<T>(e[j].l, e[j].k, m.l, m.k);
            }
        }
    }
    return eq;
}

// ---------------------------------------------------------------------------
// One Sec. 4.1 step on a deque of breakpoints (transformations (a) and (b)
// of the message update): lambda^- and lambda^+ of node i, and the deque of
// the message passed on.
//
// Entry j of the deque holds breakpoint lam_j and the tag k_j of the segment
// to its right, whose true slope at step s is Abar_s - k_j (s - k_j when
// a_i = 1).  Three conventions make every bracket the same formula:
//  * the segment left of the front has the end slope a_s (the flat left end
//    of the clipped message plus the node's unary);
//  * the back entry's tag is Abar of the step that pushed it, so one step
//    later its right segment (the flat right end plus a unary) has slope
//    a_s too, and an old back that stays interior needs no new tag;
//  * the slot after the back holds a +inf breakpoint (the sentinel).
// The message derivative at the breakpoints, v_0 = a_s lam_0 + w^-_prev - b_i
// and v_j = v_{j-1} + (Abar_s - k_{j-1}) (lam_j - lam_{j-1}), is
// non-decreasing; it is +inf at the sentinel and NaN past it, so the number p
// of breakpoints with v_j < w^- (popped at the left) and the number r with
// v_j <= w^+ (the rest are popped at the right) need no masks: comparisons
// with NaN are false.  lambda^- lies on the segment left of lam_p (the left
// end when p = 0), lambda^+ on the segment left of lam_r, which is lambda^-'s
// own when r = p.  The new deque (lambda^-, lam_p .. lam_{r-1}, lambda^+)
// takes slot p - 1 for the front, slot r for the back and r + 1 for the
// sentinel: the surviving breakpoints stay where they are.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T fmav(T a, T b, T c);
template <> __device__ __forceinline__ float fmav<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmav<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
struct DqScan {
    int p, r;  // breakpoints with v < w^- / with v <= w^+
    T vL, vR;  // v at breakpoint p - 1 / r - 1 (v_0 when p / r is 0)
};

// One breakpoint of the scan: v is the message derivative at breakpoint j.
template <typename T>
__device__ __forceinline__ void dq_count(DqScan<T> &sc, int j, T v, T lo, T hi) {
    const bool cl = v < lo;
    sc.p = cl ? j + 1 : sc.p;
    sc.vL = cl ? v : sc.vL;
    const bool ch = v <= hi;
    sc.r = ch ? j + 1 : sc.r;
    sc.vR = ch ? v : sc.vR;
}

// The solves.  E0 / E1 are entries max(p - 1, 0) and the one after it, G0 / G1
// entries max(r - 1, 0) and the one after it.  Each root is clamped to its
// segment (rounding guard), which also keeps lambda^- <= lambda^+.
template <typename T, typename G, bool kGen>
__device__ __forceinline__ void dq_solve(const DqScan<T> &sc, const StepIn<T, G> &in, const EndSlope<T, G, kGen> &es,
                                         bool empty, const Ent<T, G> &E0, const Ent<T, G> &E1, const Ent<T, G> &G0,
                                         const Ent<T, G> &G1, T &lm, T &lp, G &tnew) {
    const T lo = in.lo, hi = in.hi;
    const bool pl = sc.p > 0;
    const T rL = pl ? recip(slope_of<T, G>(in.sf, E0.k)) : es.ra;
    const T a = fmav(lo - sc.vL, rL, E0.l);
    // an empty deque (a run's first node, from an assumed zero message): a_s z - b_s
    lm = empty ? es.div(in.yi + lo) : clampv(a, pl ? E0.l : -pos_inf<T>(), pl ? E1.l : E0.l);
    tnew = pl ? E0.k : (kGen ? in.sprev : (G)(in.sf - (G)1));
    const bool rs = sc.r == sc.p;
    const T rR = rs ? rL : recip(slope_of<T, G>(in.sf, G0.k));
    const T base = rs ? lm : G0.l;
    const T b = fmav(hi - (rs ? lo : sc.vR), rR, base);
    lp = empty ? es.div(in.yi + hi) : clampv(b, base, sc.r > 0 ? G1.l : G0.l);
}

// The deque update through an accessor (put(j, e) writes logical entry j of
// the current deque, j = -1 allowed; shift(d) moves the head by d).  Returns
// the new number of breakpoints.
template <typename T, typename G, class A>
__device__ __forceinline__ int dq_update(A &R, const DqScan<T> &sc, G sf, T lm, T lp, G tnew) {
    R.put(sc.p - 1, mk_ent<T, G>(lm, tnew));
    R.put(sc.r, mk_ent<T, G>(lp, sf));
    R.put(sc.r + 1, mk_ent<T, G>(pos_inf<T>(), G{}));
    R.shift(sc.p - 1);
    return sc.r - sc.p + 2;
}

// Deques of at least this many breakpoints take the two-ended scan.
constexpr int kTwoEnded = 16;

// The scan of a deque of t breakpoints.  Below kTwoEnded breakpoints it is a
// front walk with the window's values in the window's order, stopping past
// the w^+ crossing (at the latest at the sentinel, entry t); it reads r + 1
// breakpoints, which on shallow deques is no more than a walk from the back.
// From kTwoEnded on it is two-ended: the front walk stops at the w^- crossing,
// and the w^+ crossing is found walking from the back, with values from the
// right end piece (h(z) = w^+_prev + a_s z - b_s beyond the back breakpoint),
// so a step reads the breakpoints it pops and one more at each end: the O(1)
// amortised step of Sec. 4.1 however deep the deque.  Values near the back
// differ in rounding from a front walk's; since the form follows the deque's
// own depth, in the ring and in the HBM deque alike, a state always takes the
// same arithmetic and segmented runs stay bit-identical.  Rounding cannot make
// the w^+ count fall below the w^- count: it is raised to it.
// kDeep false: the store never holds kTwoEnded breakpoints (a 16-slot ring).
template <typename T, typename G, bool kGen, bool kDeep, class A>
__device__ __forceinline__ DqScan<T> dq_scan(const A &R, int t, const StepIn<T, G> &in,
                                             const EndSlope<T, G, kGen> &es) {
    const bool deep = kDeep && t >= kTwoEnded;
    Ent<T, G> prev = R.ld(0);
    T v = es.mul(prev.l) + (in.lop - in.yi);
    DqScan<T> sc{0, 0, v, v};
    for (int j = 0; j <= t; ++j) {
        if (j > 0) {
            const Ent<T, G> e = R.ld(j);
            v = fmav(slope_of<T, G>(in.sf, prev.k), e.l - prev.l, v);
            prev = e;
        }
        if (deep ? !(v < in.lo) : !(v <= in.hi)) break;
        dq_count(sc, j, v, in.lo, in.hi);
    }
    if (deep) {
        int j = t - 1;
        Ent<T, G> b = R.ld(j);
        T u = es.mul(b.l) + (in.hip - in.yi);  // h at breakpoint j
        while (!(u <= in.hi) && j > 0) {
            const Ent<T, G> pv = R.ld(j - 1);
            u = fmav(slope_of<T, G>(in.sf, pv.k), pv.l - b.l, u);
            b = pv;
            --j;
        }
        sc.r = (u <= in.hi) ? j + 1 : 0;
        sc.vR = u;
        if (sc.r < sc.p) {
            sc.r = sc.p;
            sc.vR = sc.vL;
        }
    }
    return sc;
}

// Accessor of a CRing by logical entry.
template <typename T, int K, typename G>
struct RingAcc {
    CRing<T, K, G> &R;
    __device__ __forceinline__ Ent<T, G> ld(int j) const { return R.ld(j); }
    __device__ __forceinline__ void put(int j, const Ent<T, G> &e) const { R.put_slot((R.head + j) & (K - 1), e); }
    __device__ __forceinline__ void shift(int d) const { R.head = (R.head + d) & (K - 1); }
};

// The step in its general form: any depth (dq_scan) and an empty deque.  It
// serves a run's first node and the rare wave in which some deque is deeper
// than the window.
template <typename T, typename G, int K, bool kGen>
__device__ __forceinline__ bool dp_step_ring_general(CRing<T, K, G> &R, const StepIn<T, G> &in, T &lm, T &lp) {
    const EndSlope<T, G, kGen> es(in.sf, in.sprev);
    const int t = R.size;
    RingAcc<T, K, G> A{R};
    const DqScan<T> sc = dq_scan<T, G, kGen, (K > kTwoEnded)>(A, t, in, es);
    const int i0 = sc.p > 0 ? sc.p - 1 : 0, i1 = sc.r > 0 ? sc.r - 1 : 0;
    G tnew;
    dq_solve<T, G, kGen>(sc, in, es, t == 0, A.ld(i0), A.ld(i0 + 1), A.ld(i1), A.ld(i1 + 1), lm, lp, tnew);
    const int tn = dq_update<T, G>(A, sc, in.sf, lm, lp, tnew);
    R.size = tn < K ? tn : K;
    return tn < K;
}

// The windowed step: every lane's deque has 1 .. WN - 1 breakpoints, all of
// them and the sentinel in copied slots, read in one window from the head at
// fixed offsets and scanned branch-free.
template <typename T, typename G, int K, bool kGen, int WN>
__device__ __forceinline__ bool dp_step_window(CRing<T, K, G> &R, const StepIn<T, G> &in, T &lm, T &lp) {
    using E = Ent<T, G>;
    const EndSlope<T, G, kGen> es(in.sf, in.sprev);
    const T lo = in.lo, hi = in.hi;
    const T c = in.lop - in.yi;
    DqScan<T> sc;
    E E0, E1, G0, G1;
    G tnew;
    {
        const E *fp = R.col + R.head * 64;
        E F[WN];
#pragma unroll
        for (int j = 0; j < WN; ++j) F[j] = fp[j * 64];
        T v = es.mul(F[0].l) + c;
        sc = DqScan<T>{0, 0, v, v};
        dq_count(sc, 0, v, lo, hi);
#pragma unroll
        for (int j = 1; j < WN; ++j) {
            v = fmav(slope_of<T, G>(in.sf, F[j - 1].k), F[j].l - F[j - 1].l, v);
            dq_count(sc, j, v, lo, hi);
        }
        const E *pb = fp + (sc.p > 0 ? sc.p - 1 : 0) * 64;
        const E *qb = fp + (sc.r > 0 ? sc.r - 1 : 0) * 64;
        E0 = pb[0];
        E1 = pb[64];
        G0 = qb[0];
        G1 = qb[64];
        dq_solve<T, G, kGen>(sc, in, es, false, E0, E1, G0, G1, lm, lp, tnew);
    }
    RingAcc<T, K, G> A{R};
    const int tn = dq_update<T, G>(A, sc, in.sf, lm, lp, tnew);
    R.size = tn < K ? tn : K;
    return tn < K;
}

// One step on the LDS ring.  Deques of fewer than kRingCopies breakpoints
// (sentinel included, all in copied slots) are read in one window from the
// head at fixed offsets and scanned branch-free; in a ring with twice as many
// copied slots (every deque ring), deques of up to 2 kRingCopies - 1
// breakpoints take a window twice as wide, the same front walk without its
// branches.  Deeper ones take
// the two-ended scan.  The root step is the same step with a zero leaving
// edge (its deque update is never used).  Returns false if the ring cannot
// hold the new deque and its sentinel.
template <typename T, typename G, int K, bool kGen>
__device__ __forceinline__ bool dp_step_ring(CRing<T, K, G> &R, const StepIn<T, G> &in, T &lm, T &lp) {
    constexpr int M = kRingCopies;
    const int t = R.size;
    // Almost always every lane of the wave holds 1 .. M - 1 breakpoints: one
    // window and no selects for an empty deque, decided once for the wave.
    // Otherwise (a run's first node, or a deque deeper than the window in
    // some lane) the wider window if it holds every lane's deque, else every
    // lane takes the general step, whose front walk for the shallow lanes
    // gives the window's bits.
    if (__ballot((t == 0) | (t >= M))) {
        if constexpr (CRing<T, K, G>::kCopies >= 2 * M) {
            if (!__ballot((t == 0) | (t >= 2 * M))) return dp_step_window<T, G, K, kGen, 2 * M>(R, in, lm, lp);
        }
        return dp_step_ring_general<T, G, K, kGen>(R, in, lm, lp);
    }
    return dp_step_window<T, G, K, kGen, M>(R, in, lm, lp);
}

// The same step with the deque in HBM (the exact fallback for deques that
// outgrow every LDS ring): 2n + 4 entries per lane, the head starting at
// n + 2.  The head moves down by at most one per step and the sentinel's slot
// up by at most one, so n steps stay inside: the 4n + O(1) array of Sec. 4.1,
// two numbers per breakpoint.
template <typename T, typename G>
struct HbmDeque {
    T *lam;
    G *tag;
    int64_t head;
    int size;
    __device__ __forceinline__ void init(T *l, G *k, int64_t cap) {
        lam = l;
        tag = k;
        head = cap / 2;
        size = 0;
        put(0, mk_ent<T, G>(pos_inf<T>(), G{}));
    }
    __device__ __forceinline__ Ent<T, G> ld(int j) const { return mk_ent<T, G>(lam[head + j], tag[head + j]); }
    __device__ __forceinline__ void put(int j, const Ent<T, G> &e) const {
        lam[head + j] = e.l;
        tag[head + j] = e.k;
    }
    __device__ __forceinline__ void shift(int d) { head += d; }
};
template <typename T, typename G, bool kGen>
__device__ __forceinline__ void dp_step_hbm(HbmDeque<T, G> &D, const StepIn<T, G> &in, T &lm, T &lp) {
    const EndSlope<T, G, kGen> es(in.sf, in.sprev);
    const int t = D.size;
    const DqScan<T> sc = dq_scan<T, G, kGen, true>(D, t, in, es);
    const int i0 = sc.p > 0 ? sc.p - 1 : 0, i1 = sc.r > 0 ? sc.r - 1 : 0;
    G tnew;
    dq_solve<T, G, kGen>(sc, in, es, t == 0, D.ld(i0), D.ld(i0 + 1), D.ld(i1), D.ld(i1 + 1), lm, lp, tnew);
    D.size = dq_update<T, G>(D, sc, in.sf, lm, lp, tnew);
}

// ---------------------------------------------------------------------------
// Shared pieces.
// ---------------------------------------------------------------------------
// A problem policy (Prob) supplies its node records (Pre) through Src, and
// declares its model: Tag = the tag type, kGen = general a_i and asymmetric
// weights.  With kGen false Src provides data (b_i = y_i) and weight (w_i of
// the leaving edge, w^- = -w_i, w^+ = w_i); with kGen true it provides data,
// wlo / whi (w^-, w^+ of the leaving edge), prefix(pv, i, Abar_{i-1}) = Abar_i
// and prefix_before(i) = Abar_{i-1} (FP64; equal bits on every run).
//
// What a step needs from the node before it.
template <typename T, typename G, bool kGen> struct Carry;
template <typename T, typename G> struct Carry<T, G, false> {
    T wprev;
};
template <typename T, typename G> struct Carry<T, G, true> {
    G sprev;
    T lop, hip;
};
template <typename T, class Prob> using CarryOf = Carry<T, typename Prob::Tag, Prob::kGen>;
template <typename T, class Prob> using WsOf = SegWs<T, typename Prob::Tag>;
template <typename T, class Prob> using EntOf = Ent<T, typename Prob::Tag>;

// The carry of a run that starts at node i (node i - 1's leaving edge and
// prefix; zeros at the first node).
template <typename T, class Prob>
__device__ __forceinline__ CarryOf<T, Prob> carry_before(const typename Prob::Src &src, int64_t i) {
    CarryOf<T, Prob> cy;
    if constexpr (Prob::kGen) {
        cy.sprev = 0;
        cy.lop = (T)0;
        cy.hip = (T)0;
        if (i > 0) {
            const auto pv = src.load(i - 1);
            cy.sprev = src.prefix_before(i);
            cy.lop = src.wlo(pv);
            cy.hip = src.whi(pv);
        }
    } else {
        cy.wprev = (i > 0) ? src.weight(src.load(i - 1)) : (T)0;
    }
    return cy;
}

// Inputs of the step at node i (root: zero leaving edge); advances the carry.
template <typename T, class Prob>
__device__ __forceinline__ StepIn<T, typename Prob::Tag> step_in(const typename Prob::Src &src,
                                                                 const typename Prob::Pre &pv, int64_t i, bool root,
                                                                 CarryOf<T, Prob> &cy) {
    StepIn<T, typename Prob::Tag> in;
    in.yi = src.data(pv);
    if constexpr (Prob::kGen) {
        const T wl = src.wlo(pv), wh = src.whi(pv);
        in.sf = src.prefix(pv, i, cy.sprev);
        in.sprev = cy.sprev;
        in.lop = cy.lop;
        in.hip = cy.hip;
        in.lo = root ? (T)0 : wl;
        in.hi = root ? (T)0 : wh;
        cy.sprev = in.sf;
        cy.lop = wl;
        cy.hip = wh;
    } else {
        const T wi = src.weight(pv);
        const T w = root ? (T)0 : wi;
        in.sf = (T)(int)(i + 1);
        in.sprev = in.sf - (T)1;
        in.lop = -cy.wprev;
        in.hip = cy.wprev;
        in.lo = -w;
        in.hi = w;
        cy.wprev = wi;
    }
    return in;
}

// TV-l1 problems (Prob::kL1): the set of the Sec. 4.2 message in the ring.
template <class Prob, class = void> struct IsL1 : std::false_type {};
template <class Prob> struct IsL1<Prob, std::void_t<decltype(Prob::kL1)>> : std::bool_constant<Prob::kL1> {};

// A TV-l1 problem on FP32 data solved with its set in FP64.  A crossing at a
// breakpoint's jump keeps the part of the jump beyond the clip level, so a
// breakpoint that is crossed on many consecutive nodes carries a running sum
// of data terms in its jump.  In FP32 that sum drifts by rounding (about 1e-5
// of the data scale after a few hundred nodes), which moves the minimiser
// across a kink of the l1 term wherever two candidates are close, and it
// keeps a run started from an empty set apart from the true run bit for bit,
// so the segments would rarely meet.  In FP64 both effects vanish at FP32
// output precision.  Data are read and x written in FP32; lambda^-/lambda^+
// and the backward clip are FP64.
template <class P>
struct WideL1 {
    using Tag = TagJ<double>;
    static constexpr bool kGen = false;
    static constexpr bool kL1 = true;
    using Params = typename P::Params;
    using Pre = typename P::Pre;
    using SinkPre = typename P::SinkPre;
    struct Src {
        typename P::Src in;
        bool vec;
        __device__ __forceinline__ Src(const typename P::Src &s) : in(s), vec(s.vec) {}
        __device__ __forceinline__ Pre load(int64_t i) const { return in.load(i); }
        __device__ __forceinline__ int64_t off(int64_t i) const { return in.off(i); }
        __device__ __forceinline__ int64_t step() const { return in.step(); }
        __device__ __forceinline__ Pre load_off(int64_t o) const { return in.load_off(o); }
        __device__ __forceinline__ void load4(int64_t i, Pre *o) const { in.load4(i, o); }
        __device__ __forceinline__ double data(const Pre &p) const { return (double)in.data(p); }
        __device__ __forceinline__ double dval(const Pre &p) const { return (double)in.dval(p); }
        __device__ __forceinline__ double cval(const Pre &p) const { return (double)in.cval(p); }
        __device__ __forceinline__ double weight(const Pre &p) const { return (double)in.weight(p); }
    };
    struct Sink {
        typename P::Sink in;
        bool vec;
        __device__ __forceinline__ Sink(const typename P::Sink &s) : in(s), vec(s.vec) {}
        __device__ __forceinline__ SinkPre load(int64_t i) const { return in.load(i); }
        __device__ __forceinline__ void load4(int64_t i, SinkPre *o) const { in.load4(i, o); }
        __device__ __forceinline__ void store(int64_t i, double u, const SinkPre &p) const { in.store(i, (float)u, p); }
        __device__ __forceinline__ void store4(int64_t i, const double (&u)[4], const SinkPre (&p)[4]) const {
            const float v[4] = {(float)u[0], (float)u[1], (float)u[2], (float)u[3]};
            in.store4(i, v, p);
        }
    };
    static __device__ __forceinline__ ChainSpan span(const Params &p, int64_t c, int64_t nmax) {
        return P::span(p, c, nmax);
    }
    static __device__ __forceinline__ Src src(const Params &p, const ChainSpan &sp) { return Src(P::src(p, sp)); }
    static __device__ __forceinline__ Sink sink(const Params &p, const ChainSpan &sp) { return Sink(P::sink(p, sp)); }
};
// The problem type and working precision a TV-l1 problem Pb<T> runs with.
template <template <typename> class Pb, typename T> struct L1Run {
    using Prob = Pb<double>;
};
template <template <typename> class Pb> struct L1Run<Pb, float> {
    using Prob = WideL1<Pb<float>>;
};

// The ring as a sorted TV-l1 store (l1_core.h); a push into a full ring sets
// ovf and is dropped.
template <typename T, int K>
struct L1Ring {
    CRing<T, K, TagJ<T>> &R;
    bool ovf;
    int size;
    __device__ __forceinline__ L1Ring(CRing<T, K, TagJ<T>> &r) : R(r), ovf(false), size(r.size) {}
    __device__ __forceinline__ L1E<T> get(int j) const {
        const Ent<T, TagJ<T>> e = R.ld(j);
        return L1E<T>{e.l, e.k.k, e.k.j};
    }
    __device__ __forceinline__ void put(int j, const L1E<T> &e) const {
        R.set(j, mk_ent<T, TagJ<T>>(e.l, TagJ<T>{e.k, e.j}));
    }
    __device__ __forceinline__ void pop_front(int k) {
        R.head = (R.head + k) & (K - 1);
        size -= k;
        R.size = size;
    }
    __device__ __forceinline__ void pop_back(int k) {
        size -= k;
        R.size = size;
    }
    __device__ __forceinline__ void push_front(const L1E<T> &e) {
        if (size >= K) {
            ovf = true;
            return;
        }
        R.head = (R.head + K - 1) & (K - 1);
        R.size = ++size;
        put(0, e);
    }
    __device__ __forceinline__ void push_back(const L1E<T> &e) {
        if (size >= K) {
            ovf = true;
            return;
        }
        R.size = ++size;
        put(size - 1, e);
    }
    // insert at logical position q, shifting the shorter side
    __device__ __forceinline__ void insert(int q, const L1E<T> &e) {
        if (size >= K) {
            ovf = true;
            return;
        }
        if (q < size - q) {
            R.head = (R.head + K - 1) & (K - 1);
            for (int j = 0; j < q; ++j) put(j, get(j + 1));
        } else {
            for (int j = size; j > q; --j) put(j, get(j - 1));
        }
        R.size = ++size;
        put(q, e);
    }
};

template <typename T, class Prob, int K>
__device__ __forceinline__ void node_step(CRing<T, K, typename Prob::Tag> &R, bool &ok, int64_t i, int64_t n,
                                          const typename Prob::Src &src, const typename Prob::Pre &pv,
                                          CarryOf<T, Prob> &cy, T &lm, T &lp) {
    const bool root = (i == n - 1);
    if constexpr (IsL1<Prob>::value) {
        const T wi = src.weight(pv);
        const T w = root ? (T)0 : wi;
        L1Ring<T, K> S(R);
        l1_step<T>(S, (T)(int)(i + 1), src.data(pv), src.dval(pv), src.cval(pv), -cy.wprev, cy.wprev, -w, w, root,
                   lm, lp);
        cy.wprev = wi;
        ok = ok & (!S.ovf | root);
    } else {
        const auto in = step_in<T, Prob>(src, pv, i, root, cy);
        const bool fits = dp_step_ring<T, typename Prob::Tag, K, Prob::kGen>(R, in, lm, lp);
        ok = ok & (fits | root);
    }
    if (root) lp = lm;
}

template <typename T>
__device__ __forceinline__ void put_lam(LamPair<T> *lam, int64_t i, int64_t C, int64_t c, T lm, T lp) {
    LamPair<T> pr;
    pr.lo = lm;
    pr.hi = lp;
    lam[i * C + c] = pr;
}

template <typename T, typename G>
__device__ __forceinline__ Ent<T, G> *save_slot(const SegWs<T, G> &ws, int K, int64_t s, int kind, int64_t c) {
    return ws.st + ((s * kSaves + kind) * K) * ws.C + c;
}
template <typename T, typename G>
__device__ __forceinline__ int *size_slot(const SegWs<T, G> &ws, int64_t s, int kind, int64_t c) {
    return ws.st_size + (s * kSaves + kind) * ws.C + c;
}
template <typename T, typename G>
__device__ __forceinline__ uint32_t *hash_slot(const SegWs<T, G> &ws, int64_t s, int kind, int64_t c) {
    return ws.st_hash + (s * kSaves + kind) * ws.C + c;
}
// Save / compare the ring against saved state `kind` of segment s.
template <typename T, int K, typename G>
__device__ __forceinline__ void save_state(const SegWs<T, G> &ws, const CRing<T, K, G> &R, int64_t s, int kind,
                                           int64_t c) {
    R.save(save_slot(ws, K, s, kind, c), size_slot(ws, s, kind, c), hash_slot(ws, s, kind, c), ws.C);
}
template <typename T, int K, typename G>
__device__ __forceinline__ bool equals_state(const SegWs<T, G> &ws, const CRing<T, K, G> &R, int64_t s, int kind,
                                             int64_t c) {
    return R.equals(save_slot(ws, K, s, kind, c), size_slot(ws, s, kind, c), hash_slot(ws, s, kind, c), ws.C);
}
template <typename T, int K, typename G>
__device__ __forceinline__ void load_state(const SegWs<T, G> &ws, CRing<T, K, G> &R, int64_t s, int kind,
                                           int64_t c) {
    R.load(save_slot(ws, K, s, kind, c), size_slot(ws, s, kind, c), ws.C);
}

// Forward DP over nodes [from, b) with data loads P nodes ahead, storing the
// lambda pairs if kStore (a halo run stores nothing).  After each full tile
// hook(e) is called with the next node index e (tile edges are multiples of P
// from `from`); a true return stops the run, and fwd_run then returns e.
// Otherwise it returns b.
template <typename T, class Prob, int K, int P, bool kStore, bool kVec, class Hook>
__device__ __forceinline__ int64_t fwd_run_t(CRing<T, K, typename Prob::Tag> &R, const typename Prob::Src &src,
                                             bool &ok, CarryOf<T, Prob> &cy, int64_t from, int64_t b, int64_t n,
                                             LamPair<T> *lam, int64_t C, int64_t c, Hook hook) {
    static_assert(P % 4 == 0, "tiles hold whole groups of four nodes");
    typename Prob::Pre pre[P];
#pragma unroll
    for (int j = 0; j < P; ++j) pre[j] = src.load((from + j < b) ? from + j : b - 1);
    LamPair<T> *lq = lam + from * C + c;  // lambda pair of the next node (running pointer)
    auto node = [&](int64_t i, const typename Prob::Pre &pv) {
        T lm, lp;
        node_step<T, Prob, K>(R, ok, i, n, src, pv, cy, lm, lp);
        if (kStore) {
            LamPair<T> pr;
            pr.lo = lm;
            pr.hi = lp;
            *lq = pr;
            lq += C;
        }
    };
    int64_t i0 = from;
    // tiles whose prefetch stays inside [from, b): double-buffered, the next
    // tile's loads issued before this tile's nodes are processed (one wait per
    // tile, for loads P nodes old); no clamping, running offsets
    for (; i0 + 2 * P <= b; i0 += P) {
        typename Prob::Pre nxt[P];
        if constexpr (!kVec) {
            int64_t o = src.off(i0 + P);
            const int64_t st = src.step();
#pragma unroll
            for (int j = 0; j < P; ++j) {
                nxt[j] = src.load_off(o);
                o += st;
            }
        } else {
            // unit-stride chains (rows): one 16-byte load per stream for four
            // nodes (node indices are multiples of 4)
#pragma unroll
            for (int j = 0; j < P; j += 4) src.load4(i0 + P + j, &nxt[j]);
        }
#pragma unroll
        for (int j = 0; j < P; ++j) node(i0 + j, pre[j]);
#pragma unroll
        for (int j = 0; j < P; ++j) pre[j] = nxt[j];
        if (hook(i0 + P)) return i0 + P;
    }
    // the last full tile (its prefetch is clamped to the run's last node)
    for (; i0 + P <= b; i0 += P) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int64_t i = i0 + j;
            node(i, pre[j]);
            if constexpr (!kVec) {
                pre[j] = src.load((i + P < b) ? i + P : b - 1);
            } else if ((j & 3) == 3) {
                const int64_t q = i + P - 3;
                if (q + 3 < b) {
                    src.load4(q, &pre[j - 3]);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) pre[j - 3 + k] = src.load((q + k < b) ? q + k : b - 1);
                }
            }
        }
        if (hook(i0 + P)) return i0 + P;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (i0 + j < b) node(i0 + j, pre[j]);
    }
    return b;
}

// A source whose vec is a compile-time false never takes the 16-byte path.
template <class S, class = void> struct NeverVec : std::false_type {};
template <class S> struct NeverVec<S, std::enable_if_t<!S::vec>> : std::true_type {};

// The prefetch path is chosen once per wave: lanes whose chains all allow
// 16-byte loads take them, any other wave loads node by node.  (A per-lane
// choice would make every prefetch load conditional, and the compiler then
// waits for each load a few nodes after issuing it.)
template <typename T, class Prob, int K, int P, bool kStore, class Hook>
__device__ __forceinline__ int64_t fwd_run(CRing<T, K, typename Prob::Tag> &R, const typename Prob::Src &src,
                                           bool &ok, CarryOf<T, Prob> &cy, int64_t from, int64_t b, int64_t n,
                                           LamPair<T> *lam, int64_t C, int64_t c, Hook hook) {
    if constexpr (!NeverVec<typename Prob::Src>::value) {
        if (__ballot(!src.vec) == 0)
            return fwd_run_t<T, Prob, K, P, kStore, true>(R, src, ok, cy, from, b, n, lam, C, c, hook);
    }
    return fwd_run_t<T, Prob, K, P, kStore, false>(R, src, ok, cy, from, b, n, lam, C, c, hook);
}

// Backward clip pass over [a, b) of one chain.  All lanes of a wave share a and
// b, so node indices are wave-uniform and the lambda / sink accesses coalesce.
// Collapsed nodes are written through the sink; the un-collapsed right tail
// gets its composed interval in the lambda stream for k_seg_tail.  With kVec
// (unit-stride, element-aligned sink and b a multiple of 4) the sink is read
// and written four nodes at a time: node groups [4m, 4m + 3] are visited from
// the top, buffered, and stored with one 16-byte access per stream when the
// whole group has collapsed (the group holding the collapse point falls back
// to single stores).
//
// The sweep may start inside the segment: from node b - 1 with the state the
// sweep had entering it from the right (the composed interval, or the value
// and node of an earlier collapse).  With kRec the first pass records that
// state at the checkpoint nodes (ck_offset) that fall on a tile edge counted
// from b, so a repair that met checkpoint m redoes only
// the nodes left of it.
// Checkpoint m (1 .. kCheckpoints) of a segment starting at a sits at node
// a + CK 2^(m-1): close together where the runs usually meet, and spread out
// so that a late meeting still ends a rerun well before the segment end.
__host__ __device__ __forceinline__ int64_t ck_offset(int m, int64_t CK) { return CK << (m - 1); }
// m if node a + off is checkpoint m, else 0.
__device__ __forceinline__ int ck_index(int64_t off, int64_t CK) {
    int m = 0;
#pragma unroll
    for (int j = 1; j <= kCheckpoints; ++j) m = (off == ck_offset(j, CK)) ? j : m;
    return m;
}

template <typename T>
struct SweepIn {
    T lo, hi;   // composed interval over [b, segment end), or the collapsed value twice
    bool col;   // collapsed at node k >= b
    int64_t k;
};
template <typename T>
__device__ __forceinline__ SweepIn<T> sweep_from_end(int64_t a) {
    return SweepIn<T>{-pos_inf<T>(), pos_inf<T>(), false, a - 1};
}
// Whether the first pass recorded the sweep state at checkpoint node e of the
// segment [a, b) (both sides use this one rule).
__device__ __forceinline__ bool sweep_cp_recorded(int64_t a, int64_t b, int64_t e, int64_t CK) {
    return e < b && ck_index(e - a, CK) > 0 && (b - e) % kSweepTile == 0;
}

template <typename T, class Prob, int P, bool kVec, bool kRec>
__device__ __forceinline__ void bwd_sweep_run(const WsOf<T, Prob> &ws, const typename Prob::Sink &sink, int64_t s,
                                              int64_t c, int64_t a, int64_t b, const SweepIn<T> &in0) {
    static_assert(P % 4 == 0, "tiles hold whole groups of four nodes");
    static_assert(!kRec || P == kSweepTile, "checkpoint records sit on sweep-tile edges");
    using SP = typename Prob::SinkPre;
    LamPair<T> *__restrict__ lam = ws.lam;
    const int64_t C = ws.C;
    T glo = in0.lo, ghi = in0.hi, x = in0.lo;
    bool col = in0.col;
    int64_t k = in0.col ? in0.k : a - 1;
    // next checkpoint to record (downwards); a tile edge or never reached
    int mrec = 0;
    int64_t erec = -1;
    if (kRec) {
        mrec = kCheckpoints;
        while (mrec > 0 && a + ck_offset(mrec, ws.CK) >= b) --mrec;
        erec = mrec > 0 ? a + ck_offset(mrec, ws.CK) : -1;
    }
    LamPair<T> pre[P];
    SP spre[P];
    // slot j holds node i0 - j of the current tile (i0 = b - 1 - tile * P)
    auto refill_sink = [&](SP *dst, int jhi, int64_t q) {  // nodes q .. q+3 into slots jhi, jhi-1, jhi-2, jhi-3
        if (q >= a) {
            SP t4[4];
            sink.load4(q, t4);
#pragma unroll
            for (int m = 0; m < 4; ++m) dst[jhi - m] = t4[m];
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) dst[jhi - m] = sink.load((q + m >= a) ? q + m : a);
        }
    };
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int64_t i = (b - 1 - j >= a) ? b - 1 - j : a;
        pre[j] = lam[i * C + c];
        if (!kVec) spre[j] = sink.load(i);
        else if ((j & 3) == 3) refill_sink(spre, j, b - 1 - j);
    }
    T gx[4];
    SP gs[4];
    bool gc[4];
    auto visit = [&](int64_t i, int jj, const LamPair<T> &p, const SP &sv) {
        if (!col) {
            glo = clampv(glo, p.lo, p.hi);
            ghi = clampv(ghi, p.lo, p.hi);
            if (glo == ghi) {
                col = true;
                x = glo;
                k = i;
            }
        } else {
            x = clampv(x, p.lo, p.hi);
        }
        if (col) {
            if (kVec) {
                gx[3 - jj] = x;
                gs[3 - jj] = sv;
                gc[3 - jj] = true;
            } else {
                sink.store(i, x, sv);
            }
        } else {
            LamPair<T> g;
            g.lo = glo;
            g.hi = ghi;
            lam[i * C + c] = g;
            if (kVec) gc[3 - jj] = false;
        }
        if (kVec && jj == 3) {  // i = 4m: the group is complete
            if (gc[0] & gc[1] & gc[2] & gc[3]) {
                sink.store4(i, gx, gs);
            } else {
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    if (gc[m]) sink.store(i + m, gx[m], gs[m]);
            }
        }
    };
    int64_t i0 = b - 1;
    for (; i0 - (P - 1) >= a; i0 -= P) {
        // double-buffered: the next tile's loads go out before this tile's nodes
        LamPair<T> npre[P];
        SP nspre[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int64_t ip = (i0 - j - P >= a) ? i0 - j - P : a;
            npre[j] = lam[ip * C + c];
            if (!kVec) nspre[j] = sink.load(ip);
            else if ((j & 3) == 3) refill_sink(nspre, j, i0 - j - P);
        }
#pragma unroll
        for (int j = 0; j < P; ++j) visit(i0 - j, j & 3, pre[j], spre[j]);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            pre[j] = npre[j];
            spre[j] = nspre[j];
        }
        if (kRec && i0 - (P - 1) == erec) {  // the state now covers [erec, b)
            if (sweep_cp_recorded(a, b, erec, ws.CK)) {
                LamPair<T> r;
                r.lo = col ? x : glo;
                r.hi = col ? x : ghi;
                ws.sw_cp[(mrec - 1) * ws.S * C + s * C + c] = r;
            }
            --mrec;
            erec = mrec > 0 ? a + ck_offset(mrec, ws.CK) : -1;
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (i0 - j >= a) visit(i0 - j, j & 3, pre[j], spre[j]);
    }
    const int64_t sc = s * C + c;
    ws.seg_unc[sc] = (int)(k + 1);
    ws.seg_lo[sc] = col ? x : glo;
    ws.seg_hi[sc] = col ? x : ghi;
}

template <typename T, class Prob, int P, bool kRec = false>
__device__ __forceinline__ void bwd_sweep(const WsOf<T, Prob> &ws, const typename Prob::Params &pp, const ChainSpan &sp,
                                          int64_t s, int64_t c, int64_t a, int64_t b, const SweepIn<T> &in0) {
    const auto sink = Prob::sink(pp, sp);
    if (sink.vec && (b & 3) == 0)
        bwd_sweep_run<T, Prob, P, true, kRec>(ws, sink, s, c, a, b, in0);
    else
        bwd_sweep_run<T, Prob, P, false, kRec>(ws, sink, s, c, a, b, in0);
}

// True if the deque after node e - 1 equals the first pass's checkpoint there.
template <typename T, int K, typename G>
__device__ __forceinline__ bool meets_checkpoint(const SegWs<T, G> &ws, const CRing<T, K, G> &R, int64_t s, int64_t c,
                                                 int64_t a, int64_t e) {
    const int m = ck_index(e - a, ws.CK);
    if (m == 0) return false;
    return equals_state<T, K, G>(ws, R, s, kSaveCk + (int)m - 1, c);
}

// ---------------------------------------------------------------------------
// First pass: forward with halo and saves, then the backward sweep.
// ---------------------------------------------------------------------------
template <typename T, class Prob, int K, int P>
__global__ __launch_bounds__(64) void k_seg_main(WsOf<T, Prob> ws, typename Prob::Params pp) {
    __shared__ EntOf<T, Prob> s_ent[CRing<T, K, typename Prob::Tag>::kRows * 64];
    if (seg_stopped(ws)) return;
    const int lane = threadIdx.x;
    const int64_t g = (int64_t)blockIdx.x * 64 + lane;
    if (g == 0) *ws.ovf_count = 0;  // consumed by k_seg_fix / k_seg_ovf after this kernel
    if (g >= ws.S * ws.C) return;
    const int64_t c = g % ws.C, s = g / ws.C;
    const ChainSpan sp = Prob::span(pp, c, ws.n);
    const int64_t n = sp.n;
    const int64_t a = s * ws.L;
    if (a >= n) return;
    const int64_t b = (a + ws.L < n) ? a + ws.L : n;
    const int64_t h0 = (a > ws.H) ? a - ws.H : 0;
    const auto src = Prob::src(pp, sp);
    CRing<T, K, typename Prob::Tag> R;
    R.init(s_ent, lane);
    bool ok = true;
    auto cy = carry_before<T, Prob>(src, h0);
    const int64_t C = ws.C;
    // halo [h0, a) from an empty deque, storing nothing (a - h0 is a multiple of P)
    if (h0 < a)
        fwd_run<T, Prob, K, P, false>(R, src, ok, cy, h0, a, n, ws.lam, C, c, [](int64_t) { return false; });
    if (s > 0 && ok) save_state(ws, R, s, kSaveHalo, c);
    // own nodes; tile edges align with the checkpoints (multiples of P)
    auto saves = [&](int64_t e) {
        if (ok) {
            const int m = ck_index(e - a, ws.CK);
            if (m > 0) save_state(ws, R, s, kSaveCk + m - 1, c);
        }
        return false;
    };
    fwd_run<T, Prob, K, P, true>(R, src, ok, cy, a, b, n, ws.lam, C, c, saves);
    if (ok && b < n) save_state(ws, R, s, kSaveEnd, c);
    ws.ovf[c * ws.S + s] = ok ? 0 : 1;
    if (ok) bwd_sweep<T, Prob, kSweepTile, true>(ws, pp, sp, s, c, a, b, sweep_from_end<T>(a));
}

// ---------------------------------------------------------------------------
// Boundary check and repair, lane (s, c) for s >= 1.  If the first pass's
// deque after the halo differs from the saved end state of segment s-1, the
// segment is rerun from that end state (taken as the true incoming message;
// k_seg_fix corrects the rare cases where it is not) until the deque matches a
// first-pass checkpoint.  The backward pass is then redone left of that
// checkpoint from the first pass's recorded sweep state (the lambdas right of
// it are unchanged), or over the whole segment.
// ---------------------------------------------------------------------------
template <typename T, class Prob, int K, int P>
__global__ __launch_bounds__(64) void k_seg_repair(WsOf<T, Prob> ws, typename Prob::Params pp) {
    __shared__ EntOf<T, Prob> s_ent[CRing<T, K, typename Prob::Tag>::kRows * 64];
    if (seg_stopped(ws)) return;
    const int lane = threadIdx.x;
    const int64_t g = (int64_t)blockIdx.x * 64 + lane;
    if (g >= (ws.S - 1) * ws.C) return;
    const int64_t c = g % ws.C, s = g / ws.C + 1;
    const ChainSpan sp = Prob::span(pp, c, ws.n);
    const int64_t n = sp.n;
    const int64_t a = s * ws.L;
    if (a >= n) return;
    const int64_t b = (a + ws.L < n) ? a + ws.L : n;
    const int64_t cs = c * ws.S + s;
    if (ws.ovf[cs] || ws.ovf[cs - 1]) return;  // the chain goes to the overflow kernel
    const int64_t C = ws.C;
    bool same = (*size_slot(ws, s - 1, kSaveEnd, c) == *size_slot(ws, s, kSaveHalo, c)) &&
                (*hash_slot(ws, s - 1, kSaveEnd, c) == *hash_slot(ws, s, kSaveHalo, c));
    if (same) {
        const EntOf<T, Prob> *A = save_slot(ws, K, s - 1, kSaveEnd, c);
        const EntOf<T, Prob> *B = save_slot(ws, K, s, kSaveHalo, c);
        const int m = clamp_size<K>(*size_slot(ws, s - 1, kSaveEnd, c));
        for (int j0 = 0; j0 < m && same; j0 += 8) {
            EntOf<T, Prob> ea[8], eb[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int jj = (j0 + j < m) ? j0 + j : m - 1;
                ea[j] = A[jj * C];
                eb[j] = B[jj * C];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int jj = j0 + j;
                if (jj < m) same = same && ent_same<T>(ea[j].l, ea[j].k, eb[j].l, eb[j].k);
            }
        }
    }
    ws.mis[cs] = same ? 0 : 1;
    if (same) return;
    const auto src = Prob::src(pp, sp);
    CRing<T, K, typename Prob::Tag> R;
    R.init(s_ent, lane);
    load_state(ws, R, s - 1, kSaveEnd, c);
    bool ok = true;
    auto cy = carry_before<T, Prob>(src, a);
    const int64_t stop = fwd_run<T, Prob, K, P, true>(R, src, ok, cy, a, b, n, ws.lam, C, c,
                                                [&](int64_t e) { return !ok || meets_checkpoint(ws, R, s, c, a, e); });
    if (!ok) {
        ws.ovf[cs] = 1;
        return;
    }
    // met a checkpoint, or ends with the first pass's end deque: either way the
    // two runs coincide from some node on, so the saved end state is the true one
    const bool clean = stop < b || (b < n && equals_state(ws, R, s, kSaveEnd, c));
    ws.clean[cs] = clean ? 1 : 0;
    ws.rep_stop[s * C + c] = (int)stop;
    if (!clean && b < n) save_state(ws, R, s, kSaveEnd2, c);
    if (stop < b && sweep_cp_recorded(a, b, stop, ws.CK)) {
        // nodes [stop, b) keep their first-pass lambdas and outputs
        const LamPair<T> r = ws.sw_cp[(ck_index(stop - a, ws.CK) - 1) * ws.S * C + s * C + c];
        const int64_t k1 = (int64_t)ws.seg_unc[s * C + c] - 1;  // the first pass's collapse node
        const SweepIn<T> in0{r.lo, r.hi, k1 >= stop, k1};
        bwd_sweep<T, Prob, kSweepTile>(ws, pp, sp, s, c, a, stop, in0);
    } else {
        bwd_sweep<T, Prob, kSweepTile>(ws, pp, sp, s, c, a, b, sweep_from_end<T>(a));
    }
}

// Backward clip of a whole chain from its lambda stream (after a sequential
// forward pass); marks every segment's tail as done for k_seg_tail.
template <typename T, class Prob>
__device__ void full_backward(const WsOf<T, Prob> &ws, const typename Prob::Params &pp, const ChainSpan &sp, int64_t c) {
    const auto sink = Prob::sink(pp, sp);
    T x = (T)0;
    for (int64_t i = sp.n - 1; i >= 0; --i) {
        const LamPair<T> p = ws.lam[i * ws.C + c];
        const auto sv = sink.load(i);
        x = (i == sp.n - 1) ? p.lo : clampv(x, p.lo, p.hi);
        sink.store(i, x, sv);
    }
    for (int64_t s = 0; s * ws.L < sp.n; ++s) {
        const int64_t b = (s + 1) * ws.L < sp.n ? (s + 1) * ws.L : sp.n;
        ws.seg_unc[s * ws.C + c] = (int)b;
    }
}

// Sequential DP + backward of a whole chain with the deque in HBM.
template <typename T, class Prob>
__device__ void seg_full_chain(const WsOf<T, Prob> &ws, const typename Prob::Params &pp, const ChainSpan &sp,
                               int64_t c, int64_t slot) {
    using G = typename Prob::Tag;
    const auto src = Prob::src(pp, sp);
    auto cy = carry_before<T, Prob>(src, 0);
    if constexpr (IsL1<Prob>::value) {
        // at most one front push per node: the set starts n + 4 slots in
        L1ArrayStore<T> S;
        S.init(ws.fb_lam + slot * ws.fb_cap, ws.fb_tag + slot * ws.fb_cap, ws.fb_cap, sp.n + 4);
        for (int64_t i = 0; i < sp.n; ++i) {
            const auto pr = src.load(i);
            const bool root = (i == sp.n - 1);
            const T wi = src.weight(pr);
            const T w = root ? (T)0 : wi;
            T lm = (T)0, lp = (T)0;
            l1_step<T>(S, (T)(int)(i + 1), src.data(pr), src.dval(pr), src.cval(pr), -cy.wprev, cy.wprev, -w, w,
                       root, lm, lp);
            if (root) lp = lm;
            put_lam<T>(ws.lam, i, ws.C, c, lm, lp);
            cy.wprev = wi;
        }
    } else {
        HbmDeque<T, G> dq;
        dq.init(ws.fb_lam + slot * ws.fb_cap, ws.fb_tag + slot * ws.fb_cap, ws.fb_cap);
        for (int64_t i = 0; i < sp.n; ++i) {
            const auto pr = src.load(i);
            const bool root = (i == sp.n - 1);
            T lm = (T)0, lp = (T)0;
            const auto in = step_in<T, Prob>(src, pr, i, root, cy);
            dp_step_hbm<T, G, Prob::kGen>(dq, in, lm, lp);
            if (root) lp = lm;
            put_lam<T>(ws.lam, i, ws.C, c, lm, lp);
        }
    }
    full_backward<T, Prob>(ws, pp, sp, c);
}

template <typename T, class Prob, int K, int P>
__device__ bool fix_chain(const WsOf<T, Prob> &ws, const typename Prob::Params &pp, const ChainSpan &sp, int64_t c,
                          EntOf<T, Prob> *s_ent, int lane);

// ---------------------------------------------------------------------------
// Fix-up, one lane per chain (a no-op for almost every chain).  Walks the
// segments keeping track of whether the saved end state of the previous
// segment is the true one; where it is not, the segment is redone
// sequentially from the true state until a checkpoint matches and past the
// region the repair kernel rewrote.
// ---------------------------------------------------------------------------
template <typename T, class Prob, int K, int P>
__global__ __launch_bounds__(64) void k_seg_fix(WsOf<T, Prob> ws, typename Prob::Params pp) {
    __shared__ EntOf<T, Prob> s_ent[CRing<T, K, typename Prob::Tag>::kRows * 64];
    if (seg_stopped(ws)) return;
    const int lane = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * 64 + lane;
    if (c >= ws.C) return;
    const ChainSpan sp = Prob::span(pp, c, ws.n);
    const int64_t n = sp.n;
    if (n <= 0) return;
    const int64_t Sc = (n + ws.L - 1) / ws.L;
    const uint8_t *ovf = ws.ovf + c * ws.S;
    const uint8_t *mis = ws.mis + c * ws.S;
    const uint8_t *cln = ws.clean + c * ws.S;
    bool any_ovf = false, any_dirty = false;
    for (int64_t s = 0; s < Sc; ++s) {
        any_ovf |= ovf[s] != 0;
        if (s > 0 && s + 1 < Sc) any_dirty |= (mis[s] != 0) && (cln[s] == 0);
    }
    if (any_ovf || (any_dirty && !fix_chain<T, Prob, K, P>(ws, pp, sp, c, s_ent, lane))) {
        ws.ovf_list[atomicAdd(ws.ovf_count, 1)] = (int)c;  // solved by k_seg_ovf
        return;
    }
    // x entering each segment from the right: compose the segment maps from the
    // root's segment leftwards (seg_lo/hi are final here).  Eight segments'
    // maps are loaded before their stores, so a group costs one memory latency.
    T x = ws.seg_lo[(Sc - 1) * ws.C + c];
    for (int64_t j1 = Sc - 2; j1 >= 0; j1 -= 8) {
        T lo[8], hi[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t j = j1 - k >= 0 ? j1 - k : 0;
            lo[k] = ws.seg_lo[j * ws.C + c];
            hi[k] = ws.seg_hi[j * ws.C + c];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (j1 - k < 0) break;
            ws.seg_xb[(j1 - k) * ws.C + c] = x;
            x = clampv(x, lo[k], hi[k]);
        }
    }
}

// Returns false if the true deque outgrew the ring (the chain then goes to
// the HBM overflow kernel).
template <typename T, class Prob, int K, int P>
__device__ bool fix_chain(const WsOf<T, Prob> &ws, const typename Prob::Params &pp, const ChainSpan &sp, int64_t c,
                          EntOf<T, Prob> *s_ent, int lane) {
    const int64_t n = sp.n;
    const int64_t Sc = (n + ws.L - 1) / ws.L;
    const uint8_t *mis = ws.mis + c * ws.S;
    const uint8_t *cln = ws.clean + c * ws.S;
    const auto src = Prob::src(pp, sp);
    CRing<T, K, typename Prob::Tag> R;
    R.init(s_ent, lane);
    const int64_t C = ws.C;
    bool end_true = true, ok = true;
    // Each lane walks its own chain: a pass of the outer loop skips the
    // segments whose results stand and redoes at most one, so the lanes of a
    // wave redo their segments side by side whatever their positions, and the
    // wave costs as many segment runs as its lane with the most redos.
    int64_t s = 1;
    while (ok) {
        while (s < Sc && end_true) {
            // the pass that wrote segment s started from the true state
            if (mis[s] && !cln[s]) {
                end_true = false;
                if ((s + 1) * ws.L < n) load_state(ws, R, s, kSaveEnd2, c);
            }
            ++s;
        }
        if (s >= Sc) break;
        // R holds the true deque entering segment s: redo it until it meets the
        // first pass and is past whatever the repair kernel rewrote.
        const int64_t a = s * ws.L;
        const int64_t b = (a + ws.L < n) ? a + ws.L : n;
        const int64_t redo_to = mis[s] ? (int64_t)ws.rep_stop[s * C + c] : a;
        auto cy = carry_before<T, Prob>(src, a);
        bool met = false;
        const int64_t stop = fwd_run<T, Prob, K, P, true>(R, src, ok, cy, a, b, n, ws.lam, C, c, [&](int64_t e) {
            if (!ok) return true;
            met = met || meets_checkpoint(ws, R, s, c, a, e);
            return met && e >= redo_to;
        });
        if (!ok) break;
        if (stop == b && !met && b < n)
            met = equals_state(ws, R, s, kSaveEnd, c);
        bwd_sweep<T, Prob, kSweepTile>(ws, pp, sp, s, c, a, b, sweep_from_end<T>(a));
        end_true = met;
        ++s;
    }
    return ok;
}

// ---------------------------------------------------------------------------
// Overflowed chains, solved sequentially by a bounded pool of lanes: first with
// the largest LDS ring a workgroup may hold (160 KiB on gfx950: 256 slots of
// 8-byte entries, 128 of 16-byte ones, 64 of 32-byte ones), and only if the
// deque outgrows that too, with the deque in HBM (lane l owns deque storage
// l).  Both paths compute the same results as the segmented one.
// ---------------------------------------------------------------------------
template <typename T, typename G> struct OvfRing {
    using E = Ent<T, G>;
    static constexpr int fit(int k) {
        return (k + ring_copies<T, G>()) * 64 * (int)sizeof(E) <= 163840 ? k : fit(k / 2);
    }
    static constexpr int K = fit(512);
};

template <typename T, class Prob>
__global__ __launch_bounds__(64) void k_seg_ovf(WsOf<T, Prob> ws, typename Prob::Params pp) {
    constexpr int KB = OvfRing<T, typename Prob::Tag>::K;
    __shared__ EntOf<T, Prob> s_big[CRing<T, KB, typename Prob::Tag>::kRows * 64];
    if (seg_stopped(ws)) return;
    const int lane = threadIdx.x;
    const int64_t l = (int64_t)blockIdx.x * 64 + lane;
    const int64_t cnt = *ws.ovf_count;
    for (int64_t j = l; j < cnt; j += ws.fb_lanes) {
        const int64_t c = ws.ovf_list[j];
        const ChainSpan sp = Prob::span(pp, c, ws.n);
        if (sp.n <= 0) continue;
        const auto src = Prob::src(pp, sp);
        CRing<T, KB, typename Prob::Tag> R;
        R.init(s_big, lane);
        bool ok = true;
        auto cy = carry_before<T, Prob>(src, 0);
        fwd_run<T, Prob, KB, kTileOvf, true>(R, src, ok, cy, 0, sp.n, sp.n, ws.lam, ws.C, c,
                                             [](int64_t) { return false; });
        if (ok)
            full_backward<T, Prob>(ws, pp, sp, c);
        else
            seg_full_chain<T, Prob>(ws, pp, sp, c, l);
    }
}

// ---------------------------------------------------------------------------
// Un-collapsed tails: x_i = clip(x_b, composed interval of i .. b-1).
// ---------------------------------------------------------------------------
template <typename T, class Prob>
__global__ __launch_bounds__(64) void k_seg_tail(WsOf<T, Prob> ws, typename Prob::Params pp) {
    if (seg_stopped(ws)) return;
    const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (g >= (ws.S - 1) * ws.C) return;
    const int64_t c = g % ws.C, s = g / ws.C;
    const ChainSpan sp = Prob::span(pp, c, ws.n);
    const int64_t n = sp.n;
    const int64_t a = s * ws.L;
    if (a + ws.L >= n) return;  // the root's segment always collapses
    const int64_t b = a + ws.L;
    const int64_t C = ws.C;
    const int64_t u = ws.seg_unc[s * C + c];
    if (u >= b) return;
    const T x = ws.seg_xb[s * C + c];
    const auto sink = Prob::sink(pp, sp);
    // eight nodes' intervals (and sink inputs) loaded before their stores
    for (int64_t i1 = b - 1; i1 >= u; i1 -= 8) {
        LamPair<T> p[8];
        typename Prob::SinkPre sv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = i1 - k >= u ? i1 - k : u;
            p[k] = ws.lam[i * C + c];
            sv[k] = sink.load(i);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (i1 - k >= u) sink.store(i1 - k, clampv(x, p[k].lo, p[k].hi), sv[k]);
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
template <typename T, int K, typename G = T>
size_t seg_ws_layout(void *base, int64_t C, int64_t n, int64_t L, int64_t H, int64_t CK, SegWs<T, G> *out) {
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t S = (n + L - 1) / L;
    // HBM deques: 2n + 4 entries; TV-l1 sets (one front push and at most two
    // other insertions per node, starting n + 4 slots in): 4n + 8
    const int64_t cap = std::is_same<G, TagJ<T>>::value ? 4 * n + 8 : 2 * n + 4;
    size_t off = 0;
    const size_t o_lam = off;  off += al(sizeof(LamPair<T>) * (size_t)(n * C));
    const size_t o_st = off;   off += al(sizeof(Ent<T, G>) * (size_t)(S * kSaves * K * C));
    const size_t o_sz = off;   off += al(sizeof(int) * (size_t)(S * kSaves * C));
    const size_t o_hs = off;   off += al(sizeof(uint32_t) * (size_t)(S * kSaves * C));
    const size_t o_ovf = off;  off += al((size_t)(S * C));
    const size_t o_mis = off;  off += al((size_t)(S * C));
    const size_t o_cln = off;  off += al((size_t)(S * C));
    const size_t o_rs = off;   off += al(sizeof(int) * (size_t)(S * C));
    const size_t o_lo = off;   off += al(sizeof(T) * (size_t)(S * C));
    const size_t o_hi = off;   off += al(sizeof(T) * (size_t)(S * C));
    const size_t o_unc = off;  off += al(sizeof(int) * (size_t)(S * C));
    const size_t o_xb = off;   off += al(sizeof(T) * (size_t)(S * C));
    const int64_t fbl = (C < kOverflowLanes ? (C + 63) / 64 * 64 : kOverflowLanes);
    const size_t o_oc = off;   off += al(sizeof(int));
    const size_t o_ol = off;   off += al(sizeof(int) * (size_t)C);
    const size_t o_sw = off;   off += al(sizeof(LamPair<T>) * (size_t)(kCheckpoints * S * C));
    const size_t o_fl = off;   off += al(sizeof(T) * (size_t)(fbl * cap));
    const size_t o_ft = off;   off += al(sizeof(G) * (size_t)(fbl * cap));
    if (base && out) {
        char *p = (char *)base;
        SegWs<T, G> w;
        w.C = C;
        w.n = n;
        w.L = L;
        w.S = S;
        w.H = H;
        w.CK = CK;
        w.lam = (LamPair<T> *)(p + o_lam);
        w.st = (Ent<T, G> *)(p + o_st);
        w.st_size = (int *)(p + o_sz);
        w.st_hash = (uint32_t *)(p + o_hs);
        w.ovf = (uint8_t *)(p + o_ovf);
        w.mis = (uint8_t *)(p + o_mis);
        w.clean = (uint8_t *)(p + o_cln);
        w.rep_stop = (int *)(p + o_rs);
        w.seg_lo = (T *)(p + o_lo);
        w.seg_hi = (T *)(p + o_hi);
        w.seg_unc = (int *)(p + o_unc);
        w.seg_xb = (T *)(p + o_xb);
        w.ovf_count = (int *)(p + o_oc);
        w.ovf_list = (int *)(p + o_ol);
        w.sw_cp = (LamPair<T> *)(p + o_sw);
        w.fb_lam = (T *)(p + o_fl);
        w.fb_tag = (G *)(p + o_ft);
        w.fb_cap = cap;
        w.fb_lanes = fbl;
        w.stop = nullptr;
        *out = w;
    }
    return off;
}

template <typename T, class Prob, int K, int P>
hipError_t seg_launch(const WsOf<T, Prob> &ws, const typename Prob::Params &pp, hipStream_t stream) {
    if (ws.C <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((ws.S * ws.C + 63) / 64);
    hipLaunchKernelGGL((k_seg_main<T, Prob, K, P>), dim3(blocks), dim3(64), 0, stream, ws, pp);
    if (ws.S > 1) {
        const unsigned rb = (unsigned)(((ws.S - 1) * ws.C + 63) / 64);
        hipLaunchKernelGGL((k_seg_repair<T, Prob, K, P>), dim3(rb), dim3(64), 0, stream, ws, pp);
    }
    const unsigned fb = (unsigned)((ws.C + 63) / 64);
    hipLaunchKernelGGL((k_seg_fix<T, Prob, K, P>), dim3(fb), dim3(64), 0, stream, ws, pp);
    hipLaunchKernelGGL((k_seg_ovf<T, Prob>), dim3((unsigned)(ws.fb_lanes / 64)), dim3(64), 0, stream, ws, pp);
    if (ws.S > 1) {
        const unsigned tb = (unsigned)(((ws.S - 1) * ws.C + 63) / 64);
        hipLaunchKernelGGL((k_seg_tail<T, Prob>), dim3(tb), dim3(64), 0, stream, ws, pp);
    }
    return hipGetLastError();
}

// Ring sizes a launch may use: 16 and 32 slots, and 64 or 128 for 8-byte
// entries (40 / 72 KiB rings per wave; gfx950 gives a workgroup up to 160 KiB).
template <typename T, typename G>
constexpr int ring_max() {
    return sizeof(Ent<T, G>) <= 8 ? 128 : 32;
}
template <typename T, typename G>
constexpr bool ring64_ok() {
    return ring_max<T, G>() >= 64;
}
template <typename T, typename G>
__host__ __device__ constexpr int ring_slots_for(int K) {
    const int k = K >= 128 ? 128 : (K >= 64 ? 64 : (K >= 32 ? 32 : 16));
    return k > ring_max<T, G>() ? ring_max<T, G>() : k;
}

// Workspace bytes and launch for a plan, dispatching on its ring size.
template <typename T, typename G = T>
size_t seg_ws_bytes(int64_t C, int64_t n, const SegPlan &p) {
    switch (ring_slots_for<T, G>(p.K)) {
    case 128: return seg_ws_layout<T, 128, G>(nullptr, C, n, p.L, p.H, p.CK, nullptr);
    case 64: return seg_ws_layout<T, 64, G>(nullptr, C, n, p.L, p.H, p.CK, nullptr);
    case 32: return seg_ws_layout<T, 32, G>(nullptr, C, n, p.L, p.H, p.CK, nullptr);
    default: return seg_ws_layout<T, 16, G>(nullptr, C, n, p.L, p.H, p.CK, nullptr);
    }
}

// One segmented launch (five kernels) of plan p.  stop (device, optional):
// when it is set by the time a kernel starts, that kernel does nothing.
template <typename T, class Prob, int P>
hipError_t seg_run(void *workspace, int64_t C, int64_t n, const SegPlan &p, const typename Prob::Params &pp,
                   hipStream_t stream, const int *stop = nullptr) {
    using G = typename Prob::Tag;
    WsOf<T, Prob> ws;
    const int K = ring_slots_for<T, G>(p.K);
    if constexpr (ring_max<T, G>() >= 128) {
        if (K == 128) {
            seg_ws_layout<T, 128>(workspace, C, n, p.L, p.H, p.CK, &ws);
            ws.stop = stop;
            return seg_launch<T, Prob, 128, P>(ws, pp, stream);
        }
        if (K == 64) {
            seg_ws_layout<T, 64>(workspace, C, n, p.L, p.H, p.CK, &ws);
            ws.stop = stop;
            return seg_launch<T, Prob, 64, P>(ws, pp, stream);
        }
    }
    if (K == 32) {
        seg_ws_layout<T, 32>(workspace, C, n, p.L, p.H, p.CK, &ws);
        ws.stop = stop;
        return seg_launch<T, Prob, 32, P>(ws, pp, stream);
    }
    seg_ws_layout<T, 16>(workspace, C, n, p.L, p.H, p.CK, &ws);
    ws.stop = stop;
    return seg_launch<T, Prob, 16, P>(ws, pp, stream);
}

#pragma clang fp contract(fast)
}  // namespace tvc
