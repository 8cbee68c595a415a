// Host run of the non-convex lane kernels' per-chain bodies (nc_chain_lane of
// k_nc_chain, ncg_chain_lane of k_nc_concave), built with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Every array a lane
// touches is a separate heap block of exactly its size: each message buffer's
// breakpoints (msg_cap) and slopes (msg_cap + 1), the chain's interval list,
// the per-node edge offsets, the per-piece interval ranges and x.  An index of
// -1 or one past the end in any of them aborts the run.  Chains are random and
// ragged (empty, single-node and long ones, tied breakpoints, non-convex
// unaries), with message and interval capacities from too small (the lane must
// stop with its capacity flag, in bounds) to ample; a last pass lays the three
// buffers of several lanes side by side in one block as the dynamic-LDS launch
// of k_nc_chain does (lane l at l * 3 * (2 msg_cap + 1) doubles).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1502_07770_amd/csrc/nc_chain.hip"

using namespace tvc;

namespace {

struct Chains {
    std::vector<int64_t> coff, uoff, poff;
    std::vector<double> ulam, uslope, w, C, palpha, pC;
    std::vector<int32_t> pside;
    int64_t nodes = 0, pieces = 0;
};

Chains make_chains(std::mt19937_64 &g, int num_chains, int max_len) {
    std::uniform_real_distribution<double> U(0.0, 1.0);
    Chains ch;
    ch.coff.push_back(0);
    ch.uoff.push_back(0);
    ch.poff.push_back(0);
    for (int c = 0; c < num_chains; ++c) {
        int len = (int)(U(g) * (max_len + 1));
        if (c % 17 == 0) len = 0;
        if (c % 13 == 1) len = 1;
        for (int i = 0; i < len; ++i) {
            const int tu = 1 + (int)(U(g) * 6);
            double l = -3.0 + 6.0 * U(g);
            for (int k = 0; k < tu; ++k) {
                if (k > 0 && U(g) > 0.2) l += U(g);  // some ties
                ch.ulam.push_back(std::round(l * 8.0) / 8.0);
            }
            // slopes s_0 <= 0 <= s_t, arbitrary (non-convex) in between
            ch.uslope.push_back(-U(g) * 2.0);
            for (int k = 1; k < tu; ++k) ch.uslope.push_back(-2.0 + 4.0 * U(g));
            ch.uslope.push_back(U(g) * 2.0);
            ch.uoff.push_back(ch.uoff.back() + tu);
            ch.w.push_back(2.0 * U(g));
            ch.C.push_back(U(g) < 0.3 ? HUGE_VAL : 0.1 + 3.0 * U(g));
            const int np = (int)(U(g) * 7);  // pieces of the edge leaving this node
            for (int k = 0; k < np; ++k) {
                ch.palpha.push_back(2.0 * U(g));
                ch.pC.push_back(3.0 * U(g));
                ch.pside.push_back(U(g) < 0.5 ? 1 : -1);
            }
            ch.poff.push_back(ch.poff.back() + np);
        }
        ch.coff.push_back(ch.coff.back() + len);
    }
    ch.nodes = ch.coff.back();
    ch.pieces = ch.poff.back();
    // per-node slopes are stored with one extra slot per node (uslope[uoff[i] + i + k])
    return ch;
}

// A message buffer in two exactly-sized heap blocks.
struct Owned {
    double *l, *s;
    explicit Owned(int64_t cap) : l((double *)malloc(sizeof(double) * cap)), s((double *)malloc(sizeof(double) * (cap + 1))) {}
    ~Owned() {
        free(l);
        free(s);
    }
    NcBuf buf(int64_t cap) const { return NcBuf{l, s, 0, cap}; }
};

int runs = 0, capacity_stops = 0;

void check_flag(int f, const char *what) {
    if (f & ~(kNcFlagCapacity | kNcFlagInvalid)) {
        fprintf(stderr, "%s: unexpected flag %d\n", what, f);
        exit(1);
    }
    if (f & kNcFlagInvalid) {  // the generator makes valid chains only
        fprintf(stderr, "%s: valid chain reported invalid\n", what);
        exit(1);
    }
    capacity_stops += (f & kNcFlagCapacity) != 0;
}

template <typename T>
void run_truncated(const Chains &ch, int64_t msg_cap, int64_t map_cap, bool lds_layout) {
    const int64_t Cn = (int64_t)ch.coff.size() - 1;
    std::vector<T> ulam(ch.ulam.begin(), ch.ulam.end()), uslope(ch.uslope.begin(), ch.uslope.end());
    std::vector<T> w(ch.w.begin(), ch.w.end()), Cv(ch.C.begin(), ch.C.end());
    T *x = (T *)malloc(sizeof(T) * (ch.nodes > 0 ? ch.nodes : 1));
    int64_t *eoff = (int64_t *)malloc(sizeof(int64_t) * 3 * (ch.nodes > 0 ? ch.nodes : 1));
    NcArgs A;
    A.num_chains = Cn;
    A.num_nodes = ch.nodes;
    A.coff = ch.coff.data();
    A.uoff = ch.uoff.data();
    A.msg_cap = msg_cap;
    A.map_cap = map_cap;
    A.bufs = nullptr;
    A.eoff = eoff;
    A.flag = nullptr;
    const int64_t bstride = 2 * msg_cap + 1;
    const int lanes = 5;
    double *lds = lds_layout ? (double *)malloc(sizeof(double) * 3 * bstride * lanes) : nullptr;
    for (int64_t c = 0; c < Cn; ++c) {
        // chain c as lane index 0 of a view that starts at its offsets, so that
        // its interval list is its own block of exactly map_cap intervals
        double *maps = (double *)malloc(sizeof(double) * 3 * map_cap);
        A.maps = maps;
        A.coff = ch.coff.data() + c;
        int f;
        if (lds_layout) {
            double *base = lds + (c % lanes) * 3 * bstride;
            f = nc_chain_lane<T>(A, ulam.data(), uslope.data(), w.data(), Cv.data(), x, 0,
                                 NcBuf{base, base + msg_cap, 0, msg_cap},
                                 NcBuf{base + bstride, base + bstride + msg_cap, 0, msg_cap},
                                 NcBuf{base + 2 * bstride, base + 2 * bstride + msg_cap, 0, msg_cap});
        } else {
            Owned M(msg_cap), H(msg_cap), B(msg_cap);
            f = nc_chain_lane<T>(A, ulam.data(), uslope.data(), w.data(), (c % 2) ? Cv.data() : nullptr, x, 0,
                                 M.buf(msg_cap), H.buf(msg_cap), B.buf(msg_cap));
        }
        check_flag(f, "truncated TV lane");
        ++runs;
        free(maps);
    }
    free(lds);
    free(eoff);
    free(x);
}

template <typename T>
void run_concave(const Chains &ch, int64_t msg_cap, int64_t map_cap) {
    const int64_t Cn = (int64_t)ch.coff.size() - 1;
    std::vector<T> ulam(ch.ulam.begin(), ch.ulam.end()), uslope(ch.uslope.begin(), ch.uslope.end());
    std::vector<T> pa(ch.palpha.begin(), ch.palpha.end()), pc(ch.pC.begin(), ch.pC.end());
    T *x = (T *)malloc(sizeof(T) * (ch.nodes > 0 ? ch.nodes : 1));
    int64_t *pmap = (int64_t *)malloc(sizeof(int64_t) * 2 * (ch.pieces > 0 ? ch.pieces : 1));
    NcgArgs A;
    A.num_chains = Cn;
    A.num_nodes = ch.nodes;
    A.num_pieces = ch.pieces;
    A.coff = ch.coff.data();
    A.uoff = ch.uoff.data();
    A.poff = ch.poff.data();
    A.msg_cap = msg_cap;
    A.map_cap = map_cap;
    A.bufs = nullptr;
    A.pmap = pmap;
    A.flag = nullptr;
    for (int64_t c = 0; c < Cn; ++c) {
        double *maps = (double *)malloc(sizeof(double) * 3 * map_cap);
        A.maps = maps;
        A.coff = ch.coff.data() + c;  // chain c as lane index 0 (see run_truncated)
        Owned X(msg_cap), Y(msg_cap), U(msg_cap);
        const int f = ncg_chain_lane<T>(A, ulam.data(), uslope.data(), pa.data(), pc.data(), ch.pside.data(), x, 0,
                                        X.buf(msg_cap), Y.buf(msg_cap), U.buf(msg_cap));
        check_flag(f, "concave lane");
        ++runs;
        free(maps);
    }
    free(pmap);
    free(x);
}

}  // namespace

int main() {
    std::mt19937_64 g(20261203);
    const Chains ch = make_chains(g, 160, 90);
    const int64_t caps[][2] = {{2, 2}, {4, 8}, {8, 64}, {37, 4096}, {300, 100000}};
    for (const auto &cm : caps) {
        run_truncated<double>(ch, cm[0], cm[1], false);
        run_truncated<float>(ch, cm[0], cm[1], false);
        run_truncated<double>(ch, cm[0], cm[1], true);
        run_concave<double>(ch, cm[0], cm[1]);
        run_concave<float>(ch, cm[0], cm[1]);
    }
    printf("nc lane checks passed: %d chain runs (%d stopped at capacity), %ld nodes, %ld pieces\n", runs,
           capacity_stops, (long)ch.nodes, (long)ch.pieces);
    return 0;
}
