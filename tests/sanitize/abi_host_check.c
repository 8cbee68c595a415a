/* Host-side checks of the C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer against a host-only build of the library
 * (tests/test_sanitizers.py).  Every call here either is a pure host query
 * (workspace sizes, tuning, status strings) or carries an argument error that
 * the library must reject before touching a device, so the program never
 * launches a kernel and runs the same with or without a GPU.  It exits non-zero
 * on the first unexpected result; the sanitizers abort on any memory or UB
 * error in the library's host code. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "tvchain.h"

static int calls = 0;

static void expect_status(const char *what, tv_status got, tv_status want) {
    ++calls;
    if (got != want) {
        fprintf(stderr, "%s: status %d (%s), expected %d\n", what, (int)got, tv_status_string(got), (int)want);
        exit(1);
    }
}

static void expect_size(const char *what, size_t got, int positive) {
    ++calls;
    if ((got > 0) != (positive != 0)) {
        fprintf(stderr, "%s: size %zu, expected %s\n", what, got, positive ? "> 0" : "0");
        exit(1);
    }
}

int main(void) {
    static float buf[8192], out[8192]; /* large enough for every layout passed below */
    void *p = buf, *q = out; /* an input and a distinct output (inputs and outputs must not overlap) */
    const tv_dtype dts[2] = {TV_F32, TV_F64};

    /* status strings, including codes outside the enum */
    for (int s = -2; s <= 8; ++s) {
        const char *t = tv_status_string((tv_status)s);
        ++calls;
        if (!t || !t[0]) {
            fprintf(stderr, "empty status string for %d\n", s);
            return 1;
        }
    }

    /* chain-prox workspace queries over shapes and layouts */
    const int64_t shapes[][2] = {{1, 1}, {1, 2}, {3, 7}, {64, 256}, {4096, 4096}, {65536, 1024}, {7, 100000}};
    for (int d = 0; d < 2; ++d)
        for (size_t k = 0; k < sizeof(shapes) / sizeof(shapes[0]); ++k) {
            const tv_chain_layout rows = {shapes[k][0], shapes[k][1], 1, shapes[k][1], NULL};
            const tv_chain_layout cols = {shapes[k][0], shapes[k][1], shapes[k][0], 1, NULL};
            expect_size("prox ws rows", tv_chain_prox_workspace(&rows, dts[d]), 1);
            expect_size("prox ws cols", tv_chain_prox_workspace(&cols, dts[d]), 1);
            expect_size("dp ws", tv_chain_dp_workspace(&rows, dts[d]), 1);
            expect_size("l1 ws", tv_chain_prox_l1_workspace(&rows, dts[d]), 1);
            (void)tv_chain_prox_backward_workspace(&rows, dts[d]);  /* documented: may be 0 */
            ++calls;
            const tv_chain_layout two[2] = {rows, cols};
            expect_size("multi ws", tv_chain_prox_multi_workspace(2, two, dts[d]), 1);
            ++calls;
            if (tv_chain_prox_segment_length(&rows) < 1) {
                fprintf(stderr, "segment length < 1\n");
                return 1;
            }
        }
    const tv_chain_layout good = {16, 64, 1, 64, NULL};
    const tv_chain_layout bad_len = {16, 0, 1, 64, NULL};
    const tv_chain_layout bad_n = {-1, 64, 1, 64, NULL};
    expect_size("prox ws null layout", tv_chain_prox_workspace(NULL, TV_F32), 0);
    expect_size("prox ws bad dtype", tv_chain_prox_workspace(&good, (tv_dtype)7), 0);
    expect_size("prox ws bad chains", tv_chain_prox_workspace(&bad_n, TV_F32), 0);
    expect_size("multi ws no batches", tv_chain_prox_multi_workspace(0, &good, TV_F32), 0);
    (void)bad_len;

    /* argument errors of the chain entry points */
    for (int d = 0; d < 2; ++d) {
        expect_status("prox null y", tv_chain_prox(&good, dts[d], NULL, NULL, 0.5, p, p, 1 << 20, NULL),
                      TV_ERR_INVALID_ARG);
        expect_status("prox negative w", tv_chain_prox(&good, dts[d], p, NULL, -1.0, p, p, 1 << 20, NULL),
                      TV_ERR_INVALID_ARG);
        expect_status("prox nan w", tv_chain_prox(&good, dts[d], p, NULL, NAN, p, p, 1 << 20, NULL),
                      TV_ERR_INVALID_ARG);
        expect_status("prox no workspace", tv_chain_prox(&good, dts[d], p, NULL, 0.5, q, NULL, 0, NULL),
                      TV_ERR_WORKSPACE);
        expect_status("prox small workspace", tv_chain_prox(&good, dts[d], p, NULL, 0.5, q, p, 16, NULL),
                      TV_ERR_WORKSPACE);
        expect_status("noalloc null x", tv_chain_prox_noalloc(&good, dts[d], p, NULL, 0.5, NULL, NULL),
                      TV_ERR_INVALID_ARG);
        expect_status("dp null b", tv_chain_dp(&good, dts[d], NULL, NULL, p, p, p, p, 1 << 20, NULL),
                      TV_ERR_INVALID_ARG);
        expect_status("l1 negative c", tv_chain_prox_l1(&good, dts[d], p, p, NULL, 0.5, NULL, -1.0, p, p, 1 << 20,
                                                        NULL),
                      TV_ERR_INVALID_ARG);
        expect_status("bwd null g", tv_chain_prox_backward(&good, dts[d], p, NULL, NULL, p, 0, p, 1 << 20, NULL),
                      TV_ERR_INVALID_ARG);
        const void *ys[1] = {p}, *ws_[1] = {NULL};
        void *xs[1] = {p};
        const double wsc[1] = {-0.5};
        expect_status("multi negative w", tv_chain_prox_multi(1, &good, dts[d], ys, ws_, wsc, xs, p, 1 << 20, NULL),
                      TV_ERR_INVALID_ARG);
    }

    /* trees */
    expect_size("tree ws", tv_tree_dp_workspace(100, 25600), 1);
    expect_status("tree null parent",
                  tv_tree_dp(TV_F32, 1, 4, (const int64_t *)p, NULL, NULL, p, NULL, NULL, p, p, p, p, 1 << 20, NULL),
                  TV_ERR_INVALID_ARG);

    /* 2D ROF */
    const int64_t sides[] = {1, 2, 63, 64, 65, 512, 4096};
    for (int d = 0; d < 2; ++d)
        for (size_t a = 0; a < sizeof(sides) / sizeof(sides[0]); ++a)
            for (size_t b = 0; b < sizeof(sides) / sizeof(sides[0]); ++b) {
                expect_size("tv2d ws", tv2d_workspace(sides[a], sides[b], dts[d]), 1);
                expect_size("tv2d l1 ws", tv2d_l1_workspace(sides[a], sides[b], dts[d]), 1);
            }
    expect_size("tv2d ws empty", tv2d_workspace(0, 5, TV_F32), 0);
    tv2d_options opt = {10, 1, 1e-4, 1.0, 0, NULL, 0};
    tv2d_options bad = opt;
    expect_status("tv2d ld < W", tv2d_solve(TV_F32, p, 8, 8, 4, 0.1, p, &opt, NULL, p, 1 << 30, NULL),
                  TV_ERR_INVALID_ARG);
    expect_status("tv2d nan lambda", tv2d_solve(TV_F32, p, 8, 8, 8, NAN, p, &opt, NULL, p, 1 << 30, NULL),
                  TV_ERR_INVALID_ARG);
    bad.max_iter = -1;
    expect_status("tv2d max_iter", tv2d_solve(TV_F32, p, 8, 8, 8, 0.1, p, &bad, NULL, p, 1 << 30, NULL),
                  TV_ERR_INVALID_ARG);
    bad = opt;
    bad.tau0 = 0.0;
    expect_status("tv2d tau0", tv2d_solve(TV_F64, p, 8, 8, 8, 0.1, p, &bad, NULL, p, 1 << 30, NULL),
                  TV_ERR_INVALID_ARG);
    expect_status("tv2d small ws", tv2d_solve(TV_F32, p, 8, 8, 8, 0.1, q, &opt, NULL, p, 8, NULL),
                  TV_ERR_WORKSPACE);
    bad = opt;
    bad.lookahead = 65;
    expect_status("tv2d lookahead", tv2d_solve(TV_F32, p, 8, 8, 8, 0.1, q, &bad, NULL, p, 1 << 30, NULL),
                  TV_ERR_INVALID_ARG);
    bad.lookahead = -1;
    expect_status("tv2d lookahead < 0", tv2d_solve(TV_F64, p, 8, 8, 8, 0.1, q, &bad, NULL, p, 1 << 30, NULL),
                  TV_ERR_INVALID_ARG);
    bad = opt;
    bad.gap_tol = 1e-3;
    expect_status("tv2d l1 gap_tol", tv2d_l1_solve(TV_F32, p, 8, 8, 8, 0.5, p, &bad, NULL, p, 1 << 30, NULL),
                  TV_ERR_INVALID_ARG);

    /* batched 2D: uneven geometry through the host layout, then argument errors */
    enum { NI = 37 };
    int64_t H[NI], W[NI], off[NI];
    double lam[NI];
    int64_t o = 0;
    for (int j = 0; j < NI; ++j) {
        H[j] = 1 + (j * 97) % 300;
        W[j] = 1 + (j * 61) % 257;
        off[j] = o;
        lam[j] = 0.02 + 0.01 * j;
        o += H[j] * W[j];
    }
    for (int d = 0; d < 2; ++d) expect_size("batched ws", tv2d_batched_workspace(NI, H, W, dts[d]), 1);
    expect_size("batched ws none", tv2d_batched_workspace(0, H, W, TV_F32), 0);
    const size_t bws = tv2d_batched_workspace(NI, H, W, TV_F32);
    lam[5] = NAN;
    expect_status("batched nan lambda",
                  tv2d_solve_batched(TV_F32, NI, H, W, off, lam, p, p, &opt, NULL, p, bws, NULL), TV_ERR_INVALID_ARG);
    lam[5] = 0.1;
    off[3] += 1;
    expect_status("batched unpacked",
                  tv2d_solve_batched(TV_F32, NI, H, W, off, lam, p, p, &opt, NULL, p, bws, NULL), TV_ERR_INVALID_ARG);
    off[3] -= 1;
    opt.resume = 1;
    expect_status("batched resume",
                  tv2d_solve_batched(TV_F32, NI, H, W, off, lam, p, p, &opt, NULL, p, bws, NULL), TV_ERR_INVALID_ARG);
    opt.resume = 0;
    opt.lookahead = 99;
    expect_status("batched lookahead",
                  tv2d_solve_batched(TV_F32, NI, H, W, off, lam, p, q, &opt, NULL, p, bws, NULL), TV_ERR_INVALID_ARG);
    opt.lookahead = 0;
    expect_status("batched small ws",
                  tv2d_solve_batched(TV_F32, NI, H, W, off, lam, p, q, &opt, NULL, p, bws - 1, NULL), TV_ERR_WORKSPACE);

    /* non-convex workspace queries */
    expect_size("nc ws", tv_chain_nc_workspace(10, 1000, 64, 256), 1);
    expect_size("nc tree ws", tv_tree_nc_workspace(10, 1000, 64, 256, 64), 1);
    expect_size("nc2d ws", tv2d_nc_workspace(20, 30, 16, 64, 256), 1);

    /* tuning: round trip, rejection, restore */
    tv_tuning t0, t1, t2;
    expect_status("get tuning", tv_get_tuning(&t0), TV_OK);
    t1 = t0;
    t1.ring_slots = 24;
    expect_status("bad ring", tv_set_tuning(&t1), TV_ERR_INVALID_ARG);
    t1 = t0;
    t1.min_segment = 0;
    expect_status("bad segment", tv_set_tuning(&t1), TV_ERR_INVALID_ARG);
    t1 = t0;
    t1.ring_slots = 64;
    t1.halo = 32;
    expect_status("set tuning", tv_set_tuning(&t1), TV_OK);
    expect_status("get tuning again", tv_get_tuning(&t2), TV_OK);
    ++calls;
    if (t2.ring_slots != 64 || t2.halo != 32) {
        fprintf(stderr, "tuning did not round-trip\n");
        return 1;
    }
    expect_size("prox ws under tuning", tv_chain_prox_workspace(&good, TV_F32), 1);
    expect_status("reset tuning", tv_set_tuning(NULL), TV_OK);

    printf("host ABI checks passed: %d calls\n", calls);
    return 0;
}
