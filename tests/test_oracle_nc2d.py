"""Pins for the Sec. 5.3 non-convex 2D oracle (nc2d_pd): the Lagrangian
primal-dual iteration whose prox steps are exact non-convex chain solves with a
piecewise-linear interpolant of the quadratic proximity term.

* Convex costs and C = inf make the problem a linear program; the iteration
  reaches its optimum, computed independently by scipy's HiGHS.
* w = 0: every pixel keeps the global minimiser of its own (non-convex) cost.
* C above any reachable w |dx| gives the same iterates as C = inf.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

import oracle


def _lp_optimum(cost, steep, w_h, w_v):
    H, W, D = cost.shape
    n = H * W
    ne = H * (W - 1) + (H - 1) * W
    nv = 2 * n + ne
    A, b = [], []
    for i in range(n):
        c = cost.reshape(n, D)[i]
        pieces = [(c[0], -steep, 0.0)] + [(c[k], c[k + 1] - c[k], float(k)) for k in range(D - 1)] + \
                 [(c[-1], steep, float(D - 1))]
        for v0, s, x0 in pieces:  # f_i >= v0 + s (x - x0)
            r = np.zeros(nv)
            r[i] = s
            r[n + i] = -1
            A.append(r)
            b.append(s * x0 - v0)
    e = 2 * n
    wts = []
    for rr in range(H):
        for cc in range(W - 1):
            i = rr * W + cc
            for sgn in (1, -1):
                r = np.zeros(nv)
                r[i], r[i + 1], r[e] = sgn, -sgn, -1
                A.append(r)
                b.append(0)
            wts.append(w_h[rr, cc])
            e += 1
    for rr in range(H - 1):
        for cc in range(W):
            i = rr * W + cc
            for sgn in (1, -1):
                r = np.zeros(nv)
                r[i], r[i + W], r[e] = sgn, -sgn, -1
                A.append(r)
                b.append(0)
            wts.append(w_v[rr, cc])
            e += 1
    obj = np.zeros(nv)
    obj[n:2 * n] = 1
    obj[2 * n:] = wts
    res = linprog(obj, A_ub=np.array(A), b_ub=np.array(b), bounds=[(None, None)] * nv, method="highs")
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_convex_case_reaches_the_lp_optimum(seed):
    g = np.random.default_rng(seed)
    H, W, D = 4 + seed, 5, 6 + seed
    cost = np.cumsum(np.sort(g.normal(size=(H, W, D)), axis=2), axis=2)
    cost -= cost.min(axis=2, keepdims=True)
    w_h = g.uniform(0.2, 1.2, (H, W - 1))
    w_v = g.uniform(0.2, 1.2, (H - 1, W))
    xh, xv, E = oracle.nc2d_pd(cost, 0.0, 1.0, 20.0, w_h, w_v, np.inf, 100.0, 300)
    opt = _lp_optimum(cost, 20.0, w_h, w_v)
    assert abs(E[-1] - opt) <= 1e-7 * (1 + abs(opt)), (E[-1], opt)
    assert np.abs(xh - xv).max() <= 1e-6


def test_zero_weights_keep_each_pixels_global_minimiser():
    g = np.random.default_rng(5)
    H, W, D = 6, 7, 9
    cost = g.uniform(0, 4, (H, W, D))  # non-convex
    xh, xv, E = oracle.nc2d_pd(cost, 0.0, 1.0, 20.0, 0.0, 0.0, 2.0, 50.0, 30)
    best = np.argmin(cost, axis=2).astype(np.float64)
    assert np.array_equal(xh, best) and np.array_equal(xv, best)
    assert abs(E[-1] - cost.min(axis=2).sum()) <= 1e-9


def test_large_truncation_equals_plain_tv():
    g = np.random.default_rng(6)
    H, W, D = 5, 6, 8
    cost = g.uniform(0, 4, (H, W, D))
    a = oracle.nc2d_pd(cost, 0.0, 1.0, 20.0, 0.5, 0.5, np.inf, 100.0, 20)
    b = oracle.nc2d_pd(cost, 0.0, 1.0, 20.0, 0.5, 0.5, 0.5 * 2 * (D + 40) + 100.0, 100.0, 20)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
