"""Properties of the exact solutions that hold at any size (numpy, test-side).

These checks are independent of both the oracle's algorithm and the GPU
kernels: they restate what the problem statement fixes.

* ``kkt_residual``: optimality conditions of eq. (1D-ROF).  With
  q_e = sum_{k<=e} (x_k - y_k), x is the minimiser iff |q_e| <= w_e on every
  edge, q_e = w_e sign(x_{e+1} - x_e) wherever x_{e+1} != x_e, and the total
  sum q_{n-1} = 0.
* ``run_structure``: the jump pattern (-1, 0, +1 per edge) of a solution.
* ``dual_box_solution``: the chain (or 2D) prox via its dual, a box-constrained
  least-squares problem min |D^T p - y|^2, |p_e| <= w_e, solved by scipy's
  bounded least squares; x = y - D^T p.
* ``kkt_pq``: optimality certificate for the chain with unaries
  a_i x^2/2 - b_i x + c_i |x - d_i| and edge slopes w^-_e <= w^+_e: the edge
  subgradients q_e must satisfy q_e = q_{e-1} + a_i x_i - b_i + c_i u_i with
  u_i in the subdifferential of |x_i - d_i| and q_e in that of the edge term,
  and q_{n-1} = 0; the feasible q_e form an interval, propagated node by node.
* ``kkt_tree``: the same certificate on a forest: the interval of the edge
  subgradient from node i to its parent is a_i x_i - b_i + c_i U_i plus the sum
  of its children's intervals, intersected with the edge's subdifferential;
  a root's sum must contain 0.
"""
from __future__ import annotations

import numpy as np


def kkt_residual(y, x, w, jump_tol: float = 0.0):
    """Return (box_violation, jump_violation, total_sum) for chains along the
    last axis.  ``w`` is a scalar or has y's shape (last slot ignored)."""
    y = np.asarray(y, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = y.shape[-1]
    q = np.cumsum(x - y, axis=-1)
    total = q[..., -1]
    if n == 1:
        return 0.0, 0.0, np.abs(total).max()
    qe = q[..., :-1]
    we = np.broadcast_to(np.asarray(w, dtype=np.float64), y.shape)[..., :-1]
    box = np.maximum(np.abs(qe) - we, 0.0).max()
    d = x[..., 1:] - x[..., :-1]
    jumps = np.abs(d) > jump_tol
    s = np.sign(d)
    jv = np.where(jumps, np.abs(qe - we * s), 0.0).max()
    return float(box), float(jv), float(np.abs(total).max())


def run_structure(x):
    """-1/0/+1 per edge by exact comparison of consecutive values."""
    x = np.asarray(x)
    return np.sign(x[..., 1:] - x[..., :-1]).astype(np.int8)


def _diff_matrix(n):
    D = np.zeros((n - 1, n))
    D[np.arange(n - 1), np.arange(n - 1)] = -1.0
    D[np.arange(n - 1), np.arange(1, n)] = 1.0
    return D


def dual_box_solution_1d(y, w):
    """x = y - D^T p with p = argmin |D^T p - y|^2 s.t. |p_e| <= w_e (BVLS)."""
    from scipy.optimize import lsq_linear
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    if n == 1:
        return y.copy()
    we = np.broadcast_to(np.asarray(w, dtype=np.float64), (n - 1,))
    A = _diff_matrix(n).T
    res = lsq_linear(A, y, bounds=(-we, we), method="bvls", tol=1e-15, max_iter=10000)
    return y - A @ res.x


def dual_box_solution_2d(f, lam):
    """ROF x = f - D^T p with p = argmin |D^T p - f|^2 s.t. |p| <= lam, where D
    stacks the horizontal and vertical forward differences (BVLS)."""
    from scipy.optimize import lsq_linear
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    rows = []
    for r in range(H):
        for c in range(W - 1):
            e = np.zeros(H * W)
            e[r * W + c] = -1.0
            e[r * W + c + 1] = 1.0
            rows.append(e)
    for r in range(H - 1):
        for c in range(W):
            e = np.zeros(H * W)
            e[r * W + c] = -1.0
            e[(r + 1) * W + c] = 1.0
            rows.append(e)
    if not rows:
        return f.copy()
    D = np.array(rows)
    A = D.T
    m = D.shape[0]
    res = lsq_linear(A, f.reshape(-1), bounds=(-lam * np.ones(m), lam * np.ones(m)),
                     method="bvls", tol=1e-15, max_iter=20000)
    return (f.reshape(-1) - A @ res.x).reshape(H, W)


def kkt_pq(a, b, c, d, wm, wp, x, tol: float):
    """Largest violation of the optimality conditions of one chain (see the
    module docstring).  Values within ``tol`` of a kink (x_i = d_i, or
    x_{e+1} = x_e) count as on it; a return value near 0 certifies x."""
    a, b, c, d, x = (np.asarray(v, dtype=np.float64) for v in (a, b, c, d, x))
    wm = np.asarray(wm, dtype=np.float64)
    wp = np.asarray(wp, dtype=np.float64)
    n = x.shape[0]
    lo = hi = 0.0
    worst = 0.0
    for i in range(n):
        r = a[i] * x[i] - b[i]
        if abs(x[i] - d[i]) <= tol:
            ul, uh = -1.0, 1.0
        else:
            ul = uh = float(np.sign(x[i] - d[i]))
        ql, qh = lo + r + c[i] * ul, hi + r + c[i] * uh
        if i == n - 1:
            el = eh = 0.0
        else:
            z = x[i + 1] - x[i]
            if z > tol:
                el = eh = wp[i]
            elif z < -tol:
                el = eh = wm[i]
            else:
                el, eh = wm[i], wp[i]
        lo, hi = max(ql, el), min(qh, eh)
        if lo > hi:  # empty: record the gap and continue from its midpoint
            worst = max(worst, lo - hi)
            lo = hi = 0.5 * (lo + hi)
    return worst


def kkt_tree(parent, a, b, c, d, wm, wp, x, tol: float):
    """Largest violation of the optimality conditions on a forest (parent[i] > i,
    -1 at roots); edge i joins i to parent[i] with z = x_parent - x_i."""
    parent = np.asarray(parent)
    a, b, c, d, x, wm, wp = (np.asarray(v, dtype=np.float64) for v in (a, b, c, d, x, wm, wp))
    n = x.shape[0]
    lo = np.zeros(n)
    hi = np.zeros(n)  # sum of the children's intervals, accumulated as children finish
    worst = 0.0
    for i in range(n):
        r = a[i] * x[i] - b[i]
        ul, uh = (-1.0, 1.0) if abs(x[i] - d[i]) <= tol else (float(np.sign(x[i] - d[i])),) * 2
        ql, qh = lo[i] + r + c[i] * ul, hi[i] + r + c[i] * uh
        p = parent[i]
        if p < 0:
            el = eh = 0.0
        else:
            z = x[p] - x[i]
            if z > tol:
                el = eh = wp[i]
            elif z < -tol:
                el = eh = wm[i]
            else:
                el, eh = wm[i], wp[i]
        l2, h2 = max(ql, el), min(qh, eh)
        if l2 > h2:
            worst = max(worst, l2 - h2)
            l2 = h2 = 0.5 * (l2 + h2)
        if p >= 0:
            lo[p] += l2
            hi[p] += h2
    return worst
