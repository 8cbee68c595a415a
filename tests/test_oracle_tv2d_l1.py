"""Pins of the oracle's Sec. 5.2 TV-l1 solver (eq. (pd) with the column dual
prox and the row primal prox eq. (prox-pq)): on small images its energy
reaches the optimum of the problem written as a linear program (solved by
scipy's HiGHS, independent of any chain algorithm); lambda = 0 returns f;
shifting f shifts x."""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import oracle


def _lp_optimum(f, lam):
    """min lam sum_e |D x|_e + sum |x - f| as an LP over (x, t >= |Dx|, s >= |x - f|)."""
    H, W = f.shape
    N = H * W
    edges = [(r * W + c, r * W + c + 1) for r in range(H) for c in range(W - 1)]
    edges += [(r * W + c, (r + 1) * W + c) for r in range(H - 1) for c in range(W)]
    E = len(edges)
    D = sp.lil_matrix((max(E, 1), N))
    for e, (i, j) in enumerate(edges):
        D[e, i], D[e, j] = -1.0, 1.0
    D = D.tocsr()[:E]
    I_n = sp.identity(N, format="csr")
    I_e = sp.identity(E, format="csr")
    Z = lambda a, b: sp.csr_matrix((a, b))  # noqa: E731
    A = sp.vstack([sp.hstack([D, -I_e, Z(E, N)]), sp.hstack([-D, -I_e, Z(E, N)]),
                   sp.hstack([I_n, Z(N, E), -I_n]), sp.hstack([-I_n, Z(N, E), -I_n])]).tocsr()
    b = np.concatenate([np.zeros(2 * E), f.ravel(), -f.ravel()])
    c = np.concatenate([np.zeros(N), lam * np.ones(E), np.ones(N)])
    r = so.linprog(c, A_ub=A, b_ub=b, bounds=[(None, None)] * N + [(0, None)] * (E + N), method="highs")
    assert r.status == 0
    return r.fun


def _impulse_image(H, W, seed):
    rng = np.random.default_rng(seed)
    f = np.round(rng.uniform(0, 1, (H, W)), 1)
    m = rng.random((H, W)) < 0.25
    f[m] = rng.integers(0, 2, int(m.sum()))
    return f


@pytest.mark.parametrize("H,W,lam", [(1, 12, 0.6), (4, 5, 0.55), (6, 6, 0.3), (5, 7, 1.2), (7, 3, 0.1), (1, 1, 0.5)])
def test_energy_reaches_the_lp_optimum(H, W, lam):
    f = _impulse_image(H, W, seed=H * 10 + W)
    x, hist = oracle.tv2d_l1(f, lam, tau=1.0, max_iter=600)
    p_star = _lp_optimum(f, lam)
    assert hist[-1] == pytest.approx(oracle.tvl1_2d_objective(f, lam, x))
    assert hist[-1] - p_star <= 1e-9 * max(p_star, 1.0)
    assert hist[-1] >= p_star - 1e-9 * max(p_star, 1.0)  # never below the optimum


def test_other_step_sizes_reach_it_too():
    f = _impulse_image(6, 8, seed=3)
    p_star = _lp_optimum(f, 0.4)
    for tau in (0.3, 3.0):
        _, hist = oracle.tv2d_l1(f, 0.4, tau=tau, max_iter=3000)
        assert hist[-1] - p_star <= 1e-6 * p_star


def test_lambda_zero_returns_f():
    f = _impulse_image(9, 11, seed=4)
    x, _ = oracle.tv2d_l1(f, 0.0, max_iter=1)
    assert np.array_equal(x, f)


def test_shift_invariance():
    f = _impulse_image(10, 12, seed=5)
    x, _ = oracle.tv2d_l1(f, 0.5, max_iter=50)
    xs, _ = oracle.tv2d_l1(f + 0.375, 0.5, max_iter=50)
    assert np.abs(xs - (x + 0.375)).max() <= 1e-12


def test_single_row_iterates_are_tv_l1_chain_proxes(orc):
    """One row: every column chain is one node (prox = identity), so the dual
    iterate stays 0 and each iteration is the TV-l1 chain prox of the row,
    x^{k+1} = prox of (1/2)|x - x^k|^2 + tau lam TV(x) + tau |x - f|, i.e.
    orc.chain_prox_l1 with y = x^k, d = f, w = tau lam, c = tau (pinned by
    brute force in its own tests)."""
    rng = np.random.default_rng(41)
    f = np.repeat(rng.uniform(0, 1, 16), 10)[None, :]
    m = rng.random(f.shape) < 0.25
    f[m] = rng.integers(0, 2, int(m.sum()))
    lam, tau = 0.55, 0.7
    x = f[0].copy()
    for k in range(4):
        x = orc.chain_prox_l1(x, f[0], w_scalar=tau * lam, c_scalar=tau)
        xo, _ = orc.tv2d_l1(f, lam, tau=tau, max_iter=k + 1)
        assert np.abs(xo[0] - x).max() <= 1e-12, k


def test_single_column_iterates_soft_threshold_toward_f(orc):
    """One column: every row chain is one node, whose TV-l1 prox is the
    soft-threshold of xi toward f by tau; the dual step is the Moreau identity
    of the column's TV prox with sigma = 1/tau and xbar' = 2 x' - x."""
    rng = np.random.default_rng(42)
    col = np.repeat(rng.uniform(0, 1, 15), 10)
    m = rng.random(col.shape) < 0.25
    col[m] = rng.integers(0, 2, int(m.sum()))
    f = col[:, None].copy()
    lam, tau = 0.4, 0.8
    sigma = 1.0 / tau
    x, xbar, y = col.copy(), col.copy(), np.zeros_like(col)
    for k in range(4):
        eta = y + sigma * xbar
        y = eta - orc.chain_prox(eta, w_scalar=lam)
        xi = x - tau * y
        xn = col + np.sign(xi - col) * np.maximum(np.abs(xi - col) - tau, 0.0)
        xbar = 2.0 * xn - x
        x = xn
        xo, _ = orc.tv2d_l1(f, lam, tau=tau, max_iter=k + 1)
        assert np.abs(xo[:, 0] - x).max() <= 1e-12, k
