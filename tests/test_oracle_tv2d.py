"""Pins of the FP64 2D ROF oracle (Sec. 5.1, eq. (pd), Moreau identity).

The 2D iterate at a fixed iteration count has no closed form on a general
image; what is pinned is the limit (exact ROF solutions from an independent
bounded least-squares solve of the dual, and the reductions of the problem to
a single chain), the rigour of the duality gap (weak duality and the
strong-convexity bound 1/2 |x - x*|^2 <= P(x) - D(p)), and the fixed-count
iterates of the two degenerate shapes (one row, one column), where one of the
two chain steps is the identity and the iteration reduces to chain proxes.
"""
import numpy as np
import pytest

from tests import props


def _img(H, W, seed):
    from paper_1502_07770_amd import synth
    return synth.shapes_image(H, W, n_shapes=4, sigma=0.1, seed=seed)


@pytest.mark.parametrize("shape,lam", [((5, 7), 0.1), ((6, 6), 0.3), ((4, 9), 0.05), ((8, 5), 1.0)])
def test_matches_dual_bvls_and_gap_bounds_error(orc, shape, lam):
    f = _img(*shape, seed=sum(shape))
    xstar = props.dual_box_solution_2d(f, lam)
    HW = f.size
    Pstar = orc.rof2d_objective(f, lam, xstar)
    for iters in (5, 20, 80, 400, 1600):
        x, hist, (P, D, g), k = orc.tv2d(f, lam, max_iter=iters)
        assert k == iters
        gap_abs = g * HW
        assert gap_abs >= -1e-12                              # weak duality
        assert P - Pstar <= gap_abs + 1e-10                   # gap bounds suboptimality
        assert D <= Pstar + 1e-10
        err = np.linalg.norm(x - xstar)
        assert 0.5 * err ** 2 <= gap_abs + 1e-10              # 1-strong convexity
        assert abs(P - orc.rof2d_objective(f, lam, x)) < 1e-10
    assert np.abs(x - xstar).max() < 2e-4                     # O(1/k) in x


def test_gap_nonnegative_and_decreasing(orc):
    f = _img(48, 40, seed=2)
    x, hist, _, k = orc.tv2d(f, 0.1, max_iter=150)
    assert np.all(hist >= -1e-14)
    assert hist[-1] < 1e-2 * hist[0]
    # O(1/k^2)-type decay: the gap shrinks substantially between k and 4k
    assert hist[139] < 0.25 * hist[34]


def test_single_row_reduces_to_chain(orc):
    f = _img(1, 300, seed=4)
    lam = 0.2
    x, hist, _, _ = orc.tv2d(f, lam, max_iter=300)
    xc = orc.chain_prox(f[0], w_scalar=lam)
    gap_abs = hist[-1] * f.size
    assert np.linalg.norm(x[0] - xc) <= np.sqrt(2 * gap_abs) + 1e-12
    assert np.abs(x[0] - xc).max() < 1e-3


def test_single_column_reduces_to_chain(orc):
    f = _img(257, 1, seed=5)
    lam = 0.15
    x, hist, _, _ = orc.tv2d(f, lam, max_iter=300)
    xc = orc.chain_prox(f[:, 0], w_scalar=lam)
    gap_abs = hist[-1] * f.size
    assert np.linalg.norm(x[:, 0] - xc) <= np.sqrt(2 * gap_abs) + 1e-12
    assert np.abs(x[:, 0] - xc).max() < 1e-3


def test_column_constant_image_reduces_to_row_chain(orc):
    """f constant down columns => x is constant down columns and equals the
    chain prox of one row with weight lambda (averaging columns lowers every
    term of the objective)."""
    rng = np.random.default_rng(6)
    row = np.repeat(rng.uniform(0, 1, 12), 8) + rng.normal(0, 0.1, 96)
    f = np.tile(row, (20, 1))
    lam = 0.1
    x, hist, _, _ = orc.tv2d(f, lam, max_iter=400)
    xc = orc.chain_prox(row, w_scalar=lam)
    gap_abs = hist[-1] * f.size
    assert np.linalg.norm(x - xc[None, :]) <= np.sqrt(2 * gap_abs) + 1e-12
    assert np.abs(x - xc[None, :]).max() < 1e-3


def test_zero_lambda_is_identity(orc):
    f = _img(30, 20, seed=7)
    x, hist, _, _ = orc.tv2d(f, 0.0, max_iter=10)
    assert np.abs(x - f).max() < 1e-14
    assert np.abs(hist).max() < 1e-14


def test_huge_lambda_gives_mean(orc):
    f = _img(24, 16, seed=8)
    x, hist, _, _ = orc.tv2d(f, 1e3, max_iter=600)
    assert np.abs(x - f.mean()).max() < 1e-3
    assert hist[-1] * f.size >= 0.5 * np.sum((x - f.mean()) ** 2) - 1e-12


def test_gap_tolerance_stops_early(orc):
    f = _img(40, 32, seed=9)
    x, hist, (_, _, g), k = orc.tv2d(f, 0.1, max_iter=1000, gap_tol=1e-4)
    assert k < 1000 and g <= 1e-4 and hist[-1] == g
    assert np.all(hist[:-1] > 1e-4)


def _sched(tau0, k):
    """tau_k of eq. (pd) with theta_k = 1/sqrt(1 + 2 tau_k), tau_{k+1} = theta_k tau_k."""
    taus = [tau0]
    for _ in range(k):
        taus.append(taus[-1] / np.sqrt(1.0 + 2.0 * taus[-1]))
    return taus


@pytest.mark.parametrize("tau0", [1.0, 0.3])
def test_single_row_iterates_are_chain_proxes(orc, tau0):
    """H = 1: every column chain is one node, whose prox is the identity, so
    the dual iterate stays 0 and each iteration is one chain prox of the row:
    x^{k+1} = prox_{lam tau_k/(1 + tau_k) TV}((tau_k f + x^k)/(1 + tau_k)).
    Pins the row step's data, its weight scaling and the step schedule at a
    fixed iteration count against the chain prox (itself pinned by brute
    force)."""
    f = _img(1, 200, seed=31)
    lam = 0.2
    taus = _sched(tau0, 3)
    x = f[0].copy()
    for k in range(3):
        t = taus[k]
        b = (t * f[0] + x) / (1.0 + t)
        x = orc.chain_prox(b, w_scalar=lam * t / (1.0 + t))
        xo, _, _, _ = orc.tv2d(f, lam, tau0=tau0, max_iter=k + 1)
        assert np.abs(xo[0] - x).max() <= 1e-12 * np.ptp(f), k


@pytest.mark.parametrize("tau0", [1.0, 0.3])
def test_single_column_iterates_follow_the_moreau_identity(orc, tau0):
    """W = 1: every row chain is one node, so the row step returns its data
    b, and the column step is the Moreau identity y' = eta - prox_{lam TV}(eta),
    eta = y + sigma xbar, sigma_0 = 1/tau_0, sigma_{k+1} = sigma_k/theta_k,
    xbar' = x' + theta_k (x' - x).  Pins the dual step's sign and scaling, the
    extrapolation and the schedule at fixed iteration counts against the
    chain prox."""
    f = _img(180, 1, seed=32)
    lam = 0.15
    col = f[:, 0]
    taus = _sched(tau0, 3)
    x, xbar, y, sigma = col.copy(), col.copy(), np.zeros_like(col), 1.0 / tau0
    for k in range(3):
        t = taus[k]
        eta = y + sigma * xbar
        y = eta - orc.chain_prox(eta, w_scalar=lam)
        xn = (t * col + x - t * y) / (1.0 + t)
        theta = 1.0 / np.sqrt(1.0 + 2.0 * t)
        xbar = xn + theta * (xn - x)
        x = xn
        sigma /= theta
        xo, _, _, _ = orc.tv2d(f, lam, tau0=tau0, max_iter=k + 1)
        assert np.abs(xo[:, 0] - x).max() <= 1e-12 * np.ptp(f), k
