"""Pins of the oracle's chain-prox adjoint.

x(y, w) is piecewise affine: on a region where the run structure (fused
edges and jump signs) is fixed, x is the affine run-mean formula.  Central
finite differences whose two probes keep the run structure are therefore
exact up to rounding.  Two identities hold for every (y, w): the sum of dL/dy
equals the sum of g (shift invariance), and <dL/dy, y> + <dL/dw, w> = <g, x>
(x is positively 1-homogeneous in (y, w)).
"""
import numpy as np
import pytest

from tests import props


def _fd_check(orc, y, w, g, h=1e-6, solver=None):
    """Return (max rel err over coordinates whose probes keep the run
    structure, number checked, number skipped)."""
    n = y.shape[0]
    solve = solver or (lambda yy, ww: orc.chain_prox(yy, w=np.concatenate([ww, [0.0]])))
    x = solve(y, w)
    st = props.run_structure(x)
    dy, dw = orc.chain_adjoint(x, g)
    errs, checked, skipped = [], 0, 0
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        xp, xm = solve(y + e, w), solve(y - e, w)
        if not (np.array_equal(props.run_structure(xp), st) and np.array_equal(props.run_structure(xm), st)):
            skipped += 1
            continue
        fd = (g @ xp - g @ xm) / (2 * h)
        errs.append(abs(fd - dy[i]) / max(1.0, abs(dy[i])))
        checked += 1
    for j in range(n - 1):
        e = np.zeros(n - 1)
        e[j] = h
        if w[j] < h:
            continue
        xp, xm = solve(y, w + e), solve(y, w - e)
        if not (np.array_equal(props.run_structure(xp), st) and np.array_equal(props.run_structure(xm), st)):
            skipped += 1
            continue
        fd = (g @ xp - g @ xm) / (2 * h)
        errs.append(abs(fd - dw[j]) / max(1.0, abs(dw[j])))
        checked += 1
    return (max(errs) if errs else 0.0), checked, skipped


def test_fd_against_brute_force_tiny(orc):
    """FD of the brute-force minimiser (independent of the DP)."""
    rng = np.random.default_rng(1)
    brute = lambda yy, ww: orc.chain_brute(np.ones(yy.shape[0]), yy, -ww, ww)
    tot = 0
    for _ in range(60):
        n = int(rng.integers(2, 8))
        y = rng.normal(size=n)
        w = rng.uniform(0.05, 0.8, n - 1)
        g = rng.normal(size=n)
        err, checked, _ = _fd_check(orc, y, w, g, solver=brute)
        assert err < 1e-7
        tot += checked
    assert tot > 300


@pytest.mark.parametrize("seed", [2, 3])
def test_fd_against_oracle_prox(orc, seed):
    from paper_1502_07770_amd import synth
    y = synth.piecewise_constant(1, 120, seed=seed)[0]
    w = synth.edge_weights(119, seed=seed + 10)
    g = synth.normal(120, seed=seed + 20)
    err, checked, skipped = _fd_check(orc, y, w, g)
    assert err < 1e-7
    assert checked > 200 and skipped < 10


def test_sum_and_euler_identities(orc):
    from paper_1502_07770_amd import synth
    y = synth.piecewise_constant(16, 800, seed=4)
    w = synth.edge_weights(y.shape, seed=5)
    w[:, -1] = 0.0
    g = synth.normal(y.shape, seed=6)
    x = orc.chain_prox(y, w=w)
    dy, dw = orc.chain_adjoint(x, g)
    assert np.abs(dy.sum(axis=1) - g.sum(axis=1)).max() < 1e-9
    lhs = (dy * y).sum(axis=1) + (dw * w).sum(axis=1)
    rhs = (g * x).sum(axis=1)
    assert np.abs(lhs - rhs).max() < 1e-8 * np.abs(rhs).max()


def test_zero_weight_and_huge_weight(orc):
    rng = np.random.default_rng(7)
    y = rng.normal(size=50)
    g = rng.normal(size=50)
    # w = 0: every edge is a jump (generic data), dL/dy = g, dL/dw_e = s_e (g_e - g_{e+1})
    x = orc.chain_prox(y, w_scalar=0.0)
    dy, dw = orc.chain_adjoint(x, g)
    s = np.sign(y[1:] - y[:-1])
    assert np.abs(dy - g).max() < 1e-15
    assert np.abs(dw[:-1] - s * (g[:-1] - g[1:])).max() < 1e-14
    # huge w: one run, dL/dy = mean(g), dL/dw = 0
    x = orc.chain_prox(y, w_scalar=1e6)
    dy, dw = orc.chain_adjoint(x, g)
    assert np.abs(dy - g.mean()).max() < 1e-14
    assert np.abs(dw).max() == 0.0


def test_scalar_weight_gradient_is_edge_sum(orc):
    rng = np.random.default_rng(8)
    y = rng.normal(size=(3, 200))
    g = rng.normal(size=(3, 200))
    x = orc.chain_prox(y, w_scalar=0.4)
    _, dw = orc.chain_adjoint(x, g)
    _, dws = orc.chain_adjoint(x, g, scalar_w=True)
    assert np.abs(dw.sum(axis=1) - dws).max() < 1e-12
    # and matches FD in the scalar weight
    h = 1e-6
    xp = orc.chain_prox(y, w_scalar=0.4 + h)
    xm = orc.chain_prox(y, w_scalar=0.4 - h)
    fd = ((g * xp).sum(axis=1) - (g * xm).sum(axis=1)) / (2 * h)
    assert np.abs(fd - dws).max() < 1e-6 * max(1.0, np.abs(dws).max())
