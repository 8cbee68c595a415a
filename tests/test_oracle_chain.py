"""Pins of the FP64 chain-prox oracle (Sec. 4.1) against what the problem fixes.

Each test would catch a plausible mistake in the oracle: a wrong sign, a
dropped slope term, a transposed scan direction, an off-by-one in the
edge/weight indexing, a wrong first-node or root rule.
"""
import numpy as np
import pytest

from tests import props


def _rng(seed):
    return np.random.default_rng(seed)


# -- brute force: independent exhaustive search over sign patterns ----------

@pytest.mark.parametrize("general", [False, True])
def test_dp_matches_brute_force(orc, general):
    rng = _rng(11 + general)
    worst = 0.0
    for trial in range(1500):
        n = int(rng.integers(1, 10))
        b = rng.normal(0.0, 1.0, n) * rng.choice([0.1, 1.0, 10.0])
        if general:
            a = rng.uniform(0.2, 3.0, n)
            wp = rng.uniform(0.0, 1.5, n - 1)
            wm = -rng.uniform(0.0, 1.5, n - 1)
        else:
            a = np.ones(n)
            w = rng.uniform(0.0, 1.5, n - 1) * rng.choice([0.0, 0.1, 1.0, 10.0])
            wp, wm = w, -w
        x, _, _, _ = orc.chain_dp(a, b, wm, wp)
        xb = orc.chain_brute(a, b, wm, wp)
        scale = max(1.0, np.abs(b).max())
        worst = max(worst, np.abs(x - xb).max() / scale)
    assert worst < 1e-12, worst


def test_brute_force_objective_is_minimal(orc):
    """The brute-force point is no worse than random perturbations of it."""
    rng = _rng(3)
    for _ in range(200):
        n = int(rng.integers(2, 8))
        y = rng.normal(size=n)
        w = rng.uniform(0, 1, n - 1)
        xb = orc.chain_brute(np.ones(n), y, -w, w)
        f0 = orc.rof1d_objective(y, w, xb)
        for _ in range(20):
            xp = xb + rng.normal(0, 1e-3, n)
            assert orc.rof1d_objective(y, w, xp) >= f0 - 1e-12


# -- dual box-constrained least squares (scipy BVLS), moderate n -----------

@pytest.mark.parametrize("n", [17, 60, 150])
def test_dp_matches_dual_bvls(orc, n):
    rng = _rng(n)
    for trial in range(3):
        y = rng.normal(size=n) + np.repeat(rng.uniform(0, 1, n // 10 + 1), 10)[:n]
        w = rng.uniform(0.05, 0.8, n - 1)
        x = orc.chain_prox(y, w=np.concatenate([w, [0.0]]))
        xd = props.dual_box_solution_1d(y, w)
        assert np.abs(x - xd).max() < 1e-8


# -- optimality certificate at realistic sizes -------------------------------

@pytest.mark.parametrize("wkind", ["scalar", "edge", "zeros", "huge", "mixed"])
def test_kkt_certificate(orc, wkind):
    from paper_1502_07770_amd import synth
    rng = _rng(7)
    y = synth.piecewise_constant(32, 2000, seed=5)
    if wkind == "scalar":
        w = np.full_like(y, 0.3)
    elif wkind == "edge":
        w = rng.uniform(0.1, 1.0, y.shape)
    elif wkind == "zeros":
        w = np.zeros_like(y)
    elif wkind == "huge":
        w = np.full_like(y, 1e4)
    else:
        w = rng.uniform(0.0, 1.0, y.shape) * (rng.random(y.shape) < 0.7)
    x = orc.chain_prox(y, w=w)
    box, jump, total = props.kkt_residual(y, x, w, jump_tol=1e-10)
    assert box < 1e-9 and jump < 1e-9 and total < 1e-9, (box, jump, total)


# -- closed forms -------------------------------------------------------------

def test_zero_weight_is_identity(orc):
    y = _rng(1).normal(size=(5, 300))
    x = orc.chain_prox(y, w_scalar=0.0)
    assert np.abs(x - y).max() < 1e-13   # equal up to the DP's rounding


def test_single_node_is_identity(orc):
    y = _rng(2).normal(size=(7, 1))
    for w in (0.0, 0.5, 1e6):
        assert np.abs(orc.chain_prox(y, w_scalar=w) - y).max() < 1e-15


def test_two_nodes_closed_form(orc):
    rng = _rng(4)
    for _ in range(500):
        y1, y2 = rng.normal(size=2)
        w = rng.uniform(0, 2)
        x = orc.chain_prox(np.array([y1, y2]), w_scalar=w)
        if abs(y2 - y1) <= 2 * w:
            ref = np.array([(y1 + y2) / 2, (y1 + y2) / 2])
        else:
            s = np.sign(y2 - y1)
            ref = np.array([y1 + w * s, y2 - w * s])
        assert np.abs(x - ref).max() < 1e-14


def test_constant_solution_threshold(orc):
    """x is the constant mean(y) iff w_e >= |sum_{k<=e}(y_k - mean)| for all e."""
    rng = _rng(5)
    for _ in range(50):
        n = int(rng.integers(3, 200))
        y = rng.normal(size=n)
        thr = np.abs(np.cumsum(y - y.mean()))[:-1]
        w = thr * (1 + 1e-9) + 1e-12
        x = orc.chain_prox(y, w=np.concatenate([w, [0.0]]))
        assert np.abs(x - y.mean()).max() < 1e-10
        e = int(np.argmax(thr))
        if thr[e] > 1e-3:
            w2 = w.copy()
            w2[e] = thr[e] * 0.5
            x2 = orc.chain_prox(y, w=np.concatenate([w2, [0.0]]))
            assert np.ptp(x2) > 1e-6


def test_huge_weight_gives_mean(orc):
    y = _rng(6).normal(size=(4, 500))
    x = orc.chain_prox(y, w_scalar=1e6)
    assert np.abs(x - y.mean(axis=1, keepdims=True)).max() < 1e-9


# -- invariances ---------------------------------------------------------------

def test_invariances(orc):
    from paper_1502_07770_amd import synth
    y = synth.piecewise_constant(8, 700, seed=9)
    w = synth.edge_weights(y.shape, seed=10)
    x = orc.chain_prox(y, w=w)
    assert np.abs(orc.chain_prox(y + 3.25, w=w) - (x + 3.25)).max() < 1e-11   # shift
    assert np.abs(orc.chain_prox(-y, w=w) + x).max() < 1e-11                  # negation
    assert np.abs(orc.chain_prox(2.5 * y, w=2.5 * w) - 2.5 * x).max() < 1e-11  # homogeneity
    # reversal: edge e of the reversed chain is edge n-2-e of the original
    wr = np.concatenate([w[:, :-1][:, ::-1], np.zeros((8, 1))], axis=1)
    xr = orc.chain_prox(y[:, ::-1], w=wr)
    assert np.abs(xr[:, ::-1] - x).max() < 1e-11
    assert np.abs(x.sum(axis=1) - y.sum(axis=1)).max() < 1e-9                # mean preserved


# -- operation counts (amortised O(n) argument of Sec. 4.1) --------------------

def test_operation_counts(orc):
    from paper_1502_07770_amd import synth
    y = synth.piecewise_constant(16, 1000, seed=12)
    for w in (0.0, 0.1, 0.5, 100.0):
        _, st = orc.chain_prox(y, w_scalar=w, counts=True)
        n = y.shape[1]
        assert np.all(st[:, 0] == 2 * (n - 1))          # two breakpoints per non-root node
        assert np.all(st[:, 1] <= st[:, 0])             # each removed at most once
        assert np.all(st[:, 2] <= 2 * (n - 1))          # fits the 4n+O(1) array
        assert np.all(st[:, 2] >= 2)


def test_general_dp_lambdas_bracket_solution(orc):
    """x_i = clip(x_{i+1}, lam^-_i, lam^+_i) with lam^- <= lam^+ (Algorithm 2)."""
    rng = _rng(13)
    n = 400
    a = rng.uniform(0.5, 2, n)
    b = rng.normal(size=n)
    w = rng.uniform(0, 1, n - 1)
    x, lo, hi, _ = orc.chain_dp(a, b, -w, w)
    assert np.all(lo <= hi)
    assert np.array_equal(x[:-1], np.minimum(np.maximum(x[1:], lo), hi))
