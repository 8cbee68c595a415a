"""Pins of the oracle's Sec. 4.2 DP (piecewise-quadratic unaries
a_i x^2/2 - b_i x + c_i |x - d_i|, the unaries of the TV-l1 primal prox,
eq. (prox-pq)) and of its TV-l1 chain prox, against what the problem fixes:
brute force over every edge/node state on tiny chains, the optimality
certificate at any size, the closed forms of the decoupled and the
data-pinned cases, the c = 0 reduction to the Sec. 4.1 DP, and symmetries."""
import numpy as np
import pytest

import oracle
from tests import props


def _random(rng, n, kind):
    a = rng.uniform(0.2, 3.0, n)
    b = rng.normal(size=n) * 2
    c = rng.uniform(0.0, 1.5, n) * (rng.random(n) < 0.8)
    d = rng.normal(size=n)
    if kind == "ties":
        d = np.round(d * 2) / 2
    wp = rng.uniform(0.0, 1.0, n)
    wm = wp - rng.uniform(0.0, 1.0, n) if kind == "shifted" else -rng.uniform(0.0, 1.0, n)
    return a, b, c, d, wm, wp


@pytest.mark.parametrize("kind", ["sym", "shifted", "ties"])
def test_matches_brute_force(kind):
    rng = np.random.default_rng({"sym": 1, "shifted": 2, "ties": 3}[kind])
    for _ in range(400):
        n = int(rng.integers(1, 7))
        a, b, c, d, wm, wp = _random(rng, n, kind)
        x = oracle.chain_pq(a, b, c, d, wm, wp)[0]
        xb = oracle.chain_pq_brute(a, b, c, d, wm, wp)
        assert np.abs(x - xb).max() <= 1e-9, (a, b, c, d, wm, wp)


def test_brute_force_finds_the_minimum():
    """The brute force itself: no random perturbation of its answer does better."""
    rng = np.random.default_rng(4)
    for _ in range(50):
        n = int(rng.integers(2, 7))
        a, b, c, d, wm, wp = _random(rng, n, "sym")
        xb = oracle.chain_pq_brute(a, b, c, d, wm, wp)
        f0 = oracle.pq_objective(a, b, c, d, wm, wp, xb)
        for _ in range(50):
            xp = xb + rng.normal(size=n) * 10 ** rng.uniform(-6, 0)
            assert oracle.pq_objective(a, b, c, d, wm, wp, xp) >= f0 - 1e-12


@pytest.mark.parametrize("n", [50, 400, 3000])
def test_kkt_certificate_long_chains(n):
    rng = np.random.default_rng(n)
    for kind in ("sym", "shifted", "ties"):
        a, b, c, d, wm, wp = _random(rng, n, kind)
        x = oracle.chain_pq(a, b, c, d, wm, wp)[0]
        assert props.kkt_pq(a, b, c, d, wm, wp, x, tol=1e-9) <= 1e-8


def test_certificate_rejects_wrong_answers():
    """The certificate is not vacuous: perturbed solutions fail it."""
    rng = np.random.default_rng(5)
    a, b, c, d, wm, wp = _random(rng, 200, "sym")
    x = oracle.chain_pq(a, b, c, d, wm, wp)[0]
    bad = x.copy()
    bad[77] += 1e-3
    assert props.kkt_pq(a, b, c, d, wm, wp, bad, tol=1e-9) > 1e-5


def test_c_zero_is_the_quadratic_dp():
    rng = np.random.default_rng(6)
    for _ in range(100):
        n = int(rng.integers(1, 60))
        a, b, _, d, wm, wp = _random(rng, n, "shifted")
        x = oracle.chain_pq(a, b, np.zeros(n), d, wm, wp)[0]
        x2 = oracle.chain_dp(a, b, wm[: n - 1], wp[: n - 1])[0]
        assert np.abs(x - x2).max() <= 1e-12


def test_decoupled_nodes_soft_threshold():
    """w = 0: every node alone; the minimiser of a x^2/2 - b x + c|x - d| is
    (b - c)/a above d, (b + c)/a below d, else d."""
    rng = np.random.default_rng(7)
    n = 500
    a, b, c, d, _, _ = _random(rng, n, "sym")
    z = np.zeros(n)
    x = oracle.chain_pq(a, b, c, d, z, z)[0]
    ref = np.where((b - c) / a > d, (b - c) / a, np.where((b + c) / a < d, (b + c) / a, d))
    assert np.abs(x - ref).max() <= 1e-12


def test_large_data_weight_pins_to_d():
    """c_i >= |a_i d_i - b_i| + w_{i-1} + w_i: x = d exactly (0 is in every
    node's subdifferential at d)."""
    rng = np.random.default_rng(8)
    n = 300
    a, b, _, d, wm, wp = _random(rng, n, "sym")
    w_in = np.concatenate([[0.0], np.maximum(-wm[:-1], wp[:-1])])
    w_out = np.concatenate([np.maximum(-wm[:-1], wp[:-1]), [0.0]])
    c = np.abs(a * d - b) + w_in + w_out + 0.01
    x = oracle.chain_pq(a, b, c, d, wm, wp)[0]
    assert np.array_equal(x, d)


def test_shift_and_negation():
    rng = np.random.default_rng(9)
    n, t = 200, 0.37
    a, b, c, d, wm, wp = _random(rng, n, "shifted")
    x = oracle.chain_pq(a, b, c, d, wm, wp)[0]
    xs = oracle.chain_pq(a, b + a * t, c, d + t, wm, wp)[0]
    assert np.abs(xs - (x + t)).max() <= 1e-10
    xn = oracle.chain_pq(a, -b, c, -d, -wp, -wm)[0]
    assert np.abs(xn + x).max() <= 1e-10


def test_tv_l1_chain_prox_is_the_pq_dp():
    rng = np.random.default_rng(10)
    C, n = 12, 300
    y = rng.normal(size=(C, n))
    d = rng.normal(size=(C, n))
    w = rng.uniform(0, 1, (C, n))
    cc = rng.uniform(0, 2, (C, n))
    x = oracle.chain_prox_l1(y, d, w=w, c=cc)
    for r in range(C):
        ref = oracle.chain_pq(np.ones(n), y[r], cc[r], d[r], -w[r, :-1], w[r, :-1])[0]
        assert np.abs(x[r] - ref).max() <= 1e-13
    xs = oracle.chain_prox_l1(y, d, w_scalar=0.3, c_scalar=0.8)
    ref = oracle.chain_pq(np.ones(n), y[3], np.full(n, 0.8), d[3], np.full(n - 1, -0.3), np.full(n - 1, 0.3))[0]
    assert np.abs(xs[3] - ref).max() <= 1e-13
