"""Pins for the Sec. 3 non-convex chain oracle (piecewise-linear unaries,
truncated TV min(w|z|, C)), none of which reuse its message passing:

* the exact minimum of the energy on tiny chains from an independent Viterbi
  pass over vertex candidates (a coercive piecewise-linear energy attains its
  minimum where every x_i is a unary breakpoint plus offsets 0, +-C_e/w_e);
* that brute force is itself no larger than the energy of random points;
* closed forms: one node (an argmin breakpoint of its unary), w = 0 (nodes
  independent), C below the smallest unary spread (every node at its own
  argmin);
* invariances: a common shift of every breakpoint shifts x; reversing the chain
  keeps the minimum energy; C above any reachable w|z| equals plain TV.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def _rand_unaries(g, n, tmax=3, convex=False, scale=1.0):
    ts = g.integers(1, tmax + 1, n)
    uoff = np.concatenate([[0], np.cumsum(ts)]).astype(np.int64)
    ulam = np.concatenate([np.sort(np.round(g.normal(size=t) * 2 * scale, 1)) for t in ts])
    sl = []
    for t in ts:
        s = np.sort(g.normal(size=t + 1) * 2)
        if not convex:
            inner = s[1:-1].copy()
            g.shuffle(inner)
            s[1:-1] = inner
        s[0] = -abs(s[0]) - 0.1
        s[-1] = abs(s[-1]) + 0.1
        sl.append(s)
    return uoff, ulam, np.concatenate(sl)


def _unary_argmin(uoff, ulam, uslope, i):
    t = uoff[i + 1] - uoff[i]
    l = ulam[uoff[i]:uoff[i + 1]]
    s = uslope[uoff[i] + i:uoff[i + 1] + i + 1]
    v = np.concatenate([[0.0], np.cumsum(s[1:t] * np.diff(l))])
    return l[np.argmin(v)], v.min()


@pytest.mark.parametrize("truncated", [False, True])
def test_tiny_chains_reach_the_exact_minimum(truncated):
    g = np.random.default_rng(11 if truncated else 12)
    for _ in range(800):
        n = int(g.integers(1, 6))
        uoff, ulam, usl = _rand_unaries(g, n)
        w = g.uniform(0, 2, n - 1)
        C = g.uniform(0.1, 3, n - 1) if truncated else np.full(n - 1, np.inf)
        if truncated:
            C[g.random(n - 1) < 0.3] = np.inf
        x, _ = oracle.nc_chain(uoff, ulam, usl, w, C)
        e = oracle.nc_energy(uoff, ulam, usl, w, C, x)
        eb, xb = oracle.nc_brute(uoff, ulam, usl, w, C)
        assert abs(e - eb) <= 1e-9 * (1 + abs(eb)), (n, e, eb)
        assert abs(oracle.nc_energy(uoff, ulam, usl, w, C, xb) - eb) <= 1e-9 * (1 + abs(eb))


def test_brute_force_is_below_random_points():
    g = np.random.default_rng(13)
    for _ in range(200):
        n = int(g.integers(2, 6))
        uoff, ulam, usl = _rand_unaries(g, n)
        w = g.uniform(0, 2, n - 1)
        C = g.uniform(0.1, 3, n - 1)
        eb, _ = oracle.nc_brute(uoff, ulam, usl, w, C)
        for _ in range(50):
            xr = g.normal(size=n) * 3
            assert eb <= oracle.nc_energy(uoff, ulam, usl, w, C, xr) + 1e-12


def test_single_node_and_zero_weights():
    g = np.random.default_rng(14)
    for _ in range(100):
        n = int(g.integers(1, 30))
        uoff, ulam, usl = _rand_unaries(g, n, tmax=5)
        w = np.zeros(n - 1)
        C = np.where(g.random(n - 1) < 0.5, np.inf, 1.0)
        x, _ = oracle.nc_chain(uoff, ulam, usl, w, C)
        for i in range(n):
            xa, va = _unary_argmin(uoff, ulam, usl, i)
            # x_i is a minimiser of f_i (ties: any minimiser)
            t = uoff[i + 1] - uoff[i]
            one = oracle.nc_energy(uoff[i:i + 2] - uoff[i], ulam[uoff[i]:uoff[i + 1]],
                                   usl[uoff[i] + i:uoff[i + 1] + i + 1], [], [], [x[i]])
            assert abs(one - va) <= 1e-12 * (1 + abs(va)), (i, t)


def test_small_truncation_frees_every_node():
    """Every edge truncated at a tiny C: the minimum lies between the sum of the
    unary minima and that sum plus sum(C); the oracle's energy is in that range
    and equals the brute-force minimum."""
    g = np.random.default_rng(15)
    for _ in range(200):
        n = int(g.integers(2, 6))
        uoff, ulam, usl = _rand_unaries(g, n)
        w = g.uniform(0.5, 2, n - 1)
        C = np.full(n - 1, 1e-3)
        x, _ = oracle.nc_chain(uoff, ulam, usl, w, C)
        e = oracle.nc_energy(uoff, ulam, usl, w, C, x)
        lo = sum(_unary_argmin(uoff, ulam, usl, i)[1] for i in range(n))
        assert lo - 1e-12 <= e <= lo + C.sum() + 1e-12
        eb, _ = oracle.nc_brute(uoff, ulam, usl, w, C)
        assert abs(e - eb) <= 1e-9 * (1 + abs(eb))


def test_shift_reversal_and_large_truncation():
    g = np.random.default_rng(16)
    for _ in range(150):
        n = int(g.integers(2, 60))
        uoff, ulam, usl = _rand_unaries(g, n, tmax=4)
        w = g.uniform(0, 2, n - 1)
        C = g.uniform(0.2, 3, n - 1)
        x, _ = oracle.nc_chain(uoff, ulam, usl, w, C)
        e = oracle.nc_energy(uoff, ulam, usl, w, C, x)
        # shift
        xs, _ = oracle.nc_chain(uoff, ulam + 1.25, usl, w, C)
        assert abs(oracle.nc_energy(uoff, ulam + 1.25, usl, w, C, xs) - e) <= 1e-9 * (1 + abs(e))
        # reversal: node i -> n-1-i (breakpoints and slopes of each node unchanged)
        ts = np.diff(uoff)[::-1]
        roff = np.concatenate([[0], np.cumsum(ts)]).astype(np.int64)
        rl = np.concatenate([ulam[uoff[i]:uoff[i + 1]] for i in range(n - 1, -1, -1)])
        rs = np.concatenate([usl[uoff[i] + i:uoff[i + 1] + i + 1] for i in range(n - 1, -1, -1)])
        xr, _ = oracle.nc_chain(roff, rl, rs, w[::-1], C[::-1])
        er = oracle.nc_energy(roff, rl, rs, w[::-1], C[::-1], xr)
        assert abs(er - e) <= 1e-9 * (1 + abs(e))
        # C larger than any w|z| among breakpoint-spread points: plain TV
        span = ulam.max() - ulam.min() + 1.0
        xi, _ = oracle.nc_chain(uoff, ulam, usl, w, np.full(n - 1, np.inf))
        xb, _ = oracle.nc_chain(uoff, ulam, usl, w, w * span * 4 + 1.0)
        ei = oracle.nc_energy(uoff, ulam, usl, w, np.full(n - 1, np.inf), xi)
        eb = oracle.nc_energy(uoff, ulam, usl, w, np.full(n - 1, np.inf), xb)
        assert abs(ei - eb) <= 1e-9 * (1 + abs(ei))


def test_local_perturbations_do_not_improve_long_chains():
    g = np.random.default_rng(17)
    for _ in range(40):
        n = int(g.integers(50, 300))
        uoff, ulam, usl = _rand_unaries(g, n, tmax=6)
        w = g.uniform(0, 2, n - 1)
        C = np.where(g.random(n - 1) < 0.5, np.inf, g.uniform(0.2, 3, n - 1))
        x, mb = oracle.nc_chain(uoff, ulam, usl, w, C)
        e = oracle.nc_energy(uoff, ulam, usl, w, C, x)
        for _ in range(200):
            xp = x.copy()
            k = int(g.integers(0, n))
            m = int(g.integers(1, 6))
            xp[k:k + m] += g.normal() * 0.5
            assert e <= oracle.nc_energy(uoff, ulam, usl, w, C, xp) + 1e-9


def test_rejects_invalid_unaries():
    with pytest.raises(ValueError):
        oracle.nc_chain([0, 1], [0.0], [0.5, 1.0], [], [])       # s_0 > 0: unbounded
    with pytest.raises(ValueError):
        oracle.nc_chain([0, 2], [1.0, 0.0], [-1, 0, 1], [], [])  # unsorted breakpoints
    with pytest.raises(ValueError):
        oracle.nc_chain([0, 0], [], [0.0], [], [])               # no breakpoint


def test_lemma2_no_growth_without_truncation():
    """Lemma 2: with C = inf a min-convolution adds no breakpoints, so no message
    holds more than the unaries' breakpoints summed (hat M_i has at most
    sum_{j <= i} t_j).  An Algorithm 1 that emitted extra points would exceed it."""
    g = np.random.default_rng(18)
    for _ in range(200):
        n = int(g.integers(2, 80))
        uoff, ulam, usl = _rand_unaries(g, n, tmax=4)
        w = g.uniform(0, 2, n - 1)
        _, mb = oracle.nc_chain(uoff, ulam, usl, w, np.full(n - 1, np.inf))
        assert mb <= uoff[-1], (mb, uoff[-1])


def _rand_forest(g, n):
    """A random numbering with children before parents: node i's parent is a
    random later node, or none (a root) with probability 0.15."""
    par = np.full(n, -1, dtype=np.int64)
    for i in range(n - 1):
        if g.random() > 0.15:
            par[i] = int(g.integers(i + 1, n))
    return par


@pytest.mark.parametrize("truncated", [False, True])
def test_tree_reaches_the_exact_minimum(truncated):
    g = np.random.default_rng(21 if truncated else 22)
    for _ in range(600):
        n = int(g.integers(1, 6))
        par = _rand_forest(g, n)
        uoff, ulam, usl = _rand_unaries(g, n)
        w = g.uniform(0, 2, n)
        C = g.uniform(0.1, 3, n) if truncated else np.full(n, np.inf)
        x, _ = oracle.nc_tree(par, uoff, ulam, usl, w, C)
        e = oracle.nc_tree_energy(par, uoff, ulam, usl, w, C, x)
        eb = oracle.nc_tree_brute(par, uoff, ulam, usl, w, C)
        assert abs(e - eb) <= 1e-9 * (1 + abs(eb)), (n, par, e, eb)


def test_tree_chain_case_and_relabelling():
    g = np.random.default_rng(23)
    for _ in range(60):
        n = int(g.integers(2, 60))
        uoff, ulam, usl = _rand_unaries(g, n, tmax=4)
        w = g.uniform(0, 2, n)
        C = np.where(g.random(n) < 0.5, np.inf, g.uniform(0.2, 3, n))
        # a chain as a tree (parent = i + 1): the chain solver's energy
        par = np.arange(1, n + 1, dtype=np.int64)
        par[-1] = -1
        xt, _ = oracle.nc_tree(par, uoff, ulam, usl, w, C)
        xc, _ = oracle.nc_chain(uoff, ulam, usl, w[:-1], C[:-1])
        et = oracle.nc_tree_energy(par, uoff, ulam, usl, w, C, xt)
        assert abs(et - oracle.nc_energy(uoff, ulam, usl, w[:-1], C[:-1], xc)) <= 1e-9 * (1 + abs(et))
        # a random forest renumbered by another children-before-parents order
        par = _rand_forest(g, n)
        x1, _ = oracle.nc_tree(par, uoff, ulam, usl, w, C)
        e1 = oracle.nc_tree_energy(par, uoff, ulam, usl, w, C, x1)
        # new order: a topological order with random tie-breaks (children first)
        remaining = {i: 0 for i in range(n)}
        for i in range(n):
            if par[i] >= 0:
                remaining[int(par[i])] += 1
        ready = [i for i in range(n) if remaining[i] == 0]
        order = []
        while ready:
            k = ready.pop(int(g.integers(0, len(ready))))
            order.append(k)
            if par[k] >= 0:
                remaining[int(par[k])] -= 1
                if remaining[int(par[k])] == 0:
                    ready.append(int(par[k]))
        pos = np.empty(n, dtype=np.int64)
        pos[order] = np.arange(n)
        par2 = np.array([pos[par[k]] if par[k] >= 0 else -1 for k in order], dtype=np.int64)
        ts = np.diff(uoff)[order]
        uoff2 = np.concatenate([[0], np.cumsum(ts)]).astype(np.int64)
        ul2 = np.concatenate([ulam[uoff[k]:uoff[k + 1]] for k in order])
        us2 = np.concatenate([usl[uoff[k] + k:uoff[k + 1] + k + 1] for k in order])
        x2, _ = oracle.nc_tree(par2, uoff2, ul2, us2, w[order], C[order])
        e2 = oracle.nc_tree_energy(par2, uoff2, ul2, us2, w[order], C[order], x2)
        assert abs(e1 - e2) <= 1e-9 * (1 + abs(e1))
