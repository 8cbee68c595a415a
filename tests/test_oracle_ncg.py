"""Pins for the oracle of Sec. 3, Extensions (i): chains whose pairwise terms
are minima of one-sided linear pieces alpha |z| + C (concave on each side),
applied one piece at a time by Prop. 2."""
import numpy as np
import pytest

import oracle
from tests.test_oracle_nc import _rand_unaries


def _rand_pieces(g, n, kmax=3, allow_empty=True):
    poff, al, cc, sd = [0], [], [], []
    for e in range(n):
        ks = []
        for s in (1, -1):
            k = int(g.integers(0 if allow_empty and g.random() < 0.1 else 1, kmax + 1))
            ks += [s] * k
        g.shuffle(ks)
        for s in ks:
            a = 0.0 if g.random() < 0.25 else g.uniform(0, 2)
            c = 0.0 if g.random() < 0.25 else g.uniform(0, 3)
            al.append(a)
            cc.append(c)
            sd.append(s)
        poff.append(len(al))
    return (np.array(poff, dtype=np.int64), np.array(al), np.array(cc), np.array(sd, dtype=np.int32))


def _energy(u, p, x):
    return oracle.ncg_energy(*u, *p, x)


def test_reaches_the_exact_minimum():
    g = np.random.default_rng(31)
    for _ in range(1500):
        n = int(g.integers(1, 7))
        u = _rand_unaries(g, n)
        p = _rand_pieces(g, n)
        x, _ = oracle.ncg_chain(*u, *p)
        e = _energy(u, p, x)
        eb, _ = oracle.ncg_brute(*u, *p)
        assert np.isfinite(eb)
        assert abs(e - eb) <= 1e-9 * (1 + abs(eb)), (n, e, eb)


def test_brute_force_is_below_random_points():
    g = np.random.default_rng(32)
    for _ in range(200):
        n = int(g.integers(1, 6))
        u = _rand_unaries(g, n)
        p = _rand_pieces(g, n, allow_empty=False)
        eb, xb = oracle.ncg_brute(*u, *p)
        assert abs(_energy(u, p, xb) - eb) <= 1e-12 * (1 + abs(eb))
        for _ in range(50):
            z = g.normal(size=n) * 3
            assert _energy(u, p, z) >= eb - 1e-9


def _tv_pieces(w, C):
    poff, al, cc, sd = [0], [], [], []
    for e in range(w.size):
        for s in (1, -1):
            al.append(w[e]), cc.append(0.0), sd.append(s)
            if np.isfinite(C[e]):
                al.append(0.0), cc.append(C[e]), sd.append(s)
        poff.append(len(al))
    poff.append(len(al))
    return (np.array(poff, dtype=np.int64), np.array(al), np.array(cc), np.array(sd, dtype=np.int32))


def test_truncated_tv_as_pieces_is_the_truncated_tv_solver():
    g = np.random.default_rng(33)
    for _ in range(80):
        n = int(g.integers(2, 80))
        u = _rand_unaries(g, n, tmax=4)
        w = g.uniform(0, 2, n - 1)
        C = np.where(g.random(n - 1) < 0.3, np.inf, g.uniform(0.2, 3, n - 1))
        p = _tv_pieces(w, C)
        x, _ = oracle.ncg_chain(*u, *p)
        xr, _ = oracle.nc_chain(*u, w, C)
        er = oracle.nc_energy(*u, w, C, xr)
        assert abs(oracle.nc_energy(*u, w, C, x) - er) <= 1e-9 * (1 + abs(er))
        assert abs(_energy(u, p, x) - er) <= 1e-9 * (1 + abs(er))


def test_piece_order_does_not_matter():
    g = np.random.default_rng(34)
    for _ in range(80):
        n = int(g.integers(2, 60))
        u = _rand_unaries(g, n)
        p = _rand_pieces(g, n)
        poff, al, cc, sd = p
        perm = np.concatenate([poff[e] + g.permutation(poff[e + 1] - poff[e]) for e in range(n)]).astype(np.int64)
        q = (poff, al[perm], cc[perm], sd[perm])
        e1 = _energy(u, p, oracle.ncg_chain(*u, *p)[0])
        e2 = _energy(u, q, oracle.ncg_chain(*u, *q)[0])
        assert abs(e1 - e2) <= 1e-9 * (1 + abs(e1))


def test_dominated_pieces_change_nothing():
    g = np.random.default_rng(35)
    for _ in range(60):
        n = int(g.integers(2, 60))
        u = _rand_unaries(g, n)
        poff, al, cc, sd = _rand_pieces(g, n, allow_empty=False)
        e1 = _energy(u, (poff, al, cc, sd), oracle.ncg_chain(*u, poff, al, cc, sd)[0])
        # append to every edge a copy of one of its pieces with larger alpha and C
        al2, cc2, sd2, poff2 = [], [], [], [0]
        for e in range(n):
            k = slice(poff[e], poff[e + 1])
            al2 += list(al[k])
            cc2 += list(cc[k])
            sd2 += list(sd[k])
            if poff[e + 1] > poff[e]:
                j = int(g.integers(poff[e], poff[e + 1]))
                al2.append(al[j] + g.uniform(0, 1))
                cc2.append(cc[j] + g.uniform(0, 1))
                sd2.append(sd[j])
            poff2.append(len(al2))
        q = (np.array(poff2, dtype=np.int64), np.array(al2), np.array(cc2), np.array(sd2, dtype=np.int32))
        x2, _ = oracle.ncg_chain(*u, *q)
        assert abs(_energy(u, q, x2) - e1) <= 1e-9 * (1 + abs(e1))


def test_zero_pieces_leave_each_node_at_its_minimum():
    g = np.random.default_rng(36)
    for _ in range(40):
        n = int(g.integers(1, 50))
        u = _rand_unaries(g, n)
        poff = np.arange(n + 1, dtype=np.int64) * 2
        p = (poff, np.zeros(2 * n), np.zeros(2 * n), np.tile(np.array([1, -1], dtype=np.int32), n))
        x, _ = oracle.ncg_chain(*u, *p)
        uoff, ulam, usl = u
        # each unary's minimum over its breakpoints (the energy's constant: f_i(first breakpoint) = 0)
        best = 0.0
        for i in range(n):
            ui = (np.array([0, uoff[i + 1] - uoff[i]]), ulam[uoff[i]:uoff[i + 1]], usl[uoff[i] + i:uoff[i + 1] + i + 1])
            best += min(oracle.nc_energy(*ui, [], [], [z]) for z in ulam[uoff[i]:uoff[i + 1]])
        assert abs(_energy(u, p, x) - best) <= 1e-9 * (1 + abs(best))


def test_large_potts_cost_gives_the_best_constant():
    g = np.random.default_rng(37)
    for _ in range(40):
        n = int(g.integers(2, 40))
        u = _rand_unaries(g, n)
        poff = np.arange(n + 1, dtype=np.int64) * 2
        p = (poff, np.zeros(2 * n), np.full(2 * n, 1e6), np.tile(np.array([1, -1], dtype=np.int32), n))
        x, _ = oracle.ncg_chain(*u, *p)
        assert np.all(x == x[0])
        best = min(_energy(u, p, np.full(n, z)) for z in u[1])
        assert abs(_energy(u, p, x) - best) <= 1e-9 * (1 + abs(best))


def test_one_sided_pieces_give_an_ordered_minimiser():
    g = np.random.default_rng(38)
    for _ in range(40):
        n = int(g.integers(2, 50))
        u = _rand_unaries(g, n)
        poff = np.arange(n + 1, dtype=np.int64)
        p = (poff, g.uniform(0, 1, n), g.uniform(0, 1, n), np.ones(n, dtype=np.int32))
        x, _ = oracle.ncg_chain(*u, *p)
        assert np.all(np.diff(x) >= 0)
        assert np.isfinite(_energy(u, p, x))


def test_invalid_pieces_are_rejected():
    g = np.random.default_rng(39)
    u = _rand_unaries(g, 3)
    poff = np.array([0, 1, 2, 2], dtype=np.int64)
    for al, cc, sd in (([-1.0, 0.0], [0.0, 0.0], [1, 1]), ([0.0, 0.0], [-0.5, 0.0], [1, 1]),
                       ([0.0, 0.0], [0.0, 0.0], [1, 0]), ([np.inf, 0.0], [0.0, 0.0], [1, 1])):
        with pytest.raises(ValueError):
            oracle.ncg_chain(*u, poff, np.array(al), np.array(cc), np.array(sd, dtype=np.int32))


def _rand_forest(g, n):
    par = np.full(n, -1, dtype=np.int64)
    for i in range(n - 1):
        if g.random() > 0.15:
            par[i] = int(g.integers(i + 1, n))
    return par


def test_tree_reaches_the_exact_minimum():
    g = np.random.default_rng(41)
    for _ in range(1200):
        n = int(g.integers(1, 7))
        par = _rand_forest(g, n)
        u = _rand_unaries(g, n)
        p = _rand_pieces(g, n)
        x, _ = oracle.ncg_tree(par, *u, *p)
        e = oracle.ncg_tree_energy(par, *u, *p, x)
        eb = oracle.ncg_tree_brute(par, *u, *p)
        assert abs(e - eb) <= 1e-9 * (1 + abs(eb)), (n, par, e, eb)


def test_tree_chain_case_and_truncated_tv():
    g = np.random.default_rng(42)
    for _ in range(60):
        n = int(g.integers(2, 60))
        u = _rand_unaries(g, n, tmax=4)
        # a chain numbered as a tree: the chain solver's energy
        par = np.arange(1, n + 1, dtype=np.int64)
        par[-1] = -1
        p = _rand_pieces(g, n)
        xt, _ = oracle.ncg_tree(par, *u, *p)
        xc, _ = oracle.ncg_chain(*u, *p)
        ec = _energy(u, p, xc)
        assert abs(oracle.ncg_tree_energy(par, *u, *p, xt) - ec) <= 1e-9 * (1 + abs(ec))
        # truncated TV as pieces on a random forest: the truncated-TV tree solver's energy
        par = _rand_forest(g, n)
        w = g.uniform(0, 2, n)
        C = np.where(g.random(n) < 0.3, np.inf, g.uniform(0.2, 3, n))
        q = _tv_pieces(w, C)
        q = (q[0][:n + 1] if q[0].size > n + 1 else q[0], q[1], q[2], q[3])
        xg, _ = oracle.ncg_tree(par, *u, *q)
        xr, _ = oracle.nc_tree(par, *u, w, C)
        er = oracle.nc_tree_energy(par, *u, w, C, xr)
        assert abs(oracle.nc_tree_energy(par, *u, w, C, xg) - er) <= 1e-9 * (1 + abs(er))
