"""Pins of the oracle's Algorithm 2 on forests (orc_tree_pq: children's
clipped messages summed by merging their breakpoint sets, Sec. 4.2's extension
to trees) against what the problem fixes: brute force over every edge/node
state on tiny forests, the tree KKT certificate at any size, the chain as the
special case parent[i] = i + 1, and independence of the numbering (any order
with children before parents gives the same minimiser)."""
import numpy as np
import pytest

import oracle
from tests import props


def random_forest(n, rng, roots=1):
    """parent[i] in (i, n) for non-roots; the last `roots` nodes are roots."""
    parent = np.full(n, -1, dtype=np.int64)
    for i in range(n - roots):
        parent[i] = rng.integers(i + 1, n)
    return parent


def _data(n, rng, kind="l1"):
    a = rng.uniform(0.2, 3.0, n)
    b = rng.normal(size=n) * 2
    c = rng.uniform(0, 1.5, n) * (rng.random(n) < 0.8) if kind == "l1" else np.zeros(n)
    d = np.round(rng.normal(size=n) * 2) / 2
    wp = rng.uniform(0, 1, n)
    wm = -rng.uniform(0, 1, n) if rng.random() < 0.5 else wp - rng.uniform(0, 1, n)
    return a, b, c, d, wm, wp


@pytest.mark.parametrize("kind", ["l1", "quadratic"])
def test_matches_brute_force(kind):
    rng = np.random.default_rng(11 if kind == "l1" else 12)
    for _ in range(300):
        n = int(rng.integers(1, 7))
        parent = random_forest(n, rng, roots=int(rng.integers(1, min(n, 3) + 1)))
        args = _data(n, rng, kind)
        x = oracle.tree_pq(parent, *args)[0]
        xb = oracle.tree_pq_brute(parent, *args)
        assert np.abs(x - xb).max() <= 1e-9, (parent, args)


@pytest.mark.parametrize("n", [100, 2000])
def test_kkt_certificate(n):
    rng = np.random.default_rng(n)
    for roots in (1, 5):
        parent = random_forest(n, rng, roots)
        args = _data(n, rng)
        x = oracle.tree_pq(parent, *args)[0]
        assert props.kkt_tree(parent, *args, x, tol=1e-9) <= 1e-8
        bad = x.copy()
        bad[n // 3] += 1e-3
        assert props.kkt_tree(parent, *args, bad, tol=1e-9) > 1e-5


def test_chain_is_the_special_case():
    rng = np.random.default_rng(13)
    n = 500
    parent = np.arange(1, n + 1, dtype=np.int64)
    parent[-1] = -1
    a, b, c, d, wm, wp = _data(n, rng)
    x = oracle.tree_pq(parent, a, b, c, d, wm, wp)[0]
    xc = oracle.chain_pq(a, b, c, d, wm[:-1], wp[:-1])[0]
    assert np.abs(x - xc).max() <= 1e-12


def test_numbering_does_not_matter():
    """Relabel a forest with another order that keeps children before parents."""
    rng = np.random.default_rng(14)
    n = 300
    parent = random_forest(n, rng, roots=3)
    args = _data(n, rng)
    x = oracle.tree_pq(parent, *args)[0]
    # a random topological order: repeatedly take a random node whose children are all taken
    kids = [[] for _ in range(n)]
    for i, p in enumerate(parent):
        if p >= 0:
            kids[p].append(i)
    pending = np.array([len(k) for k in kids])
    ready = [i for i in range(n) if pending[i] == 0]
    order = []
    while ready:
        j = ready.pop(int(rng.integers(len(ready))))
        order.append(j)
        if parent[j] >= 0:
            pending[parent[j]] -= 1
            if pending[parent[j]] == 0:
                ready.append(parent[j])
    new_of = np.empty(n, dtype=np.int64)
    new_of[order] = np.arange(n)
    p2 = np.array([-1 if parent[o] < 0 else new_of[parent[o]] for o in order], dtype=np.int64)
    x2 = oracle.tree_pq(p2, *(v[order] for v in args))[0]
    assert np.abs(x2 - x[order]).max() <= 1e-10


def test_rejects_bad_numbering():
    with pytest.raises(ValueError):
        oracle.tree_pq(np.array([0, -1]), *(np.ones(2),) * 6)
