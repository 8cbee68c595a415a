"""GPU parity for the Sec. 3 non-convex trees (tv_tree_nc) against the FP64
oracle (nc_tree), compared by energy per tree (minimisers need not be unique)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth

pytestmark = pytest.mark.gpu


def _unaries(g, n, tmax=4):
    ts = g.integers(1, tmax + 1, n)
    uoff = np.concatenate([[0], np.cumsum(ts)]).astype(np.int64)
    ulam = np.concatenate([np.cumsum(np.concatenate([[g.normal() * 2], g.uniform(0, 2, t - 1)])) for t in ts])
    sl = []
    for t in ts:
        s = g.normal(size=t + 1) * 2
        s[0] = -abs(s[0]) - 0.05
        s[-1] = abs(s[-1]) + 0.05
        sl.append(s)
    return uoff, ulam, np.concatenate(sl)


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _check_trees(par, off, uoff, ulam, usl, w, C, x, tol_rel, tol_node=0.0):
    for t in range(off.size - 1):
        n0, n1 = int(off[t]), int(off[t + 1])
        p = par[n0:n1].copy()
        p[p >= 0] -= n0
        uo = uoff[n0:n1 + 1] - uoff[n0]
        l = ulam[uoff[n0]:uoff[n1]]
        s = usl[uoff[n0] + n0:uoff[n1] + n1]
        xo, _ = oracle.nc_tree(p, uo, l, s, w[n0:n1], C[n0:n1])
        eo = oracle.nc_tree_energy(p, uo, l, s, w[n0:n1], C[n0:n1], xo)
        eg = oracle.nc_tree_energy(p, uo, l, s, w[n0:n1], C[n0:n1], x[n0:n1])
        tol = tol_rel * (1 + abs(eo)) + tol_node * (n1 - n0)
        assert abs(eg - eo) <= tol, (t, n1 - n0, eo, eg)


@pytest.mark.parametrize("msg_cap", [512, 256, 128])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_random_forests_match_the_oracle(dtype, msg_cap):
    """150 trees (fewer than 1024): msg_cap 512 runs a lane per tree, 256 and
    128 a wave per tree."""
    g = np.random.default_rng(40)
    par, off = synth.post_order_forest(150, 60, seed=41)
    N = par.size
    uoff, ulam, usl = _unaries(g, N)
    w = g.uniform(0, 2, N)
    C = np.where(g.random(N) < 0.5, g.uniform(0.2, 3, N), np.inf)
    if dtype == torch.float32:
        ulam, usl, w = (a.astype(np.float32).astype(np.float64) for a in (ulam, usl, w))
        C = C.astype(np.float32).astype(np.float64)
    x = binding.tree_nc(_dev(par, torch.int64), _dev(off, torch.int64), _dev(uoff, torch.int64), _dev(ulam, dtype),
                        _dev(usl, dtype), _dev(w, dtype), _dev(C, dtype), msg_cap=msg_cap).double().cpu().numpy()
    if dtype == torch.float64:
        _check_trees(par, off, uoff, ulam, usl, w, C, x, 1e-9)
    else:
        _check_trees(par, off, uoff, ulam, usl, w, C, x, 1e-6, 8 * 2.0 ** -23 * (np.abs(ulam).max() + 1) * 4)


def test_chain_as_a_tree_equals_the_chain_solver():
    g = np.random.default_rng(42)
    n = 300
    uoff, ulam, usl = _unaries(g, n)
    w = g.uniform(0, 2, n)
    C = np.where(g.random(n) < 0.5, g.uniform(0.2, 3, n), np.inf)
    par = np.arange(1, n + 1, dtype=np.int64)
    par[-1] = -1
    off = np.array([0, n], dtype=np.int64)
    xt = binding.tree_nc(_dev(par, torch.int64), _dev(off, torch.int64), _dev(uoff, torch.int64),
                         _dev(ulam, torch.float64), _dev(usl, torch.float64), _dev(w, torch.float64),
                         _dev(C, torch.float64)).cpu().numpy()
    xc = binding.chain_nc(_dev(off, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64),
                          _dev(usl, torch.float64), _dev(w, torch.float64), _dev(C, torch.float64)).cpu().numpy()
    et = oracle.nc_energy(uoff, ulam, usl, w[:-1], C[:-1], xt)
    ec = oracle.nc_energy(uoff, ulam, usl, w[:-1], C[:-1], xc)
    assert abs(et - ec) <= 1e-9 * (1 + abs(ec))


def test_rejections():
    g = np.random.default_rng(43)
    par, off = synth.post_order_forest(8, 20, seed=44)
    N = par.size
    uoff, ulam, usl = _unaries(g, N)
    w = g.uniform(0, 2, N)
    C = np.full(N, 1.5)
    args = lambda p: (_dev(p, torch.int64), _dev(off, torch.int64), _dev(uoff, torch.int64),  # noqa: E731
                      _dev(ulam, torch.float64), _dev(usl, torch.float64), _dev(w, torch.float64),
                      _dev(C, torch.float64))
    bad = par.copy()
    bad[0] = int(off[1]) + 3  # a parent in another tree
    with pytest.raises(binding.TvChainError) as e:
        binding.tree_nc(*args(bad))
    assert e.value.status == binding.TV_ERR_INVALID_ARG
    with pytest.raises(binding.TvChainError) as e:
        binding.tree_nc(*args(par), msg_cap=2)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    with pytest.raises(binding.TvChainError) as e:
        binding.tree_nc(*args(par), stack_cap=3)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    x = binding.tree_nc(*args(par)).cpu().numpy()  # and the same call with room
    _check_trees(par, off, uoff, ulam, usl, w, C, x, 1e-9)


def test_full_batch_sampled_trees():
    """16,384 post-order trees of 256 nodes with 16-level uniform [0, 4] costs
    (slopes -/+10 outside), w = 0.5, C = 2, FP32 in, solved in one launch with
    the capacities the benchmark uses; 300 sampled trees checked."""
    T, n, D = 16384, 256, 16
    par, off = synth.post_order_forest(T, n, seed=7)
    N = par.size
    g = synth.generator(8)
    cost = g.uniform(0, 4, (N, D))
    sl = np.empty((N, D + 1))
    sl[:, 0], sl[:, D] = -10.0, 10.0
    sl[:, 1:D] = np.diff(cost, axis=1)
    uoff = np.arange(N + 1, dtype=np.int64) * D
    ulam = np.tile(np.arange(D, dtype=np.float64), N)
    usl = sl.astype(np.float32).astype(np.float64).reshape(-1)
    w, C = np.full(N, 0.5), np.full(N, 2.0)
    x = binding.tree_nc(_dev(par, torch.int64), _dev(off, torch.int64), _dev(uoff, torch.int64),
                        _dev(ulam, torch.float32), _dev(usl, torch.float32), _dev(w, torch.float32),
                        _dev(C, torch.float32), msg_cap=512, map_cap=32 * n,
                        stack_cap=48 * 1025).double().cpu().numpy()
    pick = np.sort(np.random.default_rng(45).choice(T, 300, replace=False))
    sub_off = [0]
    rows = []
    for t in pick:
        rows.append(np.arange(off[t], off[t + 1]))
        sub_off.append(sub_off[-1] + off[t + 1] - off[t])
    idx = np.concatenate(rows)
    sub_par = np.concatenate([np.where(par[r] >= 0, par[r] - r[0] + s, -1) for r, s in zip(rows, sub_off)])
    sub_uoff = np.arange(idx.size + 1, dtype=np.int64) * D
    sub_usl = usl.reshape(N, D + 1)[idx].reshape(-1)
    _check_trees(sub_par, np.array(sub_off, dtype=np.int64), sub_uoff, np.tile(np.arange(D, dtype=np.float64),
                 idx.size), sub_usl, w[idx], C[idx], x[idx], 1e-6, 8 * 2.0 ** -23 * 20)


def test_small_batch_wave_per_tree():
    """512 trees of 256 nodes (fewer than 1024: a wave per tree at msg_cap
    256), 8-level uniform [0, 4] costs, w = 0.5, C = 2, FP32 in; all trees."""
    T, n, D = 512, 256, 8
    par, off = synth.post_order_forest(T, n, seed=7)
    N = par.size
    g = synth.generator(8)
    cost = g.uniform(0, 4, (N, D))
    sl = np.empty((N, D + 1))
    sl[:, 0], sl[:, D] = -10.0, 10.0
    sl[:, 1:D] = np.diff(cost, axis=1)
    uoff = np.arange(N + 1, dtype=np.int64) * D
    ulam = np.tile(np.arange(D, dtype=np.float64), N)
    usl = sl.astype(np.float32).astype(np.float64).reshape(-1)
    w, C = np.full(N, 0.5), np.full(N, 2.0)
    x = binding.tree_nc(_dev(par, torch.int64), _dev(off, torch.int64), _dev(uoff, torch.int64),
                        _dev(ulam, torch.float32), _dev(usl, torch.float32), _dev(w, torch.float32),
                        _dev(C, torch.float32), msg_cap=256, map_cap=32 * n).double().cpu().numpy()
    _check_trees(par, off, uoff, ulam, usl, w, C, x, 1e-6, 8 * 2.0 ** -23 * 20)
