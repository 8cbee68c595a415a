"""GPU parity for concave pairwise terms on trees (tv_tree_nc_concave) against
the FP64 oracle (ncg_tree), compared by energy per tree."""
import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth
from tests.test_oracle_nc import _rand_unaries
from tests.test_oracle_ncg import _rand_pieces

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _run(par, off, u, p, dtype, **kw):
    uoff, ulam, usl = u
    poff, al, cc, sd = p
    return binding.tree_nc_concave(_dev(par, torch.int64), _dev(off, torch.int64), _dev(uoff, torch.int64),
                                   _dev(ulam, dtype), _dev(usl, dtype), _dev(poff, torch.int64), _dev(al, dtype),
                                   _dev(cc, dtype), _dev(sd, torch.int32), **kw).double().cpu().numpy()


def _check(par, off, u, p, x, trees, tol_rel, tol_node=0.0):
    uoff, ulam, usl = u
    poff, al, cc, sd = p
    for t in trees:
        n0, n1 = int(off[t]), int(off[t + 1])
        q = par[n0:n1].copy()
        q[q >= 0] -= n0
        su = (uoff[n0:n1 + 1] - uoff[n0], ulam[uoff[n0]:uoff[n1]], usl[uoff[n0] + n0:uoff[n1] + n1])
        sp = (poff[n0:n1 + 1] - poff[n0], al[poff[n0]:poff[n1]], cc[poff[n0]:poff[n1]], sd[poff[n0]:poff[n1]])
        xo, _ = oracle.ncg_tree(q, *su, *sp)
        eo = oracle.ncg_tree_energy(q, *su, *sp, xo)
        eg = oracle.ncg_tree_energy(q, *su, *sp, x[n0:n1])
        assert abs(eg - eo) <= tol_rel * (1 + abs(eo)) + tol_node * (n1 - n0), (t, n1 - n0, eo, eg)


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("msg_cap", [512, 256, 128])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_random_forests_match_the_oracle(dtype, msg_cap):
    """150 trees (fewer than 1024): msg_cap 512 runs a lane per tree, 256 and
    128 a wave per tree."""
    g = np.random.default_rng(60)
    par, off = synth.post_order_forest(150, 60, seed=61)
    N = par.size
    u = _rand_unaries(g, N)
    p = _rand_pieces(g, N)
    if dtype == torch.float32:
        u = (u[0], _f32(u[1]), _f32(u[2]))
        p = (p[0], _f32(p[1]), _f32(p[2]), p[3])
    x = _run(par, off, u, p, dtype, msg_cap=msg_cap)
    if dtype == torch.float64:
        _check(par, off, u, p, x, range(off.size - 1), 1e-9)
    else:
        _check(par, off, u, p, x, range(off.size - 1), 1e-6, 8 * 2.0 ** -23 * (np.abs(u[1]).max() + 1) * 4)


def test_chain_as_a_tree_equals_the_chain_kernel():
    g = np.random.default_rng(62)
    n = 300
    u = _rand_unaries(g, n)
    p = _rand_pieces(g, n)
    par = np.arange(1, n + 1, dtype=np.int64)
    par[-1] = -1
    off = np.array([0, n], dtype=np.int64)
    xt = _run(par, off, u, p, torch.float64)
    uoff, ulam, usl = u
    poff, al, cc, sd = p
    xc = binding.chain_nc_concave(_dev(off, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64),
                                  _dev(usl, torch.float64), _dev(poff, torch.int64), _dev(al, torch.float64),
                                  _dev(cc, torch.float64), _dev(sd, torch.int32)).cpu().numpy()
    et = oracle.ncg_energy(*u, *p, xt)
    ec = oracle.ncg_energy(*u, *p, xc)
    assert abs(et - ec) <= 1e-9 * (1 + abs(ec))


def test_rejections():
    g = np.random.default_rng(63)
    par, off = synth.post_order_forest(8, 20, seed=64)
    N = par.size
    u = _rand_unaries(g, N)
    p = _rand_pieces(g, N, allow_empty=False)
    bad = par.copy()
    bad[0] = int(off[1]) + 3  # a parent in another tree
    with pytest.raises(binding.TvChainError) as e:
        _run(bad, off, u, p, torch.float64)
    assert e.value.status == binding.TV_ERR_INVALID_ARG
    sd = p[3].copy()
    sd[0] = 0
    with pytest.raises(binding.TvChainError) as e:
        _run(par, off, u, (p[0], p[1], p[2], sd), torch.float64)
    assert e.value.status == binding.TV_ERR_INVALID_ARG
    with pytest.raises(binding.TvChainError) as e:
        _run(par, off, u, p, torch.float64, msg_cap=2)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    with pytest.raises(binding.TvChainError) as e:
        _run(par, off, u, p, torch.float64, stack_cap=3)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    x = _run(par, off, u, p, torch.float64)  # and the same call with room
    _check(par, off, u, p, x, range(off.size - 1), 1e-9)


def test_full_batch_sampled_trees():
    """16,384 post-order trees of 256 nodes, 16-level uniform [0, 4] costs,
    min(|z|, 0.25 |z| + 1, 2.5) on every edge, FP32 in; 300 sampled trees."""
    T, n = 16384, 256
    par, off = synth.post_order_forest(T, n, seed=7)
    _, u, p = synth.concave_cost_chains(T, n, 16, seed=9)
    u = (u[0], u[1], _f32(u[2]))
    x = _run(par, off, u, p, torch.float32, msg_cap=1024, map_cap=8192, stack_cap=64 * 1025)
    pick = np.sort(np.random.default_rng(65).choice(T, 300, replace=False))
    _check(par, off, u, p, x, pick, 1e-6, 8 * 2.0 ** -23 * 20)
