"""GPU parity of Algorithm 2 on batches of trees (tv_tree_dp) against the
oracle's forest DP (pinned in tests/test_oracle_tree.py to brute force, a KKT
certificate, the chain case and relabelling).  The GPU computes in FP64 for
either dtype; bars per tree relative to s = max(range of x, range of b / a, 1):
1e-11 with FP64 inputs, 1e-5 with FP32 inputs (the oracle sees the same
rounded inputs)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth

pytestmark = pytest.mark.gpu


def _tree_data(N, seed, l1=True, unit_a=False):
    rng = np.random.default_rng(seed)
    a = np.ones(N) if unit_a else rng.uniform(0.3, 2.0, N)
    b = a * (rng.normal(size=N) * 0.5 + np.repeat(rng.uniform(0, 1, N // 16 + 1), 16)[:N])
    c = rng.uniform(0, 1.0, N) * (rng.random(N) < 0.7) if l1 else np.zeros(N)
    d = np.round(rng.normal(size=N) * 2) / 2
    wp = rng.uniform(0, 0.8, N)
    wm = -rng.uniform(0, 0.8, N)
    return a, b, c, d, wm, wp


def _check(par, off, arrays, xg, trees, tol):
    a, b, c, d, wm, wp = arrays
    for t in trees:
        lo, hi = off[t], off[t + 1]
        p = par[lo:hi].copy()
        p[p >= 0] -= lo
        xo = oracle.tree_pq(p, *(v[lo:hi] for v in (a, b, c, d, wm, wp)))[0]
        s = max(np.ptp(xo), np.ptp(b[lo:hi] / a[lo:hi]), 1.0)
        assert np.abs(xg[lo:hi] - xo).max() <= tol * s, t


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("l1", [True, False])
def test_random_forests_match_oracle(dtype, tol, l1):
    par, off = synth.post_order_forest(300, 150, seed=5)
    arrays = _tree_data(par.size, seed=6, l1=l1)
    dev = [torch.tensor(v, dtype=dtype, device="cuda") for v in arrays]
    arrays = [v.double().cpu().numpy() for v in dev]
    x = binding.tree_dp(torch.tensor(par, device="cuda"), torch.tensor(off, device="cuda"), dev[1], dev[4], dev[5],
                        a=dev[0], c=dev[2] if l1 else None, d=dev[3] if l1 else None)
    _check(par, off, arrays, x.double().cpu().numpy(), range(300), tol)


def test_chain_is_the_chain_dp():
    """parent(i) = i + 1: the general chain DP's result."""
    rng = np.random.default_rng(7)
    C, n = 40, 600
    a, b, _, _, wm, wp = _tree_data(C * n, seed=8, l1=False)
    par = np.arange(1, C * n + 1, dtype=np.int64)
    par[n - 1::n] = -1
    off = np.arange(C + 1, dtype=np.int64) * n
    dev = [torch.tensor(v, device="cuda") for v in (a, b, wm, wp)]
    x = binding.tree_dp(torch.tensor(par, device="cuda"), torch.tensor(off, device="cuda"), dev[1], dev[2], dev[3],
                        a=dev[0]).cpu().numpy().reshape(C, n)
    ref = binding.chain_dp(*(v.reshape(C, n) for v in dev[1:]), a=dev[0].reshape(C, n)).cpu().numpy()
    assert np.abs(x - ref).max() <= 1e-10


def test_single_nodes_and_forest_ranges():
    """Trees of one node (x = argmin of the unary) and ranges holding several
    trees (several roots)."""
    par = np.array([-1, 2, -1, 4, 5, -1, -1], dtype=np.int64)   # ranges [0,1) [1,3) [3,7)
    off = np.array([0, 1, 3, 7], dtype=np.int64)
    arrays = _tree_data(7, seed=9)
    dev = [torch.tensor(v, device="cuda") for v in arrays]
    x = binding.tree_dp(torch.tensor(par, device="cuda"), torch.tensor(off, device="cuda"), dev[1], dev[4], dev[5],
                        a=dev[0], c=dev[2], d=dev[3]).cpu().numpy()
    _check(par, off, arrays, x, range(3), 1e-11)


def test_not_post_order_is_rejected():
    """0 is a child of 2, but 1 (a child of 3) lies between them: the subtree
    {0, 2} is not a contiguous range, so the numbering is rejected."""
    par = np.array([2, 3, 3, -1], dtype=np.int64)
    off = np.array([0, 4], dtype=np.int64)
    dev = [torch.ones(4, dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(binding.TvChainError) as e:
        binding.tree_dp(torch.tensor(par, device="cuda"), torch.tensor(off, device="cuda"), *dev)
    assert e.value.status == binding.TV_ERR_INVALID_ARG
    bad_parent = np.array([-1, 0], dtype=np.int64)     # parent below the child
    with pytest.raises(binding.TvChainError):
        binding.tree_dp(torch.tensor(bad_parent, device="cuda"), torch.tensor([0, 2], device="cuda"),
                        *(torch.ones(2, dtype=torch.float64, device="cuda") for _ in range(3)))


def test_full_size_sample_fp32():
    """65,536 trees of 256 nodes (the benchmark's batch); 300 trees checked."""
    par, off = synth.post_order_forest(65536, 256, seed=1)
    arrays = _tree_data(par.size, seed=2)
    dev = [torch.tensor(v, dtype=torch.float32, device="cuda") for v in arrays]
    x = binding.tree_dp(torch.tensor(par, device="cuda"), torch.tensor(off, device="cuda"), dev[1], dev[4], dev[5],
                        a=dev[0], c=dev[2], d=dev[3]).double().cpu().numpy()
    arrays = [v.double().cpu().numpy() for v in dev]
    rng = np.random.default_rng(3)
    _check(par, off, arrays, x, rng.choice(65536, 300, replace=False), 1e-5)
