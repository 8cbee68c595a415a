"""GPU parity for the Sec. 5.3 non-convex 2D solver (tv2d_nc_solve) against the
FP64 oracle's primal-dual iteration (nc2d_pd) and the LP optimum of the convex
case."""
import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding

pytestmark = pytest.mark.gpu


def _convex_cost(g, H, W, D):
    cost = np.cumsum(np.sort(g.normal(size=(H, W, D)), axis=2), axis=2)
    return cost - cost.min(axis=2, keepdims=True)


def test_convex_case_matches_the_oracle_optimum():
    from tests.test_oracle_nc2d import _lp_optimum
    g = np.random.default_rng(0)
    H, W, D = 5, 6, 7
    cost = _convex_cost(g, H, W, D)
    w_h = g.uniform(0.2, 1.2, (H, W - 1))
    w_v = g.uniform(0.2, 1.2, (H - 1, W))
    x = binding.tv2d_nc(torch.tensor(cost, device="cuda"), 0.0, 1.0, 20.0, torch.tensor(w_h, device="cuda"),
                        torch.tensor(w_v, device="cuda"), float("inf"), 100.0, 300).cpu().numpy()
    e = oracle.nc2d_energy(cost, 0.0, 1.0, 20.0, w_h, w_v, np.inf, x)
    opt = _lp_optimum(cost, 20.0, w_h, w_v)
    assert abs(e - opt) <= 1e-7 * (1 + abs(opt)), (e, opt)


def test_zero_weights_keep_each_minimiser():
    g = np.random.default_rng(1)
    cost = g.uniform(0, 4, (9, 11, 12))
    x = binding.tv2d_nc(torch.tensor(cost, device="cuda"), -2.0, 0.5, 30.0, 0.0, 0.0, 2.0, 50.0, 10).cpu().numpy()
    assert np.array_equal(x, -2.0 + 0.5 * np.argmin(cost, axis=2))


@pytest.mark.parametrize("iters", [1, 4])
def test_nonconvex_truncated_iterates_match_the_oracle(iters):
    """The iterates are exact chain solves of identical problems, so in FP64
    they agree with the oracle's to rounding (compared by energy per iterate,
    since a chain may have several minimisers)."""
    g = np.random.default_rng(2 + iters)
    H, W, D = 10, 13, 9
    cost = g.uniform(0, 4, (H, W, D))
    w_h, w_v, C = 0.8, 0.8, 1.5
    xh, _, E = oracle.nc2d_pd(cost, 0.0, 1.0, 20.0, w_h, w_v, C, 100.0, iters)
    x = binding.tv2d_nc(torch.tensor(cost, device="cuda"), 0.0, 1.0, 20.0, w_h, w_v, C, 100.0, iters).cpu().numpy()
    e = oracle.nc2d_energy(cost, 0.0, 1.0, 20.0, w_h, w_v, C, x)
    assert abs(e - E[-1]) <= 1e-9 * (1 + abs(E[-1])), (e, E[-1], np.abs(x - xh).max())


def test_fp32_costs_and_plain_tv():
    g = np.random.default_rng(9)
    H, W, D = 8, 9, 10
    cost = _convex_cost(g, H, W, D).astype(np.float32).astype(np.float64)
    x64 = binding.tv2d_nc(torch.tensor(cost, device="cuda"), 0.0, 1.0, 20.0, 0.5, 0.5, float("inf"), 100.0, 100)
    x32 = binding.tv2d_nc(torch.tensor(cost, dtype=torch.float32, device="cuda"), 0.0, 1.0, 20.0, 0.5, 0.5,
                          float("inf"), 100.0, 100)
    e64 = oracle.nc2d_energy(cost, 0.0, 1.0, 20.0, 0.5, 0.5, np.inf, x64.cpu().numpy())
    e32 = oracle.nc2d_energy(cost, 0.0, 1.0, 20.0, 0.5, 0.5, np.inf, x32.double().cpu().numpy())
    assert abs(e32 - e64) <= 1e-5 * (1 + abs(e64))


def test_messages_beyond_128_breakpoints_fall_back():
    """150 levels with msg_cap = 256: the first solve with 128-breakpoint
    messages runs out of room (each unary alone holds 150 breakpoints) and the
    call repeats with the caller's capacity.  w = 0 keeps every pixel at its own
    minimiser; with TV on, the energy equals the oracle's after 2 iterations.
    Random uniform costs leave many intervals per node, hence the large map_cap."""
    g = np.random.default_rng(12)
    cost = g.uniform(0, 4, (6, 7, 150))
    ct = torch.tensor(cost, device="cuda")
    x = binding.tv2d_nc(ct, 0.0, 1.0, 20.0, 0.0, 0.0, 2.0, 50.0, 3, msg_cap=256, map_cap=8192).cpu().numpy()
    assert np.array_equal(x, np.argmin(cost, axis=2).astype(np.float64))
    xh, _, E = oracle.nc2d_pd(cost, 0.0, 1.0, 20.0, 0.5, 0.5, 1.5, 100.0, 2)
    x = binding.tv2d_nc(ct, 0.0, 1.0, 20.0, 0.5, 0.5, 1.5, 100.0, 2, msg_cap=256, map_cap=8192).cpu().numpy()
    e = oracle.nc2d_energy(cost, 0.0, 1.0, 20.0, 0.5, 0.5, 1.5, x)
    assert abs(e - E[-1]) <= 1e-9 * (1 + abs(E[-1]))
