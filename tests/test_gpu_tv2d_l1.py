"""GPU parity of the 2D TV-l1 solver (tv2d_l1_solve, Sec. 5.2) with the
oracle's (pinned to the LP optimum in tests/test_oracle_tv2d_l1.py): the same
iteration with the same constant steps, compared iterate and energy after k
iterations.  The row proxes keep their TV-l1 sets in FP64 for FP32 data too
and are bitwise sequential for every plan, and the iteration is
non-expansive, so FP64 iterates agree to 1e-9 and FP32 ones to 1e-4 (of a
[0, 1] image), also at 2048 x 2048 after 30 iterations."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth

pytestmark = pytest.mark.gpu


def _impulse(H, W, seed, frac=0.25):
    rng = np.random.default_rng(seed)
    f = synth.shapes_image(H, W, sigma=0.0, seed=seed)
    m = rng.random((H, W)) < frac
    f[m] = rng.integers(0, 2, int(m.sum()))
    return f


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
@pytest.mark.parametrize("shape", [(64, 80), (130, 47)])
def test_iterates_and_energy_match_oracle(dtype, tol, shape):
    H, W = shape
    f = _impulse(H, W, seed=H + W)
    ft = torch.tensor(f, dtype=dtype, device="cuda")
    fv = ft.double().cpu().numpy()
    k = 30
    hist = torch.zeros(k, dtype=torch.float64, device="cuda")
    x, info = binding.tv2d_l1(ft, 0.55, max_iter=k, energy_every=1, energy_history=hist)
    xo, ho = oracle.tv2d_l1(fv, 0.55, tau=1.0, max_iter=k)
    assert np.abs(x.double().cpu().numpy() - xo).max() <= tol
    h = hist.cpu().numpy()
    assert np.abs(h - ho).max() <= (1e-9 if dtype == torch.float64 else 1e-6) * ho.max()
    assert info["primal"] == pytest.approx(oracle.tvl1_2d_objective(fv, 0.55, x.double().cpu().numpy()), rel=1e-12)


def test_converges_to_the_oracle_optimum():
    """Small image, many iterations: the energy reaches the oracle's converged
    energy (which the oracle tests tie to the LP optimum)."""
    f = _impulse(12, 16, seed=7)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    x, info = binding.tv2d_l1(ft, 0.4, max_iter=800, energy_every=100)
    _, ho = oracle.tv2d_l1(f, 0.4, tau=1.0, max_iter=800)
    assert info["primal"] == pytest.approx(ho[-1], rel=1e-9)


def test_lambda_zero_returns_f():
    f = _impulse(40, 50, seed=2)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    x, _ = binding.tv2d_l1(ft, 0.0, max_iter=3)
    assert torch.equal(x, ft)


def test_autotune_and_other_steps():
    f = _impulse(256, 200, seed=9)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    x, info = binding.tv2d_l1(ft, 0.5, max_iter=20, tau0=0.5, autotune=True)
    assert set(info["plans"]) == {"col", "row"}
    xo, _ = oracle.tv2d_l1(f, 0.5, tau=0.5, max_iter=20)
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-9
    binding.autotune_clear()


def test_full_size_fp32():
    """2048 x 2048 impulse-noise image, 30 iterations, against the oracle."""
    f = _impulse(2048, 2048, seed=3)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    x, info = binding.tv2d_l1(ft, 0.55, max_iter=30, energy_every=30)
    xo, ho = oracle.tv2d_l1(ft.double().cpu().numpy(), 0.55, tau=1.0, max_iter=30)
    assert np.abs(x.double().cpu().numpy() - xo).max() <= 1e-4
    assert info["primal"] == pytest.approx(ho[-1], rel=1e-6)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_segmented_rows_match_sequential(dtype):
    """The same solve with one segment per row and with the default plan:
    bit for bit (segment boundaries compare the TV-l1 sets exactly)."""
    f = _impulse(300, 1100, seed=5)
    ft = torch.tensor(f, dtype=dtype, device="cuda")
    saved = binding.get_tuning()
    try:
        binding.set_tuning(target_lanes=1, min_segment=1)
        ref, _ = binding.tv2d_l1(ft, 0.55, max_iter=12, energy_every=12)
        binding.set_tuning(**saved)
        binding.set_tuning(target_lanes=1 << 30, min_segment=32, halo=16)
        got, _ = binding.tv2d_l1(ft, 0.55, max_iter=12, energy_every=12)
    finally:
        binding.set_tuning(**saved)
    assert torch.equal(got, ref)


def test_rejects_bad_options():
    lib = binding.load()
    f = torch.zeros(8, 8, device="cuda")
    ws = torch.empty(lib.tv2d_l1_workspace(8, 8, binding.TV_F32), dtype=torch.uint8, device="cuda")
    P = ctypes.c_void_p
    for opt in (binding.Tv2dOptions(5, 1, 1e-3, 1.0, 0, None, 0), binding.Tv2dOptions(5, 1, 0.0, 1.0, 1, None, 0),
                binding.Tv2dOptions(5, 1, 0.0, 0.0, 0, None, 0), binding.Tv2dOptions(-1, 1, 0.0, 1.0, 0, None, 0)):
        st = lib.tv2d_l1_solve(binding.TV_F32, P(f.data_ptr()), 8, 8, 8, 0.5, P(f.data_ptr()), ctypes.byref(opt),
                               None, P(ws.data_ptr()), ws.numel(), None)
        assert st == binding.TV_ERR_INVALID_ARG
