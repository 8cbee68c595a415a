"""GPU parity of the TV-l1 chain prox (tv_chain_prox_l1, Sec. 4.2 with the
unaries of eq. (prox-pq)) against the FP64 oracle's Sec. 4.2 DP (pinned in
tests/test_oracle_pq.py to brute force, a KKT certificate and closed forms).

Bars per chain, relative to s = max(range of y, range of d, 1): FP64
<= 1e-11 s, FP32 <= 1e-4 s.  The oracle sees the values the GPU sees.  The
set is FP64 for FP32 data too, and segment boundaries compare sets bit for
bit, so every plan gives the sequential run's bits.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth
from tests import props

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-4, torch.float64: 1e-11}


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _rt(a, dtype):
    return _dev(a, dtype).cpu().double().numpy()


def _salt_pepper(C, n, frac, seed):
    """Piecewise-constant rows with a fraction of the samples replaced by 0 or 1."""
    rng = np.random.default_rng(seed)
    f = synth.piecewise_constant(C, n, sigma=0.02, seed=seed)
    m = rng.random(f.shape) < frac
    f[m] = rng.integers(0, 2, int(m.sum()))
    return f


def _check(y, d, xg, xo, tol):
    s = np.maximum(np.maximum(np.ptp(y, axis=1), np.ptp(d, axis=1)), 1.0)
    err = np.abs(xg - xo).max(axis=1) / s
    assert err.max() <= tol, (err.max(), int(err.argmax()))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("layout", ["rows", "cols"])
@pytest.mark.parametrize("wc", [(0.55, 1.0), (0.1, 0.3), (2.0, 0.05)])
def test_scalar_weights_match_oracle(dtype, layout, wc):
    """Salt & pepper chains (25%), the prox of the TV-l1 row step with y = d = f."""
    w, c = wc
    f = _salt_pepper(80, 700, 0.25, seed=3)
    rng = np.random.default_rng(4)
    y = _rt(f + 0.05 * rng.normal(size=f.shape), dtype)
    d = _rt(f, dtype)
    if layout == "rows":
        xg = binding.chain_prox_l1(_dev(y, dtype), _dev(d, dtype), w, c, dim=-1).double().cpu().numpy()
    else:
        xt = binding.chain_prox_l1(_dev(y.T.copy(), dtype), _dev(d.T.copy(), dtype), w, c, dim=0)
        xg = xt.double().cpu().numpy().T
    _check(y, d, xg, oracle.chain_prox_l1(y, d, w_scalar=w, c_scalar=c), TOL[dtype])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_per_edge_and_per_node_weights(dtype):
    rng = np.random.default_rng(5)
    C, n = 64, 900
    y = _rt(rng.normal(size=(C, n)), dtype)
    d = _rt(np.round(rng.normal(size=(C, n)) * 2) / 2, dtype)  # ties among the d's
    w = _rt(rng.uniform(0.0, 1.5, (C, n)), dtype)
    c = _rt(rng.uniform(0.0, 1.5, (C, n)) * (rng.random((C, n)) < 0.8), dtype)
    xg = binding.chain_prox_l1(_dev(y, dtype), _dev(d, dtype), _dev(w, dtype), _dev(c, dtype)).double().cpu().numpy()
    _check(y, d, xg, oracle.chain_prox_l1(y, d, w=w, c=c), TOL[dtype])
    if dtype == torch.float64:
        for r in range(0, C, 7):
            assert props.kkt_pq(np.ones(n), y[r], c[r], d[r], -w[r, :-1], w[r, :-1], xg[r], tol=1e-10) <= 1e-9


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_large_sets_take_the_hbm_fallback(dtype):
    """w = 20 and 50 keep 20 .. 47 breakpoints alive: beyond the 16-slot LDS set
    the chains are redone with the set in HBM; w = 0.5 chains stay on chip."""
    rng = np.random.default_rng(1)
    C, n = 48, 1024
    y = rng.normal(size=(C, n)) * 0.3 + np.repeat(rng.uniform(0, 1, (C, n // 64)), 64, axis=1)
    y = _rt(y, dtype)
    w = np.repeat(np.array([0.5, 20.0, 50.0])[np.arange(C) % 3][:, None], n, axis=1)
    w = _rt(w, dtype)
    _, st = oracle.chain_prox_l1(y, y, w=w, c_scalar=1.0, counts=True)
    assert st[1::3, 2].min() > 16 and st[0::3, 2].max() <= 16
    xg = binding.chain_prox_l1(_dev(y, dtype), _dev(y, dtype), _dev(w, dtype), 1.0).double().cpu().numpy()
    _check(y, y, xg, oracle.chain_prox_l1(y, y, w=w, c_scalar=1.0), TOL[dtype])


@pytest.fixture
def tuning():
    saved = binding.get_tuning()
    yield binding.set_tuning
    binding.set_tuning(**saved)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("halo", [0, 16, 128])
def test_segmented_matches_sequential(tuning, dtype, halo):
    """One segment per chain against fine segmentation with short and long
    halos (repairs, fix-ups and tails all run): bit for bit."""
    f = _salt_pepper(60, 2500, 0.25, seed=21)
    rng = np.random.default_rng(22)
    yt = _dev(f + 0.05 * rng.normal(size=f.shape), dtype)
    dt = _dev(f, dtype)
    wt = _dev(rng.uniform(0.1, 1.2, f.shape), dtype)
    tuning(target_lanes=1, min_segment=1)
    ref = binding.chain_prox_l1(yt, dt, wt, 0.8)
    tuning(target_lanes=1 << 30, min_segment=32, halo=halo)
    got = binding.chain_prox_l1(yt, dt, wt, 0.8)
    assert torch.equal(got, ref)
    tuning(target_lanes=1 << 30, min_segment=64, halo=halo)
    got = binding.chain_prox_l1(yt, dt, wt, 0.8, dim=-1)
    assert torch.equal(got, ref)
    y = yt.double().cpu().numpy()
    d = dt.double().cpu().numpy()
    _check(y, d, got.double().cpu().numpy(),
           oracle.chain_prox_l1(y, d, w=wt.double().cpu().numpy(), c_scalar=0.8), TOL[dtype])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_ring_sizes_agree(tuning, dtype):
    """Sets of 20 .. 47 breakpoints: with 16 ring slots they go to the large
    LDS ring or the HBM set, with 32 the smaller ones stay segmented; both
    agree with the oracle and with each other bit for bit."""
    rng = np.random.default_rng(1)
    C, n = 48, 1024
    y = rng.normal(size=(C, n)) * 0.3 + np.repeat(rng.uniform(0, 1, (C, n // 64)), 64, axis=1)
    w = np.repeat(np.array([0.5, 20.0, 50.0])[np.arange(C) % 3][:, None], n, axis=1)
    yt, wt = _dev(y, dtype), _dev(w, dtype)
    tuning(target_lanes=1 << 30, min_segment=128, ring_slots=16)
    a = binding.chain_prox_l1(yt, yt, wt, 1.0)
    tuning(target_lanes=1 << 30, min_segment=128, ring_slots=32)
    b = binding.chain_prox_l1(yt, yt, wt, 1.0)
    assert torch.equal(a, b)
    yv = yt.double().cpu().numpy()
    _check(yv, yv, b.double().cpu().numpy(), oracle.chain_prox_l1(yv, yv, w=wt.double().cpu().numpy(), c_scalar=1.0),
           TOL[dtype])


def test_autotune_picks_a_plan_and_keeps_the_result(tuning):
    f = _salt_pepper(512, 2048, 0.25, seed=30)
    t = _dev(f, torch.float32)
    ref = binding.chain_prox_l1(t, t, 0.55, 1.0)
    got, plan = binding.chain_prox_l1(t, t, 0.55, 1.0, autotune=True)
    assert plan["candidates"] >= 2 and plan["halo"] in (32, 64, 128)
    assert torch.equal(got, ref)
    again = binding.chain_prox_l1(t, t, 0.55, 1.0)
    assert torch.equal(again, got)
    binding.autotune_clear()


def test_c_zero_is_the_tv_prox():
    """No data term: the TV-l2 prox (tv_chain_prox), to rounding."""
    y = synth.piecewise_constant(40, 2000, seed=9)
    t = _dev(y, torch.float64)
    a = binding.chain_prox_l1(t, t, 0.4, 0.0).cpu().numpy()
    b = binding.chain_prox(t, 0.4).cpu().numpy()
    assert np.abs(a - b).max() <= 1e-12


def test_uneven_csr_chains_and_short_chains():
    rng = np.random.default_rng(8)
    lens = rng.integers(0, 500, size=71)
    lens[[1, 4, 6]] = [0, 1, 2]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    total = int(offs[-1])
    y = rng.normal(size=total)
    d = np.where(rng.random(total) < 0.3, rng.integers(0, 2, total).astype(float), y)
    yt, dt = _dev(y, torch.float64), _dev(d, torch.float64)
    x = torch.empty_like(yt)
    ot = torch.tensor(offs, device="cuda")
    lib = binding.load()
    lay = binding.ChainLayout(len(lens), int(lens.max()), 1, 0, ctypes.c_void_p(ot.data_ptr()))
    nbytes = lib.tv_chain_prox_l1_workspace(ctypes.byref(lay), binding.TV_F64)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    P = ctypes.c_void_p
    st = lib.tv_chain_prox_l1(ctypes.byref(lay), binding.TV_F64, P(yt.data_ptr()), P(dt.data_ptr()), None, 0.3,
                              None, 0.7, P(x.data_ptr()), P(ws.data_ptr()), nbytes,
                              P(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    xg = x.cpu().numpy()
    for ch in range(len(lens)):
        lo, hi = offs[ch], offs[ch + 1]
        if hi > lo:
            xo = oracle.chain_prox_l1(y[lo:hi], d[lo:hi], w_scalar=0.3, c_scalar=0.7)
            assert np.abs(xg[lo:hi] - xo).max() <= 1e-11 * max(np.ptp(y[lo:hi]), np.ptp(d[lo:hi]), 1.0), ch


def test_full_size_rows_fp32():
    """65,536 chains of 1,024 (the benchmark's TV-l1 workload) against the oracle."""
    f = synth.salt_pepper_chains(65536, 1024, seed=12)
    yt = _dev(f, torch.float32)
    y = yt.double().cpu().numpy()
    xg = binding.chain_prox_l1(yt, yt, 0.55, 1.0).double().cpu().numpy()
    _check(y, y, xg, oracle.chain_prox_l1(y, y, w_scalar=np.float32(0.55), c_scalar=1.0), TOL[torch.float32])


def test_rejects_bad_arguments():
    y = torch.zeros(4, 8, device="cuda")
    for bad in (-1.0, float("nan")):
        with pytest.raises(binding.TvChainError):
            binding.chain_prox_l1(y, y.clone(), bad, 1.0)
        with pytest.raises(binding.TvChainError):
            binding.chain_prox_l1(y, y.clone(), 0.5, bad)
