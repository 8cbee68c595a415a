"""GPU parity of the general chain DP (tv_chain_dp: quadratic unaries a_i > 0,
b_i, asymmetric pairwise slopes w^-_e <= w^+_e) against the FP64 oracle's
Sec. 4.1 DP (oracle.chain_dp, pinned to brute force in the CPU tests).

Bars, per chain, relative to the scale s = max(range of the oracle's x,
range of b / a): FP64 <= 1e-11 s; FP32 <= 1e-4 s (slopes are sums of a_i in
FP64 rounded once to FP32, so they are no longer exact as with a_i = 1).
The oracle always sees the values the GPU sees (FP32 inputs are rounded
first, then widened).  With a_i = 1 and w^- = -w^+ the general path must give
the same bits as tv_chain_prox.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-4, torch.float64: 1e-11}


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _rounded(a, dtype):
    return _dev(a, dtype).cpu().double().numpy()


def _oracle_rows(a, b, wm, wp):
    return np.stack([oracle.chain_dp(a[c], b[c], wm[c, :-1], wp[c, :-1])[0] for c in range(b.shape[0])])


def _check(a, b, x_gpu, x_orc, tol):
    scale = np.maximum(np.ptp(x_orc, axis=1), np.ptp(b / a, axis=1))
    scale = np.maximum(scale, 1e-30)
    err = np.abs(x_gpu - x_orc).max(axis=1) / scale
    assert err.max() <= tol, (err.max(), int(err.argmax()))
    return err.max()


def _problem(C, n, seed, kind="asym"):
    """Seeded general chain problems: a ~ U[0.25, 4], b = a y with y the
    piecewise-constant + noise rows, and edge slopes of the requested kind."""
    rng = np.random.default_rng(seed)
    y = synth.piecewise_constant(C, n, seed=seed)
    a = rng.uniform(0.25, 4.0, size=(C, n))
    b = a * y
    if kind == "asym":      # w^- <= 0 <= w^+, different magnitudes
        wm = -rng.uniform(0.0, 0.6, size=(C, n))
        wp = rng.uniform(0.0, 0.6, size=(C, n))
    elif kind == "shifted":  # both of one sign on some edges (a linear term plus a kink)
        lo = rng.uniform(-0.5, 0.5, size=(C, n))
        wm, wp = lo, lo + rng.uniform(0.0, 0.8, size=(C, n))
    elif kind == "linear":   # w^- = w^+ (no kink at all)
        wm = rng.uniform(-0.3, 0.3, size=(C, n))
        wp = wm.copy()
    else:
        raise ValueError(kind)
    return a, b, wm, wp


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["asym", "shifted", "linear"])
@pytest.mark.parametrize("layout", ["rows", "cols"])
def test_general_dp_matches_oracle(dtype, kind, layout):
    """70 chains of 900 nodes (several segments and a ragged last tile)."""
    a, b, wm, wp = _problem(70, 900, seed=5, kind=kind)
    av, bv, wmv, wpv = (_rounded(t, dtype) for t in (a, b, wm, wp))
    if layout == "rows":
        x = binding.chain_dp(_dev(bv, dtype), _dev(wmv, dtype), _dev(wpv, dtype), a=_dev(av, dtype), dim=-1)
        xg = x.double().cpu().numpy()
    else:
        t = [_dev(np.ascontiguousarray(v.T), dtype) for v in (av, bv, wmv, wpv)]
        x = binding.chain_dp(t[1], t[2], t[3], a=t[0], dim=0)
        xg = x.double().cpu().numpy().T
    _check(av, bv, xg, _oracle_rows(av, bv, wmv, wpv), TOL[dtype])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_unit_case_is_bitwise_the_tv_prox(dtype):
    """a = 1 (as None and as an explicit array), w^- = -w, w^+ = w: the general
    path computes the same bits as tv_chain_prox with per-edge weights."""
    rng = np.random.default_rng(3)
    y = synth.piecewise_constant(96, 1500, seed=3)
    w = rng.uniform(0.0, 0.8, size=y.shape)
    yt, wt = _dev(y, dtype), _dev(w, dtype)
    ref = binding.chain_prox(yt, wt, dim=-1)
    got = binding.chain_dp(yt, -wt, wt, dim=-1)
    assert torch.equal(got, ref)
    got1 = binding.chain_dp(yt, -wt, wt, a=torch.ones_like(yt), dim=0)
    assert torch.equal(got1, binding.chain_prox(yt, wt, dim=0))


@pytest.fixture
def tuning():
    saved = binding.get_tuning()
    yield binding.set_tuning
    binding.set_tuning(**saved)
    binding.autotune_clear()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("halo", [0, 16, 128])
def test_segmented_is_bitwise_sequential(tuning, dtype, halo):
    """One segment per chain vs fine segmentation with short and long halos
    (repair, fix-up and tail paths): identical bits."""
    a, b, wm, wp = _problem(50, 2100, seed=11, kind="shifted")
    ts = [_dev(v, dtype) for v in (a, b, wm, wp)]
    tuning(target_lanes=1, min_segment=1)
    ref = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0])
    tuning(target_lanes=1 << 30, min_segment=32, halo=halo)
    got = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0])
    assert torch.equal(got, ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_deep_deques_take_the_exact_fallbacks(tuning, dtype):
    """Concave ramps with large slopes keep 17 .. 110 breakpoints alive: the
    16-slot ring overflows into the large-ring pass or the HBM deque; a 32-slot
    ring keeps the shallower ones on the segmented path.  Same bits either way,
    and the oracle's values."""
    n = 1024
    rng = np.random.default_rng(2)
    rows, ws = [], []
    for k, wv in enumerate((1.0, 3.0, 5.0, 10.0, 50.0)):
        for j in range(3):
            rows.append(np.sqrt(np.arange(n) + 7 * k + j))
            ws.append(wv)
    y = np.array(rows)
    a = rng.uniform(0.8, 1.25, size=y.shape)
    b = a * y
    wp = np.repeat(np.array(ws)[:, None], n, axis=1)
    wm = -wp * rng.uniform(0.7, 1.0, size=y.shape)
    av, bv, wmv, wpv = (_rounded(t, dtype) for t in (a, b, wm, wp))
    depth = [oracle.chain_dp(av[c], bv[c], wmv[c, :-1], wpv[c, :-1])[3]["max_breakpoints"] for c in range(len(y))]
    assert min(depth) > 16 and max(depth) > 64
    ts = [_dev(v, dtype) for v in (av, bv, wmv, wpv)]
    tuning(target_lanes=1 << 30, min_segment=128, ring_slots=16)
    x16 = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0])
    tuning(target_lanes=1 << 30, min_segment=128, ring_slots=32)
    x32 = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0])
    assert torch.equal(x16, x32)
    _check(av, bv, x16.double().cpu().numpy(), _oracle_rows(av, bv, wmv, wpv), TOL[dtype])


def test_short_chains_and_csr_offsets():
    """Uneven chains (CSR offsets) of 0 .. 600 nodes, including 1- and 2-node
    chains (x = b / a for one node), through the C ABI."""
    rng = np.random.default_rng(8)
    lens = rng.integers(0, 600, size=83)
    lens[[2, 5, 9]] = [0, 1, 2]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    total = int(offs[-1])
    a = rng.uniform(0.3, 3.0, total)
    b = a * (rng.normal(size=total) + np.repeat(rng.uniform(0, 1, total // 9 + 1), 9)[:total])
    wm = -rng.uniform(0, 0.4, total)
    wp = rng.uniform(0, 0.4, total)
    ts = [_dev(v, torch.float64) for v in (a, b, wm, wp)]
    x = torch.empty_like(ts[0])
    ot = torch.tensor(offs, device="cuda")
    lib = binding.load()
    lay = binding.ChainLayout(len(lens), int(lens.max()), 1, 0, ctypes.c_void_p(ot.data_ptr()))
    nbytes = lib.tv_chain_dp_workspace(ctypes.byref(lay), binding.TV_F64)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    P = ctypes.c_void_p
    st = lib.tv_chain_dp(ctypes.byref(lay), binding.TV_F64, *(P(t.data_ptr()) for t in ts), P(x.data_ptr()),
                         P(ws.data_ptr()), nbytes, P(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    xg = x.cpu().numpy()
    for c in range(len(lens)):
        lo, hi = offs[c], offs[c + 1]
        if hi > lo:
            xo = oracle.chain_dp(a[lo:hi], b[lo:hi], wm[lo:hi - 1], wp[lo:hi - 1])[0]
            scale = max(np.ptp(xo), np.ptp(b[lo:hi] / a[lo:hi]), 1e-30)
            assert np.abs(xg[lo:hi] - xo).max() <= 1e-11 * scale, c
    assert np.array_equal(xg[offs[5]:offs[6]], b[offs[5]:offs[6]] / a[offs[5]:offs[6]])


def test_autotune_keeps_the_bits(tuning):
    a, b, wm, wp = _problem(64, 3000, seed=13, kind="asym")
    ts = [_dev(v, torch.float32) for v in (a, b, wm, wp)]
    ref = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0])
    got, plan = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0], autotune=True)
    assert plan["candidates"] >= 1 and plan["ring_slots"] in (16, 32)
    assert torch.equal(got, ref)
    assert torch.equal(binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0]), ref)


def test_full_size_rows_and_columns_fp32():
    """The 4096 x 4096 workload of the benchmark's general-DP line: data weights
    a ~ U[0.5, 2], b = a f (shapes image), w^- = -0.1 u, w^+ = 0.1 v with
    u, v ~ U[0.5, 1.5]; all 4096 row and 4096 column chains against the oracle."""
    a, b, wm, wp = synth.general_chain_problem(4096, 4096, seed=3)
    ts = [_dev(v, torch.float32) for v in (a, b, wm, wp)]
    av, bv, wmv, wpv = (t.double().cpu().numpy() for t in ts)
    xr = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0], dim=-1).double().cpu().numpy()
    xc = binding.chain_dp(ts[1], ts[2], ts[3], a=ts[0], dim=0).double().cpu().numpy()
    _check(av, bv, xr, _oracle_rows(av, bv, wmv, wpv), TOL[torch.float32])
    T = [np.ascontiguousarray(v.T) for v in (av, bv, wmv, wpv)]
    _check(T[0], T[1], np.ascontiguousarray(xc.T), _oracle_rows(*T), TOL[torch.float32])


def test_rejects_bad_arguments():
    b = torch.zeros(4, 8, device="cuda")
    with pytest.raises(binding.TvChainError):
        binding.chain_dp(b, b.clone(), b.clone(), a=torch.ones(4, 7, device="cuda"))
    lib = binding.load()
    lay = binding.ChainLayout(4, 8, 1, 8, None)
    P = ctypes.c_void_p
    same = P(b.data_ptr())
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    # x aliasing b is rejected; wm missing is rejected
    assert lib.tv_chain_dp(ctypes.byref(lay), binding.TV_F32, None, same, same, same, same, P(ws.data_ptr()),
                           1 << 20, None) == binding.TV_ERR_INVALID_ARG
