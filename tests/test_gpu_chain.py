"""GPU parity of the batched chain prox (tv_chain_prox) against the FP64 oracle.

Bars: FP64 max |x_gpu - x_oracle| <= 1e-12 x (max y - min y) per chain; FP32
<= 1e-4 x range per chain (the precision target of the chain messages).
Inputs are the seeded synthetic workloads; the oracle always sees the same
values the GPU sees (FP32 inputs are rounded first, then widened).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth
from tests import props

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-4, torch.float64: 1e-12}


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _check_rows(y64, x_gpu, x_orc, tol):
    rng = np.ptp(y64, axis=-1, keepdims=True)
    rng = np.maximum(rng, 1e-30)
    err = np.abs(x_gpu - x_orc) / rng
    assert err.max() <= tol, (err.max(), np.unravel_index(err.argmax(), err.shape))
    return err.max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("layout", ["rows", "cols"])
def test_small_piecewise_constant(dtype, layout):
    """64 chains of 256, w = 0.5 (the small FP64 workload), both layouts."""
    y = synth.piecewise_constant(64, 256, seed=1)
    y = _dev(y, dtype).cpu().double().numpy()  # the values the GPU sees
    xo = oracle.chain_prox(y, w_scalar=0.5)
    if layout == "rows":
        xg = binding.chain_prox(_dev(y, dtype), 0.5, dim=-1).double().cpu().numpy()
    else:
        xg = binding.chain_prox(_dev(y.T.copy(), dtype), 0.5, dim=0).double().cpu().numpy().T
    _check_rows(y, xg, xo, TOL[dtype])


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 4096])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_lengths_and_ragged_batches(n, dtype):
    C = 67  # not a multiple of the 64-lane wave
    y = synth.piecewise_constant(C, n, seed=n)
    y = _dev(y, dtype).cpu().double().numpy()
    xo = oracle.chain_prox(y, w_scalar=0.2)
    xg = binding.chain_prox(_dev(y, dtype), 0.2, dim=-1).double().cpu().numpy()
    _check_rows(y, xg, xo, TOL[dtype])
    xg = binding.chain_prox(_dev(y.T.copy(), dtype), 0.2, dim=0).double().cpu().numpy().T
    _check_rows(y, xg, xo, TOL[dtype])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_per_edge_weights_with_zeros_and_huge(dtype):
    rng = np.random.default_rng(5)
    y = synth.piecewise_constant(130, 700, seed=3)
    w = rng.uniform(0.0, 1.0, y.shape)
    w[rng.random(y.shape) < 0.1] = 0.0
    w[:5] = 1e4
    y = _dev(y, dtype).cpu().double().numpy()
    w = _dev(w, dtype).cpu().double().numpy()
    xo = oracle.chain_prox(y, w=w)
    xg = binding.chain_prox(_dev(y, dtype), _dev(w, dtype), dim=-1).double().cpu().numpy()
    _check_rows(y, xg, xo, TOL[dtype])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_degenerate_cases(dtype):
    n = 300
    y = np.zeros((6, n))
    y[1] = 0.7                                     # constant
    y[2] = np.linspace(0, 1, n)                    # ramp
    y[3] = (-1.0) ** np.arange(n)                  # alternating
    y[4] = np.random.default_rng(1).normal(size=n)
    y[5] = np.random.default_rng(2).normal(size=n) * 1e3
    for w in (0.0, 1e-7, 0.3, 50.0):
        yv = _dev(y, dtype).cpu().double().numpy()
        xo = oracle.chain_prox(yv, w_scalar=w)
        xg = binding.chain_prox(_dev(yv, dtype), w, dim=-1).double().cpu().numpy()
        err = np.abs(xg - xo) / np.maximum(np.ptp(yv, axis=1, keepdims=True), 1.0)
        assert err.max() <= TOL[dtype], (w, err.max())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_deep_deque_takes_exact_fallback(dtype):
    """Ramps with huge weights keep O(100s) breakpoints alive: beyond the LDS
    ring, those chains are solved again with their deque in HBM."""
    n = 2048
    rows = []
    for k in range(40):
        rows.append(np.sqrt(np.arange(n) + k))            # deep deque
        rows.append(synth.piecewise_constant(1, n, seed=k)[0])  # shallow
    y = np.array(rows)
    _, st = oracle.chain_prox(y, w_scalar=100.0, counts=True)
    assert st[:, 2].max() > 64  # the workload does exceed the ring
    y = _dev(y, dtype).cpu().double().numpy()
    xo = oracle.chain_prox(y, w_scalar=100.0)
    xg = binding.chain_prox(_dev(y, dtype), 100.0, dim=-1).double().cpu().numpy()
    err = np.abs(xg - xo) / np.ptp(y, axis=1, keepdims=True)
    assert err.max() <= TOL[dtype], err.max()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_overflow_tiers_match_the_ring_path(tuning, dtype):
    """Deques of depth 17..112: with a 16-slot ring they overflow into the
    large-ring sequential pass (up to 256 slots for float, 128 for double) or,
    deeper still, into the HBM deque; with 32, 64 or 128-slot rings more of
    them stay on the segmented path.  Every route gives the same bits."""
    n = 1024
    rows, ws = [], []
    for k, wv in enumerate((1.0, 3.0, 5.0, 10.0, 50.0)):
        for j in range(3):
            rows.append(np.sqrt(np.arange(n) + 7 * k + j))
            ws.append(wv)
    y = np.array(rows)
    w = np.repeat(np.array(ws)[:, None], n, axis=1)
    _, st = oracle.chain_prox(y, w=w, counts=True)
    assert st[:, 2].min() > 16 and st[:, 2].max() > 64
    tuning(target_lanes=1 << 30, min_segment=128, ring_slots=16)
    a = _solve(y, w, dtype)
    tuning(target_lanes=1 << 30, min_segment=128, ring_slots=32)
    b = _solve(y, w, dtype)
    assert np.array_equal(a, b)
    # 64 slots (FP32: every depth here but the deepest stays segmented; FP64 uses 32)
    tuning(target_lanes=1 << 30, min_segment=256, ring_slots=64)
    assert np.array_equal(_solve(y, w, dtype), a)
    # 128 slots (FP32: every depth here stays segmented; FP64 uses 32)
    tuning(target_lanes=1 << 30, min_segment=512, ring_slots=128)
    assert np.array_equal(_solve(y, w, dtype), a)
    yv = _dev(y, dtype).cpu().double().numpy()
    wv = _dev(w, dtype).cpu().double().numpy()
    _check_rows(yv, a.astype(np.float64), oracle.chain_prox(yv, w=wv), TOL[dtype])


def test_in_place_and_strided_dims():
    y = synth.piecewise_constant(8, 4, seed=7).reshape(2, 4, 4)
    t = _dev(y, torch.float64)
    for dim in (0, 1, 2):
        ref = np.moveaxis(oracle.chain_prox(np.moveaxis(y, dim, -1).reshape(-1, y.shape[dim]), w_scalar=0.1)
                          .reshape(np.moveaxis(y, dim, -1).shape), -1, dim)
        got = binding.chain_prox(t, 0.1, dim=dim).cpu().numpy()
        assert np.abs(got - ref).max() < 1e-12
    y2 = synth.piecewise_constant(10, 50, seed=8)
    t2 = _dev(y2, torch.float64)
    binding.chain_prox(t2, 0.3, dim=-1, out=t2)
    assert np.abs(t2.cpu().numpy() - oracle.chain_prox(y2, w_scalar=0.3)).max() < 1e-12


def test_uneven_csr_chains_via_abi():
    """Uneven chains in one buffer (CSR offsets, including empty chains)."""
    import ctypes
    lib = binding.load()
    rng = np.random.default_rng(9)
    lens = rng.integers(0, 700, size=97)
    lens[3] = 0
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    total = int(offs[-1])
    y = rng.normal(size=total) + np.repeat(rng.uniform(0, 1, total // 10 + 1), 10)[:total]
    yt = _dev(y, torch.float32)
    xt = torch.empty_like(yt)
    ot = torch.tensor(offs, device="cuda")
    lay = binding.ChainLayout(len(lens), int(lens.max()), 1, 0, ctypes.c_void_p(ot.data_ptr()))
    nbytes = lib.tv_chain_prox_workspace(ctypes.byref(lay), binding.TV_F32)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    st = lib.tv_chain_prox(ctypes.byref(lay), binding.TV_F32, ctypes.c_void_p(yt.data_ptr()), None, 0.25,
                           ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    xg = xt.double().cpu().numpy()
    yv = yt.double().cpu().numpy()
    for c in range(len(lens)):
        a, b = offs[c], offs[c + 1]
        if b > a:
            xo = oracle.chain_prox(yv[a:b], w_scalar=0.25)
            assert np.abs(xg[a:b] - xo).max() <= 1e-4 * max(np.ptp(yv[a:b]), 1e-30)


def test_rejects_bad_arguments():
    y = torch.zeros(4, 8, device="cuda")
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(binding.TvChainError) as ei:
            binding.chain_prox(y, bad)
        assert ei.value.status == binding.TV_ERR_INVALID_ARG


def test_large_rows_and_columns_fp32():
    """The 4096 x 4096 shapes image: all 4096 row chains and 4096 column chains
    (w = 0.1), launched as the benchmark launches them, against the oracle."""
    img = synth.shapes_image(4096, 4096, seed=3)
    t = _dev(img, torch.float32)
    y = t.double().cpu().numpy()
    xr = binding.chain_prox(t, 0.1, dim=-1).double().cpu().numpy()
    xc = binding.chain_prox(t, 0.1, dim=0).double().cpu().numpy()
    _check_rows(y, xr, oracle.chain_prox(y, w_scalar=0.1), 1e-4)
    _check_rows(y.T, xc.T, oracle.chain_prox(np.ascontiguousarray(y.T), w_scalar=0.1), 1e-4)
    box, jump, total = props.kkt_residual(y, xr, 0.1, jump_tol=1e-5)
    assert box < 1e-3 and total < 1e-2


# -- segment-parallel forward / backward -------------------------------------

@pytest.fixture
def tuning():
    saved = binding.get_tuning()
    yield binding.set_tuning
    binding.set_tuning(**saved)


def _solve(y, w, dtype, dim=-1):
    t = _dev(y, dtype)
    wt = _dev(w, dtype) if isinstance(w, np.ndarray) else w
    return binding.chain_prox(t, wt, dim=dim).cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("wval", [0.1, 0.5, 3.0])
def test_segmented_is_bitwise_sequential(tuning, dtype, wval):
    """Cutting chains into segments (repair until the deques meet, fix-up where
    they never meet, collapse-based backward) gives bit-identical output."""
    y = synth.piecewise_constant(70, 2000, seed=21)
    tuning(target_lanes=1, min_segment=1)             # one segment per chain
    assert binding.segment_length(70, 2000) >= 2000
    ref = _solve(y, wval, dtype)
    for min_seg in (8, 16, 64, 256):
        tuning(target_lanes=1 << 30, min_segment=min_seg)
        L = binding.segment_length(70, 2000)
        assert L <= max(min_seg, 8)
        got = _solve(y, wval, dtype)
        assert np.array_equal(got, ref), (min_seg, np.abs(got - ref).max())
    yv = _dev(y, dtype).cpu().double().numpy()
    _check_rows(yv, ref.astype(np.float64), oracle.chain_prox(yv, w_scalar=wval), TOL[dtype])


@pytest.mark.parametrize("ring", [16, 32])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_window_widths_give_the_same_bits(tuning, ring, dtype):
    """Square-root ramps with w in [0.2, 0.8] keep 8 to 15 breakpoints alive,
    next to shallow piecewise-constant chains in the same waves: in FP32 those
    waves take the 16-entry window (rings of 8-byte entries), FP64 the general
    step.  Segmented runs equal the one-segment-per-chain run bit for bit, for
    16- and 32-slot rings, and the oracle within the bar."""
    n = 1024
    rows, ws = [], []
    pc = synth.piecewise_constant(96, n, seed=33)
    for k in range(96):
        if k % 3 == 0:
            rows.append(pc[k])
            ws.append(0.1)
        else:
            rows.append(np.sqrt(np.arange(n) + 5 * k))
            ws.append((0.2, 0.3, 0.5, 0.8)[k % 4])
    y = np.array(rows)
    w = np.repeat(np.array(ws)[:, None], n, axis=1)
    _, st = oracle.chain_prox(y, w=w, counts=True)
    deep = st[:, 2]
    assert ((deep >= 8) & (deep <= 15)).sum() >= 48 and deep.min() < 8
    tuning(target_lanes=1, min_segment=1, ring_slots=ring)
    ref = _solve(y, w, dtype)
    for min_seg in (32, 128):
        tuning(target_lanes=1 << 30, min_segment=min_seg, ring_slots=ring)
        got = _solve(y, w, dtype)
        assert np.array_equal(got, ref), (min_seg, np.abs(got - ref).max())
    yv = _dev(y, dtype).cpu().double().numpy()
    wv = _dev(w, dtype).cpu().double().numpy()
    _check_rows(yv, ref.astype(np.float64), oracle.chain_prox(yv, w=wv), TOL[dtype])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_segmented_columns_edge_weights_and_overflow(tuning, dtype):
    """Column layout, per-edge weights, and chains whose deques overflow the
    ring mixed with shallow ones, all under fine segmentation."""
    n = 1500
    rows = []
    for k in range(24):
        rows.append(np.sqrt(np.arange(n) + k))
        rows.append(synth.piecewise_constant(1, n, seed=100 + k)[0])
    y = np.array(rows)
    w = np.where(np.arange(48)[:, None] % 2 == 0, 100.0, synth.edge_weights((48, n), seed=5))
    tuning(target_lanes=1, min_segment=1)
    ref = _solve(y.T.copy(), w.T.copy(), dtype, dim=0).T
    tuning(target_lanes=1 << 30, min_segment=16)
    got = _solve(y.T.copy(), w.T.copy(), dtype, dim=0).T
    assert np.array_equal(got, ref)
    yv = _dev(y, dtype).cpu().double().numpy()
    wv = _dev(w, dtype).cpu().double().numpy()
    _check_rows(yv, ref.astype(np.float64), oracle.chain_prox(yv, w=wv), TOL[dtype])


@pytest.mark.parametrize("halo", [0, 8, 16, 64])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_segmented_halo_mismatches_are_repaired(tuning, dtype, halo):
    """Short halos leave many segment boundaries unconverged: those are found
    by exact state comparison and redone, so the output stays bit-identical."""
    y = synth.piecewise_constant(130, 3000, seed=31)
    for wval in (0.1, 0.6):
        tuning(target_lanes=1, min_segment=1)
        ref = _solve(y, wval, dtype)
        tuning(target_lanes=1 << 30, min_segment=64, halo=halo)
        got = _solve(y, wval, dtype)
        assert np.array_equal(got, ref), (halo, wval)


def test_segmented_uneven_lengths(tuning):
    """Lengths that are not multiples of the segment or tile, including n < L."""
    for n in (1, 7, 9, 63, 129, 1001):
        y = synth.piecewise_constant(65, n, seed=n)
        tuning(target_lanes=1, min_segment=1)
        ref = _solve(y, 0.3, torch.float32)
        tuning(target_lanes=1 << 30, min_segment=8)
        got = _solve(y, 0.3, torch.float32)
        assert np.array_equal(got, ref), n


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_multi_batch_launch_equals_separate_calls(dtype):
    """Rows and columns of an image (and a third batch of other length and
    weight) in one tv_chain_prox_multi launch: bit-identical to separate calls."""
    img = _dev(synth.shapes_image(700, 900, seed=41), dtype)
    other = _dev(synth.piecewise_constant(300, 2500, seed=42), dtype)
    xs = binding.chain_prox_multi([(img, -1), (img, 0), (other, -1)], w=[0.1, 0.1, 0.45])
    assert torch.equal(xs[0], binding.chain_prox(img, 0.1, dim=-1))
    assert torch.equal(xs[1], binding.chain_prox(img, 0.1, dim=0))
    assert torch.equal(xs[2], binding.chain_prox(other, 0.45, dim=-1))
    ov = other.double().cpu().numpy()
    _check_rows(ov, xs[2].double().cpu().numpy(), oracle.chain_prox(ov, w_scalar=0.45), TOL[dtype])


def test_multi_batch_full_size_rows_and_columns_fp32():
    """The 4096 x 4096 rows + columns step as one launch, against separate calls
    and the oracle on sampled chains."""
    img = synth.shapes_image(4096, 4096, seed=3)
    t = _dev(img, torch.float32)
    xr, xc = binding.chain_prox_multi([(t, -1), (t, 0)], w=0.1)
    assert torch.equal(xr, binding.chain_prox(t, 0.1, dim=-1))
    assert torch.equal(xc, binding.chain_prox(t, 0.1, dim=0))
    yv = t.double().cpu().numpy()
    rows = np.random.default_rng(5).choice(4096, size=48, replace=False)
    _check_rows(yv[rows], xr.double().cpu().numpy()[rows], oracle.chain_prox(yv[rows], w_scalar=0.1),
                TOL[torch.float32])
    cols = np.ascontiguousarray(yv[:, rows].T)
    _check_rows(cols, xc.double().cpu().numpy()[:, rows].T, oracle.chain_prox(cols, w_scalar=0.1),
                TOL[torch.float32])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_autotuned_plan_gives_identical_results(dtype):
    """The autotuner times the candidate plans and keeps the fastest for the
    shape; the prox is bit-identical under every plan."""
    img = _dev(synth.shapes_image(600, 1000, seed=51), dtype)
    ref_r = binding.chain_prox(img, 0.1, dim=-1)
    ref_c = binding.chain_prox(img, 0.1, dim=0)
    try:
        plan = binding.autotune_chain_prox([(img, -1), (img, 0)], w=0.1)
        assert plan["candidates"] >= 2 and plan["ring_slots"] in (16, 32) and plan["ms"] > 0
        xr, xc = binding.chain_prox_multi([(img, -1), (img, 0)], w=0.1)
        assert torch.equal(xr, ref_r) and torch.equal(xc, ref_c)
        one = binding.autotune_chain_prox([(img, 0)], w=0.1)
        assert binding.segment_length(1000, 600) == one["segment_length"]
        assert torch.equal(binding.chain_prox(img, 0.1, dim=0), ref_c)
    finally:
        binding.autotune_clear()


def test_maximum_length_fp32_chain():
    """The longest FP32 chain the ABI accepts (2^24 - 1 nodes, slopes still exact
    integers in float), against the oracle; and a length of 2^24 is rejected."""
    n = (1 << 24) - 1
    y = synth.piecewise_constant(1, n, seed=61)[0]
    t = _dev(y, torch.float32)
    x = binding.chain_prox(t, 0.3, dim=-1)
    yv = t.double().cpu().numpy()
    xo = oracle.chain_prox(yv[None], w_scalar=0.3)[0]
    assert np.abs(x.double().cpu().numpy() - xo).max() <= TOL[torch.float32] * np.ptp(yv)
    with pytest.raises(binding.TvChainError):
        binding.chain_prox(torch.zeros(1 << 24, dtype=torch.float32, device="cuda"), 0.3, dim=-1)


def test_many_tiny_chains_and_single_node_chains():
    """A million chains of 1, 2 and 3 nodes (closed forms of the prox)."""
    rng = np.random.default_rng(62)
    for n in (1, 2, 3):
        y = rng.normal(size=(1 << 20, n))
        x = binding.chain_prox(_dev(y, torch.float64), 0.25, dim=-1).cpu().numpy()
        assert np.abs(x - oracle.chain_prox(y, w_scalar=0.25)).max() < 1e-12
        if n == 1:
            assert np.array_equal(x, y)
