"""Host-side checks of the C ABI (no GPU): the built library exports every
function that include/tvchain.h declares, and argument errors are reported
before any HIP call (so they are testable on a machine without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1502_07770_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvchain.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(tv\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libtvchain.so not built")
    return binding.load()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("tv_chain_prox", "tv_chain_prox_backward", "tv_chain_prox_multi", "tv2d_solve",
              "tv2d_solve_batched", "tv_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if getattr(lib, n, None) is None]
    assert not missing, missing
    # the binding describes every declared function
    assert set(_declared()) <= set(binding._SIG)


def test_status_strings(lib):
    for code in range(7):
        assert lib.tv_status_string(code)
    assert lib.tv_status_string(99) == b"unknown status"


def test_tuning_round_trip_and_rejections(lib):
    saved = binding.get_tuning()
    try:
        binding.set_tuning(target_lanes=4096, min_segment=32, halo=40, ring_slots=32)
        assert binding.get_tuning() == {"target_lanes": 4096, "min_segment": 32, "halo": 40, "ring_slots": 32}
        bad = binding.Tuning(0, 1, 0, 16)
        assert lib.tv_set_tuning(ctypes.byref(bad)) == binding.TV_ERR_INVALID_ARG
        bad = binding.Tuning(4096, 1, 0, 24)
        assert lib.tv_set_tuning(ctypes.byref(bad)) == binding.TV_ERR_INVALID_ARG
        bad = binding.Tuning(4096, 1, 0, 256)
        assert lib.tv_set_tuning(ctypes.byref(bad)) == binding.TV_ERR_INVALID_ARG
        for k in (16, 32, 64, 128):
            binding.set_tuning(target_lanes=4096, min_segment=32, halo=40, ring_slots=k)
            assert binding.get_tuning()["ring_slots"] == k
        assert lib.tv_get_tuning(None) == binding.TV_ERR_INVALID_ARG
    finally:
        binding.set_tuning(**saved)


def _lay(C, n, es, cs):
    return binding.ChainLayout(C, n, es, cs, None)


def test_workspace_queries(lib):
    rows = _lay(64, 1000, 1, 1000)
    assert lib.tv_chain_prox_workspace(ctypes.byref(rows), binding.TV_F32) > 0
    assert lib.tv_chain_prox_workspace(ctypes.byref(rows), 7) == 0          # bad dtype
    assert lib.tv_chain_prox_workspace(ctypes.byref(_lay(4, 0, 1, 1)), binding.TV_F32) == 0
    assert lib.tv_chain_prox_workspace(ctypes.byref(_lay(4, 1 << 24, 1, 1 << 24)), binding.TV_F32) == 0
    assert lib.tv2d_workspace(64, 48, binding.TV_F32) > 0
    assert lib.tv2d_workspace(0, 48, binding.TV_F32) == 0
    lays = (binding.ChainLayout * 2)(_lay(64, 100, 1, 100), _lay(100, 64, 100, 1))
    assert lib.tv_chain_prox_multi_workspace(2, lays, binding.TV_F32) > 0
    assert lib.tv_chain_prox_multi_workspace(0, lays, binding.TV_F32) == 0
    assert lib.tv_chain_prox_multi_workspace(9, lays, binding.TV_F32) == 0


def test_argument_errors_before_any_hip_call(lib):
    rows = _lay(8, 100, 1, 100)
    P = ctypes.c_void_p
    buf, out, ws = P(0x10000000), P(0x20000000), P(0x30000000)
    call = lib.tv_chain_prox
    # negative / NaN weight, null pointers
    assert call(ctypes.byref(rows), 0, buf, None, -1.0, out, ws, 1 << 30, None) == binding.TV_ERR_INVALID_ARG
    assert call(ctypes.byref(rows), 0, buf, None, float("nan"), out, ws, 1 << 30, None) == binding.TV_ERR_INVALID_ARG
    assert call(ctypes.byref(rows), 0, None, None, 0.1, out, ws, 1 << 30, None) == binding.TV_ERR_INVALID_ARG
    # x aliasing y (or overlapping its range) is rejected
    assert call(ctypes.byref(rows), 0, buf, None, 0.1, buf, ws, 1 << 30, None) == binding.TV_ERR_INVALID_ARG
    assert call(ctypes.byref(rows), 0, buf, None, 0.1, P(0x10000000 + 4 * 799), ws, 1 << 30,
                None) == binding.TV_ERR_INVALID_ARG
    # workspace missing or short
    assert call(ctypes.byref(rows), 0, buf, None, 0.1, out, None, 0, None) == binding.TV_ERR_WORKSPACE
    assert call(ctypes.byref(rows), 0, buf, None, 0.1, out, ws, 256, None) == binding.TV_ERR_WORKSPACE
    # multi: overlapping outputs, bad batch counts, NaN weight
    lays = (binding.ChainLayout * 2)(rows, rows)
    ys = (P * 2)(buf, buf)
    same = (P * 2)(out, out)
    wsc = (ctypes.c_double * 2)(0.1, 0.1)
    m = lib.tv_chain_prox_multi
    assert m(2, lays, 0, ys, None, wsc, same, ws, 1 << 30, None) == binding.TV_ERR_INVALID_ARG
    assert m(0, lays, 0, ys, None, wsc, same, ws, 1 << 30, None) == binding.TV_ERR_INVALID_ARG
    xs = (P * 2)(out, P(0x40000000))
    bad = (ctypes.c_double * 2)(0.1, float("nan"))
    assert m(2, lays, 0, ys, None, bad, xs, ws, 1 << 30, None) == binding.TV_ERR_INVALID_ARG
    assert m(2, lays, 0, ys, None, wsc, xs, None, 0, None) == binding.TV_ERR_WORKSPACE
    # the autotuner validates like the multi launch
    res = binding.TuningResult()
    at = lib.tv_chain_prox_autotune
    assert at(2, lays, 0, ys, None, wsc, same, ws, 1 << 30, None, ctypes.byref(res)) == binding.TV_ERR_INVALID_ARG
    assert at(2, lays, 0, ys, None, wsc, xs, None, 0, None, ctypes.byref(res)) == binding.TV_ERR_WORKSPACE
    assert lib.tv2d_autotune(0, buf, 64, 48, 40, 0.1, 1.0, ws, 1 << 30, None, None, None) == binding.TV_ERR_INVALID_ARG
    assert lib.tv2d_autotune(0, buf, 64, 48, 48, 0.1, 0.0, ws, 1 << 30, None, None, None) == binding.TV_ERR_INVALID_ARG
    assert lib.tv2d_autotune(0, buf, 64, 48, 48, 0.1, 1.0, ws, 16, None, None, None) == binding.TV_ERR_WORKSPACE


def test_chain_dp_argument_errors_and_workspace(lib):
    """tv_chain_dp: host-visible argument errors come back before any HIP call."""
    P = ctypes.c_void_p
    rows = _lay(8, 100, 1, 100)
    a, b, wm, wp, x, ws = (P(0x10000000 * k) for k in range(1, 7))
    assert lib.tv_chain_dp_workspace(ctypes.byref(rows), binding.TV_F32) > \
        lib.tv_chain_prox_workspace(ctypes.byref(rows), binding.TV_F32)  # + FP64 prefix sums
    assert lib.tv_chain_dp_workspace(ctypes.byref(rows), 5) == 0
    assert lib.tv_chain_dp_workspace(ctypes.byref(_lay(4, 1 << 24, 1, 1 << 24)), binding.TV_F32) == 0
    dp = lib.tv_chain_dp
    big = 1 << 30
    assert dp(ctypes.byref(rows), 0, a, None, wm, wp, x, ws, big, None) == binding.TV_ERR_INVALID_ARG  # no b
    assert dp(ctypes.byref(rows), 0, a, b, None, wp, x, ws, big, None) == binding.TV_ERR_INVALID_ARG  # no wm
    assert dp(ctypes.byref(rows), 0, a, b, wm, None, x, ws, big, None) == binding.TV_ERR_INVALID_ARG  # no wp
    assert dp(ctypes.byref(rows), 0, a, b, wm, wp, None, ws, big, None) == binding.TV_ERR_INVALID_ARG  # no x
    for alias in (a, b, wm, wp):  # x overlapping any input
        assert dp(ctypes.byref(rows), 0, a, b, wm, wp, alias, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert dp(ctypes.byref(rows), 0, a, b, wm, wp, P(0x20000000 + 4 * 799), ws, big,
              None) == binding.TV_ERR_INVALID_ARG
    assert dp(ctypes.byref(rows), 0, None, b, wm, wp, x, None, 0, None) == binding.TV_ERR_WORKSPACE
    assert dp(ctypes.byref(rows), 0, None, b, wm, wp, x, ws, 256, None) == binding.TV_ERR_WORKSPACE
    assert dp(ctypes.byref(_lay(0, 100, 1, 100)), 0, None, None, None, None, None, None, 0, None) == binding.TV_OK
    res = binding.TuningResult()
    at = lib.tv_chain_dp_autotune
    assert at(ctypes.byref(rows), 0, a, b, wm, wp, b, ws, big, None, ctypes.byref(res)) == binding.TV_ERR_INVALID_ARG
    assert at(ctypes.byref(rows), 0, a, b, wm, wp, x, None, 0, None, ctypes.byref(res)) == binding.TV_ERR_WORKSPACE


def test_chain_prox_l1_argument_errors(lib):
    """tv_chain_prox_l1: host-visible argument errors before any HIP call."""
    P = ctypes.c_void_p
    rows = _lay(8, 100, 1, 100)
    y, d, w, c, x, ws = (P(0x10000000 * k) for k in range(1, 7))
    assert lib.tv_chain_prox_l1_workspace(ctypes.byref(rows), binding.TV_F32) > 0
    assert lib.tv_chain_prox_l1_workspace(ctypes.byref(rows), 3) == 0
    f = lib.tv_chain_prox_l1
    big = 1 << 30
    assert f(ctypes.byref(rows), 0, None, d, None, 0.1, None, 1.0, x, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert f(ctypes.byref(rows), 0, y, None, None, 0.1, None, 1.0, x, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert f(ctypes.byref(rows), 0, y, d, None, -0.1, None, 1.0, x, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert f(ctypes.byref(rows), 0, y, d, None, 0.1, None, float("inf"), x, ws, big,
             None) == binding.TV_ERR_INVALID_ARG
    for alias in (y, d, w, c):
        assert f(ctypes.byref(rows), 0, y, d, w, 0.1, c, 1.0, alias, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert f(ctypes.byref(rows), 0, y, d, w, 0.1, c, 1.0, x, None, 0, None) == binding.TV_ERR_WORKSPACE
    assert f(ctypes.byref(rows), 0, y, d, w, 0.1, c, 1.0, x, ws, 64, None) == binding.TV_ERR_WORKSPACE


def test_tv2d_l1_argument_errors(lib):
    P = ctypes.c_void_p
    buf, ws = P(0x10000000), P(0x30000000)
    assert lib.tv2d_l1_workspace(64, 48, binding.TV_F32) > lib.tv2d_workspace(64, 48, binding.TV_F32)
    assert lib.tv2d_l1_workspace(0, 48, binding.TV_F32) == 0
    ok = binding.Tv2dOptions(5, 1, 0.0, 1.0, 0, None, 0)
    solve = lib.tv2d_l1_solve
    big = 1 << 30
    assert solve(0, buf, 64, 48, 40, 0.5, buf, ctypes.byref(ok), None, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert solve(0, buf, 64, 48, 48, -0.5, buf, ctypes.byref(ok), None, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert solve(0, buf, 64, 48, 48, 0.5, None, ctypes.byref(ok), None, ws, big, None) == binding.TV_ERR_INVALID_ARG
    for bad in (binding.Tv2dOptions(5, 1, 1e-3, 1.0, 0, None, 0), binding.Tv2dOptions(5, 1, 0.0, 1.0, 1, None, 0),
                binding.Tv2dOptions(5, 1, 0.0, float("nan"), 0, None, 0)):
        assert solve(0, buf, 64, 48, 48, 0.5, buf, ctypes.byref(bad), None, ws, big, None) == binding.TV_ERR_INVALID_ARG
    assert solve(0, buf, 64, 48, 48, 0.5, buf, ctypes.byref(ok), None, ws, 16, None) == binding.TV_ERR_WORKSPACE
    assert lib.tv2d_l1_autotune(0, buf, 64, 48, 48, 0.5, 0.0, ws, big, None, None, None) == binding.TV_ERR_INVALID_ARG


def test_tv2d_lookahead_out_of_range_is_rejected(lib):
    """tv2d_options.lookahead outside 0 .. 64 is an argument error of the ROF
    and the batched solve, found on the host before any device call."""
    P = ctypes.c_void_p
    buf, out, ws = P(0x10000000), P(0x20000000), P(0x30000000)
    big = 1 << 30
    H = (ctypes.c_int64 * 1)(16)
    W = (ctypes.c_int64 * 1)(16)
    off = (ctypes.c_int64 * 1)(0)
    lam = (ctypes.c_double * 1)(0.1)
    for la in (-1, 65):
        bad = binding.Tv2dOptions(5, 1, 1e-4, 1.0, 0, None, 0, la)
        assert lib.tv2d_solve(0, buf, 16, 16, 16, 0.1, out, ctypes.byref(bad), None, ws, big,
                              None) == binding.TV_ERR_INVALID_ARG
        assert lib.tv2d_solve_batched(0, 1, H, W, off, lam, buf, out, ctypes.byref(bad), None, ws, big,
                                      None) == binding.TV_ERR_INVALID_ARG


def test_tree_dp_argument_errors(lib):
    P = ctypes.c_void_p
    buf, x = P(0x10000000), P(0x20000000)
    assert lib.tv_tree_dp_workspace(10, 100) > 0
    assert lib.tv_tree_dp_workspace(0, 100) == 0
    f = lib.tv_tree_dp
    assert f(0, 1, 4, None, buf, None, buf, None, None, buf, buf, x, buf, 1 << 20, None) == binding.TV_ERR_INVALID_ARG
    assert f(0, 1, 4, buf, buf, None, buf, buf, None, buf, buf, x, buf, 1 << 20, None) == binding.TV_ERR_INVALID_ARG
    assert f(0, 1, 4, buf, buf, None, buf, None, None, buf, buf, buf, buf, 1 << 20, None) == binding.TV_ERR_INVALID_ARG
    assert f(7, 1, 4, buf, buf, None, buf, None, None, buf, buf, x, buf, 1 << 20, None) == binding.TV_ERR_INVALID_ARG
    assert f(0, 1, 4, buf, buf, None, buf, None, None, buf, buf, x, None, 0, None) == binding.TV_ERR_WORKSPACE
    assert f(0, 0, 0, None, None, None, None, None, None, None, None, None, None, 0, None) == binding.TV_OK


def test_workspace_covers_every_autotune_candidate(lib):
    """The workspace queries reserve room for the largest candidate plan, so a
    plan chosen after the workspace was allocated always fits."""
    rows = _lay(4096, 4096, 1, 4096)
    big = lib.tv_chain_prox_workspace(ctypes.byref(rows), binding.TV_F32)
    saved = binding.get_tuning()
    try:
        # a coarser default plan needs less, but the query keeps the candidates' maximum
        binding.set_tuning(target_lanes=4096, min_segment=4096, halo=0)
        assert lib.tv_chain_prox_workspace(ctypes.byref(rows), binding.TV_F32) <= big
        assert binding.segment_length(4096, 4096) == 4096
    finally:
        binding.set_tuning(**saved)


def test_nc_chain_argument_errors(lib):
    assert lib.tv_chain_nc_workspace(4, 100, 64, 256) > 0
    assert lib.tv_chain_nc_workspace(-1, 100, 64, 256) == 0
    assert lib.tv_chain_nc_workspace(4, 100, 0, 256) == 0
    assert lib.tv_chain_nc_workspace(4, 100, 64, 0) == 0
    # zero chains: nothing to do, no device call
    assert lib.tv_chain_nc(binding.TV_F32, 0, 0, None, None, None, None, None, None, None, 8, 8, None, 0,
                           None) == binding.TV_OK
    # null arrays and a bad dtype are rejected on the host
    assert lib.tv_chain_nc(binding.TV_F32, 1, 4, None, None, None, None, None, None, None, 8, 8, None, 0,
                           None) == binding.TV_ERR_INVALID_ARG
    assert lib.tv_chain_nc(7, 1, 4, None, None, None, None, None, None, None, 8, 8, None, 0,
                           None) == binding.TV_ERR_INVALID_ARG
    assert lib.tv_chain_nc(binding.TV_F64, 1 << 31, 4, None, None, None, None, None, None, None, 8, 8, None, 0,
                           None) == binding.TV_ERR_INVALID_ARG


def test_nc2d_argument_errors(lib):
    assert lib.tv2d_nc_workspace(16, 20, 8, 64, 256) > 0
    assert lib.tv2d_nc_workspace(0, 20, 8, 64, 256) == 0
    assert lib.tv2d_nc_workspace(16, 20, 1, 64, 256) == 0   # D < 2
    assert lib.tv2d_nc_workspace(16, 20, 8, 4, 256) == 0    # msg_cap < D
    # null arrays, bad steps and bad dtype are rejected on the host
    assert lib.tv2d_nc_solve(binding.TV_F32, None, 4, 4, 4, 0.0, 1.0, 10.0, None, 0.5, None, 0.5, 1.0, 10.0, 1,
                             None, 64, 64, None, 0, None) == binding.TV_ERR_INVALID_ARG
    assert lib.tv2d_nc_solve(7, None, 4, 4, 4, 0.0, 1.0, 10.0, None, 0.5, None, 0.5, 1.0, 10.0, 1,
                             None, 64, 64, None, 0, None) == binding.TV_ERR_INVALID_ARG


def test_nc_tree_argument_errors(lib):
    assert lib.tv_tree_nc_workspace(4, 100, 64, 256, 1000) > 0
    assert lib.tv_tree_nc_workspace(4, 100, 64, 256, 0) == 0
    assert lib.tv_tree_nc(binding.TV_F64, 0, 0, None, None, None, None, None, None, None, None, 8, 8, 8, None, 0,
                          None) == binding.TV_OK
    assert lib.tv_tree_nc(binding.TV_F64, 1, 4, None, None, None, None, None, None, None, None, 8, 8, 8, None, 0,
                          None) == binding.TV_ERR_INVALID_ARG


def test_nc_concave_argument_errors(lib):
    assert lib.tv_chain_nc_concave_workspace(4, 100, 300, 64, 256) > 0
    assert lib.tv_chain_nc_concave_workspace(4, 100, -1, 64, 256) == 0
    assert lib.tv_chain_nc_concave_workspace(4, 100, 300, 0, 256) == 0
    assert lib.tv_chain_nc_concave(binding.TV_F64, 0, 0, 0, None, None, None, None, None, None, None, None, None,
                                   8, 8, None, 0, None) == binding.TV_OK
    assert lib.tv_chain_nc_concave(binding.TV_F64, 1, 4, 3, None, None, None, None, None, None, None, None, None,
                                   8, 8, None, 0, None) == binding.TV_ERR_INVALID_ARG
    assert lib.tv_chain_nc_concave(binding.TV_F64, 1 << 31, 4, 3, None, None, None, None, None, None, None, None,
                                   None, 8, 8, None, 0, None) == binding.TV_ERR_INVALID_ARG


def test_nc_tree_concave_argument_errors(lib):
    assert lib.tv_tree_nc_concave_workspace(4, 100, 300, 64, 256, 1000) > 0
    assert lib.tv_tree_nc_concave_workspace(4, 100, 300, 64, 256, 0) == 0
    assert lib.tv_tree_nc_concave(binding.TV_F64, 0, 0, 0, None, None, None, None, None, None, None, None, None,
                                  None, 8, 8, 8, None, 0, None) == binding.TV_OK
    assert lib.tv_tree_nc_concave(binding.TV_F64, 1, 4, 3, None, None, None, None, None, None, None, None, None,
                                  None, 8, 8, 8, None, 0, None) == binding.TV_ERR_INVALID_ARG
