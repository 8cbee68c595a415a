"""FP64 CPU oracle for "Total variation on a tree" (arXiv 1502.07770).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the GPU library (``paper_1502_07770_amd``) and never imports it; the GPU
library never imports this package.

The arithmetic lives in ``tv_oracle.c`` (plain C, FP64, optional OpenMP over
independent chains); this module is a ctypes wrapper that converts numpy
arrays.  Functions and the passages they follow:

* ``chain_prox``      -- eq. (1D-ROF) solved by the Sec. 4.1 O(n) algorithm
                         (Algorithm 2 specialised to quadratic unaries).
* ``chain_dp``        -- the same algorithm for general a_i > 0, b_i and
                         asymmetric slopes w^-_i <= w^+_i (Sec. 4 / 4.1), with
                         lambda^+- and breakpoint counters exposed.
* ``chain_brute``     -- brute force over all edge sign patterns (tiny n).
* ``chain_adjoint``   -- gradient of <g, x(y, w)> from the run structure of x.
* ``tv2d``            -- Sec. 5.1 ROF via Lagrangian decomposition and the
                         accelerated primal-dual iteration eq. (pd), with an
                         FP64 duality gap.
* ``nc_chain``        -- Sec. 3 (non-convex case) on a chain: piecewise-linear
                         unaries, truncated TV, Lemma 1, Algorithm 1 and its
                         reversal, the truncation, and the backward pass through
                         the mappings pi; ``nc_brute`` is its independent pin;
                         ``nc_tree`` the same on a forest (children's messages
                         summed, Lemma 1), pinned by ``nc_tree_brute``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tv_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Counts(ctypes.Structure):
    _fields_ = [("pushes", ctypes.c_int64), ("pops", ctypes.c_int64),
                ("max_breakpoints", ctypes.c_int64)]


# A sanitized build (AddressSanitizer + UndefinedBehaviorSanitizer), for
# running the oracle's own tests under the sanitizers; ORACLE_LIBRARY makes
# this module load it (or any other build) instead of liboracle.so.
SAN_LIB_PATH = os.path.join(_HERE, "liboracle_san.so")
if os.environ.get("ORACLE_LIBRARY"):
    _LIB_PATH = os.environ["ORACLE_LIBRARY"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile tv_oracle.c into liboracle.so (gcc, -O2, OpenMP, IEEE FP64), or
    with sanitize into liboracle_san.so (-O1, ASan + UBSan, aborting on the
    first error; load it into a process that preloads libasan)."""
    out = SAN_LIB_PATH if sanitize else _LIB_PATH
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        opt = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer"] if sanitize else ["-O2"])
        cmd = ["gcc"] + opt + ["-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    lib.orc_chain_dp.argtypes = [I64, P, P, P, P, P, P, P, P, P]
    lib.orc_chain_dp.restype = ctypes.c_int
    lib.orc_chain_prox_tv.argtypes = [I64, I64, I64, I64, P, P, D, P, P, ctypes.c_int]
    lib.orc_chain_prox_tv.restype = ctypes.c_int
    lib.orc_chain_brute.argtypes = [I64, P, P, P, P, P]
    lib.orc_chain_brute.restype = ctypes.c_int
    lib.orc_rof1d_objective.argtypes = [I64, P, P, D, P]
    lib.orc_rof1d_objective.restype = D
    lib.orc_chain_adjoint.argtypes = [I64, I64, I64, I64, P, P, P, P, P, ctypes.c_int]
    lib.orc_chain_adjoint.restype = ctypes.c_int
    lib.orc_tv2d.argtypes = [I64, I64, P, D, D, I64, D, P, P, P, ctypes.c_int]
    lib.orc_tv2d.restype = I64
    lib.orc_rof2d_objective.argtypes = [I64, I64, P, D, P]
    lib.orc_rof2d_objective.restype = D
    lib.orc_chain_pq.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_chain_pq.restype = ctypes.c_int
    lib.orc_chain_pq_brute.argtypes = [I64, P, P, P, P, P, P, P]
    lib.orc_chain_pq_brute.restype = ctypes.c_int
    lib.orc_pq_objective.argtypes = [I64, P, P, P, P, P, P, P]
    lib.orc_pq_objective.restype = D
    lib.orc_chain_prox_l1.argtypes = [I64, I64, I64, I64, P, P, P, D, P, D, P, P, ctypes.c_int]
    lib.orc_chain_prox_l1.restype = ctypes.c_int
    lib.orc_tvl1_2d_objective.argtypes = [I64, I64, P, D, P]
    lib.orc_tvl1_2d_objective.restype = D
    lib.orc_tv2d_l1.argtypes = [I64, I64, P, D, D, I64, P, P, ctypes.c_int]
    lib.orc_tv2d_l1.restype = I64
    lib.orc_tree_pq.argtypes = [I64, P, P, P, P, P, P, P, P, P, P]
    lib.orc_tree_pq.restype = ctypes.c_int
    lib.orc_tree_pq_brute.argtypes = [I64, P, P, P, P, P, P, P, P]
    lib.orc_tree_pq_brute.restype = ctypes.c_int
    lib.orc_tree_pq_objective.argtypes = [I64, P, P, P, P, P, P, P, P]
    lib.orc_tree_pq_objective.restype = D
    lib.orc_nc_chain.argtypes = [I64, P, P, P, P, P, P, P]
    lib.orc_nc_chain.restype = ctypes.c_int
    lib.orc_nc_energy.argtypes = [I64, P, P, P, P, P, P]
    lib.orc_nc_energy.restype = D
    lib.orc_nc_brute.argtypes = [I64, P, P, P, P, P, P, P]
    lib.orc_nc_brute.restype = ctypes.c_int
    lib.orc_nc_tree.argtypes = [I64, P, P, P, P, P, P, P, P]
    lib.orc_nc_tree.restype = ctypes.c_int
    lib.orc_nc_tree_energy.argtypes = [I64, P, P, P, P, P, P, P]
    lib.orc_nc_tree_energy.restype = D
    lib.orc_nc_tree_brute.argtypes = [I64, P, P, P, P, P, P, P]
    lib.orc_nc_tree_brute.restype = ctypes.c_int
    lib.orc_ncg_chain.argtypes = [I64, P, P, P, P, P, P, P, P, P]
    lib.orc_ncg_chain.restype = ctypes.c_int
    lib.orc_ncg_energy.argtypes = [I64, P, P, P, P, P, P, P, P]
    lib.orc_ncg_energy.restype = D
    lib.orc_ncg_brute.argtypes = [I64, P, P, P, P, P, P, P, P, P]
    lib.orc_ncg_brute.restype = ctypes.c_int
    lib.orc_ncg_tree.argtypes = [I64, P, P, P, P, P, P, P, P, P, P]
    lib.orc_ncg_tree.restype = ctypes.c_int
    lib.orc_ncg_tree_energy.argtypes = [I64, P, P, P, P, P, P, P, P, P]
    lib.orc_ncg_tree_energy.restype = D
    lib.orc_ncg_tree_brute.argtypes = [I64, P, P, P, P, P, P, P, P, P]
    lib.orc_ncg_tree_brute.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    """OpenMP threads the oracle uses when ``threads <= 0``."""
    return int(_load().orc_num_threads())


def chain_dp(a, b, wm, wp):
    """Sec. 4.1 DP on one chain with f_i = a_i x^2/2 - b_i x and pairwise slopes
    (wm[e], wp[e]) on edge (e, e+1).  Returns (x, lam_lo, lam_hi, counts) with
    counts = dict(pushes, pops, max_breakpoints)."""
    a, b = _f64(a), _f64(b)
    n = a.shape[0]
    wm = _f64(np.zeros(0) if n == 1 else wm)
    wp = _f64(np.zeros(0) if n == 1 else wp)
    assert b.shape == (n,) and wm.shape == (n - 1,) and wp.shape == (n - 1,)
    x = np.empty(n)
    llo = np.empty(max(n, 1))
    lhi = np.empty(max(n, 1))
    seq = np.empty(4 * n + 9)
    cnt = _Counts()
    # pad the edge arrays so the C side may read index n-1 safely
    wm_p = np.concatenate([wm, [0.0]])
    wp_p = np.concatenate([wp, [0.0]])
    rc = _load().orc_chain_dp(n, _ptr(a), _ptr(b), _ptr(wm_p), _ptr(wp_p), _ptr(x),
                              _ptr(llo), _ptr(lhi), _ptr(seq), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("orc_chain_dp failed")
    return x, llo[: n - 1].copy(), lhi[: n - 1].copy(), dict(
        pushes=cnt.pushes, pops=cnt.pops, max_breakpoints=cnt.max_breakpoints)


def chain_prox(y, w=None, w_scalar: float = 0.0, threads: int = 0, counts: bool = False):
    """eq. (1D-ROF) for a batch of chains.  ``y`` is (n,) or (C, n); ``w`` is
    None (use ``w_scalar``) or an array of the same shape as y whose slot i is
    the weight of edge (i, i+1) (the last slot is ignored).  Returns x (and the
    per-chain counters when ``counts``)."""
    y = _f64(y)
    squeeze = y.ndim == 1
    y2 = y.reshape(1, -1) if squeeze else y
    C, n = y2.shape
    w2 = None
    if w is not None:
        w2 = _f64(w).reshape(C, n)
    x = np.empty_like(y2)
    cnt = (_Counts * max(C, 1))() if counts else None
    rc = _load().orc_chain_prox_tv(C, n, 1, n, _ptr(y2), _ptr(w2), float(w_scalar), _ptr(x),
                                   cnt, int(threads))
    if rc != 0:
        raise ValueError("orc_chain_prox_tv: invalid argument (negative or NaN weight?)")
    out = x.reshape(-1) if squeeze else x
    if counts:
        stats = np.array([[c.pushes, c.pops, c.max_breakpoints] for c in cnt[:C]], dtype=np.int64)
        return out, stats
    return out


def chain_pq(a, b, c, d, wm, wp):
    """Sec. 4.2 DP on one chain with piecewise-quadratic unaries
    f_i = a_i x^2/2 - b_i x + c_i |x - d_i| and edge slopes (wm[e], wp[e]) on
    edge (e, e+1).  Returns (x, lam_lo, lam_hi, counts)."""
    a, b, c, d = _f64(a), _f64(b), _f64(c), _f64(d)
    n = a.shape[0]
    assert b.shape == c.shape == d.shape == (n,)
    wm_p = np.concatenate([_f64(wm).reshape(-1)[: max(n - 1, 0)], [0.0]])
    wp_p = np.concatenate([_f64(wp).reshape(-1)[: max(n - 1, 0)], [0.0]])
    x = np.empty(n)
    llo = np.empty(max(n, 1))
    lhi = np.empty(max(n, 1))
    buf = np.empty(3 * (3 * n + 4))
    cnt = _Counts()
    rc = _load().orc_chain_pq(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(wm_p), _ptr(wp_p), _ptr(x),
                              _ptr(llo), _ptr(lhi), _ptr(buf), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("orc_chain_pq failed")
    return x, llo[: n - 1].copy(), lhi[: n - 1].copy(), dict(
        pushes=cnt.pushes, pops=cnt.pops, max_breakpoints=cnt.max_breakpoints)


def chain_pq_brute(a, b, c, d, wm, wp):
    """Brute-force minimiser of the Sec. 4.2 chain objective for n <= 6."""
    a, b, c, d = _f64(a), _f64(b), _f64(c), _f64(d)
    n = a.shape[0]
    wm_p = np.concatenate([_f64(wm).reshape(-1)[: max(n - 1, 0)], [0.0]])
    wp_p = np.concatenate([_f64(wp).reshape(-1)[: max(n - 1, 0)], [0.0]])
    x = np.empty(n)
    rc = _load().orc_chain_pq_brute(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(wm_p), _ptr(wp_p), _ptr(x))
    if rc != 0:
        raise ValueError("orc_chain_pq_brute: n must be in [1, 6]")
    return x


def pq_objective(a, b, c, d, wm, wp, x) -> float:
    """Objective of the Sec. 4.2 chain problem at x."""
    a, b, c, d, x = _f64(a), _f64(b), _f64(c), _f64(d), _f64(x)
    n = a.shape[0]
    wm_p = np.concatenate([_f64(wm).reshape(-1)[: max(n - 1, 0)], [0.0]])
    wp_p = np.concatenate([_f64(wp).reshape(-1)[: max(n - 1, 0)], [0.0]])
    return float(_load().orc_pq_objective(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(wm_p), _ptr(wp_p),
                                          _ptr(x)))


def chain_prox_l1(y, d, w=None, w_scalar: float = 0.0, c=None, c_scalar: float = 1.0, threads: int = 0,
                  counts: bool = False):
    """TV-l1 chain prox for a batch of chains (rows of y): argmin sum w|dx| +
    sum (x - y)^2/2 + sum c |x - d|.  w, c: arrays shaped like y (slot i of w =
    edge (i, i+1), the last slot ignored) or None for the scalars."""
    y = _f64(y)
    squeeze = y.ndim == 1
    y2 = y.reshape(1, -1) if squeeze else y
    C, n = y2.shape
    d2 = _f64(d).reshape(C, n)
    w2 = None if w is None else _f64(w).reshape(C, n)
    c2 = None if c is None else _f64(c).reshape(C, n)
    x = np.empty_like(y2)
    cnt = (_Counts * max(C, 1))() if counts else None
    rc = _load().orc_chain_prox_l1(C, n, 1, n, _ptr(y2), _ptr(d2), _ptr(w2), float(w_scalar), _ptr(c2),
                                   float(c_scalar), _ptr(x), cnt, int(threads))
    if rc != 0:
        raise ValueError("orc_chain_prox_l1: invalid argument")
    out = x.reshape(-1) if squeeze else x
    if counts:
        stats = np.array([[q.pushes, q.pops, q.max_breakpoints] for q in cnt[:C]], dtype=np.int64)
        return out, stats
    return out


def chain_brute(a, b, wm, wp):
    """Brute-force minimiser of the Sec. 4.1 objective for n <= 12."""
    a, b = _f64(a), _f64(b)
    n = a.shape[0]
    wm_p = np.concatenate([_f64(wm).reshape(-1), [0.0]])
    wp_p = np.concatenate([_f64(wp).reshape(-1), [0.0]])
    x = np.empty(n)
    rc = _load().orc_chain_brute(n, _ptr(a), _ptr(b), _ptr(wm_p), _ptr(wp_p), _ptr(x))
    if rc != 0:
        raise ValueError("orc_chain_brute: n must be in [1, 12]")
    return x


def rof1d_objective(y, w, x, w_scalar: float = 0.0) -> float:
    """Objective of eq. (1D-ROF) for one chain."""
    y, x = _f64(y), _f64(x)
    wa = None if w is None else _f64(w)
    return float(_load().orc_rof1d_objective(y.shape[0], _ptr(y), _ptr(wa), float(w_scalar), _ptr(x)))


def chain_adjoint(x, g, scalar_w: bool = False, threads: int = 0):
    """Gradient of <g, x(y, w)>: returns (dy, dw) where dw has the shape of x
    (slot i = edge (i, i+1), last slot 0), or a per-chain sum when
    ``scalar_w``."""
    x, g = _f64(x), _f64(g)
    squeeze = x.ndim == 1
    x2 = x.reshape(1, -1) if squeeze else x
    g2 = g.reshape(x2.shape)
    C, n = x2.shape
    dy = np.empty_like(x2)
    dw = None if scalar_w else np.empty_like(x2)
    dws = np.empty(C) if scalar_w else None
    _load().orc_chain_adjoint(C, n, 1, n, _ptr(x2), _ptr(g2), _ptr(dy), _ptr(dw), _ptr(dws),
                              int(threads))
    if squeeze:
        return dy.reshape(-1), (dws[0] if scalar_w else dw.reshape(-1))
    return dy, (dws if scalar_w else dw)


def tv2d(f, lam: float, tau0: float = 1.0, max_iter: int = 200, gap_tol: float = 0.0,
         threads: int = 0):
    """Sec. 5.1 ROF solve.  Returns (x, gap_hist, (P, D, gap_norm), iters)."""
    f = _f64(f)
    H, W = f.shape
    x = np.empty_like(f)
    hist = np.zeros(max(int(max_iter), 1))
    out3 = np.zeros(3)
    k = _load().orc_tv2d(H, W, _ptr(f), float(lam), float(tau0), int(max_iter), float(gap_tol),
                         _ptr(x), _ptr(hist), _ptr(out3), int(threads))
    if k < 0:
        raise ValueError("orc_tv2d: invalid argument")
    return x, hist[:k].copy(), (float(out3[0]), float(out3[1]), float(out3[2])), int(k)


def rof2d_objective(f, lam: float, x) -> float:
    """Primal ROF objective lam (TV_h + TV_v)(x) + |x - f|^2 / 2."""
    f, x = _f64(f), _f64(x)
    H, W = f.shape
    return float(_load().orc_rof2d_objective(H, W, _ptr(f), float(lam), _ptr(x)))


def tvl1_2d_objective(f, lam: float, x) -> float:
    """TV-l1 objective lam (TV_h + TV_v)(x) + |x - f|_1."""
    f, x = _f64(f), _f64(x)
    H, W = f.shape
    return float(_load().orc_tvl1_2d_objective(H, W, _ptr(f), float(lam), _ptr(x)))


def tv2d_l1(f, lam: float, tau: float = 1.0, max_iter: int = 200, threads: int = 0):
    """Sec. 5.2 TV-l1 by row/column decomposition, eq. (pd) with constant steps
    tau, sigma = 1/tau, theta = 1.  Returns (x, energy history)."""
    f = _f64(f)
    H, W = f.shape
    x = np.empty_like(f)
    hist = np.empty(max(max_iter, 1))
    k = _load().orc_tv2d_l1(H, W, _ptr(f), float(lam), float(tau), int(max_iter), _ptr(x), _ptr(hist), int(threads))
    if k < 0:
        raise ValueError("orc_tv2d_l1: invalid argument")
    return x, hist[:k].copy()


def _tree_args(parent, a, b, c, d, wm, wp):
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    n = parent.shape[0]
    return n, parent, _f64(a), _f64(b), _f64(c), _f64(d), _f64(wm), _f64(wp)


def tree_pq(parent, a, b, c, d, wm, wp):
    """Algorithm 2 on a forest (parent[i] > i, -1 at roots) with unaries
    a_i x^2/2 - b_i x + c_i |x - d_i| and edge slopes (wm[i], wp[i]) on the edge
    from i to its parent (z = x_parent - x_i).  Returns (x, lam_lo, lam_hi)."""
    n, parent, a, b, c, d, wm, wp = _tree_args(parent, a, b, c, d, wm, wp)
    x, llo, lhi = np.empty(n), np.empty(n), np.empty(n)
    rc = _load().orc_tree_pq(n, _ptr(parent), _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(wm), _ptr(wp), _ptr(x),
                             _ptr(llo), _ptr(lhi))
    if rc != 0:
        raise ValueError("orc_tree_pq: parent[i] must exceed i (or be -1)")
    return x, llo, lhi


def tree_pq_brute(parent, a, b, c, d, wm, wp):
    """Brute-force minimiser of the forest objective for n <= 6."""
    n, parent, a, b, c, d, wm, wp = _tree_args(parent, a, b, c, d, wm, wp)
    x = np.empty(n)
    rc = _load().orc_tree_pq_brute(n, _ptr(parent), _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(wm), _ptr(wp), _ptr(x))
    if rc != 0:
        raise ValueError("orc_tree_pq_brute: n must be in [1, 6]")
    return x


def tree_pq_objective(parent, a, b, c, d, wm, wp, x) -> float:
    n, parent, a, b, c, d, wm, wp = _tree_args(parent, a, b, c, d, wm, wp)
    return float(_load().orc_tree_pq_objective(n, _ptr(parent), _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(wm),
                                               _ptr(wp), _ptr(_f64(x))))


def _nc_args(uoff, ulam, uslope, w, C):
    uoff = np.ascontiguousarray(uoff, dtype=np.int64)
    n = uoff.size - 1
    ulam, uslope = _f64(ulam), _f64(uslope)
    if ulam.size != uoff[-1] or uslope.size != uoff[-1] + n:
        raise ValueError("unary arrays do not match the offsets")
    w = _f64(np.broadcast_to(w, (max(n - 1, 0),)))
    C = _f64(np.broadcast_to(C, (max(n - 1, 0),)))
    return n, uoff, ulam, uslope, w, C


def nc_chain(uoff, ulam, uslope, w, C):
    """Sec. 3 on a chain: piecewise-linear unaries (node i: breakpoints
    ulam[uoff[i]:uoff[i+1]], slopes uslope[uoff[i]+i : uoff[i+1]+i+1]) and
    truncated TV min(w_e |x_{e+1} - x_e|, C_e) (C_e = inf: plain TV).
    Returns (x, largest number of message breakpoints)."""
    n, uoff, ulam, uslope, w, C = _nc_args(uoff, ulam, uslope, w, C)
    x = np.empty(n)
    mb = ctypes.c_int64(0)
    rc = _load().orc_nc_chain(n, _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(w), _ptr(C), _ptr(x), ctypes.byref(mb))
    if rc != 0:
        raise ValueError("orc_nc_chain: invalid input (%d)" % rc)
    return x, int(mb.value)


def nc_energy(uoff, ulam, uslope, w, C, x) -> float:
    """sum_i f_i(x_i) + sum_e min(w_e |x_{e+1} - x_e|, C_e), with f_i(first breakpoint) = 0."""
    n, uoff, ulam, uslope, w, C = _nc_args(uoff, ulam, uslope, w, C)
    x = _f64(x)
    return float(_load().orc_nc_energy(n, _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(w), _ptr(C), _ptr(x)))


def nc_brute(uoff, ulam, uslope, w, C):
    """Exact minimum energy and a minimiser for n <= 5 (vertex candidates, Viterbi)."""
    n, uoff, ulam, uslope, w, C = _nc_args(uoff, ulam, uslope, w, C)
    x = np.empty(n)
    e = ctypes.c_double(0.0)
    rc = _load().orc_nc_brute(n, _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(w), _ptr(C), _ptr(x), ctypes.byref(e))
    if rc != 0:
        raise ValueError("orc_nc_brute: invalid input (%d)" % rc)
    return float(e.value), x


def _ncg_args(uoff, ulam, uslope, poff, alpha, C, side):
    uoff = np.ascontiguousarray(uoff, dtype=np.int64)
    n = uoff.size - 1
    ulam, uslope = _f64(ulam), _f64(uslope)
    if ulam.size != uoff[-1] or uslope.size != uoff[-1] + n:
        raise ValueError("unary arrays do not match the offsets")
    poff = np.ascontiguousarray(poff, dtype=np.int64)
    alpha, C = _f64(alpha), _f64(C)
    side = np.ascontiguousarray(side, dtype=np.int32)
    if poff.size != n + 1 or not (alpha.size == C.size == side.size == poff[-1]):
        raise ValueError("piece arrays do not match the offsets")
    return n, uoff, ulam, uslope, poff, alpha, C, side


def ncg_chain(uoff, ulam, uslope, poff, alpha, C, side):
    """Sec. 3, Extensions (i), on a chain: unaries as for nc_chain; the
    pairwise term of edge e is the minimum of its pieces k in
    [poff[e], poff[e+1]), alpha[k] |z| + C[k] on the side side[k] (+1: z > 0,
    -1: z < 0) of z = x_{e+1} - x_e, and 0 at z = 0.  Returns (x, largest
    number of message breakpoints)."""
    n, uoff, ulam, uslope, poff, alpha, C, side = _ncg_args(uoff, ulam, uslope, poff, alpha, C, side)
    x = np.empty(n)
    mb = ctypes.c_int64(0)
    rc = _load().orc_ncg_chain(n, _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(poff), _ptr(alpha), _ptr(C),
                               _ptr(side), _ptr(x), ctypes.byref(mb))
    if rc != 0:
        raise ValueError("orc_ncg_chain: invalid input (%d)" % rc)
    return x, int(mb.value)


def ncg_energy(uoff, ulam, uslope, poff, alpha, C, side, x) -> float:
    n, uoff, ulam, uslope, poff, alpha, C, side = _ncg_args(uoff, ulam, uslope, poff, alpha, C, side)
    x = _f64(x)
    return float(_load().orc_ncg_energy(n, _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(poff), _ptr(alpha), _ptr(C),
                                        _ptr(side), _ptr(x)))


def ncg_brute(uoff, ulam, uslope, poff, alpha, C, side):
    """Exact minimum energy and a minimiser for n <= 6 (unary breakpoints, Viterbi)."""
    n, uoff, ulam, uslope, poff, alpha, C, side = _ncg_args(uoff, ulam, uslope, poff, alpha, C, side)
    x = np.empty(n)
    e = ctypes.c_double(0.0)
    rc = _load().orc_ncg_brute(n, _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(poff), _ptr(alpha), _ptr(C),
                               _ptr(side), _ptr(x), ctypes.byref(e))
    if rc != 0:
        raise ValueError("orc_ncg_brute: invalid input (%d)" % rc)
    return float(e.value), x


def ncg_tree(parent, uoff, ulam, uslope, poff, alpha, C, side):
    """ncg_chain's pairwise terms on a forest (parent[i] > i, -1 at roots): the
    pieces [poff[i], poff[i+1]) belong to the edge from i to its parent, with
    z = x_parent - x_i.  Returns (x, largest number of message breakpoints)."""
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    n, uoff, ulam, uslope, poff, alpha, C, side = _ncg_args(uoff, ulam, uslope, poff, alpha, C, side)
    if parent.size != n:
        raise ValueError("parent must hold one entry per node")
    x = np.empty(n)
    mb = ctypes.c_int64(0)
    rc = _load().orc_ncg_tree(n, _ptr(parent), _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(poff), _ptr(alpha),
                              _ptr(C), _ptr(side), _ptr(x), ctypes.byref(mb))
    if rc != 0:
        raise ValueError("orc_ncg_tree: invalid input (%d)" % rc)
    return x, int(mb.value)


def ncg_tree_energy(parent, uoff, ulam, uslope, poff, alpha, C, side, x) -> float:
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    n, uoff, ulam, uslope, poff, alpha, C, side = _ncg_args(uoff, ulam, uslope, poff, alpha, C, side)
    x = _f64(x)
    return float(_load().orc_ncg_tree_energy(n, _ptr(parent), _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(poff),
                                             _ptr(alpha), _ptr(C), _ptr(side), _ptr(x)))


def ncg_tree_brute(parent, uoff, ulam, uslope, poff, alpha, C, side) -> float:
    """Exact minimum energy of a forest of n <= 6 nodes (unary breakpoints, min-sum)."""
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    n, uoff, ulam, uslope, poff, alpha, C, side = _ncg_args(uoff, ulam, uslope, poff, alpha, C, side)
    e = ctypes.c_double(0.0)
    rc = _load().orc_ncg_tree_brute(n, _ptr(parent), _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(poff), _ptr(alpha),
                                    _ptr(C), _ptr(side), ctypes.byref(e))
    if rc != 0:
        raise ValueError("orc_ncg_tree_brute: invalid input (%d)" % rc)
    return float(e.value)


def grid_unaries(cost, d0: float, dd: float, steep: float):
    """Piecewise-linear unaries through the costs of a cost volume cost[..., D]
    at the levels d0 + k dd (k = 0..D-1), slopes -steep / +steep outside.
    Returns (uoff, ulam, uslope) in the layout of nc_chain, pixels in C order."""
    cost = np.asarray(cost, dtype=np.float64)
    D = cost.shape[-1]
    c2 = cost.reshape(-1, D)
    n = c2.shape[0]
    lev = d0 + dd * np.arange(D)
    sl = np.empty((n, D + 1))
    sl[:, 0] = -steep
    sl[:, D] = steep
    sl[:, 1:D] = np.diff(c2, axis=1) / dd
    return (np.arange(n + 1, dtype=np.int64) * D), np.tile(lev, n), sl.reshape(-1)


def nc2d_pd(cost, d0: float, dd: float, steep: float, w_h, w_v, C: float, tau0: float, iters: int):
    """Sec. 5.3: TV^C_h + TV^C_v + sum f_i on an H x W grid (f_i piecewise-linear
    through cost[i, j, :] at d0 + k dd), by the Lagrangian splitting
    min_{x_h, x_v} max_y Psi_h(x_h) + Psi_v(x_v) + <x_h - x_v, y>,
    Psi = TV^C + f / 2, with the primal-dual iteration
      x_h <- prox_{tau Psi_h}(x_h - tau ybar),  x_v <- prox_{tau Psi_v}(x_v + tau ybar),
      y <- y + sigma (x_h - x_v),  ybar <- 2 y_new - y_old,
    tau_k = tau0 / k, sigma_k = 1 / (2 tau_k) (L^2 = 2), theta = 1.  Each prox
    is the exact minimiser, over every row (or column) chain, of Psi plus the
    piecewise-linear interpolant on the levels of |x - z|^2 / (2 tau) (Sec. 5.3),
    solved by nc_chain.  w_h: H x (W-1) horizontal edge weights, w_v: (H-1) x W.
    Starts from x_h = x_v = the per-pixel minimiser of f, y = 0.  Returns
    (x_h, x_v, energies of x_h after each iteration)."""
    cost = np.asarray(cost, dtype=np.float64)
    H, W, D = cost.shape
    lev = d0 + dd * np.arange(D)
    uoff, ulam, usl = grid_unaries(cost, d0, dd, steep)
    usl = usl.reshape(H, W, D + 1)
    x0 = lev[np.argmin(cost, axis=2)]
    xh, xv = x0.copy(), x0.copy()
    y = np.zeros((H, W))
    ybar = y.copy()
    w_h = np.broadcast_to(np.asarray(w_h, dtype=np.float64), (H, W - 1))
    w_v = np.broadcast_to(np.asarray(w_v, dtype=np.float64), (H - 1, W))

    def prox(z, tau, horizontal):
        # unary of pixel i: f_i / 2 + PL interpolant of (x - z_i)^2 / (2 tau) on the levels
        q = (lev[None, None, :-1] + lev[None, None, 1:] - 2 * z[:, :, None]) / (2 * tau)  # quad slopes between levels
        sl = 0.5 * usl.copy()
        sl[:, :, 1:D] += q
        sl[:, :, 0] += (lev[0] - z) / tau        # the quadratic's slope at the ends, added to the steep sides
        sl[:, :, D] += (lev[-1] - z) / tau
        sl[:, :, 0] = np.minimum(sl[:, :, 0], 0.0)
        sl[:, :, D] = np.maximum(sl[:, :, D], 0.0)
        out = np.empty((H, W))
        if horizontal:
            for r in range(H):
                o = np.arange(W + 1, dtype=np.int64) * D
                out[r], _ = nc_chain(o, np.tile(lev, W), sl[r].reshape(-1), w_h[r], np.full(W - 1, C))
        else:
            for c in range(W):
                o = np.arange(H + 1, dtype=np.int64) * D
                out[:, c], _ = nc_chain(o, np.tile(lev, H), sl[:, c].reshape(-1), w_v[:, c], np.full(H - 1, C))
        return out

    energies = []
    for k in range(1, iters + 1):
        tau = tau0 / k
        sigma = 1.0 / (2.0 * tau)
        xh = prox(xh - tau * ybar, tau, True)
        xv = prox(xv + tau * ybar, tau, False)
        y_new = y + sigma * (xh - xv)
        ybar = 2 * y_new - y
        y = y_new
        energies.append(nc2d_energy(cost, d0, dd, steep, w_h, w_v, C, xh))
    return xh, xv, np.array(energies)


def nc2d_energy(cost, d0: float, dd: float, steep: float, w_h, w_v, C: float, x) -> float:
    """TV^C_h + TV^C_v + sum f_i at x (f_i through the costs, as in nc2d_pd; the
    absolute cost values are used, not nc_chain's f(first level) = 0)."""
    cost = np.asarray(cost, dtype=np.float64)
    H, W, D = cost.shape
    lev = d0 + dd * np.arange(D)
    x = np.asarray(x, dtype=np.float64)
    e = 0.0
    for i in range(H):
        for j in range(W):
            z = x[i, j]
            c = cost[i, j]
            if z <= lev[0]:
                e += c[0] - steep * (z - lev[0])
            elif z >= lev[-1]:
                e += c[-1] + steep * (z - lev[-1])
            else:
                k = min(int((z - d0) // dd), D - 2)
                t = (z - lev[k]) / dd
                e += c[k] * (1 - t) + c[k + 1] * t
    w_h = np.broadcast_to(np.asarray(w_h, dtype=np.float64), (H, W - 1))
    w_v = np.broadcast_to(np.asarray(w_v, dtype=np.float64), (H - 1, W))
    e += np.minimum(w_h * np.abs(np.diff(x, axis=1)), C).sum()
    e += np.minimum(w_v * np.abs(np.diff(x, axis=0)), C).sum()
    return float(e)


def _nc_tree_args(parent, uoff, ulam, uslope, w, C):
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    n = parent.size
    uoff = np.ascontiguousarray(uoff, dtype=np.int64)
    ulam, uslope = _f64(ulam), _f64(uslope)
    if uoff.size != n + 1 or ulam.size != uoff[-1] or uslope.size != uoff[-1] + n:
        raise ValueError("unary arrays do not match the offsets")
    w = _f64(np.broadcast_to(w, (n,)))
    C = _f64(np.broadcast_to(C, (n,)))
    return n, parent, uoff, ulam, uslope, w, C


def nc_tree(parent, uoff, ulam, uslope, w, C):
    """Sec. 3 on a forest (parent[i] > i, -1 at roots; w[i], C[i] on the edge
    from i to its parent): x and the largest number of message breakpoints."""
    n, parent, uoff, ulam, uslope, w, C = _nc_tree_args(parent, uoff, ulam, uslope, w, C)
    x = np.empty(n)
    mb = ctypes.c_int64(0)
    rc = _load().orc_nc_tree(n, _ptr(parent), _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(w), _ptr(C), _ptr(x),
                             ctypes.byref(mb))
    if rc != 0:
        raise ValueError("orc_nc_tree: invalid input (%d)" % rc)
    return x, int(mb.value)


def nc_tree_energy(parent, uoff, ulam, uslope, w, C, x) -> float:
    n, parent, uoff, ulam, uslope, w, C = _nc_tree_args(parent, uoff, ulam, uslope, w, C)
    x = _f64(x)
    return float(_load().orc_nc_tree_energy(n, _ptr(parent), _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(w),
                                            _ptr(C), _ptr(x)))


def nc_tree_brute(parent, uoff, ulam, uslope, w, C) -> float:
    """Exact minimum energy of a forest of n <= 5 nodes (vertex candidates, min-sum)."""
    n, parent, uoff, ulam, uslope, w, C = _nc_tree_args(parent, uoff, ulam, uslope, w, C)
    e = ctypes.c_double(0.0)
    rc = _load().orc_nc_tree_brute(n, _ptr(parent), _ptr(uoff), _ptr(ulam), _ptr(uslope), _ptr(w), _ptr(C),
                                   ctypes.byref(e))
    if rc != 0:
        raise ValueError("orc_nc_tree_brute: invalid input (%d)" % rc)
    return float(e.value)
