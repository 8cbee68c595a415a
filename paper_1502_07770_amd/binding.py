"""ctypes binding of libtvchain.so (argument marshalling only).

Every computation runs in the HIP kernels of ``libtvchain.so``; this module
only converts torch tensors (device memory) and the current HIP stream into
the C ABI declared in ``include/tvchain.h``.  There is no CPU fallback: if the
library is missing or no GPU is visible, calls raise ``TvChainError``.

Functions mirror the C entry points:

* ``chain_prox(y, w, dim)``            -> tv_chain_prox (eq. (1D-ROF), Sec. 4.1)
* ``chain_prox_multi(items, w)``      -> tv_chain_prox_multi (several batches, one launch)
* ``autotune_chain_prox(items, w)``   -> tv_chain_prox_autotune (plan per shape)
* ``chain_prox_backward(x, g, ...)``   -> tv_chain_prox_backward
* ``prox(y, w, dim)``                  -> autograd-aware chain prox
* ``tv2d(f, lam, ...)``                -> tv2d_solve (Sec. 5.1)
* ``tv2d_batched(images, lams, ...)``  -> tv2d_solve_batched
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Union

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtvchain.so")

TV_OK = 0
TV_ERR_INVALID_ARG = 1
TV_ERR_WORKSPACE = 2
TV_ERR_NO_DEVICE = 3
TV_ERR_HIP = 4
TV_ERR_NOT_CONVERGED = 5
TV_ERR_NONFINITE = 6
TV_F32 = 0
TV_F64 = 1


class TvChainError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        msg = "%s: status %d (%s)" % (what or "tvchain", self.status, status_string(self.status))
        super().__init__(msg)


class ChainLayout(ctypes.Structure):
    _fields_ = [("num_chains", ctypes.c_int64), ("length", ctypes.c_int64),
                ("elem_stride", ctypes.c_int64), ("chain_stride", ctypes.c_int64),
                ("offsets", ctypes.c_void_p)]


class Tv2dOptions(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("gap_every", ctypes.c_int), ("gap_tol", ctypes.c_double),
                ("tau0", ctypes.c_double), ("resume", ctypes.c_int), ("gap_history", ctypes.c_void_p),
                ("use_graph", ctypes.c_int), ("lookahead", ctypes.c_int)]


# Chunks of gap_every iterations the host may enqueue ahead of the device in a
# solve that can stop early (tv2d_options.lookahead); these calls read their
# stats back at once, so the host waits for the device anyway.
DEFAULT_LOOKAHEAD = 4


def _lookahead(lookahead: Optional[int], gap_tol: float) -> int:
    if lookahead is None:
        return DEFAULT_LOOKAHEAD if gap_tol > 0.0 else 0
    return int(lookahead)


class Tuning(ctypes.Structure):
    _fields_ = [("target_lanes", ctypes.c_int64), ("min_segment", ctypes.c_int64), ("halo", ctypes.c_int64),
                ("ring_slots", ctypes.c_int64)]


class TuningResult(ctypes.Structure):
    _fields_ = [("segment_length", ctypes.c_int64), ("halo", ctypes.c_int64), ("ring_slots", ctypes.c_int),
                ("candidates", ctypes.c_int), ("ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {"segment_length": int(self.segment_length), "halo": int(self.halo),
                "ring_slots": int(self.ring_slots), "candidates": int(self.candidates), "ms": float(self.ms)}


class Tv2dStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("gap_norm", ctypes.c_double),
                ("primal", ctypes.c_double), ("dual", ctypes.c_double), ("device_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {"iters": int(self.iters), "status": int(self.status), "gap_norm": float(self.gap_norm),
                "primal": float(self.primal), "dual": float(self.dual), "device_ms": float(self.device_ms)}


def _stats_buffer(n: int, device) -> torch.Tensor:
    """Device memory for n tv2d_stats records (the 2D solves write them from
    their last kernel)."""
    return torch.empty(n * ctypes.sizeof(Tv2dStats), dtype=torch.uint8, device=device)


def _read_stats(buf: torch.Tensor, n: int) -> list:
    """The n records of a stats buffer, read after the work queued before on
    the current stream (the copy to the host waits for it)."""
    raw = buf.cpu().numpy().tobytes()
    return [r.as_dict() for r in (Tv2dStats * n).from_buffer_copy(raw)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SIG = {
    "tv_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tv_chain_prox_workspace": (ctypes.c_size_t, [_P, ctypes.c_int]),
    "tv_chain_prox": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_double, _P, _P, ctypes.c_size_t, _P]),
    "tv_chain_prox_noalloc": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_double, _P, _P]),
    "tv_chain_prox_backward_workspace": (ctypes.c_size_t, [_P, ctypes.c_int]),
    "tv_chain_prox_backward": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, ctypes.c_int, _P,
                                              ctypes.c_size_t, _P]),
    "tv_chain_prox_multi_workspace": (ctypes.c_size_t, [ctypes.c_int, _P, ctypes.c_int]),
    "tv_chain_prox_multi": (ctypes.c_int, [ctypes.c_int, _P, ctypes.c_int, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                           _P]),
    "tv_chain_prox_autotune": (ctypes.c_int, [ctypes.c_int, _P, ctypes.c_int, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                              _P, _P]),
    "tv_autotune_clear": (None, []),
    "tv_chain_prox_l1_workspace": (ctypes.c_size_t, [_P, ctypes.c_int]),
    "tv_chain_prox_l1": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_double, _P, ctypes.c_double, _P,
                                        _P, ctypes.c_size_t, _P]),
    "tv_chain_prox_l1_autotune": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_double, _P,
                                                 ctypes.c_double, _P, _P, ctypes.c_size_t, _P, _P]),
    "tv2d_l1_workspace": (ctypes.c_size_t, [_I64, _I64, ctypes.c_int]),
    "tv2d_l1_solve": (ctypes.c_int, [ctypes.c_int, _P, _I64, _I64, _I64, ctypes.c_double, _P, _P, _P, _P,
                                     ctypes.c_size_t, _P]),
    "tv2d_l1_autotune": (ctypes.c_int, [ctypes.c_int, _P, _I64, _I64, _I64, ctypes.c_double, ctypes.c_double, _P,
                                        ctypes.c_size_t, _P, _P, _P]),
    "tv_chain_nc_workspace": (ctypes.c_size_t, [_I64, _I64, _I64, _I64]),
    "tv_chain_nc": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _I64, _I64, _P,
                                   ctypes.c_size_t, _P]),
    "tv_chain_nc_concave_workspace": (ctypes.c_size_t, [_I64, _I64, _I64, _I64, _I64]),
    "tv_chain_nc_concave": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                           _I64, _I64, _P, ctypes.c_size_t, _P]),
    "tv_tree_nc_concave_workspace": (ctypes.c_size_t, [_I64, _I64, _I64, _I64, _I64, _I64]),
    "tv_tree_nc_concave": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                          _I64, _I64, _I64, _P, ctypes.c_size_t, _P]),
    "tv_tree_nc_workspace": (ctypes.c_size_t, [_I64, _I64, _I64, _I64, _I64]),
    "tv_tree_nc": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _I64, _I64, _P,
                                  ctypes.c_size_t, _P]),
    "tv2d_nc_workspace": (ctypes.c_size_t, [_I64, _I64, _I64, _I64, _I64]),
    "tv2d_nc_solve": (ctypes.c_int, [ctypes.c_int, _P, _I64, _I64, _I64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, _P, ctypes.c_double, _P, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, _P, _I64, _I64, _P, ctypes.c_size_t, _P]),
    "tv_tree_dp_workspace": (ctypes.c_size_t, [_I64, _I64]),
    "tv_tree_dp": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                  _P]),
    "tv_chain_dp_workspace": (ctypes.c_size_t, [_P, ctypes.c_int]),
    "tv_chain_dp": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "tv_chain_dp_autotune": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, _P]),
    "tv2d_autotune": (ctypes.c_int, [ctypes.c_int, _P, _I64, _I64, _I64, ctypes.c_double, ctypes.c_double, _P,
                                     ctypes.c_size_t, _P, _P, _P]),
    "tv2d_batched_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, ctypes.c_double, _P,
                                             ctypes.c_size_t, _P, _P, _P]),
    "tv_set_tuning": (ctypes.c_int, [_P]),
    "tv_get_tuning": (ctypes.c_int, [_P]),
    "tv_chain_prox_segment_length": (_I64, [_P]),
    "tv2d_workspace": (ctypes.c_size_t, [_I64, _I64, ctypes.c_int]),
    "tv2d_solve": (ctypes.c_int, [ctypes.c_int, _P, _I64, _I64, _I64, ctypes.c_double, _P, _P, _P, _P,
                                  ctypes.c_size_t, _P]),
    "tv2d_batched_workspace": (ctypes.c_size_t, [ctypes.c_int, _P, _P, ctypes.c_int]),
    "tv2d_solve_batched": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                          ctypes.c_size_t, _P]),
}


def load() -> ctypes.CDLL:
    """Load libtvchain.so; raises TvChainError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TvChainError(TV_ERR_NO_DEVICE, "libtvchain.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIG.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().tv_status_string(int(status)).decode()
    except Exception:  # library missing: still give a readable message
        return "status %d" % status


def _check(status: int, what: str) -> None:
    if status != TV_OK:
        raise TvChainError(status, what)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return TV_F32
    if t.dtype == torch.float64:
        return TV_F64
    raise TypeError("tvchain supports float32 and float64 tensors, got %s" % t.dtype)


def _require_gpu(*ts: torch.Tensor) -> None:
    for t in ts:
        if t is not None and not t.is_cuda:
            raise TvChainError(TV_ERR_INVALID_ARG, "tvchain tensors must live on the GPU")


def _stream_ptr(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def get_tuning() -> dict:
    t = Tuning()
    _check(load().tv_get_tuning(ctypes.byref(t)), "tv_get_tuning")
    return {"target_lanes": int(t.target_lanes), "min_segment": int(t.min_segment), "halo": int(t.halo),
            "ring_slots": int(t.ring_slots)}


def set_tuning(target_lanes: Optional[int] = None, min_segment: Optional[int] = None,
               halo: Optional[int] = None, ring_slots: Optional[int] = None) -> None:
    """Set the process-wide segmentation of chain-prox launches (None keeps the
    current value).  Results do not depend on it; only speed does."""
    cur = get_tuning()
    t = Tuning(int(target_lanes if target_lanes is not None else cur["target_lanes"]),
               int(min_segment if min_segment is not None else cur["min_segment"]),
               int(halo if halo is not None else cur["halo"]),
               int(ring_slots if ring_slots is not None else cur["ring_slots"]))
    _check(load().tv_set_tuning(ctypes.byref(t)), "tv_set_tuning")


def reset_tuning() -> None:
    _check(load().tv_set_tuning(None), "tv_set_tuning")


def segment_length(num_chains: int, length: int) -> int:
    lay = ChainLayout(int(num_chains), int(length), 1, int(length), None)
    return int(load().tv_chain_prox_segment_length(ctypes.byref(lay)))


# ---------------------------------------------------------------------------
# layouts
# ---------------------------------------------------------------------------

def _chain_view(y: torch.Tensor, dim: int):
    """Return (tensor to pass, layout, restore) for chains along ``dim``.

    1-D tensors are one chain.  2-D tensors are passed with their own strides
    (rows: dim=-1/1, columns: dim=0).  Anything else is moved to a contiguous
    (chains, n) view and restored afterwards."""
    if y.dim() == 1:
        y1 = y.contiguous()
        return y1, ChainLayout(1, y1.shape[0], 1, y1.shape[0], None), lambda t: t
    d = dim % y.dim()
    if y.dim() == 2 and y.is_contiguous():
        R, C = y.shape
        if d == 1:
            return y, ChainLayout(R, C, 1, C, None), lambda t: t
        return y, ChainLayout(C, R, C, 1, None), lambda t: t
    moved = torch.movedim(y, d, -1)
    shp = moved.shape
    flat = moved.reshape(-1, shp[-1]).contiguous()
    lay = ChainLayout(flat.shape[0], flat.shape[1], 1, flat.shape[1], None)
    return flat, lay, (lambda t: torch.movedim(t.reshape(shp), -1, d))


def chain_prox(y: torch.Tensor, w: Union[float, torch.Tensor] = 0.0, dim: int = -1,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Exact TV prox of every chain of ``y`` along ``dim`` (eq. (1D-ROF)).

    ``w`` is a float (one weight for every edge) or a tensor shaped like ``y``
    whose entry at node i is the weight of edge (i, i+1) along ``dim``."""
    _require_gpu(y)
    lib = load()
    if y.numel() == 0:
        return torch.empty_like(y) if out is None else out
    wv = None
    w_scalar = 0.0
    if isinstance(w, torch.Tensor):
        _require_gpu(w)
        if w.shape != y.shape or w.dtype != y.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "per-edge w must match y's shape and dtype")
        if w.stride() != y.stride():
            y, w = y.contiguous(), w.contiguous()
        wv, _, _ = _chain_view(w, dim)
    else:
        w_scalar = float(w)
    yv, lay, restore = _chain_view(y, dim)
    xv = torch.empty_like(yv)
    code = _dtype_code(y)
    nbytes = lib.tv_chain_prox_workspace(ctypes.byref(lay), code)
    ws = _workspace(nbytes, y.device)
    st = lib.tv_chain_prox(ctypes.byref(lay), code, _ptr(yv), _ptr(wv), w_scalar, _ptr(xv), _ptr(ws),
                           nbytes, ctypes.c_void_p(_stream_ptr(y.device)))
    _check(st, "tv_chain_prox")
    res = restore(xv)
    if out is not None:
        out.copy_(res)
        return out
    return res


def chain_prox_noalloc(y: torch.Tensor, x: torch.Tensor, w: Union[float, torch.Tensor] = 0.0) -> torch.Tensor:
    """chain_prox of the rows of a contiguous 2D ``y`` into the preallocated ``x``
    through tv_chain_prox_noalloc: the library call allocates nothing (its
    workspace is the library's fixed per-GPU scratch), so it may run where
    allocation is not allowed.  Raises TvChainError(TV_ERR_WORKSPACE) when the
    problem needs more scratch than the library holds."""
    _require_gpu(y, x)
    if y.dim() != 2 or not y.is_contiguous() or x.shape != y.shape or x.dtype != y.dtype or not x.is_contiguous():
        raise TvChainError(TV_ERR_INVALID_ARG, "y and x must be contiguous 2D tensors of one shape and dtype")
    wv, w_scalar = (w, 0.0) if isinstance(w, torch.Tensor) else (None, float(w))
    if wv is not None and (wv.shape != y.shape or wv.dtype != y.dtype or not wv.is_contiguous()):
        raise TvChainError(TV_ERR_INVALID_ARG, "per-edge w must be contiguous and match y")
    lay = ChainLayout(y.shape[0], y.shape[1], 1, y.shape[1], None)
    st = load().tv_chain_prox_noalloc(ctypes.byref(lay), _dtype_code(y), _ptr(y), _ptr(wv), w_scalar, _ptr(x),
                                      ctypes.c_void_p(_stream_ptr(y.device)))
    _check(st, "tv_chain_prox_noalloc")
    return x


def chain_dp(b: torch.Tensor, wm: torch.Tensor, wp: torch.Tensor, a: Optional[torch.Tensor] = None,
             dim: int = -1, out: Optional[torch.Tensor] = None, autotune: bool = False):
    """Sec. 4.1 chain DP with general quadratic unaries and asymmetric weights
    (tv_chain_dp): per chain along ``dim``, the minimiser of
    sum_i a_i x_i^2 / 2 - b_i x_i + sum_e f_e(x_{e+1} - x_e) with
    f_e(z) = wm_e z (z < 0), wp_e z (z >= 0).  ``wm``, ``wp`` (and ``a``, None
    meaning all ones) are shaped like ``b``; entry i along ``dim`` belongs to
    edge (i, i+1).  With ``autotune`` the call times the candidate plans and
    returns (x, chosen plan)."""
    _require_gpu(b, wm, wp, *([a] if a is not None else []))
    lib = load()
    for t in (wm, wp) + ((a,) if a is not None else ()):
        if t.shape != b.shape or t.dtype != b.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "a, wm and wp must match b's shape and dtype")
    if b.numel() == 0:
        x = torch.empty_like(b) if out is None else out
        return (x, None) if autotune else x
    ts = [b, wm, wp] + ([a] if a is not None else [])
    if any(t.stride() != b.stride() for t in ts):
        ts = [t.contiguous() for t in ts]
    views = [_chain_view(t, dim) for t in ts]
    bv, lay, restore = views[0]
    wmv, wpv = views[1][0], views[2][0]
    av = views[3][0] if a is not None else None
    xv = torch.empty_like(bv)
    code = _dtype_code(b)
    nbytes = lib.tv_chain_dp_workspace(ctypes.byref(lay), code)
    ws = _workspace(nbytes, b.device)
    stream = ctypes.c_void_p(_stream_ptr(b.device))
    chosen = None
    if autotune:
        res = TuningResult()
        st = lib.tv_chain_dp_autotune(ctypes.byref(lay), code, _ptr(av), _ptr(bv), _ptr(wmv), _ptr(wpv),
                                      _ptr(xv), _ptr(ws), nbytes, stream, ctypes.byref(res))
        _check(st, "tv_chain_dp_autotune")
        chosen = res.as_dict()
    else:
        st = lib.tv_chain_dp(ctypes.byref(lay), code, _ptr(av), _ptr(bv), _ptr(wmv), _ptr(wpv), _ptr(xv),
                             _ptr(ws), nbytes, stream)
        _check(st, "tv_chain_dp")
    res_x = restore(xv)
    if out is not None:
        out.copy_(res_x)
        res_x = out
    return (res_x, chosen) if autotune else res_x


def chain_prox_l1(y: torch.Tensor, d: torch.Tensor, w: Union[float, torch.Tensor] = 0.0,
                  c: Union[float, torch.Tensor] = 1.0, dim: int = -1,
                  out: Optional[torch.Tensor] = None, autotune: bool = False):
    """TV-l1 chain prox (tv_chain_prox_l1) of every chain along ``dim``:
    argmin sum w|x_{i+1} - x_i| + sum (x - y)^2/2 + sum c|x - d|.  ``w`` and
    ``c`` are floats or tensors shaped like ``y`` (w at node i is the weight of
    edge (i, i+1)).  With ``autotune`` the call times the candidate plans and
    returns (x, chosen plan)."""
    _require_gpu(y, d)
    lib = load()
    if y.numel() == 0:
        return torch.empty_like(y) if out is None else out
    ts = [y, d] + [t for t in (w, c) if isinstance(t, torch.Tensor)]
    for t in ts:
        _require_gpu(t)
        if t.shape != y.shape or t.dtype != y.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "d, w and c must match y's shape and dtype")
    if any(t.stride() != y.stride() for t in ts):
        y, d = y.contiguous(), d.contiguous()
        w = w.contiguous() if isinstance(w, torch.Tensor) else w
        c = c.contiguous() if isinstance(c, torch.Tensor) else c
    yv, lay, restore = _chain_view(y, dim)
    dv = _chain_view(d, dim)[0]
    wv = _chain_view(w, dim)[0] if isinstance(w, torch.Tensor) else None
    cv = _chain_view(c, dim)[0] if isinstance(c, torch.Tensor) else None
    ws_ = 0.0 if wv is not None else float(w)
    cs_ = 0.0 if cv is not None else float(c)
    xv = torch.empty_like(yv)
    code = _dtype_code(y)
    nbytes = lib.tv_chain_prox_l1_workspace(ctypes.byref(lay), code)
    ws = _workspace(nbytes, y.device)
    stream = ctypes.c_void_p(_stream_ptr(y.device))
    chosen = None
    if autotune:
        r = TuningResult()
        st = lib.tv_chain_prox_l1_autotune(ctypes.byref(lay), code, _ptr(yv), _ptr(dv), _ptr(wv), ws_, _ptr(cv), cs_,
                                           _ptr(xv), _ptr(ws), nbytes, stream, ctypes.byref(r))
        _check(st, "tv_chain_prox_l1_autotune")
        chosen = r.as_dict()
    else:
        st = lib.tv_chain_prox_l1(ctypes.byref(lay), code, _ptr(yv), _ptr(dv), _ptr(wv), ws_, _ptr(cv), cs_,
                                  _ptr(xv), _ptr(ws), nbytes, stream)
        _check(st, "tv_chain_prox_l1")
    res = restore(xv)
    if out is not None:
        out.copy_(res)
        res = out
    return (res, chosen) if autotune else res


MAX_CHAIN_BATCHES = 8


def autotune_clear() -> None:
    """Forget every plan chosen by the autotuners."""
    load().tv_autotune_clear()


def _multi_args(items, w):
    if not 1 <= len(items) <= MAX_CHAIN_BATCHES:
        raise TvChainError(TV_ERR_INVALID_ARG, "chain_prox_multi takes 1..%d batches" % MAX_CHAIN_BATCHES)
    ys = [y for y, _ in items]
    _require_gpu(*ys)
    dev, code = ys[0].device, _dtype_code(ys[0])
    if any(y.device != dev or _dtype_code(y) != code for y in ys):
        raise TvChainError(TV_ERR_INVALID_ARG, "chain_prox_multi batches must share dtype and device")
    wl = list(w) if isinstance(w, (list, tuple)) else [float(w)] * len(items)
    views = [_chain_view(y, d) for y, d in items]
    xs = [torch.empty_like(v) for v, _, _ in views]
    nb = len(items)
    lays = (ChainLayout * nb)(*[lay for _, lay, _ in views])
    yp = (ctypes.c_void_p * nb)(*[v.data_ptr() for v, _, _ in views])
    xp = (ctypes.c_void_p * nb)(*[x.data_ptr() for x in xs])
    wsc = (ctypes.c_double * nb)(*[float(v) for v in wl])
    return dev, code, nb, views, xs, lays, yp, xp, wsc


def autotune_chain_prox(items, w: Union[float, list] = 0.0) -> dict:
    """Autotune the launch of these chain batches (tv_chain_prox_autotune): later
    chain_prox / chain_prox_multi calls with the same total number of chains and
    length use the fastest plan.  Returns the chosen plan."""
    lib = load()
    dev, code, nb, views, xs, lays, yp, xp, wsc = _multi_args(items, w)
    nbytes = lib.tv_chain_prox_multi_workspace(nb, lays, code)
    ws = _workspace(nbytes, dev)
    res = TuningResult()
    st = lib.tv_chain_prox_autotune(nb, lays, code, yp, None, wsc, xp, _ptr(ws), nbytes,
                                    ctypes.c_void_p(_stream_ptr(dev)), ctypes.byref(res))
    _check(st, "tv_chain_prox_autotune")
    return res.as_dict()


def chain_prox_multi(items, w: Union[float, list] = 0.0) -> list:
    """Exact TV prox of several batches of chains in one launch
    (tv_chain_prox_multi).  ``items`` is a list of ``(y, dim)`` pairs (one
    dtype, one device); ``w`` is one scalar weight for every batch or a list
    with one per batch.  Returns the outputs in the order of ``items``;
    they are bit-identical to separate ``chain_prox`` calls."""
    lib = load()
    dev, code, nb, views, xs, lays, yp, xp, wsc = _multi_args(items, w)
    nbytes = lib.tv_chain_prox_multi_workspace(nb, lays, code)
    ws = _workspace(nbytes, dev)
    st = lib.tv_chain_prox_multi(nb, lays, code, yp, None, wsc, xp, _ptr(ws), nbytes,
                                 ctypes.c_void_p(_stream_ptr(dev)))
    _check(st, "tv_chain_prox_multi")
    return [restore(x) for x, (_, _, restore) in zip(xs, views)]


def chain_prox_backward(x: torch.Tensor, grad_x: torch.Tensor, dim: int = -1,
                        per_edge_w: bool = False, need_y: bool = True, need_w: bool = True):
    """Adjoint of ``chain_prox``: returns (grad_y, grad_w); grad_w has x's shape
    when ``per_edge_w`` and otherwise holds one sum per chain (shape of x
    without ``dim``), either may be None."""
    _require_gpu(x, grad_x)
    lib = load()
    xv, lay, restore = _chain_view(x, dim)
    gv, lay_g, _ = _chain_view(grad_x.to(x.dtype), dim)
    if (lay_g.elem_stride, lay_g.chain_stride) != (lay.elem_stride, lay.chain_stride):
        xv = xv.contiguous()
        gv = gv.contiguous()
        xv, lay, restore = _chain_view(xv, dim)
        gv, _, _ = _chain_view(gv, dim)
    gy = torch.empty_like(xv) if need_y else None
    if need_w:
        gw = torch.empty_like(xv) if per_edge_w else torch.empty(lay.num_chains, dtype=x.dtype, device=x.device)
    else:
        gw = None
    code = _dtype_code(x)
    nbytes = lib.tv_chain_prox_backward_workspace(ctypes.byref(lay), code)
    ws = _workspace(nbytes, x.device)
    st = lib.tv_chain_prox_backward(ctypes.byref(lay), code, _ptr(xv), _ptr(gv), _ptr(gy), _ptr(gw),
                                    1 if per_edge_w else 0, _ptr(ws), nbytes,
                                    ctypes.c_void_p(_stream_ptr(x.device)))
    _check(st, "tv_chain_prox_backward")
    gy_out = restore(gy) if gy is not None else None
    if gw is not None:
        if per_edge_w:
            gw = restore(gw)
        else:
            d = dim % x.dim()
            shp = list(x.shape)
            del shp[d]
            gw = gw.reshape(shp) if shp else gw.reshape(())
    return gy_out, gw


class _ProxFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, w_t, w_scalar, dim):
        x = chain_prox(y, w_t if w_t is not None else w_scalar, dim)
        ctx.save_for_backward(x)
        ctx.dim = dim
        ctx.per_edge = w_t is not None
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        need_y = ctx.needs_input_grad[0]
        need_w = ctx.per_edge and ctx.needs_input_grad[1]
        gy, gw = chain_prox_backward(x, gx.contiguous(), ctx.dim, per_edge_w=True, need_y=need_y,
                                     need_w=need_w)
        return gy, gw, None, None


def prox(y: torch.Tensor, w: Union[float, torch.Tensor] = 0.0, dim: int = -1) -> torch.Tensor:
    """Differentiable chain prox: gradients flow to ``y`` and, when ``w`` is a
    per-edge tensor, to ``w`` (through the run-structure adjoint)."""
    if isinstance(w, torch.Tensor):
        return _ProxFn.apply(y, w, 0.0, dim)
    return _ProxFn.apply(y, None, float(w), dim)


# ---------------------------------------------------------------------------
# 2D ROF (tv2d_solve)
# ---------------------------------------------------------------------------

class Tv2dSolver:
    """Owns the device workspace of one H x W problem so that solves can be
    resumed (the workspace holds x, y, xbar and the schedule position)."""

    def __init__(self, H: int, W: int, dtype=torch.float32, device="cuda"):
        self.H, self.W = int(H), int(W)
        self.dtype = dtype
        self.device = torch.device(device)
        self.code = _dtype_code(torch.empty(0, dtype=dtype))
        lib = load()
        self.nbytes = int(lib.tv2d_workspace(self.H, self.W, self.code))
        if self.nbytes == 0:
            raise TvChainError(TV_ERR_INVALID_ARG, "tv2d_workspace")
        self.ws = _workspace(self.nbytes, self.device)

    def autotune(self, f: torch.Tensor, lam: float, tau0: float = 1.0) -> dict:
        """Choose the fastest plans of the column and row launches for this
        image size (tv2d_autotune).  Resets the solver state (no resume after
        it).  Returns {"col": plan, "row": plan}."""
        _require_gpu(f)
        if f.shape != (self.H, self.W) or f.dtype != self.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "f must be (%d, %d) %s" % (self.H, self.W, self.dtype))
        if f.stride(1) != 1:
            f = f.contiguous()
        col, row = TuningResult(), TuningResult()
        st = load().tv2d_autotune(self.code, _ptr(f), self.H, self.W, f.stride(0), float(lam), float(tau0),
                                  _ptr(self.ws), self.nbytes, ctypes.c_void_p(_stream_ptr(f.device)),
                                  ctypes.byref(col), ctypes.byref(row))
        _check(st, "tv2d_autotune")
        return {"col": col.as_dict(), "row": row.as_dict()}

    def solve(self, f: torch.Tensor, lam: float, max_iter: int = 200, gap_every: int = 10,
              gap_tol: float = 0.0, tau0: float = 1.0, resume: bool = False,
              gap_history: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
              use_graph: bool = False, lookahead: Optional[int] = None):
        """Run the Sec. 5.1 decomposition.  Returns (x, stats dict).  With
        gap_tol > 0 a solve that stops at max_iter above the tolerance raises
        nothing: stats['status'] says TV_ERR_NOT_CONVERGED.  ``lookahead``:
        tv2d_options.lookahead (default DEFAULT_LOOKAHEAD with gap_tol > 0,
        else 0)."""
        _require_gpu(f)
        if f.shape != (self.H, self.W) or f.dtype != self.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "f must be (%d, %d) %s" % (self.H, self.W, self.dtype))
        if f.stride(1) != 1:
            f = f.contiguous()
        ld = f.stride(0)
        x = out if out is not None else torch.empty((self.H, self.W), dtype=self.dtype, device=f.device)
        if x.stride(1) != 1 or x.stride(0) != ld:
            x = torch.empty_strided((self.H, self.W), (ld, 1), dtype=self.dtype, device=f.device)
        hist_ptr = None
        if gap_history is not None:
            if gap_history.dtype != torch.float64 or not gap_history.is_cuda:
                raise TvChainError(TV_ERR_INVALID_ARG, "gap_history must be a float64 GPU tensor")
            hist_ptr = gap_history.data_ptr()
        opt = Tv2dOptions(int(max_iter), int(gap_every), float(gap_tol), float(tau0), 1 if resume else 0, hist_ptr,
                          1 if use_graph else 0, _lookahead(lookahead, gap_tol))
        sbuf = _stats_buffer(1, f.device)
        st = load().tv2d_solve(self.code, _ptr(f), self.H, self.W, ld, float(lam), _ptr(x), ctypes.byref(opt),
                               _ptr(sbuf), _ptr(self.ws), self.nbytes, ctypes.c_void_p(_stream_ptr(f.device)))
        _check(st, "tv2d_solve")
        info = _read_stats(sbuf, 1)[0]
        if out is not None and x is not out:
            out.copy_(x)
            x = out
        return x, info


def tv2d(f: torch.Tensor, lam: float, max_iter: int = 200, gap_every: int = 10, gap_tol: float = 0.0,
         tau0: float = 1.0, gap_history: Optional[torch.Tensor] = None, use_graph: bool = False,
         lookahead: Optional[int] = None):
    """2D ROF min_x lam (TV_h + TV_v)(x) + |x - f|^2 / 2 by the row/column chain
    decomposition (Sec. 5.1).  Returns (x, stats)."""
    s = Tv2dSolver(f.shape[0], f.shape[1], f.dtype, f.device)
    return s.solve(f, lam, max_iter=max_iter, gap_every=gap_every, gap_tol=gap_tol, tau0=tau0,
                   gap_history=gap_history, use_graph=use_graph, lookahead=lookahead)


def tv2d_batched(images, lams, max_iter: int = 200, gap_every: int = 10, gap_tol: float = 0.0,
                 tau0: float = 1.0, packed: Optional[torch.Tensor] = None, autotune: bool = False,
                 tuned: Optional[dict] = None, use_graph: bool = False, lookahead: Optional[int] = None):
    """Solve many 2D ROF problems of different sizes in one call
    (tv2d_solve_batched).  ``images`` is a list of (H_j, W_j) GPU tensors of one
    dtype (or a list of shapes when ``packed`` holds them back to back);
    ``lams`` the per-image weights.  Each image stops at its own gap_tol.
    ``lookahead`` as for Tv2dSolver.solve.
    Returns (list of x_j views into one packed output, list of stats dicts)."""
    if packed is None:
        _require_gpu(*images)
        dtype = images[0].dtype
        shapes = [tuple(im.shape) for im in images]
        packed = torch.cat([im.reshape(-1) for im in images]).contiguous()
    else:
        _require_gpu(packed)
        dtype = packed.dtype
        shapes = [tuple(s) for s in images]
    n = len(shapes)
    Hs = (ctypes.c_int64 * n)(*[s[0] for s in shapes])
    Ws = (ctypes.c_int64 * n)(*[s[1] for s in shapes])
    offs, o = [], 0
    for s in shapes:
        offs.append(o)
        o += s[0] * s[1]
    Os = (ctypes.c_int64 * n)(*offs)
    Ls = (ctypes.c_double * n)(*[float(v) for v in lams])
    code = _dtype_code(packed)
    lib = load()
    nbytes = int(lib.tv2d_batched_workspace(n, Hs, Ws, code))
    if nbytes == 0:
        raise TvChainError(TV_ERR_INVALID_ARG, "tv2d_batched_workspace")
    ws = _workspace(nbytes, packed.device)
    if autotune:  # choose the launch plans first (tv2d_batched_autotune); the solve below uses them
        col, row = TuningResult(), TuningResult()
        st = lib.tv2d_batched_autotune(code, n, Hs, Ws, Os, Ls, _ptr(packed), float(tau0), _ptr(ws), nbytes,
                                       ctypes.c_void_p(_stream_ptr(packed.device)), ctypes.byref(col),
                                       ctypes.byref(row))
        _check(st, "tv2d_batched_autotune")
        if tuned is not None:
            tuned.update({"col": col.as_dict(), "row": row.as_dict()})
    x = torch.empty_like(packed)
    opt = Tv2dOptions(int(max_iter), int(gap_every), float(gap_tol), float(tau0), 0, None, 1 if use_graph else 0,
                      _lookahead(lookahead, gap_tol))
    sbuf = _stats_buffer(n, packed.device)
    st = lib.tv2d_solve_batched(code, n, Hs, Ws, Os, Ls, _ptr(packed), _ptr(x), ctypes.byref(opt), _ptr(sbuf),
                                _ptr(ws), nbytes, ctypes.c_void_p(_stream_ptr(packed.device)))
    _check(st, "tv2d_solve_batched")
    outs = [x[offs[j]:offs[j] + shapes[j][0] * shapes[j][1]].view(shapes[j]) for j in range(n)]
    return outs, _read_stats(sbuf, n)


def tv2d_l1(f: torch.Tensor, lam: float, max_iter: int = 200, energy_every: int = 10, tau0: float = 1.0,
            energy_history: Optional[torch.Tensor] = None, autotune: bool = False):
    """2D TV-l1, min_x lam (TV_h + TV_v)(x) + |x - f|_1, by the row/column
    decomposition (tv2d_l1_solve, Sec. 5.2).  Returns (x, stats) with
    stats["primal"] the FP64 energy of x; with ``autotune`` the launch plans are
    tuned first and stats["plans"] holds them."""
    _require_gpu(f)
    lib = load()
    H, W = f.shape
    f = f.contiguous()
    code = _dtype_code(f)
    nbytes = lib.tv2d_l1_workspace(H, W, code)
    ws = _workspace(nbytes, f.device)
    stream = ctypes.c_void_p(_stream_ptr(f.device))
    plans = None
    if autotune:
        col, row = TuningResult(), TuningResult()
        _check(lib.tv2d_l1_autotune(code, _ptr(f), H, W, W, float(lam), float(tau0), _ptr(ws), nbytes, stream,
                                    ctypes.byref(col), ctypes.byref(row)), "tv2d_l1_autotune")
        plans = {"col": col.as_dict(), "row": row.as_dict()}
    x = torch.empty_like(f)
    opt = Tv2dOptions(int(max_iter), int(energy_every), 0.0, float(tau0), 0,
                      ctypes.c_void_p(energy_history.data_ptr()) if energy_history is not None else None, 0, 0)
    sbuf = _stats_buffer(1, f.device)
    _check(lib.tv2d_l1_solve(code, _ptr(f), H, W, W, float(lam), _ptr(x), ctypes.byref(opt), _ptr(sbuf),
                             _ptr(ws), nbytes, stream), "tv2d_l1_solve")
    r = _read_stats(sbuf, 1)[0]
    info = {"iters": r["iters"], "status": r["status"], "primal": r["primal"], "device_ms": r["device_ms"]}
    if plans is not None:
        info["plans"] = plans
    return x, info


def tree_dp(parent: torch.Tensor, offsets: torch.Tensor, b: torch.Tensor, wm: torch.Tensor, wp: torch.Tensor,
            a: Optional[torch.Tensor] = None, c: Optional[torch.Tensor] = None,
            d: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Algorithm 2 on a batch of trees (tv_tree_dp): parent (int64, -1 at roots,
    each tree numbered in depth-first post-order), offsets (int64, num_trees + 1
    node ranges), per-node b, wm, wp and optional a, c, d (1-D tensors of one
    float dtype).  Returns x."""
    _require_gpu(parent, offsets, b, wm, wp)
    lib = load()
    if parent.dtype != torch.int64 or offsets.dtype != torch.int64:
        raise TvChainError(TV_ERR_INVALID_ARG, "parent and offsets must be int64")
    ts = [t.contiguous() if t is not None else None for t in (a, b, c, d, wm, wp)]
    for t in ts:
        if t is not None and (t.dtype != b.dtype or t.shape != b.shape):
            raise TvChainError(TV_ERR_INVALID_ARG, "per-node arrays must match b")
    parent, offsets = parent.contiguous(), offsets.contiguous()
    T, N = offsets.numel() - 1, b.numel()
    x = torch.empty_like(ts[1])
    nbytes = lib.tv_tree_dp_workspace(T, N)
    ws = _workspace(nbytes, b.device)
    st = lib.tv_tree_dp(_dtype_code(b), T, N, _ptr(offsets), _ptr(parent), *(_ptr(t) for t in ts), _ptr(x), _ptr(ws),
                        nbytes, ctypes.c_void_p(_stream_ptr(b.device)))
    _check(st, "tv_tree_dp")
    return x


def chain_nc(chain_offsets: torch.Tensor, unary_offsets: torch.Tensor, ulam: torch.Tensor, uslope: torch.Tensor,
             w: torch.Tensor, C: Optional[torch.Tensor] = None, msg_cap: int = 256,
             map_cap: Optional[int] = None) -> torch.Tensor:
    """Sec. 3 non-convex chains (tv_chain_nc): chain_offsets (int64, chains + 1
    node ranges), unary_offsets (int64, nodes + 1; node i has breakpoints
    ulam[unary_offsets[i]:unary_offsets[i+1]] and slopes
    uslope[unary_offsets[i]+i : unary_offsets[i+1]+i+1]), per-node w and C of the
    edge to the next node (C None or inf: plain TV).  msg_cap bounds a
    message's breakpoints (up to 256: a wave per chain, 128 or less: smaller
    LDS and more waves per CU; larger: a lane per chain), map_cap the intervals
    kept per chain (default: 32 per
    node of the longest chain; cost-volume chains need about 8 to 12).  Returns x
    (one value per node)."""
    _require_gpu(chain_offsets, unary_offsets, ulam, uslope, w)
    lib = load()
    if chain_offsets.dtype != torch.int64 or unary_offsets.dtype != torch.int64:
        raise TvChainError(TV_ERR_INVALID_ARG, "offsets must be int64")
    N = unary_offsets.numel() - 1
    ts = [t.contiguous() if t is not None else None for t in (ulam, uslope, w, C)]
    for t in ts:
        if t is not None and t.dtype != ulam.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "float arrays must share one dtype")
    if ts[2].numel() != N or (ts[3] is not None and ts[3].numel() != N):
        raise TvChainError(TV_ERR_INVALID_ARG, "w and C hold one value per node")
    chain_offsets, unary_offsets = chain_offsets.contiguous(), unary_offsets.contiguous()
    nchains = chain_offsets.numel() - 1
    if map_cap is None:
        longest = int((chain_offsets[1:] - chain_offsets[:-1]).max().item()) if nchains > 0 else 1
        map_cap = max(64, 32 * longest)
    x = torch.empty(N, dtype=ulam.dtype, device=ulam.device)
    nbytes = lib.tv_chain_nc_workspace(nchains, N, msg_cap, map_cap)
    if nbytes == 0:
        raise TvChainError(TV_ERR_INVALID_ARG, "tv_chain_nc_workspace")
    ws = _workspace(nbytes, ulam.device)
    st = lib.tv_chain_nc(_dtype_code(ulam), nchains, N, _ptr(chain_offsets), _ptr(unary_offsets),
                         *(_ptr(t) for t in ts), _ptr(x), msg_cap, map_cap, _ptr(ws), nbytes,
                         ctypes.c_void_p(_stream_ptr(ulam.device)))
    _check(st, "tv_chain_nc")
    return x


def chain_nc_concave(chain_offsets: torch.Tensor, unary_offsets: torch.Tensor, ulam: torch.Tensor,
                     uslope: torch.Tensor, piece_offsets: torch.Tensor, piece_alpha: torch.Tensor,
                     piece_C: torch.Tensor, piece_side: torch.Tensor, msg_cap: int = 256,
                     map_cap: Optional[int] = None) -> torch.Tensor:
    """Sec. 3 Extensions (i) (tv_chain_nc_concave): chains as for chain_nc whose
    pairwise term on the edge from node i to i + 1 is the minimum of the pieces
    piece_offsets[i] .. piece_offsets[i+1] - 1, alpha |z| + C on the side
    piece_side (+1: z = x_{i+1} - x_i > 0, -1: z < 0), and 0 at z = 0.
    piece_offsets int64 (nodes + 1), piece_side int32.  msg_cap up to 256: a
    wave per chain (128 or less: smaller LDS), larger: a lane per chain.
    map_cap defaults to 8
    per piece of the chain with the most pieces (at least 64; about 3 per piece
    on 16-level cost chains).  Returns x."""
    _require_gpu(chain_offsets, unary_offsets, ulam, uslope, piece_offsets, piece_alpha, piece_C, piece_side)
    lib = load()
    if chain_offsets.dtype != torch.int64 or unary_offsets.dtype != torch.int64 or \
            piece_offsets.dtype != torch.int64:
        raise TvChainError(TV_ERR_INVALID_ARG, "offsets must be int64")
    if piece_side.dtype != torch.int32:
        raise TvChainError(TV_ERR_INVALID_ARG, "piece_side must be int32")
    N = unary_offsets.numel() - 1
    ts = [t.contiguous() for t in (ulam, uslope, piece_alpha, piece_C)]
    for t in ts:
        if t.dtype != ulam.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "float arrays must share one dtype")
    P = ts[2].numel()
    if piece_offsets.numel() != N + 1 or ts[3].numel() != P or piece_side.numel() != P:
        raise TvChainError(TV_ERR_INVALID_ARG, "piece arrays do not match")
    chain_offsets, unary_offsets = chain_offsets.contiguous(), unary_offsets.contiguous()
    piece_offsets, piece_side = piece_offsets.contiguous(), piece_side.contiguous()
    nchains = chain_offsets.numel() - 1
    if map_cap is None:
        co = chain_offsets.cpu()
        po = piece_offsets.cpu()
        most = int((po[co[1:]] - po[co[:-1]]).max().item()) if nchains > 0 else 1
        map_cap = max(64, 8 * most)
    x = torch.empty(N, dtype=ulam.dtype, device=ulam.device)
    nbytes = lib.tv_chain_nc_concave_workspace(nchains, N, P, msg_cap, map_cap)
    if nbytes == 0:
        raise TvChainError(TV_ERR_INVALID_ARG, "tv_chain_nc_concave_workspace")
    ws = _workspace(nbytes, ulam.device)
    st = lib.tv_chain_nc_concave(_dtype_code(ulam), nchains, N, P, _ptr(chain_offsets), _ptr(unary_offsets),
                                 _ptr(ts[0]), _ptr(ts[1]), _ptr(piece_offsets), _ptr(ts[2]), _ptr(ts[3]),
                                 _ptr(piece_side), _ptr(x), msg_cap, map_cap, _ptr(ws), nbytes,
                                 ctypes.c_void_p(_stream_ptr(ulam.device)))
    _check(st, "tv_chain_nc_concave")
    return x


def tree_nc_concave(parent: torch.Tensor, tree_offsets: torch.Tensor, unary_offsets: torch.Tensor,
                    ulam: torch.Tensor, uslope: torch.Tensor, piece_offsets: torch.Tensor,
                    piece_alpha: torch.Tensor, piece_C: torch.Tensor, piece_side: torch.Tensor,
                    msg_cap: int = 256, map_cap: Optional[int] = None,
                    stack_cap: Optional[int] = None) -> torch.Tensor:
    """Sec. 3 Extensions (i) on trees (tv_tree_nc_concave): the trees of tree_nc
    with the pieces of chain_nc_concave on the edge from each node to its parent
    (z = x_parent - x_i).  Fewer than 1024 trees with msg_cap up to 256 run a
    wave per tree, otherwise a lane per tree.  Defaults: 8 intervals per piece
    of the tree with the
    most pieces (at least 64), room for min(64, largest tree) waiting messages
    of msg_cap breakpoints.  Returns x."""
    _require_gpu(parent, tree_offsets, unary_offsets, ulam, uslope, piece_offsets, piece_alpha, piece_C, piece_side)
    lib = load()
    for t in (parent, tree_offsets, unary_offsets, piece_offsets):
        if t.dtype != torch.int64:
            raise TvChainError(TV_ERR_INVALID_ARG, "parent and offsets must be int64")
    if piece_side.dtype != torch.int32:
        raise TvChainError(TV_ERR_INVALID_ARG, "piece_side must be int32")
    ts = [t.contiguous() for t in (ulam, uslope, piece_alpha, piece_C)]
    for t in ts:
        if t.dtype != ulam.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "float arrays must share one dtype")
    N = parent.numel()
    P = ts[2].numel()
    if unary_offsets.numel() != N + 1 or piece_offsets.numel() != N + 1 or ts[3].numel() != P or \
            piece_side.numel() != P:
        raise TvChainError(TV_ERR_INVALID_ARG, "arrays do not match the nodes")
    parent, tree_offsets = parent.contiguous(), tree_offsets.contiguous()
    unary_offsets, piece_offsets, piece_side = (unary_offsets.contiguous(), piece_offsets.contiguous(),
                                                piece_side.contiguous())
    T = tree_offsets.numel() - 1
    to = tree_offsets.cpu()
    biggest = int((to[1:] - to[:-1]).max().item()) if T > 0 else 1
    if map_cap is None:
        po = piece_offsets.cpu()
        most = int((po[to[1:]] - po[to[:-1]]).max().item()) if T > 0 else 1
        map_cap = max(64, 8 * most)
    if stack_cap is None:
        stack_cap = max(1, min(64, biggest)) * (2 * msg_cap + 1)
    x = torch.empty(N, dtype=ulam.dtype, device=ulam.device)
    nbytes = lib.tv_tree_nc_concave_workspace(T, N, P, msg_cap, map_cap, stack_cap)
    if nbytes == 0:
        raise TvChainError(TV_ERR_INVALID_ARG, "tv_tree_nc_concave_workspace")
    ws = _workspace(nbytes, ulam.device)
    st = lib.tv_tree_nc_concave(_dtype_code(ulam), T, N, P, _ptr(tree_offsets), _ptr(parent), _ptr(unary_offsets),
                                _ptr(ts[0]), _ptr(ts[1]), _ptr(piece_offsets), _ptr(ts[2]), _ptr(ts[3]),
                                _ptr(piece_side), _ptr(x), msg_cap, map_cap, stack_cap, _ptr(ws), nbytes,
                                ctypes.c_void_p(_stream_ptr(ulam.device)))
    _check(st, "tv_tree_nc_concave")
    return x


def tv2d_nc(cost: torch.Tensor, d0: float, dd: float, steep: float, w_h, w_v, C: float, tau0: float, iters: int,
            msg_cap: Optional[int] = None, map_cap: Optional[int] = None) -> torch.Tensor:
    """Sec. 5.3 non-convex 2D (tv2d_nc_solve): cost is an H x W x D tensor of
    unary costs at the levels d0 + k dd; w_h (H x (W-1)) and w_v ((H-1) x W)
    are tensors or floats; C the truncation (inf: plain TV).  Returns x (H x W)."""
    _require_gpu(cost)
    lib = load()
    if cost.dim() != 3:
        raise TvChainError(TV_ERR_INVALID_ARG, "cost must be H x W x D")
    H, W, D = cost.shape
    cost = cost.contiguous()
    wh = w_h.contiguous() if isinstance(w_h, torch.Tensor) else None
    wv = w_v.contiguous() if isinstance(w_v, torch.Tensor) else None
    for t in (wh, wv):
        if t is not None and t.dtype != cost.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "weights must match the cost dtype")
    if msg_cap is None:
        msg_cap = max(256, 2 * D)
    if map_cap is None:
        map_cap = 32 * max(H, W)
    x = torch.empty((H, W), dtype=cost.dtype, device=cost.device)
    nbytes = lib.tv2d_nc_workspace(H, W, D, msg_cap, map_cap)
    if nbytes == 0:
        raise TvChainError(TV_ERR_INVALID_ARG, "tv2d_nc_workspace")
    ws = _workspace(nbytes, cost.device)
    st = lib.tv2d_nc_solve(_dtype_code(cost), _ptr(cost), H, W, D, float(d0), float(dd), float(steep), _ptr(wh),
                           0.0 if wh is not None else float(w_h), _ptr(wv), 0.0 if wv is not None else float(w_v),
                           float(C), float(tau0), int(iters), _ptr(x), msg_cap, map_cap, _ptr(ws), nbytes,
                           ctypes.c_void_p(_stream_ptr(cost.device)))
    _check(st, "tv2d_nc_solve")
    return x


def tree_nc(parent: torch.Tensor, offsets: torch.Tensor, unary_offsets: torch.Tensor, ulam: torch.Tensor,
            uslope: torch.Tensor, w: torch.Tensor, C: Optional[torch.Tensor] = None, msg_cap: int = 256,
            map_cap: Optional[int] = None, stack_cap: Optional[int] = None) -> torch.Tensor:
    """Sec. 3 non-convex trees (tv_tree_nc): parent (int64, global, -1 at roots,
    each tree in depth-first post-order), offsets (int64, trees + 1), unaries as
    for chain_nc, per-node w and C of the edge to the parent.  Fewer than 1024
    trees with msg_cap up to 256 run a wave per tree, otherwise a lane per
    tree.  Defaults: 32
    intervals per node and room for min(64, largest tree) waiting messages of
    msg_cap breakpoints per tree.  Returns x."""
    _require_gpu(parent, offsets, unary_offsets, ulam, uslope, w)
    lib = load()
    for t in (parent, offsets, unary_offsets):
        if t.dtype != torch.int64:
            raise TvChainError(TV_ERR_INVALID_ARG, "parent and offsets must be int64")
    N = parent.numel()
    ts = [t.contiguous() if t is not None else None for t in (ulam, uslope, w, C)]
    for t in ts:
        if t is not None and t.dtype != ulam.dtype:
            raise TvChainError(TV_ERR_INVALID_ARG, "float arrays must share one dtype")
    parent, offsets, unary_offsets = parent.contiguous(), offsets.contiguous(), unary_offsets.contiguous()
    T = offsets.numel() - 1
    biggest = int((offsets[1:] - offsets[:-1]).max().item()) if T > 0 else 1
    if map_cap is None:
        map_cap = max(64, 32 * biggest)
    if stack_cap is None:
        stack_cap = max(1, min(64, biggest)) * (2 * msg_cap + 1)
    x = torch.empty(N, dtype=ulam.dtype, device=ulam.device)
    nbytes = lib.tv_tree_nc_workspace(T, N, msg_cap, map_cap, stack_cap)
    if nbytes == 0:
        raise TvChainError(TV_ERR_INVALID_ARG, "tv_tree_nc_workspace")
    ws = _workspace(nbytes, ulam.device)
    st = lib.tv_tree_nc(_dtype_code(ulam), T, N, _ptr(offsets), _ptr(parent), _ptr(unary_offsets),
                        *(_ptr(t) for t in ts), _ptr(x), msg_cap, map_cap, stack_cap, _ptr(ws), nbytes,
                        ctypes.c_void_p(_stream_ptr(ulam.device)))
    _check(st, "tv_tree_nc")
    return x
