#!/usr/bin/env python3
"""Benchmark of the batched exact TV-chain prox (and the 2D ROF solvers) on one MI355X.

Headline workload (one "step"): the 4096 x 4096 FP32 shapes-plus-noise image
(30 rectangles/disks, intensities U[0,1], noise sigma 0.1, seed 3); the exact
chain prox (w = 0.1) of all 4096 row chains and all 4096 column chains of
length 4096, i.e. 33,554,432 chain nodes.  Inputs are resident in HBM before
timing starts.  value = Gelem/s = nodes / time.

Also on the same JSON line:
  roofline     -- one tv_chain_prox_multi launch (its kernels: k_seg_main,
                  k_seg_repair, k_seg_fix, k_seg_ovf, k_seg_tail) timed with HIP events;
                  algorithmic bytes 8 B/node (y read, x written) / duration vs the
                  8 TB/s HBM peak; traffic from the committed rocprofv3
                  FETCH_SIZE/WRITE_SIZE summary when it was taken on the current
                  kernel sources, else null.
  cpu_baseline -- the FP64 C oracle on the host cores, same workload; with
                  the extras, "parity" holds each extra's max error against
                  the oracle on the inputs that extra times (sampled).
  extras       -- 2D ROF time-to-gap 1e-4 in FP32 vs FP64 (512^2 and 4096^2),
                  200 iterations at 512^2, forward+backward of 65,536 chains of
                  1,024 with per-edge weights, the general chain DP (data weights,
                  asymmetric edge slopes) on the 4096^2 rows and columns, the
                  TV-l1 chain prox of 65,536 salt & pepper chains, 100 iterations
                  of 2D TV-l1 at 4096^2, 65,536 trees of 256 nodes, the 1000 rows
                  of a 64-level synthetic cost volume as non-convex chains
                  (truncated TV), 5 iterations of the non-convex 2D solver on
                  that volume, 16,384 non-convex trees of 256 nodes, and a batch
                  of 256 uneven images.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras | --extras LIST]
       python bench.py --rocprof-summary DIR   (print a summary of rocprofv3 output)
       python bench.py --copy-calibration      (a plain copy of known size, for counters)
"""
from __future__ import annotations

import argparse
import ctypes
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gelem/s batched TV-chain prox (%HBM peak); 2D TV time-to-gap 1e-4 FP32 vs FP64"
HBM_PEAK_GBS = 8000.0
SIDE = 4096
W_CHAIN = 0.1
SEED = 3
KERNEL_SOURCES = ["paper_1502_07770_amd/csrc/chain_core.h", "paper_1502_07770_amd/csrc/seg_kernels.h",
                  "paper_1502_07770_amd/csrc/chain_kernels.hip", "paper_1502_07770_amd/csrc/api_chain.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "chain_prox_4096_rows_cols_traffic.json")


def kernel_source_hash() -> str:
    """Hash of the chain-prox kernel sources with comments and whitespace
    removed: a counter record stays valid across comment edits only."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def committed_traffic():
    """HBM bytes per bench step launch from the committed counter summary, only
    if taken on the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


class Timer:
    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def __call__(self, fn, reps):
        torch = self.torch
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        for _ in range(reps):
            fn()
        b.record(self.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps


def bench_chain(steps: int, warmup: int, autotune: bool = True):
    """The headline step: rows and columns of the image in ONE tv_chain_prox_multi
    launch.  Also times the two batches as separate tv_chain_prox calls."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth

    lib = binding.load()
    dev = torch.device("cuda:0")
    img = synth.shapes_image(SIDE, SIDE, seed=SEED)
    y = torch.tensor(img, dtype=torch.float32, device=dev)
    xr = torch.empty_like(y)
    xc = torch.empty_like(y)
    rows = binding.ChainLayout(SIDE, SIDE, 1, SIDE, None)
    cols = binding.ChainLayout(SIDE, SIDE, SIDE, 1, None)
    lays = (binding.ChainLayout * 2)(rows, cols)
    yp = (ctypes.c_void_p * 2)(y.data_ptr(), y.data_ptr())
    xp = (ctypes.c_void_p * 2)(xr.data_ptr(), xc.data_ptr())
    wsc = (ctypes.c_double * 2)(W_CHAIN, W_CHAIN)
    nb = lib.tv_chain_prox_multi_workspace(2, lays, binding.TV_F32)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)

    def step():
        st = lib.tv_chain_prox_multi(2, lays, binding.TV_F32, yp, None, wsc, xp, ctypes.c_void_p(ws.data_ptr()),
                                     nb, sp)
        if st != 0:
            raise binding.TvChainError(st, "tv_chain_prox_multi")

    # setup (not timed): the autotuner picks the launch plan for this shape
    plan = None
    if autotune:
        res = binding.TuningResult()
        st = lib.tv_chain_prox_autotune(2, lays, binding.TV_F32, yp, None, wsc, xp, ctypes.c_void_p(ws.data_ptr()),
                                        nb, sp, ctypes.byref(res))
        if st != 0:
            raise binding.TvChainError(st, "tv_chain_prox_autotune")
        plan = res.as_dict()
    else:
        plan = {"segment_length": int(lib.tv_chain_prox_segment_length(ctypes.byref(
            binding.ChainLayout(2 * SIDE, SIDE, 1, SIDE, None)))), "halo": binding.get_tuning()["halo"],
                "ring_slots": binding.get_tuning()["ring_slots"], "candidates": 0, "ms": None}
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    assert torch.isfinite(xr).all() and torch.isfinite(xc).all()
    # the same work as two separate calls (context)
    sep = []
    for lay in (rows, cols):
        nbs = lib.tv_chain_prox_workspace(ctypes.byref(lay), binding.TV_F32)
        wss = torch.empty(nbs, dtype=torch.uint8, device=dev)
        out = torch.empty_like(y)
        call = lambda: lib.tv_chain_prox(ctypes.byref(lay), binding.TV_F32, ctypes.c_void_p(y.data_ptr()),  # noqa
                                         None, W_CHAIN, ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(wss.data_ptr()), nbs, sp)
        call()
        sep.append(Timer(torch, stream)(call, max(3, steps // 2)))
    nodes = 2 * SIDE * SIDE
    ms_step = total_ms / steps
    copy_gbs = measured_copy_gbs(torch, stream)
    return dict(ms_per_step=ms_step, gelem=nodes / (ms_step * 1e-3) / 1e9, launch_ms=float(np.mean(launch_ms)),
                separate_ms=sep, nodes=nodes, img=img, plan=plan, x_rows=xr.cpu().numpy(),
                x_cols=xc.cpu().numpy(), copy_gbs=copy_gbs)


def measured_copy_gbs(torch, stream):
    """Bandwidth of a plain 1 GiB device-to-device copy (reads 1 GiB, writes
    1 GiB), HIP events on the bench stream: the achievable HBM rate next to
    the 8 TB/s peak."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return round(2.0 * (1 << 30) / (ms * 1e-3) / 1e9, 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(img, x_rows, x_cols):
    """The FP64 C oracle on the host cores, same workload; its outputs also
    give the step's max error (per chain, relative to the chain's data range)."""
    import numpy as np
    import oracle
    threads = oracle.num_threads()
    y = np.ascontiguousarray(img.astype(np.float32).astype(np.float64))
    yt = np.ascontiguousarray(y.T)
    times = []
    for _ in range(3):
        t = time.perf_counter()
        xo_r = oracle.chain_prox(y, w_scalar=W_CHAIN)
        xo_c = oracle.chain_prox(yt, w_scalar=W_CHAIN)
        times.append(time.perf_counter() - t)
    dt = float(np.median(times))
    nodes = 2 * y.size
    err_r = np.abs(x_rows.astype(np.float64) - xo_r) / np.ptp(y, axis=1, keepdims=True)
    err_c = np.abs(x_cols.astype(np.float64).T - xo_c) / np.ptp(yt, axis=1, keepdims=True)
    return {"value": round(nodes / dt / 1e9, 4), "unit": "Gelem/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "full workload: 4096 row + 4096 column chains of 4096 (FP64 C oracle, OpenMP over "
                      "chains), median of 3 runs of %.3f s" % dt,
            "max_err_vs_step": float(max(err_r.max(), err_c.max())),
            "max_err_note": "max over chains of |x_gpu - x_oracle| / (max y - min y) of the chain, FP32 step "
                            "against the FP64 oracle (bar 1e-4)"}


def oracle_parity(pick=None):
    """Max error of each extra's result against the FP64 oracle, on the inputs
    that line times (a seeded sample of its chains, trees or images where the
    oracle on all of them would take minutes; 2D solves at a fixed iteration
    count, the same on both sides).  Each entry holds max_err, the bar the GPU
    tests hold that result to, ok, what the error measures and the sample.
    FP32 results are compared with the oracle run on the FP32-rounded inputs."""
    import numpy as np
    import torch
    import oracle
    from paper_1502_07770_amd import binding, synth
    out = {}
    f64 = lambda t: t.double().cpu().numpy()  # noqa: E731
    dev = lambda a, t=torch.float32: torch.tensor(np.asarray(a), dtype=t, device="cuda")  # noqa: E731
    pick_rng = np.random.default_rng(2024)

    def want(key):
        return pick is None or key in pick

    def rec(key, err, bar, measure, sample, **extra):
        out[key] = dict(max_err=float(err), bar=bar, ok=bool(err <= bar), measure=measure, sample=sample, **extra)
        log("parity %s: %.3g (bar %g)" % (key, err, bar))

    rel_img = "max |x - x_oracle| / (max f - min f)"
    for key, side, seed, iters in (("tv2d_512", 512, 11, 200), ("tv2d_4096", SIDE, SEED, 5)):
        if not want(key):
            continue
        img = synth.shapes_image(side, side, seed=seed)
        for name, dt, bar in (("fp32", torch.float32, 1e-4), ("fp64", torch.float64, 1e-9)):
            f = dev(img, dt)
            x, info = binding.tv2d(f, 0.1, max_iter=iters, gap_every=iters)
            fv = f64(f)
            xo, _, (_, _, go), _ = oracle.tv2d(fv, 0.1, max_iter=iters)
            rec("%s_%s" % (key, name), np.abs(f64(x) - xo).max() / np.ptp(fv), bar, rel_img,
                "whole image, %d iterations" % iters, gap=info["gap_norm"], gap_oracle=float(go))
            del f, x

    if want("adjoint"):
        C, n, S = 65536, 1024, 2048
        y = dev(synth.piecewise_constant(C, n, seed=5))
        w = dev(synth.edge_weights((C, n), seed=6))
        g = dev(synth.normal((C, n), seed=7))
        x = binding.chain_prox(y, w, dim=-1)
        dy, dw = binding.chain_prox_backward(x, g, dim=-1, per_edge_w=True)
        rows = np.sort(pick_rng.choice(C, S, replace=False))
        ri = torch.tensor(rows, device="cuda")
        yv, wv, gv, xg, dyg, dwg = (f64(t.index_select(0, ri)) for t in (y, w, g, x, dy, dw))
        del y, w, g, x, dy, dw
        wv[:, -1] = 0.0  # the last slot is no edge
        xo = oracle.chain_prox(yv, w=wv)
        dyo, dwo = oracle.chain_adjoint(xo, gv)
        same = ((xg[:, 1:] == xg[:, :-1]) == (xo[:, 1:] == xo[:, :-1])).all(axis=1)
        sample = "%d of the 65,536 chains (seeded choice)" % S
        rec("adjoint_fwd", (np.abs(xg - xo) / np.ptp(yv, axis=1, keepdims=True)).max(), 1e-4,
            "max over chains of |x - x_oracle| / (max y - min y)", sample)
        rec("adjoint_dy", np.abs(dyg - dyo)[same].max(initial=0.0) / max(1.0, np.abs(dyo).max()), 1e-4,
            "max |dy - dy_oracle| / max(1, max |dy_oracle|) over chains whose run structure matches the oracle's",
            sample, run_structure_mismatch=round(1.0 - float(same.mean()), 5), run_structure_mismatch_bar=0.02)
        rec("adjoint_dw", np.abs(dwg - dwo)[same].max(initial=0.0) / max(1.0, np.abs(dwo).max()), 1e-4,
            "max |dw - dw_oracle| / max(1, max |dw_oracle|) over the same chains", sample)

    if want("general_dp"):
        a, b, wm, wp = (dev(v) for v in synth.general_chain_problem(SIDE, SIDE, seed=SEED))
        S = 128
        worst = 0.0
        for dim in (-1, 0):
            xg = binding.chain_dp(b, wm, wp, a=a, dim=dim)
            idx = np.sort(pick_rng.choice(SIDE, S, replace=False))
            for c in idx:
                sl = (int(c), slice(None)) if dim == -1 else (slice(None), int(c))
                av, bv, wmv, wpv, xv = (f64(t[sl]) for t in (a, b, wm, wp, xg))
                xo = oracle.chain_dp(av, bv, wmv[:-1], wpv[:-1])[0]
                scale = max(np.ptp(xo), np.ptp(bv / av), 1e-30)
                worst = max(worst, np.abs(xv - xo).max() / scale)
            del xg
        rec("general_dp", worst, 1e-4, "max over chains of |x - x_oracle| / max(range x_oracle, range b/a)",
            "%d row and %d column chains (seeded choice)" % (S, S))
        del a, b, wm, wp

    if want("tv_l1"):
        S = 4096
        f = dev(synth.salt_pepper_chains(65536, 1024, seed=12))
        ft = f.t().contiguous()
        rows = torch.tensor(np.sort(pick_rng.choice(65536, S, replace=False)), device="cuda")
        xr = f64(binding.chain_prox_l1(f, f, 0.55, 1.0, dim=-1).index_select(0, rows))
        xc = f64(binding.chain_prox_l1(ft, ft, 0.55, 1.0, dim=0).index_select(1, rows).t())
        yv = f64(f.index_select(0, rows))
        del f, ft
        xo = oracle.chain_prox_l1(yv, yv, w_scalar=0.55, c_scalar=1.0)
        s = np.maximum(np.ptp(yv, axis=1), 1.0)
        err = max((np.abs(xr - xo).max(axis=1) / s).max(), (np.abs(xc - xo).max(axis=1) / s).max())
        rec("tv_l1", err, 1e-4, "max over chains of |x - x_oracle| / max(range y, 1), row and column layouts",
            "%d of the 65,536 chains (seeded choice)" % S)

    if want("tv2d_l1"):
        iters = 10
        f = dev(tv2d_l1_image())
        x, info = binding.tv2d_l1(f, 0.55, max_iter=iters, energy_every=iters)
        fv = f64(f)
        xo, ho = oracle.tv2d_l1(fv, 0.55, tau=1.0, max_iter=iters)
        rec("tv2d_l1", np.abs(f64(x) - xo).max(), 1e-4, "max |x - x_oracle| (f in [0, 1])",
            "whole 4096 x 4096 image, %d iterations" % iters, energy=info["primal"], energy_oracle=float(ho[-1]))
        del f, x

    if want("tree"):
        par, off, vals = tree_inputs()
        ts = [dev(v) for v in vals]
        xg = f64(binding.tree_dp(torch.tensor(par, device="cuda"), torch.tensor(off, device="cuda"), ts[1], ts[4],
                                 ts[5], a=ts[0], c=ts[2], d=ts[3]))
        a, b, c, d, wm, wp = (f64(t) for t in ts)
        del ts
        worst = 0.0
        for t in pick_rng.choice(65536, 300, replace=False):
            lo, hi = off[t], off[t + 1]
            p = par[lo:hi].copy()
            p[p >= 0] -= lo
            xo = oracle.tree_pq(p, *(v[lo:hi] for v in (a, b, c, d, wm, wp)))[0]
            worst = max(worst, np.abs(xg[lo:hi] - xo).max() / max(np.ptp(xo), np.ptp(b[lo:hi] / a[lo:hi]), 1.0))
        rec("tree", worst, 1e-5, "max over trees of |x - x_oracle| / max(range x_oracle, range b/a, 1)",
            "300 of the 65,536 trees (seeded choice)")

    def energy_rec(key, diffs, sample):
        d = np.array(diffs)  # (|E_gpu - E_oracle|, 1 + |E_oracle|, nodes) per chain or tree
        rec(key, float((d[:, 0] / d[:, 1]).max()), 1e-5,
            "max |E(x) - E(x_oracle)| / (1 + |E(x_oracle)|) (minimisers need not be unique)", sample,
            within_test_tolerance=bool((d[:, 0] <= 1e-5 * d[:, 1] + 1e-4 * d[:, 2]).all()))

    if want("nc"):
        coff, uoff, ulam, usl, _ = synth.cost_volume_chains(1000, 1482, 64, seed=1)
        N = uoff.size - 1
        ulam, usl = (v.astype(np.float32).astype(np.float64) for v in (ulam, usl))
        w, Cc = np.full(N, np.float32(0.6), dtype=np.float64), np.full(N, 2.0)  # the FP32 weights
        x = f64(binding.chain_nc(dev(coff, torch.int64), dev(uoff, torch.int64), dev(ulam), dev(usl), dev(w),
                                 dev(Cc), msg_cap=256))
        diffs = []
        for c in pick_rng.choice(coff.size - 1, 64, replace=False):
            n0, n1 = int(coff[c]), int(coff[c + 1])
            uo = uoff[n0:n1 + 1] - uoff[n0]
            lc, sc = ulam[uoff[n0]:uoff[n1]], usl[uoff[n0] + n0:uoff[n1] + n1]
            xo, _ = oracle.nc_chain(uo, lc, sc, w[n0:n1 - 1], Cc[n0:n1 - 1])
            eo = oracle.nc_energy(uo, lc, sc, w[n0:n1 - 1], Cc[n0:n1 - 1], xo)
            eg = oracle.nc_energy(uo, lc, sc, w[n0:n1 - 1], Cc[n0:n1 - 1], x[n0:n1])
            diffs.append((abs(eg - eo), 1.0 + abs(eo), n1 - n0))
        energy_rec("nc", diffs, "64 of the 1000 rows (seeded choice)")

    if want("nc2d"):
        cost, _ = synth.cost_volume(1000, 1482, 64, seed=1)
        crop = np.ascontiguousarray(cost[:128, :160].astype(np.float32).astype(np.float64))
        del cost
        iters = 5
        x = f64(binding.tv2d_nc(dev(crop), 0.0, 1.0, 10.0, 0.6, 0.6, 2.0, 100.0, iters))
        _, _, E = oracle.nc2d_pd(crop, 0.0, 1.0, 10.0, 0.6, 0.6, 2.0, 100.0, iters)
        e = oracle.nc2d_energy(crop, 0.0, 1.0, 10.0, 0.6, 0.6, 2.0, x)
        rec("nc2d", abs(e - E[-1]) / (1 + abs(E[-1])), 1e-5,
            "|E(x) - E(x_oracle)| / (1 + |E(x_oracle)|) after the same iterations",
            "the top-left 128 x 160 crop of the 64-level cost volume, %d iterations" % iters)

    if want("nc_tree"):
        par, off, uoff, ulam, usl, w, Cc = nc_tree_inputs()
        x = f64(binding.tree_nc(dev(par, torch.int64), dev(off, torch.int64), dev(uoff, torch.int64), dev(ulam),
                                dev(usl), dev(w), dev(Cc), msg_cap=512, map_cap=32 * 256, stack_cap=48 * 1025))
        ulam, usl = (v.astype(np.float32).astype(np.float64) for v in (ulam, usl))
        diffs = []
        for t in pick_rng.choice(off.size - 1, 32, replace=False):
            n0, n1 = int(off[t]), int(off[t + 1])
            p = par[n0:n1].copy()
            p[p >= 0] -= n0
            uo = uoff[n0:n1 + 1] - uoff[n0]
            lc, sc = ulam[uoff[n0]:uoff[n1]], usl[uoff[n0] + n0:uoff[n1] + n1]
            xo, _ = oracle.nc_tree(p, uo, lc, sc, w[n0:n1], Cc[n0:n1])
            eo = oracle.nc_tree_energy(p, uo, lc, sc, w[n0:n1], Cc[n0:n1], xo)
            eg = oracle.nc_tree_energy(p, uo, lc, sc, w[n0:n1], Cc[n0:n1], x[n0:n1])
            diffs.append((abs(eg - eo), 1.0 + abs(eo), n1 - n0))
        energy_rec("nc_tree", diffs, "32 of the 16,384 trees (seeded choice)")

    if want("batched"):
        packed, shapes, lams = batched_inputs()
        iters = 20
        xs, _ = binding.tv2d_batched(shapes, lams, max_iter=iters, gap_every=iters, packed=dev(packed))
        worst, offs = 0.0, np.concatenate([[0], np.cumsum([h * w_ for h, w_ in shapes])])
        picked = pick_rng.choice(len(shapes), 8, replace=False)
        for j in picked:
            fv = packed[offs[j]:offs[j + 1]].astype(np.float64).reshape(shapes[j])
            xo = oracle.tv2d(fv, lams[j], max_iter=iters)[0]
            worst = max(worst, np.abs(f64(xs[j]) - xo).max() / max(np.ptp(fv), 1e-12))
        del xs
        rec("batched", worst, 1e-4, rel_img, "8 of the 256 images (seeded choice), %d iterations" % iters)
    torch.cuda.empty_cache()
    return out


def tv2d_l1_image():
    """The 2D TV-l1 input: the 4096 x 4096 shapes image (no Gaussian noise) with
    25% of the pixels replaced by 0 or 1."""
    import numpy as np
    from paper_1502_07770_amd import synth
    rng = np.random.default_rng(SEED)
    f = synth.shapes_image(SIDE, SIDE, sigma=0.0, seed=SEED)
    m = rng.random(f.shape) < 0.25
    f[m] = rng.integers(0, 2, int(m.sum()))
    return f


def tree_inputs():
    """The tree line's forest and data: 65,536 post-order trees of 256 nodes,
    a ~ U[0.3, 2], b = a N(0, 1), c ~ U[0, 1] on 70% of the nodes (0 elsewhere),
    d ~ N(0, 1), w^- ~ -U[0, 0.8], w^+ ~ U[0, 0.8]."""
    from paper_1502_07770_amd import synth
    par, off = synth.post_order_forest(65536, 256, seed=1)
    g = synth.generator(2)
    N = par.size
    a = g.uniform(0.3, 2.0, N)
    vals = [a, a * g.normal(size=N), g.uniform(0, 1, N) * (g.random(N) < 0.7), g.normal(size=N),
            -g.uniform(0, 0.8, N), g.uniform(0, 0.8, N)]
    return par, off, vals


def nc_tree_inputs():
    """The non-convex tree line's input: 16,384 post-order trees of 256 nodes,
    unaries through uniform [0, 4] costs at 16 levels (slopes -/+10 outside),
    w = 0.5, C = 2 on every edge.  Returns (par, off, uoff, ulam, uslope, w, C)."""
    import numpy as np
    from paper_1502_07770_amd import synth
    T, n, D = 16384, 256, 16
    par, off = synth.post_order_forest(T, n, seed=7)
    N = par.size
    g = synth.generator(8)
    cost = g.uniform(0, 4, (N, D))
    sl = np.empty((N, D + 1))
    sl[:, 0], sl[:, D] = -10.0, 10.0
    sl[:, 1:D] = np.diff(cost, axis=1)
    return (par, off, np.arange(N + 1, dtype=np.int64) * D, np.tile(np.arange(D, dtype=np.float64), N),
            sl.reshape(-1), np.full(N, 0.5), np.full(N, 2.0))


def batched_inputs():
    """The batched line's 256 uneven images, packed FP32, with their shapes and
    lambdas."""
    import numpy as np
    from paper_1502_07770_amd import synth
    specs = synth.uneven_batch_specs(256, seed=11)
    packed = np.concatenate([synth.shapes_image(s["H"], s["W"], sigma=s["sigma"], seed=s["seed"]).ravel()
                             .astype(np.float32) for s in specs])
    return packed, [(s["H"], s["W"]) for s in specs], [s["lam"] for s in specs]


def bench_tv2d(side: int, seed: int, iters_fixed: int | None, hist_iters: int, max_iter: int):
    """2D ROF (Sec. 5.1) on a side x side shapes image, FP32 and FP64 iterates
    (FP64 gaps).  The gap after every iteration (gap_every = 1) over hist_iters
    iterations gives the iterations each per-pixel tolerance takes and the
    relative gap (P - D) / P.  Time to gap: solves with gap_every = 1 that stop
    on the device at the tolerance (gap checks included), timed with HIP events
    around the whole call ("ms": the binding's default lookahead of 4 chunks,
    so at most 4 iterations of launches follow the stop), by the device clock
    from the first iteration to the stop ("device_ms"), and with HIP events
    around the fully asynchronous call ("ms_lookahead_0": every iteration up to
    max_iter enqueued, those after the stop returning at once).  At 1e-7 the FP32 iterate's gap floor
    (about 1e-6 to 1e-7 per pixel) separates it from FP64."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    img = synth.shapes_image(side, side, seed=seed)
    out = {"image": "%dx%d shapes+noise sigma 0.1, lambda 0.1" % (side, side), "max_iter": max_iter}
    tm = Timer(torch, torch.cuda.current_stream())
    for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        f = torch.tensor(img, dtype=dt, device="cuda")
        s = binding.Tv2dSolver(side, side, dt)
        r = {"plans": s.autotune(f, 0.1)}  # setup, not timed
        s.solve(f, 0.1, max_iter=2, gap_every=1)  # warm-up
        torch.cuda.synchronize()
        if iters_fixed:
            for graph in (False, True):
                s.solve(f, 0.1, max_iter=20, gap_every=10, use_graph=graph)  # warm-up (graph capture)
                res = {}
                ms = tm(lambda: res.update(info=s.solve(f, 0.1, max_iter=iters_fixed, gap_every=10,
                                                         use_graph=graph)[1]), 1)
                r["ms_%d_iters%s" % (iters_fixed, "_graph" if graph else "")] = round(ms, 3)
            r["gap_after_%d" % iters_fixed] = res["info"]["gap_norm"]
        hist = torch.zeros(hist_iters, dtype=torch.float64, device="cuda")
        _, info = s.solve(f, 0.1, max_iter=hist_iters, gap_every=1, gap_history=hist)
        h = hist.cpu().numpy()
        hw = float(side * side)
        r["gap_history_iters"] = hist_iters
        r["gap_norm_final"] = float(h[-1])
        r["rel_gap_final"] = float(h[-1] * hw / info["primal"])
        for tol in (1e-4, 1e-5, 1e-6, 1e-7):
            hit = np.nonzero(h <= tol)[0]
            r["iters_to_gap_%g" % tol] = int(hit[0]) + 1 if hit.size else None
        ttg = {}
        for tol in (1e-4, 1e-5, 1e-6, 1e-7):
            res = {}
            ms = tm(lambda: res.update(info=s.solve(f, 0.1, max_iter=max_iter, gap_every=1, gap_tol=tol)[1]), 1)
            ms0 = tm(lambda: s.solve(f, 0.1, max_iter=max_iter, gap_every=1, gap_tol=tol, lookahead=0), 1)
            info = res["info"]
            ttg["%g" % tol] = {"ms": round(ms, 3), "device_ms": round(info["device_ms"], 3),
                               "ms_lookahead_0": round(ms0, 3), "iters": info["iters"],
                               "reached": info["status"] == binding.TV_OK,
                               "rel_gap": float(info["gap_norm"] * hw / info["primal"])}
        r["time_to_gap"] = ttg
        out[name] = r
    return out


def bench_adjoint(steps: int):
    import torch
    from paper_1502_07770_amd import binding, synth
    C, n = 65536, 1024
    y = torch.tensor(synth.piecewise_constant(C, n, seed=5), dtype=torch.float32, device="cuda")
    w = torch.tensor(synth.edge_weights((C, n), seed=6), dtype=torch.float32, device="cuda")
    g = torch.tensor(synth.normal((C, n), seed=7), dtype=torch.float32, device="cuda")
    tm = Timer(torch, torch.cuda.current_stream())
    plan = binding.autotune_chain_prox([(y, -1)], w=0.55)  # setup, not timed (scalar w of the same scale)
    fwd = lambda: binding.chain_prox(y, w, dim=-1)  # noqa: E731
    x = fwd()
    bwd = lambda: binding.chain_prox_backward(x, g, dim=-1, per_edge_w=True)  # noqa: E731
    fwd(); bwd()
    f_ms = tm(fwd, steps)
    b_ms = tm(bwd, steps)
    nodes = C * n
    # chains whose FP32 run structure (the runs of equal x the adjoint reduces
    # over) differs from the FP64 one (the FP64 prox matches the oracle to
    # 1e-12 in the tests)
    x64 = binding.chain_prox(y.double(), w.double(), dim=-1)
    same = ((x[:, 1:] == x[:, :-1]) == (x64[:, 1:] == x64[:, :-1])).all(dim=1)
    mismatch = 1.0 - same.double().mean().item()
    del x64
    return {"workload": "65536 chains x 1024, per-edge w ~ U[0.1,1], FP32", "plan": plan,
            "fwd_ms": round(f_ms, 3), "bwd_ms": round(b_ms, 3),
            "fwd_gelem_s": round(nodes / f_ms / 1e6, 2), "bwd_gelem_s": round(nodes / b_ms / 1e6, 2),
            "fwd_bwd_gelem_s": round(nodes / (f_ms + b_ms) / 1e6, 2),
            "fwd_hbm_frac": round(nodes * 12 / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bwd_hbm_frac": round(nodes * 16 / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "run_structure_mismatch_vs_fp64": round(mismatch, 5)}


def bench_general_dp(steps: int, autotune: bool = True):
    """The general chain DP (tv_chain_dp: data weights a_i, asymmetric edge
    slopes) over all row and all column chains of a 4096 x 4096 image, FP32;
    rows and columns are separate calls (each autotuned just before it is
    timed: both have the same chain count and length, so they share a plan
    key).  Algorithmic bytes: a, b, w^-, w^+ read and x written, 20 B/node."""
    import torch
    from paper_1502_07770_amd import binding, synth
    a, b, wm, wp = (torch.tensor(v, dtype=torch.float32, device="cuda")
                    for v in synth.general_chain_problem(SIDE, SIDE, seed=SEED))
    tm = Timer(torch, torch.cuda.current_stream())
    out = {"workload": "4096 row + 4096 column chains of 4096, a ~ U[0.5,2], b = a f (shapes image), "
                       "w- = -0.1 U[0.5,1.5], w+ = 0.1 U[0.5,1.5], FP32"}
    for name, dim in (("rows", -1), ("cols", 0)):
        plan = None
        if autotune:
            _, plan = binding.chain_dp(b, wm, wp, a=a, dim=dim, autotune=True)  # setup, not timed
        else:
            binding.chain_dp(b, wm, wp, a=a, dim=dim)
        ms = tm(lambda: binding.chain_dp(b, wm, wp, a=a, dim=dim), steps)  # noqa: B023
        out[name] = {"plan": plan, "ms": round(ms, 4)}
    tot = out["rows"]["ms"] + out["cols"]["ms"]
    nodes = 2 * SIDE * SIDE
    out["gelem_s"] = round(nodes / tot / 1e6, 2)
    out["hbm_frac"] = round(nodes * 20 / (tot * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def bench_l1(steps: int, autotune: bool = True):
    """TV-l1 chain prox (tv_chain_prox_l1) of 65,536 salt & pepper chains of
    1,024 (25% impulses), y = d = f, w = 0.55, c = 1, FP32, as row chains
    (unit stride) and as column chains (the same data transposed).
    Algorithmic bytes: y and d read, x written, 12 B/node."""
    import torch
    from paper_1502_07770_amd import binding, synth
    f = torch.tensor(synth.salt_pepper_chains(65536, 1024, seed=12), dtype=torch.float32, device="cuda")
    ft = f.t().contiguous()
    tm = Timer(torch, torch.cuda.current_stream())
    out = {"workload": "65536 chains x 1024, piecewise-constant + 25% salt & pepper, y = d, w = 0.55, c = 1, FP32"}
    nodes = f.numel()
    for name, t, dim in (("rows", f, -1), ("cols", ft, 0)):
        plan = None
        if autotune:  # setup, not timed; rows and columns share a plan key, so each is tuned just before it
            _, plan = binding.chain_prox_l1(t, t, 0.55, 1.0, dim=dim, autotune=True)
        else:
            binding.chain_prox_l1(t, t, 0.55, 1.0, dim=dim)
        ms = tm(lambda: binding.chain_prox_l1(t, t, 0.55, 1.0, dim=dim), steps)  # noqa: B023
        out[name] = {"plan": plan, "ms": round(ms, 4), "gelem_s": round(nodes / ms / 1e6, 2),
                     "hbm_frac": round(nodes * 12 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def bench_tv2d_l1():
    """2D TV-l1 (Sec. 5.2) on a 4096 x 4096 shapes image with 25% salt & pepper
    noise, lambda = 0.55, constant steps tau = sigma = 1, FP32: autotuned plans
    (setup), then 100 iterations timed; FP64 energy at the end."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    ft = torch.tensor(tv2d_l1_image(), dtype=torch.float32, device="cuda")
    _, info = binding.tv2d_l1(ft, 0.55, max_iter=1, autotune=True)  # setup, not timed
    e0 = binding.tv2d_l1(ft, 0.55, max_iter=0)[1]["primal"]
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, st = binding.tv2d_l1(ft, 0.55, max_iter=100, energy_every=100)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) * 1e3
    return {"image": "4096x4096 shapes + 25% salt & pepper, lambda 0.55, tau = sigma = 1, FP32",
            "plans": info.get("plans"), "ms_100_iters": round(dt, 2), "ms_per_iter": round(dt / 100, 3),
            "energy_f": e0, "energy_100": st["primal"]}


def bench_nc(steps: int):
    """Sec. 3 non-convex chains (tv_chain_nc): the 1000 rows (1482 nodes) of a
    synthetic stereo-like cost volume with 64 levels (piecewise-linear unaries
    through the level costs, 64 breakpoints each), truncated TV w = 0.6, C = 2,
    FP32 in, FP64 inside.  Algorithmic bytes: the unary (64 breakpoints + 65
    slopes) and w, C read and x written, 4 B each: 524 B/node."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    H, W, D = 1000, 1482, 64
    coff, uoff, ulam, usl, dt = synth.cost_volume_chains(H, W, D, seed=1)
    N = uoff.size - 1
    dev = lambda a, t=torch.float32: torch.tensor(a, dtype=t, device="cuda")  # noqa: E731
    args = (dev(coff, torch.int64), dev(uoff, torch.int64), dev(ulam), dev(usl), dev(np.full(N, 0.6)),
            dev(np.full(N, 2.0)))
    del ulam, usl
    run = lambda: binding.chain_nc(*args, msg_cap=256)  # noqa: E731
    x = run()
    tm = Timer(torch, torch.cuda.current_stream())
    ms = tm(run, steps)
    err = float(np.abs(x.cpu().numpy().reshape(H, W) - dt).mean())
    return {"workload": "1000 rows x 1482 of a 64-level synthetic cost volume, truncated TV w 0.6, C 2, FP32 in, "
                        "FP64 messages", "ms": round(ms, 2), "mnode_s": round(N / ms / 1e3, 2),
            "hbm_frac": round(N * 524 / (ms * 1e-3) / 8e12, 5), "mean_abs_x_minus_true_disparity": round(err, 3)}


def bench_nc2d(iters: int):
    """Sec. 5.3 non-convex 2D (tv2d_nc_solve) on a 1000 x 1482 synthetic cost
    volume with 64 levels (the stereo pair's size), truncated TV w = 0.6, C = 2,
    tau0 = 100: `iters` primal-dual iterations (each one row and one column
    non-convex chain solve), FP32 costs.  Reports the time per iteration and the
    energy before and after."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    H, W, D = 1000, 1482, 64
    cost, dt = synth.cost_volume(H, W, D, seed=1)
    ct = torch.tensor(cost, dtype=torch.float32, device="cuda")
    run = lambda k: binding.tv2d_nc(ct, 0.0, 1.0, 10.0, 0.6, 0.6, 2.0, 100.0, k)  # noqa: E731
    run(1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    x = run(iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3
    x = x.double().cpu().numpy()
    x0 = np.argmin(cost, axis=2).astype(np.float64)
    return {"workload": "1000 x 1482 x 64 synthetic cost volume, truncated TV w 0.6, C 2, tau0 100, FP32 costs",
            "iters": iters, "ms": round(ms, 1), "ms_per_iter": round(ms / iters, 1),
            "mean_abs_x_minus_true_disparity": round(float(np.abs(x - dt).mean()), 3),
            "mean_abs_init_minus_true_disparity": round(float(np.abs(x0 - dt).mean()), 3)}


def bench_nc_concave(steps: int):
    """Sec. 3 Extensions (i) (tv_chain_nc_concave): 16,384 chains of 256 nodes
    (concave_cost_chains), 16-level uniform [0, 4] costs, and on every edge
    min(|z|, 0.25 |z| + 1, 2.5), three pieces per side, FP32 in, FP64
    messages, msg_cap 128 (a wave per chain).  Capacities from the oracle on 256 of the chains: messages up to
    37 breakpoints, up to 4,857 intervals per chain."""
    import torch
    from paper_1502_07770_amd import binding, synth
    coff, (uoff, ulam, usl), (poff, al, cc, sd) = synth.concave_cost_chains(16384, 256, 16, seed=9)
    f32 = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")  # noqa: E731
    i64 = lambda a: torch.tensor(a, dtype=torch.int64, device="cuda")  # noqa: E731
    args = (i64(coff), i64(uoff), f32(ulam), f32(usl), i64(poff), f32(al), f32(cc),
            torch.tensor(sd, dtype=torch.int32, device="cuda"))
    run = lambda: binding.chain_nc_concave(*args, msg_cap=128, map_cap=8192)  # noqa: E731
    run()
    ms = Timer(torch, torch.cuda.current_stream())(run, steps)
    N = int(coff[-1])
    return {"workload": "16384 chains x 256 nodes, 16-level uniform random costs, pairwise min(|z|, 0.25|z| + 1, "
                        "2.5), FP32 in, FP64 messages", "ms": round(ms, 2), "mnode_s": round(N / ms / 1e3, 2)}


def bench_nc_concave_rows(steps: int):
    """Sec. 3 Extensions (i) on the 1000 rows (1482 nodes, 64 levels) of the
    synthetic cost volume (concave_cost_volume_rows) with min(0.6 |z|,
    0.15 |z| + 1, 2) on every edge, FP32 in, msg_cap 256 (a wave per row)."""
    import torch
    from paper_1502_07770_amd import binding, synth
    coff, (uoff, ulam, usl), (poff, al, cc, sd) = synth.concave_cost_volume_rows(1000, 1482, 64, seed=1)
    f32 = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")  # noqa: E731
    i64 = lambda a: torch.tensor(a, dtype=torch.int64, device="cuda")  # noqa: E731
    args = (i64(coff), i64(uoff), f32(ulam), f32(usl), i64(poff), f32(al), f32(cc),
            torch.tensor(sd, dtype=torch.int32, device="cuda"))
    run = lambda: binding.chain_nc_concave(*args, msg_cap=256, map_cap=64 * 1482)  # noqa: E731
    run()
    ms = Timer(torch, torch.cuda.current_stream())(run, steps)
    N = int(coff[-1])
    return {"workload": "1000 cost-volume rows x 1482 nodes, 64 levels, pairwise min(0.6|z|, 0.15|z| + 1, 2), "
                        "FP32 in, FP64 messages", "ms": round(ms, 2), "mnode_s": round(N / ms / 1e3, 2)}


def bench_nc_tree_concave(steps: int):
    """Sec. 3 Extensions (i) on trees (tv_tree_nc_concave): the 16,384 trees of
    bench_nc_tree (post_order_forest, seed 7) with the unaries and pairwise
    terms of bench_nc_concave (min(|z|, 0.25 |z| + 1, 2.5), three pieces per
    side), FP32 in, FP64 messages.  Capacities from the oracle on all the
    trees: messages up to 506 breakpoints, at most 4,875 intervals per tree."""
    import torch
    from paper_1502_07770_amd import binding, synth
    par, off = synth.post_order_forest(16384, 256, seed=7)
    _, (uoff, ulam, usl), (poff, al, cc, sd) = synth.concave_cost_chains(16384, 256, 16, seed=9)
    f32 = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")  # noqa: E731
    i64 = lambda a: torch.tensor(a, dtype=torch.int64, device="cuda")  # noqa: E731
    args = (i64(par), i64(off), i64(uoff), f32(ulam), f32(usl), i64(poff), f32(al), f32(cc),
            torch.tensor(sd, dtype=torch.int32, device="cuda"))
    run = lambda: binding.tree_nc_concave(*args, msg_cap=1024, map_cap=8192, stack_cap=64 * 1025)  # noqa: E731
    run()
    ms = Timer(torch, torch.cuda.current_stream())(run, steps)
    N = int(off[-1])
    return {"workload": "16384 post-order trees x 256 nodes, 16-level uniform random costs, pairwise min(|z|, "
                        "0.25|z| + 1, 2.5), FP32 in, FP64 messages", "ms": round(ms, 2),
            "mnode_s": round(N / ms / 1e3, 2)}


def bench_nc_tree_small(steps: int):
    """Sec. 3 non-convex trees, a small batch: 512 post-order trees of 256 nodes
    (fewer trees than SIMDs), 8-level uniform [0, 4] costs, truncated TV
    w = 0.5, C = 2, FP32 in.  The oracle finds messages of at most 140
    breakpoints, so msg_cap 256 runs a wave per tree; msg_cap 512 the lane
    kernel on the same trees, for comparison.  The same for concave pairwise
    terms on these trees (tv_tree_nc_concave)."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    T, n, D = 512, 256, 8
    par, off = synth.post_order_forest(T, n, seed=7)
    N = par.size
    g = synth.generator(8)
    cost = g.uniform(0, 4, (N, D))
    sl = np.empty((N, D + 1))
    sl[:, 0], sl[:, D] = -10.0, 10.0
    sl[:, 1:D] = np.diff(cost, axis=1)
    dev = lambda a, t=torch.float32: torch.tensor(a, dtype=t, device="cuda")  # noqa: E731
    args = (dev(par, torch.int64), dev(off, torch.int64), dev(np.arange(N + 1, dtype=np.int64) * D, torch.int64),
            dev(np.tile(np.arange(D, dtype=np.float64), N)), dev(sl.reshape(-1)), dev(np.full(N, 0.5)),
            dev(np.full(N, 2.0)))
    out = {"workload": "512 post-order trees x 256 nodes, 8-level uniform random costs, truncated TV w 0.5, C 2, "
                       "FP32 in, FP64 messages"}
    for name, cap in (("ms", 256), ("ms_lane", 512)):
        run = lambda: binding.tree_nc(*args, msg_cap=cap, map_cap=32 * n)  # noqa: E731
        run()
        out[name] = round(Timer(torch, torch.cuda.current_stream())(run, steps), 2)
    out["mnode_s"] = round(N / out["ms"] / 1e3, 2)
    # the same trees with 8-level concave_cost_chains unaries and min(|z|, 0.25 |z| + 1, 2.5)
    # (messages up to 200 breakpoints)
    _, (uoff, ulam, usl), (poff, al, cc, sd) = synth.concave_cost_chains(T, n, D, seed=9)
    cargs = (args[0], args[1], dev(uoff, torch.int64), dev(ulam), dev(usl), dev(poff, torch.int64), dev(al), dev(cc),
             dev(sd, torch.int32))
    for name, cap in (("concave_ms", 256), ("concave_ms_lane", 512)):
        run = lambda: binding.tree_nc_concave(*cargs, msg_cap=cap, map_cap=32 * n)  # noqa: E731
        run()
        out[name] = round(Timer(torch, torch.cuda.current_stream())(run, steps), 2)
    return out


def bench_nc_tree(steps: int):
    """Sec. 3 non-convex trees (tv_tree_nc): 16,384 random post-order trees of
    256 nodes (post_order_forest), unaries through uniform [0, 4] costs at 16
    levels (slopes -/+10 outside), truncated TV w = 0.5, C = 2, FP32 in, FP64
    messages.  Capacities from the oracle on all the trees: messages up to
    356 breakpoints, at most 3,114 intervals per tree; up to 39 messages wait
    on a tree's stack (40 trees sampled)."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    par, off, uoff, ulam, usl, w, C = nc_tree_inputs()
    N, n = par.size, 256
    dev = lambda a, t=torch.float32: torch.tensor(a, dtype=t, device="cuda")  # noqa: E731
    args = (dev(par, torch.int64), dev(off, torch.int64), dev(uoff, torch.int64), dev(ulam), dev(usl), dev(w),
            dev(C))
    run = lambda: binding.tree_nc(*args, msg_cap=512, map_cap=32 * n, stack_cap=48 * 1025)  # noqa: E731
    run()
    ms = Timer(torch, torch.cuda.current_stream())(run, steps)
    return {"workload": "16384 post-order trees x 256 nodes, 16-level uniform random costs, truncated TV w 0.5, C 2, "
                        "FP32 in, FP64 messages", "ms": round(ms, 2), "mnode_s": round(N / ms / 1e3, 2)}


def bench_tree(steps: int):
    """Algorithm 2 on 65,536 random post-order trees of 256 nodes (tv_tree_dp)
    with a ~ U[0.3, 2], TV-l1 data terms on 70% of the nodes, asymmetric edge
    slopes, FP32 inputs (FP64 inside).  Algorithmic bytes: parent (8 B), a, b, c,
    d, w^-, w^+ read and x written (4 B each): 36 B/node."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    par, off, vals = tree_inputs()
    N = par.size
    a_t, b_t, c_t, d_t, wm_t, wp_t = (torch.tensor(v, dtype=torch.float32, device="cuda") for v in vals)
    pt, ot = torch.tensor(par, device="cuda"), torch.tensor(off, device="cuda")
    tm = Timer(torch, torch.cuda.current_stream())
    run = lambda: binding.tree_dp(pt, ot, b_t, wm_t, wp_t, a=a_t, c=c_t, d=d_t)  # noqa: E731
    run()
    ms = tm(run, steps)
    return {"workload": "65536 post-order trees x 256 nodes, a ~ U[0.3,2], l1 terms on 70% of nodes, FP32 in, FP64 DP",
            "ms": round(ms, 3), "gelem_s": round(N / ms / 1e6, 2),
            "hbm_frac": round(N * 36 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_batched():
    """256 uneven images in one batched solve, each stopping on the device at
    its own gap (gap_every = 1): HIP-event time of the call and the device time
    to the last image's stop, for gap 1e-4 and 1e-5 per pixel."""
    import numpy as np
    import torch
    from paper_1502_07770_amd import binding, synth
    t = time.perf_counter()
    packed, shapes, lams = batched_inputs()
    gen_s = time.perf_counter() - t
    f = torch.from_numpy(packed).cuda()
    tuned = {}
    binding.tv2d_batched(shapes, lams, max_iter=1, gap_every=1, packed=f, autotune=True, tuned=tuned)  # setup
    tm = Timer(torch, torch.cuda.current_stream())
    out = {"workload": "256 images, H,W ~ U{64..2048}, lambda ~ U[0.02,0.3], sigma ~ U[0.05,0.2], FP32",
           "pixels": int(packed.size), "max_iter": 200, "gap_every": 1, "generate_s": round(gen_s, 1),
           "plans": tuned}
    for tol in (1e-4, 1e-5):
        for graph in (False, True):
            res = {}
            ms = tm(lambda: res.update(r=binding.tv2d_batched(shapes, lams, max_iter=200, gap_every=1, gap_tol=tol,
                                                              packed=f, use_graph=graph)), 1)
            infos = res["r"][1]
            iters = [i["iters"] for i in infos]
            out["gap_%g%s" % (tol, "_graph" if graph else "")] = {
                "ms": round(ms, 1), "device_ms": round(max(i["device_ms"] for i in infos), 1),
                "all_reached": all(i["status"] == binding.TV_OK for i in infos),
                "iters_min": min(iters), "iters_median": int(np.median(iters)), "iters_max": max(iters)}
    return out


def c4_iters(iters: int):
    """The batched line's 256 images for profiling runs: its two launches
    autotuned (setup), then `iters` iterations with one gap evaluation."""
    import torch
    from paper_1502_07770_amd import binding
    packed, shapes, lams = batched_inputs()
    f = torch.from_numpy(packed).cuda()
    tuned = {}
    binding.tv2d_batched(shapes, lams, max_iter=1, gap_every=1, packed=f, autotune=True, tuned=tuned)
    torch.cuda.synchronize()
    log("plans", tuned)
    binding.tv2d_batched(shapes, lams, max_iter=iters, gap_every=iters, gap_tol=0.0, packed=f)
    torch.cuda.synchronize()
    log("c4: %d iterations done" % iters)


def rocprof_summary(d):
    """Print per-kernel call counts and average durations from rocprofv3 output
    (kernel_stats CSV or the results database) and, if counter CSVs are present,
    per-dispatch FETCH_SIZE / WRITE_SIZE."""
    import csv
    import sqlite3
    stats = sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True))
    if stats:
        with open(stats[0]) as fh:
            rows = list(csv.DictReader(fh))
        print("kernel stats (%s):" % os.path.relpath(stats[0], d))
        for r in rows[:15]:
            print("  %-60s calls=%-6s avg_us=%.1f" % (r["Name"].split("(")[0][:60], r["Calls"],
                                                       float(r["AverageNs"]) / 1e3))
    dbs = sorted(glob.glob(os.path.join(d, "**", "*results.db"), recursive=True))
    if dbs and not stats:
        con = sqlite3.connect(dbs[0])
        print("kernel stats (%s):" % os.path.relpath(dbs[0], d))
        call_us = {}
        for name, calls, total, avg in con.execute(
                "select name, total_calls, total_duration, average from top_kernels limit 25"):
            short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
            print("  %-60s calls=%-6d total_us=%-10.1f avg_us=%.1f" % (short[:60], calls, total, avg))
            if short.startswith("tvc::k_seg_"):
                prob = short.split(",")[1].strip().split("<")[0] if "," in short else short
                call_us[prob] = call_us.get(prob, 0.0) + avg
            elif short.startswith("tvc::k_prefix_"):  # the general DP's prefix pass
                call_us["tvc::GenProb"] = call_us.get("tvc::GenProb", 0.0) + avg
        for prob, us in sorted(call_us.items()):
            print("  one launch with %s (sum of the k_seg_* (and k_prefix_*) averages): %.1f us" % (prob, us))
    for cnt in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(cnt) as fh:
            rows = list(csv.DictReader(fh))
        agg = {}
        for r in rows:
            key = (r["Kernel_Name"].split("(")[0][:60], r["Counter_Name"])
            agg.setdefault(key, []).append(float(r["Counter_Value"]))
        print("counters (%s):" % os.path.relpath(cnt, d))
        for (k, c), v in sorted(agg.items()):
            print("  %-60s %-12s dispatches=%-4d mean=%.1f" % (k, c, len(v), sum(v) / len(v)))


def _counter_means(d, counter):
    import csv
    out = {}
    for cnt in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(cnt) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.setdefault(r["Kernel_Name"].split("(")[0].replace("void ", ""), []).append(
                        float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in out.items()}


def traffic_from_counters(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """HBM bytes of one tv_chain_prox_multi launch (the bench step) from
    FETCH_SIZE / WRITE_SIZE (KiB per dispatch, averaged over the steps of the
    run; the separate-call timing dispatches are excluded), each scaled by what the
    counter reads for a plain 1 GiB device copy (reads 1 GiB, writes 1 GiB)."""
    gib = float(1 << 30)
    cf = _counter_means(copy_fetch_dir, "FETCH_SIZE")
    cw = _counter_means(copy_write_dir, "WRITE_SIZE")
    copy_k = [k for k in cf if "copyBuffer" in k][0]
    f_scale = gib / (cf[copy_k] * 1024.0)
    w_scale = gib / (cw[copy_k] * 1024.0)
    step = lambda k: k.startswith("tvc::k_seg_") and "MultiProb" in k  # noqa: E731
    fe = {k: v for k, v in _counter_means(fetch_dir, "FETCH_SIZE").items() if step(k)}
    wr = {k: v for k, v in _counter_means(write_dir, "WRITE_SIZE").items() if step(k)}
    fetch_b = sum(fe.values()) * 1024.0 * f_scale
    write_b = sum(wr.values()) * 1024.0 * w_scale
    rec = {"workload": "tv_chain_prox_multi, 4096 row + 4096 column chains of 4096 in one launch, FP32, w = 0.1",
           "kernel_source_hash": kernel_source_hash(),
           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
           "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
           "bytes_per_launch": round(fetch_b + write_b),
           "alg_bytes_per_launch": 8 * 2 * SIDE * SIDE,
           "per_kernel_fetch_kib": {k: round(v, 1) for k, v in fe.items()},
           "per_kernel_write_kib": {k: round(v, 1) for k, v in wr.items()}}
    return rec


def copy_calibration():
    """A plain device-to-device copy of 1 GiB (reads 1 GiB, writes 1 GiB)."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="all",
                    help="comma-separated subset of tv2d_512,tv2d_4096,adjoint,general_dp,tv_l1,tv2d_l1,tree,nc,"
                         "nc2d,nc_tree,nc_tree_small,nc_concave,nc_tree_concave,nc_concave_rows,batched")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default plan (profiling runs: no candidate dispatches in the trace)")
    ap.add_argument("--rocprof-summary", metavar="DIR")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--c4-iters", type=int, metavar="N",
                    help="run the batched line's autotune and N iterations only (for profiling runs)")
    ap.add_argument("--plan", metavar="L,H,K",
                    help="fixed plan for the headline launch (segment length, halo, ring slots) instead of the "
                         "autotuner's: for profiling runs that must launch exactly the plan the default run picks")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 --pmc output folders; writes the traffic record read by the roofline")
    args = ap.parse_args()
    if args.traffic_from:
        rec = traffic_from_counters(*args.traffic_from)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec, indent=1))
        return
    if args.rocprof_summary:
        rocprof_summary(args.rocprof_summary)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the workload's chains are independent and one MI355X holds "
              "all of them (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    from paper_1502_07770_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    if args.copy_calibration:
        copy_calibration()
        return

    log("bench: chain prox 4096x4096 rows+cols, steps=%d warmup=%d" % (args.steps, args.warmup))
    if args.c4_iters:
        c4_iters(args.c4_iters)
        return
    if args.plan:
        from paper_1502_07770_amd import binding
        L, H, K = (int(v) for v in args.plan.split(","))
        binding.set_tuning(target_lanes=1 << 30, min_segment=L, halo=H, ring_slots=K)
    r = bench_chain(args.steps, args.warmup, autotune=not (args.no_autotune or args.plan))
    log("bench: %.3f ms/step, %.1f Gelem/s (one launch %.3f ms; separate row / column calls %.3f / %.3f ms)" % (
        r["ms_per_step"], r["gelem"], r["launch_ms"], r["separate_ms"][0], r["separate_ms"][1]))
    alg_bytes = 8.0 * r["nodes"]
    achieved = alg_bytes / (r["launch_ms"] * 1e-3) / 1e9
    traffic = committed_traffic()
    out = {
        "metric": METRIC,
        "value": round(r["gelem"], 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "exact TV chain prox of all 4096 row and 4096 column chains (length 4096) of a "
                        "4096x4096 FP32 shapes+noise image (sigma 0.1, seed 3), w = 0.1, in one launch",
            "nodes_per_step": r["nodes"],
            "launch_ms": round(r["launch_ms"], 4),
            "separate_row_col_calls_ms": [round(v, 4) for v in r["separate_ms"]],
            "autotuned_plan": r["plan"],
        },
        "hbm_pct": round(100.0 * r["gelem"] * 8.0 / HBM_PEAK_GBS, 2),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "one tv_chain_prox_multi launch over rows + columns (k_seg_main, k_seg_repair, k_seg_fix, "
                      "k_seg_ovf, k_seg_tail)",
            "alg_bytes_per_launch": alg_bytes,
            "measured_copy_gbs": r["copy_gbs"],
            "frac_of_measured_copy": round(achieved / r["copy_gbs"], 4),
        },
    }
    if not args.no_cpu:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(r["img"], r["x_rows"], r["x_cols"])
    if not args.no_extras:
        extras = {}
        runs = [("tv2d_512", "2D 512x512", lambda: bench_tv2d(512, 11, 200, 200, 2000)),
                ("tv2d_4096", "2D 4096x4096", lambda: bench_tv2d(4096, SEED, None, 60, 500)),
                ("adjoint", "adjoint 65536x1024", lambda: bench_adjoint(5)),
                ("general_dp", "general chain DP 4096x4096 rows, cols",
                 lambda: bench_general_dp(10, autotune=not args.no_autotune)),
                ("tv_l1", "TV-l1 chain prox 65536x1024", lambda: bench_l1(10, autotune=not args.no_autotune)),
                ("tv2d_l1", "2D TV-l1 4096x4096", bench_tv2d_l1),
                ("tree", "trees 65536x256", lambda: bench_tree(5)),
                ("nc", "non-convex chains 1000x1482, 64 levels", lambda: bench_nc(3)),
                ("nc2d", "non-convex 2D 1000x1482, 64 levels", lambda: bench_nc2d(5)),
                ("nc_tree", "non-convex trees 16384x256", lambda: bench_nc_tree(3)),
                ("nc_tree_small", "non-convex trees 512x256", lambda: bench_nc_tree_small(3)),
                ("nc_concave", "concave pairwise chains 16384x256", lambda: bench_nc_concave(3)),
                ("nc_tree_concave", "concave pairwise trees 16384x256", lambda: bench_nc_tree_concave(3)),
                ("nc_concave_rows", "concave pairwise cost-volume rows 1000x1482", lambda: bench_nc_concave_rows(3)),
                ("batched", "batched 256 images", bench_batched)]
        pick = None if args.extras == "all" else set(args.extras.split(","))
        try:
            for key, what, fn in runs:
                if pick is None or key in pick:
                    log("bench: " + what)
                    extras[key] = fn()
        except Exception as e:  # report what finished
            extras["error"] = repr(e)
        out["extras"] = extras
    if not (args.no_cpu or args.no_extras):
        log("bench: oracle parity of the extras")
        try:
            out["cpu_baseline"]["parity"] = oracle_parity(None if args.extras == "all"
                                                          else set(args.extras.split(",")))
        except Exception as e:  # report what finished
            out["cpu_baseline"]["parity_error"] = repr(e)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
