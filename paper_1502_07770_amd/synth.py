"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no arithmetic of the method: it only draws inputs.  All
randomness comes from ``numpy.random.Generator(PCG64(seed))`` and is returned
as FP64 arrays; callers cast to the precision they run in.

Workloads (stand-ins for the paper's signals and images, which are not
available; the noise level sigma = 0.1 and weight 0.1 mirror Sec. 5.1's
experiments, Figs. 5 and 6):

* ``piecewise_constant``: chains whose clean signal is piecewise constant with
  segment lengths Geometric(p = 1/seg_mean) on {1, 2, ...} (the last segment
  truncated), levels U[0, 1], plus N(0, sigma^2) noise.
* ``shapes_image``: an H x W image of ``n_shapes`` axis-aligned rectangles or
  disks (probability 1/2 each) painted in order over a zero background, with
  intensities U[0, 1], plus N(0, sigma^2) noise (no clipping).  Rectangle sides
  are U[W/20, W/3] x U[H/20, H/3], disk radii U[min(H,W)/40, min(H,W)/6], and
  centres uniform over the image.
* ``uneven_batch_specs``: per-image (H, W, lambda, sigma, seed) for a batch of
  images with H, W uniform on {64, ..., 2048}, lambda U[0.02, 0.3], sigma
  U[0.05, 0.2].
* ``general_chain_problem``: inputs of the general chain DP (quadratic unaries
  a_i x^2 / 2 - b_i x, edge slopes w^- <= w^+) on an H x W image: data weights
  a ~ U[0.5, 2], b = a f with f the shapes image, w^- = -w u and w^+ = w v with
  u, v ~ U[0.5, 1.5] per edge (asymmetric TV of weight about w).
* ``salt_pepper_chains``: piecewise-constant chains (levels U[0, 1], no
  Gaussian noise) with a fraction of the samples (25%) replaced by 0 or 1 with
  probability 1/2 each -- impulse noise, the TV-l1 model's setting (Sec. 5.2).
* ``post_order_forest``: num_trees random trees of n nodes each, numbered in
  depth-first post-order: node j adopts k of the pending subtree roots (the
  most recent ones), k in {0, 1, 2, 3} with probabilities 0.4, 0.3, 0.2, 0.1
  (at most the number pending), and the last node adopts all that remain.
  Returns (parent with global indices and -1 at roots, offsets).
* ``edge_weights`` (U[lo, hi]) and ``normal`` (N(0, 1)) helpers.
"""
from __future__ import annotations

import numpy as np


def generator(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def piecewise_constant(num_chains: int, n: int, seg_mean: float = 20.0, sigma: float = 0.1,
                       seed: int = 0) -> np.ndarray:
    """(num_chains, n) FP64 piecewise-constant-plus-noise chains."""
    g = generator(seed)
    p = 1.0 / float(seg_mean)
    k = int(2 * n / seg_mean) + 64
    lengths = g.geometric(p, size=(num_chains, k))
    levels = g.uniform(0.0, 1.0, size=(num_chains, k))
    ends = np.cumsum(lengths, axis=1)
    short = np.nonzero(ends[:, -1] < n)[0]
    for c in short:  # essentially never: extend the rare row that falls short
        while ends[c, -1] < n:
            extra = g.geometric(p, size=k)
            lengths[c] = np.concatenate([lengths[c], extra])[-k:]
            ends[c] = np.cumsum(lengths[c])
    marks = np.zeros((num_chains, n + 1), dtype=np.int32)
    rows = np.repeat(np.arange(num_chains), k)
    e = ends.reshape(-1)
    keep = e < n
    marks[rows[keep], e[keep]] = 1
    seg = np.cumsum(marks[:, :n], axis=1)
    y = np.take_along_axis(levels, seg, axis=1)
    y += g.normal(0.0, sigma, size=(num_chains, n))
    return y


def shapes_image(H: int, W: int, n_shapes: int = 30, sigma: float = 0.1, seed: int = 0) -> np.ndarray:
    """(H, W) FP64 image of random rectangles and disks plus Gaussian noise."""
    g = generator(seed)
    img = np.zeros((H, W))
    m = min(H, W)
    for _ in range(n_shapes):
        is_rect = g.random() < 0.5
        inten = g.uniform(0.0, 1.0)
        cy = g.uniform(0.0, H)
        cx = g.uniform(0.0, W)
        if is_rect:
            sw = g.uniform(W / 20.0, W / 3.0)
            sh = g.uniform(H / 20.0, H / 3.0)
            r0, r1 = int(np.ceil(cy - sh / 2)), int(np.floor(cy + sh / 2))
            c0, c1 = int(np.ceil(cx - sw / 2)), int(np.floor(cx + sw / 2))
            r0, c0 = max(r0, 0), max(c0, 0)
            r1, c1 = min(r1, H - 1), min(c1, W - 1)
            if r0 <= r1 and c0 <= c1:
                img[r0:r1 + 1, c0:c1 + 1] = inten
        else:
            rad = g.uniform(m / 40.0, m / 6.0)
            r0, r1 = max(int(np.floor(cy - rad)), 0), min(int(np.ceil(cy + rad)), H - 1)
            c0, c1 = max(int(np.floor(cx - rad)), 0), min(int(np.ceil(cx + rad)), W - 1)
            if r0 <= r1 and c0 <= c1:
                rr = np.arange(r0, r1 + 1)[:, None]
                cc = np.arange(c0, c1 + 1)[None, :]
                mask = (rr - cy) ** 2 + (cc - cx) ** 2 <= rad * rad
                sub = img[r0:r1 + 1, c0:c1 + 1]
                sub[mask] = inten
    img += g.normal(0.0, sigma, size=(H, W))
    return img


def uneven_batch_specs(num_images: int = 256, side_lo: int = 64, side_hi: int = 2048,
                       lam_lo: float = 0.02, lam_hi: float = 0.3,
                       sigma_lo: float = 0.05, sigma_hi: float = 0.2, seed: int = 0):
    """List of dicts (H, W, lam, sigma, seed) for a batch of uneven images."""
    g = generator(seed)
    Hs = g.integers(side_lo, side_hi + 1, size=num_images)
    Ws = g.integers(side_lo, side_hi + 1, size=num_images)
    lams = g.uniform(lam_lo, lam_hi, size=num_images)
    sigmas = g.uniform(sigma_lo, sigma_hi, size=num_images)
    seeds = g.integers(0, 2 ** 31 - 1, size=num_images)
    return [dict(H=int(Hs[i]), W=int(Ws[i]), lam=float(lams[i]), sigma=float(sigmas[i]),
                 seed=int(seeds[i])) for i in range(num_images)]


def edge_weights(shape, lo: float = 0.1, hi: float = 1.0, seed: int = 0) -> np.ndarray:
    return generator(seed).uniform(lo, hi, size=shape)


def normal(shape, seed: int = 0) -> np.ndarray:
    return generator(seed).normal(0.0, 1.0, size=shape)


def general_chain_problem(H: int, W: int, w: float = 0.1, seed: int = 0):
    """(a, b, wm, wp), each H x W, for the general chain DP over the rows or the
    columns of a shapes image (see the module docstring)."""
    f = shapes_image(H, W, seed=seed)
    g = generator(seed + 7919)
    a = g.uniform(0.5, 2.0, size=(H, W))
    wm = -w * g.uniform(0.5, 1.5, size=(H, W))
    wp = w * g.uniform(0.5, 1.5, size=(H, W))
    return a, a * f, wm, wp


def salt_pepper_chains(num_chains: int, n: int, frac: float = 0.25, seed: int = 0) -> np.ndarray:
    """Piecewise-constant chains with salt & pepper noise (see the module docstring)."""
    f = piecewise_constant(num_chains, n, sigma=0.0, seed=seed)
    g = generator(seed + 104729)
    m = g.random(f.shape) < frac
    f[m] = g.integers(0, 2, int(m.sum())).astype(np.float64)
    return f


def post_order_forest(num_trees: int, n: int, seed: int = 0):
    """Random post-order trees (see the module docstring)."""
    g = generator(seed)
    T = int(num_trees)
    parent = np.full((T, n), -1, dtype=np.int64)
    stack = np.zeros((T, n), dtype=np.int64)
    sp = np.zeros(T, dtype=np.int64)
    rows = np.arange(T)
    for j in range(n - 1):
        k = np.minimum(g.choice(4, size=T, p=[0.4, 0.3, 0.2, 0.1]), sp)
        for r in range(3):
            m = k > r
            parent[rows[m], stack[rows[m], sp[m] - 1]] = j
            sp[m] -= 1
        stack[rows, sp] = j
        sp += 1
    pending = np.arange(n)[None, :] < sp[:, None]
    tt, cc = np.nonzero(pending)
    parent[tt, stack[tt, cc]] = n - 1
    base = (np.arange(T, dtype=np.int64) * n)[:, None]
    glob = np.where(parent >= 0, parent + base, -1).reshape(-1)
    offsets = np.arange(T + 1, dtype=np.int64) * n
    return glob, offsets


def cost_volume(H: int, W: int, D: int, seed: int = 0, outliers: float = 0.1):
    """A synthetic stereo-like cost volume: a piecewise-smooth true disparity map
    (the shapes image scaled to [0, D-1]) and per pixel the matching cost
    min(|d - d_true|, 4) at the integer levels d = 0..D-1 plus N(0, 0.1) noise,
    uniform [0, 4] costs on an `outliers` fraction of pixels.  Returns
    (cost [H, W, D], true disparities [H, W])."""
    g = generator(seed)
    dt = shapes_image(H, W, sigma=0.0, seed=seed)
    dt = (dt - dt.min()) / max(dt.max() - dt.min(), 1e-9) * (D - 1)
    lev = np.arange(D, dtype=np.float64)
    cost = np.minimum(np.abs(lev[None, None, :] - dt[:, :, None]), 4.0) + g.normal(0, 0.1, (H, W, D))
    bad = g.random((H, W)) < outliers
    cost[bad] = g.uniform(0, 4, (int(bad.sum()), D))
    return cost, dt


def cost_volume_chains(H: int, W: int, D: int, seed: int = 0, outliers: float = 0.1, steep: float = 10.0):
    """Rows of the cost volume of cost_volume() as non-convex chains: the costs
    joined linearly between the integer levels, slopes -steep / +steep outside
    [0, D-1].  Returns chain_offsets (H + 1), unary_offsets (H W + 1), ulam
    (H W D), uslope (H W (D + 1)) and the true disparities."""
    cost, dt = cost_volume(H, W, D, seed=seed, outliers=outliers)
    lev = np.arange(D, dtype=np.float64)
    n = H * W
    slopes = np.empty((n, D + 1))
    slopes[:, 0] = -steep
    slopes[:, D] = steep
    slopes[:, 1:D] = np.diff(cost.reshape(n, D), axis=1)
    chain_offsets = (np.arange(H + 1, dtype=np.int64) * W)
    unary_offsets = (np.arange(n + 1, dtype=np.int64) * D)
    ulam = np.tile(lev, n)
    return chain_offsets, unary_offsets, ulam, slopes.reshape(-1), dt


def concave_cost_chains(num_chains: int, n: int, D: int, seed: int = 0, steep: float = 10.0,
                        pieces=((1.0, 0.0), (0.25, 1.0), (0.0, 2.5))):
    """Chains of n nodes with uniform [0, 4] costs at the D integer levels
    (joined linearly, slopes -steep / +steep outside) and, on every edge, the
    pairwise term min over `pieces` (alpha, C) of alpha |z| + C on both sides
    (default: min(|z|, 0.25 |z| + 1, 2.5)).  Returns chain_offsets, (unary
    offsets, ulam, uslope) and (piece offsets, alpha, C, side int32)."""
    g = generator(seed)
    N = int(num_chains) * int(n)
    cost = g.uniform(0, 4, (N, D))
    sl = np.empty((N, D + 1))
    sl[:, 0], sl[:, D] = -steep, steep
    sl[:, 1:D] = np.diff(cost, axis=1)
    k = 2 * len(pieces)
    al = np.array([a for a, _ in pieces] * 2, dtype=np.float64)
    cc = np.array([c for _, c in pieces] * 2, dtype=np.float64)
    sd = np.array([1] * len(pieces) + [-1] * len(pieces), dtype=np.int32)
    unaries = (np.arange(N + 1, dtype=np.int64) * D, np.tile(np.arange(D, dtype=np.float64), N), sl.reshape(-1))
    pcs = (np.arange(N + 1, dtype=np.int64) * k, np.tile(al, N), np.tile(cc, N), np.tile(sd, N))
    return np.arange(int(num_chains) + 1, dtype=np.int64) * int(n), unaries, pcs


def concave_cost_volume_rows(H: int, W: int, D: int, seed: int = 0,
                             pieces=((0.6, 0.0), (0.15, 1.0), (0.0, 2.0))):
    """The rows of cost_volume_chains() with, on every edge, the pairwise term
    min over `pieces` (alpha, C) of alpha |z| + C on both sides (default:
    min(0.6 |z|, 0.15 |z| + 1, 2)).  Returns chain_offsets, (unary offsets,
    ulam, uslope) and (piece offsets, alpha, C, side int32)."""
    coff, uoff, ulam, usl, _ = cost_volume_chains(H, W, D, seed=seed)
    N = uoff.size - 1
    k = 2 * len(pieces)
    al = np.array([a for a, _ in pieces] * 2, dtype=np.float64)
    cc = np.array([c for _, c in pieces] * 2, dtype=np.float64)
    sd = np.array([1] * len(pieces) + [-1] * len(pieces), dtype=np.int32)
    pcs = (np.arange(N + 1, dtype=np.int64) * k, np.tile(al, N), np.tile(cc, N), np.tile(sd, N))
    return coff, (uoff, ulam, usl), pcs
