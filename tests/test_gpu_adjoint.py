"""GPU parity of the chain-prox adjoint (tv_chain_prox_backward) and the
autograd wrapper.

The gradient is defined by the run structure of x (exact equality of
consecutive values).  FP32 and FP64 solutions share it except near
degenerate points, so the FP32 gradient is compared with the FP64 oracle's
gradient on every chain whose jump pattern matches, and the fraction of
chains that differ is bounded.  The oracle's gradient is itself pinned by
FP64 central finite differences on sampled chains.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth
from tests import props

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _workload(C, n, seed):
    y = synth.piecewise_constant(C, n, seed=seed)
    w = synth.edge_weights((C, n), lo=0.1, hi=1.0, seed=seed + 1)
    w[:, -1] = 0.0
    g = synth.normal((C, n), seed=seed + 2)
    return y, w, g


def _compare(C, n, seed, dtype, tol):
    y, w, g = _workload(C, n, seed)
    yt, wt, gt = _dev(y, dtype), _dev(w, dtype), _dev(g, dtype)
    xt = binding.chain_prox(yt, wt, dim=-1)
    dy, dw = binding.chain_prox_backward(xt, gt, dim=-1, per_edge_w=True)
    yv, wv, gv = (t.double().cpu().numpy() for t in (yt, wt, gt))
    xo = oracle.chain_prox(yv, w=wv)
    dyo, dwo = oracle.chain_adjoint(xo, gv)
    same = (props.run_structure(xt.double().cpu().numpy()) == props.run_structure(xo)).all(axis=1)
    dyg, dwg = dy.double().cpu().numpy(), dw.double().cpu().numpy()
    ey = np.abs(dyg - dyo)[same].max(initial=0.0) / max(1.0, np.abs(dyo).max())
    ew = np.abs(dwg - dwo)[same].max(initial=0.0) / max(1.0, np.abs(dwo).max())
    return ey, ew, 1.0 - same.mean(), (yv, wv, gv, xt, dyg, dwg, same)


def test_fp64_adjoint_matches_oracle():
    ey, ew, frac, _ = _compare(300, 700, seed=1, dtype=torch.float64, tol=1e-12)
    assert frac < 0.01  # a near-tie at a clip bound may flip by one rounding
    assert ey < 1e-12 and ew < 1e-12


def test_fp32_adjoint_full_size():
    """65,536 chains of 1,024 nodes, per-edge w ~ U[0.1, 1], g ~ N(0, 1)."""
    ey, ew, frac, (yv, wv, gv, xt, dyg, dwg, same) = _compare(65536, 1024, seed=5, dtype=torch.float32, tol=1e-4)
    assert frac < 0.02, frac          # chains whose FP32 run structure differs from FP64
    assert ey < 1e-4 and ew < 1e-4, (ey, ew)
    # identities on the GPU output (any x): sum dy = sum g; Euler <dy,y> + <dw,w> = <g,x>
    x = xt.double().cpu().numpy()
    assert np.abs(dyg.sum(axis=1) - gv.sum(axis=1)).max() < 1e-3
    lhs = (dyg * yv).sum(axis=1) + (dwg * wv).sum(axis=1)
    rhs = (gv * x).sum(axis=1)
    assert np.abs(lhs - rhs).max() < 1e-3 * max(1.0, np.abs(rhs).max())


def test_fp32_gradient_against_finite_differences():
    """FP64 central differences (h = 1e-6) of the oracle on 64 sampled chains of
    the large workload, compared with the GPU FP32 gradient where the run
    structure is unchanged by the probes."""
    C, n = 65536, 1024
    y, w, g = _workload(C, n, seed=5)
    rows = np.random.default_rng(0).choice(C, size=64, replace=False)
    ys, ws_, gs = y[rows], w[rows], g[rows]
    yt, wt, gt = _dev(ys, torch.float32), _dev(ws_, torch.float32), _dev(gs, torch.float32)
    xt = binding.chain_prox(yt, wt, dim=-1)
    dy, dw = binding.chain_prox_backward(xt, gt, dim=-1, per_edge_w=True)
    dy, dw = dy.double().cpu().numpy(), dw.double().cpu().numpy()
    yv, wv, gv = (t.double().cpu().numpy() for t in (yt, wt, gt))
    h = 1e-6
    rng = np.random.default_rng(1)
    checked = 0
    for k in range(64):
        x0 = oracle.chain_prox(yv[k], w=wv[k])
        if not np.array_equal(props.run_structure(x0), props.run_structure(xt[k].double().cpu().numpy())):
            continue
        st0 = props.run_structure(x0)
        idx = rng.choice(n, size=24, replace=False)
        eidx = rng.choice(n - 1, size=24, replace=False)
        Yp = np.repeat(yv[k][None], 2 * len(idx), axis=0)
        Yp[np.arange(len(idx)), idx] += h
        Yp[len(idx) + np.arange(len(idx)), idx] -= h
        Xp = oracle.chain_prox(Yp, w=np.repeat(wv[k][None], 2 * len(idx), axis=0))
        Wp = np.repeat(wv[k][None], 2 * len(eidx), axis=0)
        Wp[np.arange(len(eidx)), eidx] += h
        Wp[len(eidx) + np.arange(len(eidx)), eidx] -= h
        Xw = oracle.chain_prox(np.repeat(yv[k][None], 2 * len(eidx), axis=0), w=Wp)
        for j, i in enumerate(idx):
            a, b = Xp[j], Xp[len(idx) + j]
            if np.array_equal(props.run_structure(a), st0) and np.array_equal(props.run_structure(b), st0):
                fd = (gv[k] @ a - gv[k] @ b) / (2 * h)
                assert abs(fd - dy[k, i]) <= 1e-4 * max(1.0, abs(fd)), (k, i, fd, dy[k, i])
                checked += 1
        for j, e in enumerate(eidx):
            a, b = Xw[j], Xw[len(eidx) + j]
            if np.array_equal(props.run_structure(a), st0) and np.array_equal(props.run_structure(b), st0):
                fd = (gv[k] @ a - gv[k] @ b) / (2 * h)
                assert abs(fd - dw[k, e]) <= 1e-4 * max(1.0, abs(fd)), (k, e, fd, dw[k, e])
                checked += 1
    assert checked > 1500


def test_autograd_and_scalar_weight():
    y, w, g = _workload(40, 300, seed=9)
    yt = _dev(y, torch.float64).requires_grad_(True)
    wt = _dev(w, torch.float64).requires_grad_(True)
    gt = _dev(g, torch.float64)
    x = binding.prox(yt, wt, dim=-1)
    (x * gt).sum().backward()
    xo = oracle.chain_prox(y, w=w)
    dyo, dwo = oracle.chain_adjoint(xo, g)
    assert np.abs(yt.grad.cpu().numpy() - dyo).max() < 1e-12
    assert np.abs(wt.grad.cpu().numpy()[:, :-1] - dwo[:, :-1]).max() < 1e-12
    # scalar weight: per-chain sum of the edge gradients
    x2 = binding.chain_prox(_dev(y, torch.float64), 0.4, dim=-1)
    _, dws = binding.chain_prox_backward(x2, gt, dim=-1, per_edge_w=False)
    xo2 = oracle.chain_prox(y, w_scalar=0.4)
    _, dwso = oracle.chain_adjoint(xo2, g, scalar_w=True)
    assert np.abs(dws.cpu().numpy() - dwso).max() < 1e-12
    # scalar-weight autograd: gradient flows to y only
    y3 = _dev(y, torch.float64).requires_grad_(True)
    (binding.prox(y3, 0.4, dim=-1) * gt).sum().backward()
    dyo2, _ = oracle.chain_adjoint(xo2, g)
    assert np.abs(y3.grad.cpu().numpy() - dyo2).max() < 1e-12


def test_column_layout_backward():
    y, w, g = _workload(50, 200, seed=11)
    xt = binding.chain_prox(_dev(y.T.copy(), torch.float64), _dev(w.T.copy(), torch.float64), dim=0)
    dy, dw = binding.chain_prox_backward(xt, _dev(g.T.copy(), torch.float64), dim=0, per_edge_w=True)
    xo = oracle.chain_prox(y, w=w)
    dyo, dwo = oracle.chain_adjoint(xo, g)
    assert np.abs(dy.cpu().numpy().T - dyo).max() < 1e-12
    assert np.abs(dw.cpu().numpy().T[:, :-1] - dwo[:, :-1]).max() < 1e-12


def _designed_runs(n, seed):
    """Chains whose run structure is set by hand: ends exactly at the 1024-node
    chunk edges, one run over the whole chain, ends next to chunk edges, long
    random runs, short random runs and all-singleton runs."""
    rng = np.random.default_rng(seed)
    rows = []
    def from_bounds(bounds):
        x = np.zeros(n)
        level = 0.0
        prev = 0
        for bnd in list(bounds) + [n]:
            level += rng.choice([-1.0, 1.0]) * rng.uniform(0.1, 1.0)
            x[prev:bnd] = level
            prev = bnd
        return x
    rows.append(from_bounds(range(1024, n, 1024)))
    rows.append(np.full(n, 0.7))
    rows.append(from_bounds(sorted({1023, 1025, 2047, 2049, 3071})))
    long_runs = np.cumsum(rng.geometric(1 / 300, size=64))
    rows.append(from_bounds(long_runs[long_runs < n]))
    rows.append(from_bounds(np.unique(rng.integers(1, n, size=n // 5))))
    rows.append(rng.normal(size=n))
    rows.append(from_bounds([1]))
    rows.append(from_bounds([n - 1]))
    return np.array(rows)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
@pytest.mark.parametrize("n", [4100, 1024, 2048, 37])
def test_rows_adjoint_across_chunks(dtype, tol, n):
    """Unit-stride adjoint (wave per chain, 1024-node chunks): runs crossing,
    ending at and spanning chunk edges, against the oracle's formulas."""
    x = _designed_runs(n, seed=n)
    g = synth.normal(x.shape, seed=n + 1)
    xt, gt = _dev(x, dtype), _dev(g, dtype)
    dy, dw = binding.chain_prox_backward(xt, gt, dim=-1, per_edge_w=True)
    _, dws = binding.chain_prox_backward(xt, gt, dim=-1, per_edge_w=False, need_y=False)
    xv, gv = xt.double().cpu().numpy(), gt.double().cpu().numpy()
    dyo, dwo = oracle.chain_adjoint(xv, gv)
    _, dwso = oracle.chain_adjoint(xv, gv, scalar_w=True)
    scale = max(1.0, np.abs(dyo).max())
    assert np.abs(dy.double().cpu().numpy() - dyo).max() <= tol * scale
    assert np.abs(dw.double().cpu().numpy()[:, :-1] - dwo[:, :-1]).max() <= tol * scale
    assert (dw.double().cpu().numpy()[:, -1] == 0).all()
    assert np.abs(dws.double().cpu().numpy() - dwso).max() <= tol * max(1.0, np.abs(dwso).max()) * 10


def test_rows_adjoint_csr_chains():
    """Uneven chains given by CSR offsets go through the unit-stride adjoint."""
    import ctypes
    rng = np.random.default_rng(3)
    lens = [1, 2, 1023, 1024, 1025, 3000, 0, 77]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xs = [np.repeat(rng.normal(size=max(1, L // 50 + 1)), 50)[:L] for L in lens]
    x = np.concatenate(xs)
    g = rng.normal(size=x.size)
    xt, gt = _dev(x, torch.float64), _dev(g, torch.float64)
    dy = torch.empty_like(xt)
    dw = torch.empty_like(xt)
    ot = torch.tensor(offs, device="cuda")
    lib = binding.load()
    lay = binding.ChainLayout(len(lens), max(lens), 1, 1, ctypes.c_void_p(ot.data_ptr()))
    st = lib.tv_chain_prox_backward(ctypes.byref(lay), binding.TV_F64, ctypes.c_void_p(xt.data_ptr()),
                                    ctypes.c_void_p(gt.data_ptr()), ctypes.c_void_p(dy.data_ptr()),
                                    ctypes.c_void_p(dw.data_ptr()), 1, None, 0,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    dyv, dwv = dy.cpu().numpy(), dw.cpu().numpy()
    for c, L in enumerate(lens):
        if L == 0:
            continue
        sl = slice(offs[c], offs[c + 1])
        dyo, dwo = oracle.chain_adjoint(x[sl][None], g[sl][None])
        assert np.abs(dyv[sl] - dyo[0]).max() < 1e-12
        assert np.abs(dwv[sl][:-1] - dwo[0][:-1]).max(initial=0.0) < 1e-12
