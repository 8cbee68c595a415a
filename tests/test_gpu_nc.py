"""GPU parity for the Sec. 3 non-convex chains (tv_chain_nc) against the FP64
oracle.  Minimisers of a non-convex energy need not be unique, so each chain is
compared by energy: the GPU's x must reach the oracle's minimum energy (FP64:
to 1e-9 relative; FP32: inputs rounded to FP32 first, and the energy of the
FP32-rounded output within the rounding of x times the largest slope)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth

pytestmark = pytest.mark.gpu


def _rand_batch(g, num_chains, nmax, tmax=5, trunc_frac=0.5, ragged=True):
    lens = g.integers(1, nmax + 1, num_chains) if ragged else np.full(num_chains, nmax)
    coff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    N = int(coff[-1])
    ts = g.integers(1, tmax + 1, N)
    uoff = np.concatenate([[0], np.cumsum(ts)]).astype(np.int64)
    ulam = np.concatenate([np.cumsum(np.concatenate([[g.normal() * 2], g.uniform(0, 2, t - 1)])) for t in ts])
    sl = []
    for t in ts:
        s = g.normal(size=t + 1) * 2
        s[0] = -abs(s[0]) - 0.05
        s[-1] = abs(s[-1]) + 0.05
        sl.append(s)
    usl = np.concatenate(sl)
    w = g.uniform(0, 2, N)
    C = np.where(g.random(N) < trunc_frac, g.uniform(0.1, 3, N), np.inf)
    return coff, uoff, ulam, usl, w, C


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _check(coff, uoff, ulam, usl, w, C, x, tol_rel, tol_abs_per_node=0.0):
    worst = 0.0
    for c in range(coff.size - 1):
        n0, n1 = int(coff[c]), int(coff[c + 1])
        if n1 <= n0:
            continue
        uo = uoff[n0:n1 + 1] - uoff[n0]
        l = ulam[uoff[n0]:uoff[n1]]
        s = usl[uoff[n0] + n0:uoff[n1] + n1]
        xo, _ = oracle.nc_chain(uo, l, s, w[n0:n1 - 1], C[n0:n1 - 1])
        eo = oracle.nc_energy(uo, l, s, w[n0:n1 - 1], C[n0:n1 - 1], xo)
        eg = oracle.nc_energy(uo, l, s, w[n0:n1 - 1], C[n0:n1 - 1], x[n0:n1])
        tol = tol_rel * (1 + abs(eo)) + tol_abs_per_node * (n1 - n0)
        assert eg <= eo + tol and eg >= eo - tol, (c, n1 - n0, eo, eg)
        worst = max(worst, abs(eg - eo))
    return worst


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_random_ragged_batches(dtype):
    g = np.random.default_rng(3)
    for trial in range(3):
        coff, uoff, ulam, usl, w, C = _rand_batch(g, 150, 120, trunc_frac=(0.0, 0.5, 1.0)[trial])
        if dtype == torch.float32:  # the oracle sees the rounded inputs
            ulam, usl, w = (a.astype(np.float32).astype(np.float64) for a in (ulam, usl, w))
            C = C.astype(np.float32).astype(np.float64)
        x = binding.chain_nc(_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, dtype), _dev(usl, dtype),
                             _dev(w, dtype), _dev(C, dtype)).double().cpu().numpy()
        if dtype == torch.float64:
            _check(coff, uoff, ulam, usl, w, C, x, 1e-9)
        else:
            # x rounded to FP32: |dx| <= 2^-24 |x| per node, times slopes up to ~8
            _check(coff, uoff, ulam, usl, w, C, x, 1e-6, 8 * 2.0 ** -23 * (np.abs(ulam).max() + 1) * 4)


def test_plain_tv_without_C_and_single_nodes():
    g = np.random.default_rng(4)
    coff, uoff, ulam, usl, w, _ = _rand_batch(g, 64, 40, trunc_frac=0.0)
    coff = np.concatenate([coff, coff[-1] + np.arange(1, 4)]).astype(np.int64)  # three 1-node chains
    extra_t = 3
    N0 = uoff.size - 1
    uoff = np.concatenate([uoff, uoff[-1] + extra_t * np.arange(1, 4)]).astype(np.int64)
    ulam = np.concatenate([ulam, np.tile([-1.0, 0.5, 2.0], 3)])
    usl = np.concatenate([usl, np.tile([-1.0, 0.5, -0.25, 1.0], 3)])
    w = np.concatenate([w, np.ones(3)])
    x = binding.chain_nc(_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64),
                         _dev(usl, torch.float64), _dev(w, torch.float64), None).cpu().numpy()
    _check(coff, uoff, ulam, usl, w, np.full(w.size, np.inf), x, 1e-9)
    # a 1-node chain sits at its unary's minimum: f(-1) = 0, f(0.5) = 0.75, f(2) = 0.375
    assert np.allclose(x[N0:], -1.0)


def test_cost_volume_rows():
    coff, uoff, ulam, usl, dt = synth.cost_volume_chains(24, 160, 32, seed=5)
    N = uoff.size - 1
    w = np.full(N, 0.6)
    C = np.full(N, 2.0)
    for dtype in (torch.float64, torch.float32):
        l, s, ww, cc = ulam, usl, w, C
        if dtype == torch.float32:
            l, s, ww, cc = (a.astype(np.float32).astype(np.float64) for a in (ulam, usl, w, C))
        x = binding.chain_nc(_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(l, dtype), _dev(s, dtype),
                             _dev(ww, dtype), _dev(cc, dtype), msg_cap=512).double().cpu().numpy()
        _check(coff, uoff, l, s, ww, cc, x, 1e-9 if dtype == torch.float64 else 1e-5, 1e-4)


def test_rejections():
    g = np.random.default_rng(7)
    coff, uoff, ulam, usl, w, C = _rand_batch(g, 8, 30)
    args = [_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64)]
    bad = usl.copy()
    bad[0] = 0.5  # unbounded below
    with pytest.raises(binding.TvChainError) as e:
        binding.chain_nc(*args, _dev(bad, torch.float64), _dev(w, torch.float64), _dev(C, torch.float64))
    assert e.value.status == binding.TV_ERR_INVALID_ARG
    with pytest.raises(binding.TvChainError) as e:  # a message longer than msg_cap
        binding.chain_nc(*args, _dev(usl, torch.float64), _dev(w, torch.float64), _dev(C, torch.float64), msg_cap=2)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    with pytest.raises(binding.TvChainError) as e:  # too few mapping intervals
        binding.chain_nc(*args, _dev(usl, torch.float64), _dev(w, torch.float64), _dev(C, torch.float64), map_cap=1)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    # the same call with room succeeds afterwards
    x = binding.chain_nc(*args, _dev(usl, torch.float64), _dev(w, torch.float64), _dev(C, torch.float64))
    _check(coff, uoff, ulam, usl, w, C, x.cpu().numpy(), 1e-9)


def test_hbm_message_buffers_match_lds_ones():
    """msg_cap too large for LDS puts the message buffers in the workspace: the
    same results as the LDS path."""
    g = np.random.default_rng(8)
    coff, uoff, ulam, usl, w, C = _rand_batch(g, 70, 80)
    args = [_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64), _dev(usl, torch.float64),
            _dev(w, torch.float64), _dev(C, torch.float64)]
    a = binding.chain_nc(*args, msg_cap=512)   # one lane per chain, buffers in LDS
    b = binding.chain_nc(*args, msg_cap=8192)  # one lane per chain, buffers in HBM
    assert torch.equal(a, b)
    _check(coff, uoff, ulam, usl, w, C, b.cpu().numpy(), 1e-9)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_wave_kernel_matches_the_oracle(dtype):
    """msg_cap <= 256 selects a wave per chain (prefix-minimum form of Algorithm 1):
    the same minimum energies as the oracle and as the one-lane kernel."""
    g = np.random.default_rng(21)
    for trial in range(3):
        coff, uoff, ulam, usl, w, C = _rand_batch(g, 120, 150, trunc_frac=(0.0, 0.5, 1.0)[trial])
        if trial == 1:
            w[g.random(w.size) < 0.2] = 0.0
        if dtype == torch.float32:
            ulam, usl, w = (a.astype(np.float32).astype(np.float64) for a in (ulam, usl, w))
            C = C.astype(np.float32).astype(np.float64)
        args = [_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, dtype), _dev(usl, dtype),
                _dev(w, dtype), _dev(C, dtype)]
        xw = binding.chain_nc(*args, msg_cap=256).double().cpu().numpy()
        xl = binding.chain_nc(*args, msg_cap=1024).double().cpu().numpy()
        if dtype == torch.float64:
            _check(coff, uoff, ulam, usl, w, C, xw, 1e-9)
        else:
            _check(coff, uoff, ulam, usl, w, C, xw, 1e-6, 8 * 2.0 ** -23 * (np.abs(ulam).max() + 1) * 4)
        del xl


def test_wave_kernel_cost_volume_and_capacity():
    coff, uoff, ulam, usl, _ = synth.cost_volume_chains(32, 300, 64, seed=8)
    N = uoff.size - 1
    w = np.full(N, 0.6)
    C = np.full(N, 2.0)
    args = [_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64), _dev(usl, torch.float64),
            _dev(w, torch.float64), _dev(C, torch.float64)]
    x = binding.chain_nc(*args, msg_cap=256).cpu().numpy()
    _check(coff, uoff, ulam, usl, w, C, x, 1e-9)
    x = binding.chain_nc(*args, msg_cap=128).cpu().numpy()  # the 16 KiB wave variant
    _check(coff, uoff, ulam, usl, w, C, x, 1e-9)
    with pytest.raises(binding.TvChainError) as e:  # 64-breakpoint unaries do not fit 40
        binding.chain_nc(*args, msg_cap=40)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    with pytest.raises(binding.TvChainError) as e:
        binding.chain_nc(*args, msg_cap=256, map_cap=100)
    assert e.value.status == binding.TV_ERR_WORKSPACE


def test_full_bench_size_sampled_rows():
    """The bench's workload (1000 rows x 1482 of the 64-level cost volume, FP32,
    w = 0.6, C = 2, msg_cap = 256: the wave kernel), checked on 8 sampled rows."""
    coff, uoff, ulam, usl, _ = synth.cost_volume_chains(1000, 1482, 64, seed=1)
    N = uoff.size - 1
    w = np.full(N, 0.6)
    C = np.full(N, 2.0)
    x = binding.chain_nc(_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float32),
                         _dev(usl, torch.float32), _dev(w, torch.float32), _dev(C, torch.float32),
                         msg_cap=256).double().cpu().numpy()
    l32, s32 = ulam.astype(np.float32).astype(np.float64), usl.astype(np.float32).astype(np.float64)
    rows = np.random.default_rng(0).choice(1000, 8, replace=False)
    sub = np.concatenate([[0], np.cumsum(np.full(8, 1482))]).astype(np.int64)
    nodes = np.concatenate([np.arange(r * 1482, (r + 1) * 1482) for r in rows])
    uo = np.arange(nodes.size + 1, dtype=np.int64) * 64
    ll = np.concatenate([l32[i * 64:(i + 1) * 64] for i in nodes])
    ss = np.concatenate([s32[i * 65 + 0:i * 65 + 65] for i in nodes])
    _check(sub, uo, ll, ss, w[nodes], C[nodes], x[nodes], 1e-6, 1e-4)


def test_chain_ranges_outside_the_nodes_are_rejected():
    g = np.random.default_rng(30)
    coff, uoff, ulam, usl, w, C = _rand_batch(g, 6, 20)
    bad = coff.copy()
    bad[-1] += 5  # past num_nodes
    for cap in (256, 1024):  # wave and lane kernels
        with pytest.raises(binding.TvChainError) as e:
            binding.chain_nc(_dev(bad, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64),
                             _dev(usl, torch.float64), _dev(w, torch.float64), _dev(C, torch.float64), msg_cap=cap)
        assert e.value.status == binding.TV_ERR_INVALID_ARG
