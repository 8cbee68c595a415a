"""GPU parity for Sec. 3, Extensions (i) (tv_chain_nc_concave): chains whose
pairwise terms are minima of one-sided linear pieces, against the FP64 oracle
(ncg_chain), compared by energy per chain (minimisers need not be unique)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1502_07770_amd import binding, synth
from tests.test_oracle_nc import _rand_unaries
from tests.test_oracle_ncg import _rand_pieces

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _batch(g, lengths, tmax=3):
    """Chains of the given lengths, concatenated: unaries, pieces (the last node
    of each chain gets pieces too; they are ignored), chain offsets."""
    N = int(sum(lengths))
    uoff, ulam, usl = _rand_unaries(g, N, tmax=tmax)
    poff, al, cc, sd = _rand_pieces(g, N)
    coff = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return coff, (uoff, ulam, usl), (poff, al, cc, sd)


def _sub(coff, u, p, c):
    """Chain c as a stand-alone problem for the oracle."""
    n0, n1 = int(coff[c]), int(coff[c + 1])
    uoff, ulam, usl = u
    poff, al, cc, sd = p
    uo = uoff[n0:n1 + 1] - uoff[n0]
    su = (uo, ulam[uoff[n0]:uoff[n1]], usl[uoff[n0] + n0:uoff[n1] + n1])
    po = poff[n0:n1 + 1] - poff[n0]
    sp = (po, al[poff[n0]:poff[n1]], cc[poff[n0]:poff[n1]], sd[poff[n0]:poff[n1]])
    return n0, n1, su, sp


def _run(coff, u, p, dtype, **kw):
    uoff, ulam, usl = u
    poff, al, cc, sd = p
    return binding.chain_nc_concave(_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, dtype),
                                    _dev(usl, dtype), _dev(poff, torch.int64), _dev(al, dtype), _dev(cc, dtype),
                                    _dev(sd, torch.int32), **kw).double().cpu().numpy()


def _check(coff, u, p, x, chains, tol_rel, tol_node=0.0):
    for c in chains:
        n0, n1, su, sp = _sub(coff, u, p, c)
        if n1 == n0:
            continue
        xo, _ = oracle.ncg_chain(*su, *sp)
        eo = oracle.ncg_energy(*su, *sp, xo)
        eg = oracle.ncg_energy(*su, *sp, x[n0:n1])
        assert abs(eg - eo) <= tol_rel * (1 + abs(eo)) + tol_node * (n1 - n0), (c, n1 - n0, eo, eg)


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_random_chains_match_the_oracle(dtype):
    g = np.random.default_rng(50)
    lengths = np.concatenate([[0, 1, 2], g.integers(1, 90, 197)])
    coff, u, p = _batch(g, lengths)
    if dtype == torch.float32:
        u = (u[0], _f32(u[1]), _f32(u[2]))
        p = (p[0], _f32(p[1]), _f32(p[2]), p[3])
    x = _run(coff, u, p, dtype)
    if dtype == torch.float64:
        _check(coff, u, p, x, range(lengths.size), 1e-9)
    else:
        _check(coff, u, p, x, range(lengths.size), 1e-6, 8 * 2.0 ** -23 * (np.abs(u[1]).max() + 1) * 4)


def test_truncated_tv_pieces_match_the_truncated_tv_solver():
    g = np.random.default_rng(51)
    lengths = g.integers(2, 120, 100)
    N = int(lengths.sum())
    coff = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    uoff, ulam, usl = _rand_unaries(g, N, tmax=4)
    w = g.uniform(0, 2, N)
    C = np.where(g.random(N) < 0.3, np.inf, g.uniform(0.2, 3, N))
    poff, al, cc, sd = [0], [], [], []
    for i in range(N):
        for s in (1, -1):
            al.append(w[i]), cc.append(0.0), sd.append(s)
            if np.isfinite(C[i]):
                al.append(0.0), cc.append(C[i]), sd.append(s)
        poff.append(len(al))
    p = (np.array(poff, dtype=np.int64), np.array(al), np.array(cc), np.array(sd, dtype=np.int32))
    x = _run(coff, (uoff, ulam, usl), p, torch.float64)
    xt = binding.chain_nc(_dev(coff, torch.int64), _dev(uoff, torch.int64), _dev(ulam, torch.float64),
                          _dev(usl, torch.float64), _dev(w, torch.float64), _dev(C, torch.float64)).cpu().numpy()
    for c in range(lengths.size):
        n0, n1 = int(coff[c]), int(coff[c + 1])
        uo = uoff[n0:n1 + 1] - uoff[n0]
        su = (uo, ulam[uoff[n0]:uoff[n1]], usl[uoff[n0] + n0:uoff[n1] + n1])
        e1 = oracle.nc_energy(*su, w[n0:n1 - 1], C[n0:n1 - 1], x[n0:n1])
        e2 = oracle.nc_energy(*su, w[n0:n1 - 1], C[n0:n1 - 1], xt[n0:n1])
        assert abs(e1 - e2) <= 1e-9 * (1 + abs(e2)), (c, e1, e2)


def test_rejections():
    g = np.random.default_rng(52)
    lengths = np.array([10, 12, 7])
    coff, u, p = _batch(g, lengths)
    poff, al, cc, sd = p
    for bad in ("side", "alpha", "C"):
        al2, cc2, sd2 = al.copy(), cc.copy(), sd.copy()
        k = int(poff[3])  # a piece of an edge inside the first chain
        if bad == "side":
            sd2[k] = 0
        elif bad == "alpha":
            al2[k] = -0.5
        else:
            cc2[k] = np.inf
        with pytest.raises(binding.TvChainError) as e:
            _run(coff, u, (poff, al2, cc2, sd2), torch.float64)
        assert e.value.status == binding.TV_ERR_INVALID_ARG
    with pytest.raises(binding.TvChainError) as e:
        _run(coff, u, p, torch.float64, msg_cap=2)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    with pytest.raises(binding.TvChainError) as e:
        _run(coff, u, p, torch.float64, map_cap=1)
    assert e.value.status == binding.TV_ERR_WORKSPACE
    x = _run(coff, u, p, torch.float64)  # and the same call with room
    _check(coff, u, p, x, range(3), 1e-9)


def test_full_size_sampled_chains():
    """16,384 chains of 256 nodes, 16-level costs, min(|z|, 0.25 |z| + 1, 2.5)
    on every edge (three pieces per side), FP32, in the benchmark's launch."""
    coff, u, p = synth.concave_cost_chains(16384, 256, 16, seed=9)
    u = (u[0], u[1], _f32(u[2]))
    x = _run(coff, u, p, torch.float32, msg_cap=128, map_cap=8192)
    pick = np.sort(np.random.default_rng(53).choice(coff.size - 1, 300, replace=False))
    _check(coff, u, p, x, pick, 1e-6, 8 * 2.0 ** -23 * 20)


@pytest.mark.parametrize("msg_cap", [8192, 256, 128])
def test_lane_and_wave_kernels_match_the_oracle(msg_cap):
    """msg_cap above 256: a lane per chain with the messages in the workspace;
    256 and 128: a wave per chain with the messages in LDS (two sizes)."""
    g = np.random.default_rng(54)
    lengths = np.concatenate([[0, 1], g.integers(1, 80, 118)])
    coff, u, p = _batch(g, lengths)
    x = _run(coff, u, p, torch.float64, msg_cap=msg_cap)
    _check(coff, u, p, x, range(lengths.size), 1e-9)


@pytest.mark.parametrize("kind", ["potts", "monotone", "equal"])
def test_special_piece_sets(kind):
    """Potts (0, C) on both sides; one-sided pieces (x non-decreasing along the
    chain); no pieces at all (every chain at one value)."""
    g = np.random.default_rng(55)
    lengths = g.integers(1, 70, 80)
    N = int(lengths.sum())
    coff = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    u = _rand_unaries(g, N)
    if kind == "potts":
        p = (np.arange(N + 1, dtype=np.int64) * 2, np.zeros(2 * N), g.uniform(0, 3, 2 * N),
             np.tile(np.array([1, -1], dtype=np.int32), N))
    elif kind == "monotone":
        p = (np.arange(N + 1, dtype=np.int64), g.uniform(0, 1, N), g.uniform(0, 1, N), np.ones(N, dtype=np.int32))
    else:
        p = (np.zeros(N + 1, dtype=np.int64), np.zeros(0), np.zeros(0), np.zeros(0, dtype=np.int32))
    x = _run(coff, u, p, torch.float64)
    _check(coff, u, p, x, range(lengths.size), 1e-9)
    for c in range(lengths.size):
        seg = x[coff[c]:coff[c + 1]]
        if kind == "monotone":
            assert np.all(np.diff(seg) >= 0)
        if kind == "equal":
            assert np.all(seg == seg[0])


def test_cost_volume_rows_sampled():
    """The 1000 rows (1482 nodes, 64 levels) of the synthetic cost volume with
    min(0.6 |z|, 0.15 |z| + 1, 2), FP32 in, in the benchmark's launch (a wave
    per row); 24 sampled rows checked."""
    coff, u, p = synth.concave_cost_volume_rows(1000, 1482, 64, seed=1)
    u = (u[0], _f32(u[1]), _f32(u[2]))
    x = _run(coff, u, p, torch.float32, msg_cap=256, map_cap=64 * 1482)
    pick = np.sort(np.random.default_rng(56).choice(1000, 24, replace=False))
    _check(coff, u, p, x, pick, 1e-6, 8 * 2.0 ** -23 * 70)
