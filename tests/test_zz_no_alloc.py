"""tv_chain_prox_noalloc (the entry point for callers that cannot allocate):
called through the C ABI with caller-owned inputs and outputs only, it must
give what tv_chain_prox gives with a caller workspace -- bit for bit, since
both run the same kernels under the same plan -- on two calls in a row, the
second with a smaller problem (the scratch keeps the first call's contents),
and reject a problem larger than its scratch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1502_07770_amd import binding, synth

pytestmark = pytest.mark.gpu

P = ctypes.c_void_p


def _with_workspace(lib, lay, code, y, w, w_scalar):
    x = torch.empty_like(y)
    nb = lib.tv_chain_prox_workspace(ctypes.byref(lay), code)
    ws = torch.empty(nb, dtype=torch.uint8, device=y.device)
    st = lib.tv_chain_prox(ctypes.byref(lay), code, P(y.data_ptr()), P(w.data_ptr()) if w is not None else None,
                           w_scalar, P(x.data_ptr()), P(ws.data_ptr()), nb, None)
    assert st == binding.TV_OK
    return x


def _noalloc(lib, lay, code, y, w, w_scalar):
    x = torch.full_like(y, float("nan"))
    torch.cuda.synchronize()
    st = lib.tv_chain_prox_noalloc(ctypes.byref(lay), code, P(y.data_ptr()),
                                   P(w.data_ptr()) if w is not None else None, w_scalar, P(x.data_ptr()), None)
    assert st == binding.TV_OK, binding.status_string(st)
    return x


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_the_workspace_call(dtype):
    lib = binding.load()
    code = binding.TV_F32 if dtype == torch.float32 else binding.TV_F64
    cases = [(300, 2000, 0.5, False), (70, 900, 0.2, True)]  # the second call is smaller
    for C, n, wval, per_edge in cases:
        y = torch.tensor(synth.piecewise_constant(C, n, seed=C + n), dtype=dtype, device="cuda")
        w = torch.tensor(synth.edge_weights((C, n), seed=n), dtype=dtype, device="cuda") if per_edge else None
        lay = binding.ChainLayout(C, n, 1, n, None)
        ref = _with_workspace(lib, lay, code, y, w, wval)
        got = _noalloc(lib, lay, code, y, w, wval)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (C, n, (got - ref).abs().max().item())
        # the same rows through the binding's wrapper of the entry point
        x2 = binding.chain_prox_noalloc(y, torch.empty_like(y), w if per_edge else wval)
        assert torch.equal(x2, ref)


def test_noalloc_rejects_a_problem_beyond_its_scratch():
    lib = binding.load()
    C, n = 4096, 4096  # 16.8 M nodes: its lambda stream alone exceeds the scratch
    lay = binding.ChainLayout(C, n, 1, n, None)
    assert lib.tv_chain_prox_workspace(ctypes.byref(lay), binding.TV_F32) > (64 << 20)
    y = torch.zeros((C, n), dtype=torch.float32, device="cuda")
    x = torch.empty_like(y)
    st = lib.tv_chain_prox_noalloc(ctypes.byref(lay), binding.TV_F32, P(y.data_ptr()), None, 0.1,
                                   P(x.data_ptr()), None)
    assert st == binding.TV_ERR_WORKSPACE
