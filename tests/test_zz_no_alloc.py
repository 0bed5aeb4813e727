"""ttm_chain_noalloc (the entry point for callers that cannot allocate)
against ttm_chain, through the C interface.

Two calls in a row on the library's per-GPU scratch, the second with a
smaller problem, each compared bit for bit with ttm_chain on a caller
workspace (the same kernels in the same order) and with the FP64 oracle at
the form's tolerance; a shape whose workspace exceeds the scratch is refused
before anything is launched.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2411_13532_amd import _lib, chain, workloads
from tests import pins

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-5, "bf16": 2e-2}
DT = {torch.float64: _lib.TTM_F64, torch.float32: _lib.TTM_F32, torch.bfloat16: _lib.TTM_BF16}


def _noalloc(X, A, B, C, math):
    lib = _lib.load()
    J = (A.shape[0], B.shape[0], C.shape[0])
    Y = torch.full(J, float("nan"), dtype=torch.float64 if math == "f64" else torch.float32, device=DEV)
    s = _lib.shape(tuple(X.shape), J)
    rc = lib.ttm_chain_noalloc(ctypes.byref(s), ctypes.c_void_p(X.data_ptr()), DT[X.dtype],
                               ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                               ctypes.c_void_p(C.data_ptr()), DT[A.dtype], ctypes.c_void_p(Y.data_ptr()),
                               DT[Y.dtype], _lib.MATH[math],
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.TTM_OK, _lib.status_string(rc)
    return Y


CASES = [("bf16x3", torch.bfloat16), ("bf16", torch.bfloat16), ("f32", torch.float32), ("f64", torch.float64)]


@pytest.mark.parametrize("math,xdt", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_chain_twice(math, xdt):
    fdt = torch.float64 if math == "f64" else torch.float32
    # first call: several row tiles and k chunks; second: a smaller problem
    # on the same scratch, so stale contents of the first would show
    for k, (I, J) in enumerate((((64, 600, 256), (20, 40, 70)), ((7, 100, 64), (5, 12, 20)))):
        p = workloads.random_problem(I, J, seed=71 + k)
        X = torch.from_numpy(p["X"]).to(DEV).to(xdt).contiguous()
        A, B, C = (torch.from_numpy(p[n]).to(DEV).to(fdt).contiguous() for n in "ABC")
        ws = _lib.load().ttm_chain_workspace_size(ctypes.byref(_lib.shape(I, J)), DT[xdt], _lib.MATH[math])
        assert 0 < ws <= _lib.TTM_NOALLOC_SCRATCH_BYTES
        Yn = _noalloc(X, A, B, C, math)
        Yw = chain(X, A, B, C, math=math)
        torch.cuda.synchronize()
        assert torch.equal(Yn, Yw), (math, k)
        Xs = X.float().cpu().numpy() if xdt == torch.bfloat16 else X.cpu().numpy()
        ref = oracle.chain(Xs, *(t.cpu().numpy() for t in (A, B, C)))
        err = pins.rel_fro(Yn.double().cpu().numpy(), ref)
        print(f"[noalloc {math} call {k}] rel err {err:.3e}", flush=True)
        assert err <= TOL[math]


def test_noalloc_refuses_shapes_beyond_the_scratch():
    lib = _lib.load()
    s = _lib.shape((1024, 1024, 1024), (128, 128, 128))
    assert lib.ttm_chain_workspace_size(ctypes.byref(s), _lib.TTM_BF16, _lib.MATH["bf16x3"]) > \
        _lib.TTM_NOALLOC_SCRATCH_BYTES
    # refused by the host check before any launch: the pointers are never used
    fake = [ctypes.c_void_p((1 << 40) + (k << 34)) for k in range(5)]
    rc = lib.ttm_chain_noalloc(ctypes.byref(s), fake[0], _lib.TTM_BF16, fake[1], fake[2], fake[3], _lib.TTM_F32,
                               fake[4], _lib.TTM_F32, _lib.MATH["bf16x3"], None)
    assert rc == _lib.TTM_ERR_WORKSPACE
