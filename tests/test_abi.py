"""The C interface of libttm: exported symbols and argument validation.

Runs on the CPU: every call here fails validation before any HIP call is
made (pointers are plain integers that are never dereferenced).
"""
import ctypes
import os
import re

import pytest

from paper_2411_13532_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ttm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)
    assert not _lib.MISSING


def test_slab_kernel_selection_range(lib):
    for mode in (-1, 4, 5, 100):
        assert lib.ttm_set_slab_kernel(mode) == -1
    for mode in (3, 2, 1, 0):
        assert lib.ttm_set_slab_kernel(mode) == 0


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert lib.ttm_status_string(code)
    assert lib.ttm_version() >= 10000


def test_supported_combinations(lib):
    F64, F32, BF16 = _lib.TTM_F64, _lib.TTM_F32, _lib.TTM_BF16
    m = _lib.MATH
    ok = [(F64, F64, F64, m["f64"]), (F32, F32, F32, m["f32"]), (F32, F32, F32, m["bf16"]),
          (F32, F32, F32, m["bf16x3"]), (BF16, F32, F32, m["f32"]), (BF16, F32, F32, m["bf16"]),
          (BF16, F32, F32, m["bf16x3"])]
    for c in ok:
        assert lib.ttm_chain_supported(*c) == 1, c
    bad = [(F64, F64, F64, m["f32"]), (F32, F64, F32, m["f32"]), (BF16, BF16, F32, m["bf16"]),
           (F32, F32, BF16, m["f32"]), (F64, F32, F32, m["bf16x3"]), (F32, F32, F32, 9)]
    for c in bad:
        assert lib.ttm_chain_supported(*c) == 0, c


def shp(I, J):
    return ctypes.byref(_lib.shape(I, J))


def test_workspace_query(lib):
    m = _lib.MATH
    assert lib.ttm_chain_workspace_size(shp((64, 64, 64), (16, 16, 16)), _lib.TTM_F64, m["f64"]) > 0
    ws_c3 = lib.ttm_chain_workspace_size(shp((1024, 1024, 1024), (128, 128, 128)), _lib.TTM_BF16, m["bf16x3"])
    # factors (hi+lo) plus the mode-2 partials V (I1 x J2 x J3 float) and mode-1 split partials
    assert 64 << 20 <= ws_c3 <= 160 << 20
    assert lib.ttm_chain_workspace_size(shp((0, 4, 4), (2, 2, 2)), _lib.TTM_F32, m["f32"]) == 0
    assert lib.ttm_chain_workspace_size(shp((4, 4, 4), (2, 2, 2)), _lib.TTM_F64, m["f32"]) == 0
    assert lib.ttm_chain_workspace_size(None, _lib.TTM_F32, m["f32"]) == 0
    assert lib.ttm_chain_backward_workspace_size(shp((8, 9, 10), (2, 3, 4)), _lib.TTM_F32, m["f32"]) > 0
    assert lib.ttm_chain_backward_workspace_size(shp((8, 9, 10), (2, 3, 4)), _lib.TTM_F32, m["bf16"]) == 0


FAKE = 1 << 40   # an address that is never dereferenced


def call_chain(lib, I=(8, 8, 8), J=(4, 4, 4), X=FAKE, A=FAKE + (1 << 30), B=FAKE + (2 << 30),
               C=FAKE + (3 << 30), Y=FAKE + (4 << 30), ws=FAKE + (5 << 30), ws_bytes=1 << 30,
               xdt=_lib.TTM_F32, fdt=_lib.TTM_F32, ydt=_lib.TTM_F32, math=_lib.MATH["f32"], shape=True):
    s = shp(I, J) if shape else None
    P = ctypes.c_void_p
    return lib.ttm_chain(s, P(X), xdt, P(A), P(B), P(C), fdt, P(Y), ydt, math, P(ws), ws_bytes, P(0))


def test_chain_validation_errors(lib):
    E = _lib
    assert call_chain(lib, shape=False) == E.TTM_ERR_INVALID_ARG
    assert call_chain(lib, I=(0, 8, 8)) == E.TTM_ERR_INVALID_ARG
    assert call_chain(lib, J=(4, -1, 4)) == E.TTM_ERR_INVALID_ARG
    assert call_chain(lib, X=0) == E.TTM_ERR_INVALID_ARG
    assert call_chain(lib, C=0) == E.TTM_ERR_INVALID_ARG
    assert call_chain(lib, Y=0) == E.TTM_ERR_INVALID_ARG
    assert call_chain(lib, X=FAKE + 4) == E.TTM_ERR_INVALID_ARG          # X not 16-byte aligned
    assert call_chain(lib, A=FAKE + (1 << 30) + 2) == E.TTM_ERR_INVALID_ARG
    assert call_chain(lib, math=E.MATH["f64"]) == E.TTM_ERR_UNSUPPORTED
    assert call_chain(lib, ydt=E.TTM_BF16) == E.TTM_ERR_UNSUPPORTED
    assert call_chain(lib, ws=0) == E.TTM_ERR_WORKSPACE
    assert call_chain(lib, ws_bytes=16) == E.TTM_ERR_WORKSPACE
    assert call_chain(lib, Y=FAKE + 256) == E.TTM_ERR_ALIAS              # Y inside X
    assert call_chain(lib, ws=FAKE + (1 << 30)) == E.TTM_ERR_ALIAS       # workspace over A
    assert call_chain(lib, Y=FAKE + (5 << 30) + 4096) == E.TTM_ERR_ALIAS  # Y inside the workspace


def test_backward_validation_errors(lib):
    E = _lib
    P = ctypes.c_void_p
    s = shp((8, 8, 8), (4, 4, 4))
    base = [P(FAKE + (k << 30)) for k in range(5)]   # G, X, A, B, C
    outs = [P(FAKE + ((6 + k) << 30)) for k in range(4)]
    ws = P(FAKE + (12 << 30))

    def bw(ins=base, o=outs, dt=E.TTM_F32, math=E.MATH["f32"], wsz=1 << 30, w=ws):
        return lib.ttm_chain_backward(s, *ins, dt, *o, math, w, wsz, P(0))

    assert bw(o=[P(0)] * 4) == E.TTM_ERR_INVALID_ARG
    assert bw(ins=[P(0)] + base[1:]) == E.TTM_ERR_INVALID_ARG
    assert bw(math=E.MATH["bf16x3"]) == E.TTM_ERR_UNSUPPORTED
    assert bw(dt=E.TTM_BF16) == E.TTM_ERR_UNSUPPORTED
    assert bw(wsz=8) == E.TTM_ERR_WORKSPACE
    assert bw(o=[base[1]] + outs[1:]) == E.TTM_ERR_ALIAS          # dX over X
    assert bw(o=[outs[0], outs[0], P(0), P(0)]) == E.TTM_ERR_ALIAS  # two outputs on one buffer


def test_batched_plan_validation_errors(lib):
    import numpy as np
    E = _lib
    P = ctypes.c_void_p
    h = P()
    dims = np.ones((3, 6), dtype=np.int64)
    ptr = dims.ctypes.data_as(P)
    assert lib.ttm_batched_plan_create(0, ptr, E.TTM_F32, E.MATH["f32"], None, P(0), ctypes.byref(h)) == E.TTM_ERR_INVALID_ARG
    assert lib.ttm_batched_plan_create(3, None, E.TTM_F32, E.MATH["f32"], None, P(0), ctypes.byref(h)) == E.TTM_ERR_INVALID_ARG
    assert lib.ttm_batched_plan_create(3, ptr, E.TTM_F32, E.MATH["bf16"], None, P(0), ctypes.byref(h)) == E.TTM_ERR_UNSUPPORTED
    assert lib.ttm_batched_plan_create(3, ptr, E.TTM_BF16, E.MATH["f32"], None, P(0), ctypes.byref(h)) == E.TTM_ERR_UNSUPPORTED
    big = dims.copy()
    big[1, 2] = 17
    assert lib.ttm_batched_plan_create(3, big.ctypes.data_as(P), E.TTM_F32, E.MATH["f32"], None, P(0),
                                       ctypes.byref(h)) == E.TTM_ERR_INVALID_ARG
    zero = dims.copy()
    zero[2, 5] = 0
    assert lib.ttm_batched_plan_create(3, zero.ctypes.data_as(P), E.TTM_F32, E.MATH["f32"], None, P(0),
                                       ctypes.byref(h)) == E.TTM_ERR_INVALID_ARG
    assert lib.ttm_batched_plan_destroy(None) == E.TTM_ERR_INVALID_ARG
    assert lib.ttm_batched_plan_totals(None, None) == E.TTM_ERR_INVALID_ARG
    assert lib.ttm_chain_batched(None, P(FAKE), P(FAKE), P(FAKE), P(FAKE), P(FAKE), P(0)) == E.TTM_ERR_INVALID_ARG
    assert lib.ttm_batched_plan_set_config(None, 256, 1, 1, P(0)) == E.TTM_ERR_INVALID_ARG


def test_timing_collect_empty(lib):
    assert lib.ttm_timing_enable(0) == 0
    names = ctypes.create_string_buffer(64 * 4)
    counts = (ctypes.c_int64 * 4)()
    ms = (ctypes.c_double * 4)()
    assert lib.ttm_timing_collect(names, counts, ms, 4) == 0
    assert lib.ttm_timing_collect(None, None, None, 4) == _lib.TTM_ERR_INVALID_ARG


def test_python_binding_rejects_cpu_tensors():
    import torch
    from paper_2411_13532_amd import chain
    X = torch.zeros(4, 4, 4)
    A = torch.zeros(2, 4)
    with pytest.raises(ValueError):
        chain(X, A, A, A)


def test_compact_validation_errors(lib):
    dims = (ctypes.c_int64 * 3)(8, 16, 32)
    coef = _lib.CompactCoef(1 / 3, 14 / 9, 1 / 9, 0.1)
    X, Y, ws = 0x100000, 0x900000, 0x2000000
    need = lib.ttm_compact_workspace_size(16, _lib.TTM_F64)
    assert need >= (4 * 16 + 2) * 8 and need % 256 == 0
    assert lib.ttm_compact_workspace_size(2, _lib.TTM_F64) == 0
    assert lib.ttm_compact_workspace_size(16, _lib.TTM_BF16) == 0
    call = lambda **kw: lib.ttm_compact_apply(kw.get("dims", dims), kw.get("mode", 2), kw.get("X", X),
                                              kw.get("Y", Y), kw.get("dt", _lib.TTM_F64),
                                              ctypes.byref(kw.get("coef", coef)), kw.get("ws", ws),
                                              kw.get("wsb", need), 0, None)
    assert call(mode=0) == _lib.TTM_ERR_INVALID_ARG
    assert call(mode=4) == _lib.TTM_ERR_INVALID_ARG
    assert call(dt=_lib.TTM_BF16) == _lib.TTM_ERR_UNSUPPORTED
    assert call(dims=(ctypes.c_int64 * 3)(2, 16, 32), mode=1) == _lib.TTM_ERR_UNSUPPORTED
    assert call(dims=(ctypes.c_int64 * 3)(0, 16, 32)) == _lib.TTM_ERR_INVALID_ARG
    assert call(X=0) == _lib.TTM_ERR_INVALID_ARG
    assert call(X=X + 4) == _lib.TTM_ERR_INVALID_ARG                 # misaligned for float64
    assert call(Y=X + 8 * 100) == _lib.TTM_ERR_ALIAS                  # Y overlaps X
    assert call(wsb=need - 8) == _lib.TTM_ERR_WORKSPACE
    assert call(ws=0) == _lib.TTM_ERR_WORKSPACE
    assert call(coef=_lib.CompactCoef(0.5, 14 / 9, 1 / 9, 0.1)) == _lib.TTM_ERR_INVALID_ARG   # not dominant
    assert call(coef=_lib.CompactCoef(1 / 3, 14 / 9, 1 / 9, 0.0)) == _lib.TTM_ERR_INVALID_ARG
    assert call(coef=_lib.CompactCoef(1 / 3, float("nan"), 1 / 9, 0.1)) == _lib.TTM_ERR_INVALID_ARG
    assert lib.ttm_compact_apply(dims, 2, X, Y, _lib.TTM_F64, None, ws, need, 0, None) == _lib.TTM_ERR_INVALID_ARG


# ---------------------------------------------------------------------------
# Failure of the HIP runtime itself.  Where no GPU is visible every HIP call
# fails, so a fully valid request reaches its first launch (or allocation)
# and must come back as TTM_ERR_HIP instead of crashing or reporting success.
# The pointers are well-formed device-looking addresses that no kernel ever
# receives: the launch itself fails.  Skipped where a GPU is visible.
# ---------------------------------------------------------------------------
def _no_gpu():
    try:
        import torch
        return not torch.cuda.is_available()
    except Exception:
        return True


needs_no_gpu = pytest.mark.skipif(not _no_gpu(), reason="forces HIP failures; only where no GPU is visible")
FAKE = 1 << 40


def fake(k):
    return ctypes.c_void_p(FAKE + (k << 32))


@needs_no_gpu
@pytest.mark.parametrize("math", ["f64", "f32", "bf16", "bf16x3"])
def test_launch_failure_maps_to_hip_error(lib, math):
    m = _lib.MATH[math]
    fdt = _lib.TTM_F64 if math == "f64" else _lib.TTM_F32
    xdt = _lib.TTM_BF16 if math in ("bf16", "bf16x3") else fdt
    s = _lib.shape((64, 300, 128), (16, 20, 40))
    ws = lib.ttm_chain_workspace_size(ctypes.byref(s), xdt, m)
    assert ws > 0
    rc = lib.ttm_chain(ctypes.byref(s), fake(0), xdt, fake(1), fake(2), fake(3), fdt, fake(4), fdt, m,
                       fake(5), ws, None)
    assert rc == _lib.TTM_ERR_HIP


@needs_no_gpu
def test_backward_and_copy_failures_map_to_hip_error(lib):
    s = _lib.shape((32, 64, 64), (8, 8, 8))
    ws = lib.ttm_chain_backward_workspace_size(ctypes.byref(s), _lib.TTM_F32, _lib.MATH["f32"])
    rc = lib.ttm_chain_backward(ctypes.byref(s), fake(0), fake(1), fake(2), fake(3), fake(4), _lib.TTM_F32,
                                fake(5), fake(6), fake(7), fake(8), _lib.MATH["f32"], fake(9), ws, None)
    assert rc == _lib.TTM_ERR_HIP
    assert lib.ttm_stream_copy(fake(0), fake(1), 4096, None) == _lib.TTM_ERR_HIP


@needs_no_gpu
def test_plan_create_failure_returns_no_plan(lib):
    import numpy as np
    dims = np.array([[5, 6, 7, 5, 6, 7]] * 4, dtype=np.int64)
    for _ in range(200):       # repeated failures: nothing is handed out
        h = ctypes.c_void_p(1234)
        rc = lib.ttm_batched_plan_create(4, dims.ctypes.data_as(ctypes.c_void_p), _lib.TTM_F32, _lib.MATH["f32"],
                                         None, None, ctypes.byref(h))
        assert rc == _lib.TTM_ERR_HIP
        assert h.value is None
