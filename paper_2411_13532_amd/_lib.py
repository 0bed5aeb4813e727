"""ctypes loader for libttm.so (the HIP library built from csrc/).

Argument marshalling only: every computation runs in the library's kernels.
Loading fails loudly when the shared object has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttm.so")

# status codes and enums (include/ttm.h)
TTM_OK = 0
TTM_ERR_INVALID_ARG = -1
TTM_ERR_UNSUPPORTED = -2
TTM_ERR_WORKSPACE = -3
TTM_ERR_ALIAS = -4
TTM_ERR_HIP = -5

TTM_F64, TTM_F32, TTM_BF16 = 0, 1, 2
TTM_NOALLOC_SCRATCH_BYTES = 64 << 20
MATH = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}

# every exported entry point and its C signature
P = ctypes.c_void_p
I64 = ctypes.c_int64
SZ = ctypes.c_size_t
INT = ctypes.c_int


class Shape(ctypes.Structure):
    _fields_ = [("I", ctypes.c_int64 * 3), ("J", ctypes.c_int64 * 3)]


PShape = ctypes.POINTER(Shape)


class CompactCoef(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("h", ctypes.c_double)]

SIGNATURES = {
    "ttm_status_string": (ctypes.c_char_p, [INT]),
    "ttm_version": (INT, []),
    "ttm_set_slab_kernel": (INT, [INT]),
    "ttm_chain_supported": (INT, [INT, INT, INT, INT]),
    "ttm_chain_workspace_size": (SZ, [PShape, INT, INT]),
    "ttm_chain": (INT, [PShape, P, INT, P, P, P, INT, P, INT, INT, P, SZ, P]),
    "ttm_chain_noalloc": (INT, [PShape, P, INT, P, P, P, INT, P, INT, INT, P]),
    "ttm_chain_backward_workspace_size": (SZ, [PShape, INT, INT]),
    "ttm_chain_backward": (INT, [PShape, P, P, P, P, P, INT, P, P, P, P, INT, P, SZ, P]),
    "ttm_batched_plan_create": (INT, [I64, P, INT, INT, ctypes.c_char_p, P, ctypes.POINTER(P)]),
    "ttm_batched_plan_destroy": (INT, [P]),
    "ttm_batched_plan_totals": (INT, [P, P]),
    "ttm_chain_batched": (INT, [P, P, P, P, P, P, P]),
    "ttm_chain_batched_graph": (INT, [P, P, P, P, P, P, P]),
    "ttm_chain_batched_loop": (INT, [P, P, P, P, P, P, P]),
    "ttm_batched_autotune": (INT, [P, P, P, P, P, P, P, INT, ctypes.POINTER(ctypes.c_double)]),
    "ttm_batched_plan_config": (INT, [P, P]),
    "ttm_batched_plan_set_config": (INT, [P, INT, INT, INT, P]),
    "ttm_stream_copy": (INT, [P, P, SZ, P]),
    "ttm_reorder": (INT, [P, P, P, P, INT, INT, P]),
    "ttm_hosvd_workspace_size": (SZ, [PShape]),
    "ttm_hosvd": (INT, [PShape, P, P, P, P, P, P, SZ, P]),
    "ttm_compact_workspace_size": (SZ, [I64, INT]),
    "ttm_compact_apply": (INT, [P, INT, P, P, INT, ctypes.POINTER(CompactCoef), P, SZ, INT, P]),
    "ttm_timing_enable": (INT, [INT]),
    "ttm_timing_collect": (INT, [P, P, P, INT]),
}

_lib = None
MISSING: list = []


class TTMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})")


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libttm.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2411_13532_amd.build` (or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            try:
                fn = getattr(lib, name)
            except AttributeError:
                MISSING.append(name)
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(status: int) -> str:
    return load().ttm_status_string(status).decode()


def check(status: int, where: str) -> None:
    if status != TTM_OK:
        raise TTMError(status, where)


def shape(I, J) -> Shape:
    s = Shape()
    for n in range(3):
        s.I[n] = int(I[n])
        s.J[n] = int(J[n])
    return s
