"""PyTorch-facing binding of libttm.

Torch provides device memory and the current HIP stream; every step of the
chain runs in the library's HIP kernels (see include/ttm.h for the C
interface these functions wrap one to one).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MATH, TTM_BF16, TTM_F32, TTM_F64, check

_DT = {torch.float64: TTM_F64, torch.float32: TTM_F32, torch.bfloat16: TTM_BF16}


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("libttm works on GPU tensors only")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous (row-major)")


def _math_id(math: str) -> int:
    try:
        return MATH[math]
    except KeyError:
        raise ValueError(f"math must be one of {sorted(MATH)}") from None


def chain_workspace_size(I, J, x_dtype: torch.dtype, math: str) -> int:
    s = _lib.shape(I, J)
    return int(_lib.load().ttm_chain_workspace_size(ctypes.byref(s), _DT[x_dtype], _math_id(math)))


def chain(X: torch.Tensor, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, math: str = "f32",
          out: torch.Tensor | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Y = X x1 A x2 B x3 C with X (I1,I2,I3) and factors (J_n, I_n), all on one GPU.

    math: "f64" (all float64), "f32", "bf16" or "bf16x3" (float32 factors; X
    float32 or bfloat16).  Y is float64 for "f64", else float32.
    """
    _need_cuda(X, A, B, C, out, workspace)
    if X.dim() != 3 or A.dim() != 2 or B.dim() != 2 or C.dim() != 2:
        raise ValueError("X must be 3-way and A, B, C matrices")
    I = tuple(X.shape)
    J = (A.shape[0], B.shape[0], C.shape[0])
    if (A.shape[1], B.shape[1], C.shape[1]) != I:
        raise ValueError(f"factor widths {A.shape[1], B.shape[1], C.shape[1]} do not match X {I}")
    m = _math_id(math)
    ydt = torch.float64 if math == "f64" else torch.float32
    if out is None:
        out = torch.empty(J, dtype=ydt, device=X.device)
    s = _lib.shape(I, J)
    lib = _lib.load()
    ws_bytes = int(lib.ttm_chain_workspace_size(ctypes.byref(s), _DT.get(X.dtype, -1), m))
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=X.device)
    fdt = _DT.get(A.dtype, -1)
    if B.dtype != A.dtype or C.dtype != A.dtype:
        raise ValueError("A, B and C must share one dtype")
    rc = lib.ttm_chain(ctypes.byref(s), _ptr(X), _DT.get(X.dtype, -1), _ptr(A), _ptr(B), _ptr(C), fdt,
                       _ptr(out), _DT.get(out.dtype, -1), m, _ptr(workspace), workspace.numel(),
                       _stream(X.device))
    check(rc, "ttm_chain")
    return out


def chain_noalloc(X: torch.Tensor, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, math: str = "f32",
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """ttm_chain_noalloc: as :func:`chain`, with the library's per-GPU scratch
    as workspace (no workspace allocation; `out` may be given to allocate
    nothing at all)."""
    _need_cuda(X, A, B, C, out)
    if X.dim() != 3 or A.dim() != 2 or B.dim() != 2 or C.dim() != 2:
        raise ValueError("X must be 3-way and A, B, C matrices")
    I = tuple(X.shape)
    J = (A.shape[0], B.shape[0], C.shape[0])
    if (A.shape[1], B.shape[1], C.shape[1]) != I:
        raise ValueError(f"factor widths {A.shape[1], B.shape[1], C.shape[1]} do not match X {I}")
    if B.dtype != A.dtype or C.dtype != A.dtype:
        raise ValueError("A, B and C must share one dtype")
    m = _math_id(math)
    if out is None:
        out = torch.empty(J, dtype=torch.float64 if math == "f64" else torch.float32, device=X.device)
    s = _lib.shape(I, J)
    rc = _lib.load().ttm_chain_noalloc(ctypes.byref(s), _ptr(X), _DT.get(X.dtype, -1), _ptr(A), _ptr(B), _ptr(C),
                                       _DT.get(A.dtype, -1), _ptr(out), _DT.get(out.dtype, -1), m, _stream(X.device))
    check(rc, "ttm_chain_noalloc")
    return out


def chain_backward_workspace_size(I, J, dtype: torch.dtype, math: str) -> int:
    s = _lib.shape(I, J)
    return int(_lib.load().ttm_chain_backward_workspace_size(ctypes.byref(s), _DT[dtype], _math_id(math)))


def chain_backward(G, X, A, B, C, math: str = "f32", need=(True, True, True, True), workspace=None):
    """(dX, dA, dB, dC) for dL/dY = G; entries not in `need` come back as None."""
    _need_cuda(G, X, A, B, C, workspace)
    I = tuple(X.shape)
    J = (A.shape[0], B.shape[0], C.shape[0])
    if tuple(G.shape) != J:
        raise ValueError("G must have the output shape")
    outs = [torch.empty_like(t) if n else None for t, n in zip((X, A, B, C), need)]
    s = _lib.shape(I, J)
    lib = _lib.load()
    m = _math_id(math)
    ws_bytes = int(lib.ttm_chain_backward_workspace_size(ctypes.byref(s), _DT.get(X.dtype, -1), m))
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=X.device)
    rc = lib.ttm_chain_backward(ctypes.byref(s), _ptr(G), _ptr(X), _ptr(A), _ptr(B), _ptr(C),
                                _DT.get(X.dtype, -1), *[_ptr(o) for o in outs], m,
                                _ptr(workspace), workspace.numel(), _stream(X.device))
    check(rc, "ttm_chain_backward")
    return tuple(outs)


class TTMChain(torch.autograd.Function):
    """Differentiable Y = X x1 A x2 B x3 C whose backward is the library's adjoint kernels."""

    @staticmethod
    def forward(ctx, X, A, B, C, math="f32"):
        ctx.save_for_backward(X, A, B, C)
        ctx.math = math
        return chain(X.contiguous(), A.contiguous(), B.contiguous(), C.contiguous(), math=math)

    @staticmethod
    def backward(ctx, G):
        X, A, B, C = ctx.saved_tensors
        need = tuple(bool(n) for n in ctx.needs_input_grad[:4])
        grads = chain_backward(G.contiguous(), X, A, B, C, math=ctx.math, need=need)
        return (*grads, None)


def ttm_chain(X, A, B, C, math="f32"):
    return TTMChain.apply(X, A, B, C, math)


class BatchedPlan:
    """A ragged batch of independent chains run by one persistent kernel.

    dims: (count, 6) integer array of (I1, I2, I3, J1, J2, J3) per cuboid.
    Buffers passed to run() are the cuboids' tensors stored back to back.
    """

    def __init__(self, dims, dtype=torch.float32, tune_cache: str | None = None, device=None):
        import numpy as np
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int64).reshape(-1, 6))
        self.dims = d
        self.count = d.shape[0]
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        math = "f64" if dtype == torch.float64 else "f32"
        with torch.cuda.device(self.device):
            rc = self._lib.ttm_batched_plan_create(
                self.count, d.ctypes.data_as(ctypes.c_void_p), _DT[dtype], MATH[math],
                tune_cache.encode() if tune_cache else None, _stream(self.device), ctypes.byref(h))
        check(rc, "ttm_batched_plan_create")
        self._h = h
        tot = (ctypes.c_int64 * 5)()
        check(self._lib.ttm_batched_plan_totals(h, tot), "ttm_batched_plan_totals")
        self.totals = tuple(int(v) for v in tot)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.ttm_batched_plan_destroy(h)
            self._h = None

    def empty_output(self):
        return torch.empty(self.totals[4], dtype=self.dtype, device=self.device)

    def _args(self, X, A, B, C, Y):
        _need_cuda(X, A, B, C, Y)
        for t, n in zip((X, A, B, C, Y), self.totals):
            if t.numel() != n or t.dtype != self.dtype:
                raise ValueError(f"buffer has {t.numel()} {t.dtype} elements, plan expects {n} {self.dtype}")
        return [_ptr(t) for t in (X, A, B, C, Y)]

    def run(self, X, A, B, C, Y=None, mode: str = "persistent"):
        """mode: "persistent" (one launch), "graph" (replay of the plan's HIP graph)
        or "loop" (one launch per cuboid, for comparison)."""
        if Y is None:
            Y = self.empty_output()
        args = self._args(X, A, B, C, Y)
        fn = {"persistent": self._lib.ttm_chain_batched, "graph": self._lib.ttm_chain_batched_graph,
              "loop": self._lib.ttm_chain_batched_loop}[mode]
        check(fn(self._h, *args, _stream(self.device)), f"ttm_chain_batched[{mode}]")
        return Y

    def autotune(self, X, A, B, C, Y=None, reps: int = 10) -> float:
        if Y is None:
            Y = self.empty_output()
        args = self._args(X, A, B, C, Y)
        best = ctypes.c_double()
        check(self._lib.ttm_batched_autotune(self._h, *args, _stream(self.device), reps, ctypes.byref(best)),
              "ttm_batched_autotune")
        return best.value

    def config(self):
        out = (ctypes.c_int * 4)()
        check(self._lib.ttm_batched_plan_config(self._h, out), "ttm_batched_plan_config")
        return {"threads": out[0], "blocks_per_cu": out[1], "blocks": out[2], "variant": out[3]}

    def set_config(self, threads: int, blocks_per_cu: int, variant: int) -> None:
        """Pin the launch shape (ttm_batched_plan_set_config)."""
        check(self._lib.ttm_batched_plan_set_config(self._h, int(threads), int(blocks_per_cu), int(variant),
                                                    _stream(self.device)), "ttm_batched_plan_set_config")


COMPACT6 = (1.0 / 3.0, 14.0 / 9.0, 1.0 / 9.0)   # alpha, a, b of Sec. 4.2 Eq. (cfds)


def compact_apply(X: torch.Tensor, mode: int, h: float | None = None, coef=COMPACT6,
                  out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                  prepared: bool = False) -> torch.Tensor:
    """The periodic compact first-derivative scheme (alpha, a, b) = coef with grid
    spacing h (default 2 pi / n) applied along mode 1, 2 or 3 of X (float64 or
    float32), i.e. X x_mode A_c^-1 B_c, by fused stencil + cyclic tridiagonal solve.
    prepared=True reuses the coefficients an earlier call with the same fiber
    length, coef and dtype left in `workspace`."""
    _need_cuda(X, out, workspace)
    if X.dim() != 3:
        raise ValueError("X must be 3-way")
    if X.dtype not in (torch.float64, torch.float32):
        raise ValueError("X must be float64 or float32")
    n = X.shape[mode - 1] if 1 <= mode <= 3 else 0
    if h is None:
        h = 2.0 * 3.141592653589793 / max(n, 1)
    if out is None:
        out = torch.empty_like(X)
    lib = _lib.load()
    dt = _DT[X.dtype]
    if prepared and workspace is None:
        raise ValueError("prepared=True needs the workspace of the earlier call")
    if workspace is None:
        workspace = torch.empty(max(int(lib.ttm_compact_workspace_size(n, dt)), 256), dtype=torch.uint8,
                                device=X.device)
    dims = (ctypes.c_int64 * 3)(*X.shape)
    c = _lib.CompactCoef(float(coef[0]), float(coef[1]), float(coef[2]), float(h))
    rc = lib.ttm_compact_apply(dims, int(mode), _ptr(X), _ptr(out), dt, ctypes.byref(c), _ptr(workspace),
                               workspace.numel(), 1 if prepared else 0, _stream(X.device))
    check(rc, "ttm_compact_apply")
    return out


def stream_copy(dst: torch.Tensor, src: torch.Tensor) -> None:
    """dst <- src (same byte size, 16-byte multiple) with the library's copy kernel."""
    _need_cuda(dst, src)
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src must have the same size in bytes")
    check(_lib.load().ttm_stream_copy(_ptr(dst), _ptr(src), nbytes, _stream(src.device)), "ttm_stream_copy")


def set_slab_kernel(mode: int) -> None:
    """0: automatic (default: X and C through LDS for bf16 X with the bf16
    forms, else direct-to-LDS 256-byte chunks where that applies);
    1: register-staged everywhere; 2: direct-to-LDS 256-byte chunks; 3: 512-byte
    chunks; 4: copy-wave direct-to-LDS kernel; 5: X and C through LDS, eight
    waves over 256-row tiles (see ttm_set_slab_kernel)."""
    check(_lib.load().ttm_set_slab_kernel(int(mode)), "ttm_set_slab_kernel")


def timing_enable(on: bool = True) -> None:
    check(_lib.load().ttm_timing_enable(1 if on else 0), "ttm_timing_enable")


def timing_collect(max_entries: int = 32) -> dict:
    """{kernel name: (launches, total ms)} since the last collect."""
    names = ctypes.create_string_buffer(64 * max_entries)
    counts = (ctypes.c_int64 * max_entries)()
    ms = (ctypes.c_double * max_entries)()
    n = _lib.load().ttm_timing_collect(names, counts, ms, max_entries)
    if n < 0:
        check(n, "ttm_timing_collect")
    out = {}
    for k in range(n):
        name = names.raw[64 * k:64 * k + 64].split(b"\0", 1)[0].decode()
        out[name] = (int(counts[k]), float(ms[k]))
    return out


def reorder(X: torch.Tensor, perm, out: torch.Tensor | None = None, accumulate: bool = False) -> torch.Tensor:
    """ttm_reorder: X (3-way, float32 or float64) moved to the layout whose
    axis k is X's axis perm[k] (a directional layout change, Sec. 4.1); with
    accumulate=True the result is added to `out` instead of written."""
    _need_cuda(X, out)
    if X.dim() != 3 or X.dtype not in (torch.float32, torch.float64):
        raise ValueError("X must be a 3-way float32 or float64 tensor")
    import numpy as np
    p = np.ascontiguousarray(np.asarray(perm, dtype=np.int32))
    if sorted(int(k) for k in p) != [0, 1, 2]:
        raise ValueError("perm must be a permutation of (0, 1, 2)")
    yshape = tuple(X.shape[int(k)] for k in p)
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs out")
        out = torch.empty(yshape, dtype=X.dtype, device=X.device)
    elif tuple(out.shape) != yshape or out.dtype != X.dtype:
        raise ValueError("out has the wrong shape or dtype")
    dims = np.ascontiguousarray(np.asarray(X.shape, dtype=np.int64))
    rc = _lib.load().ttm_reorder(dims.ctypes.data_as(ctypes.c_void_p), p.ctypes.data_as(ctypes.c_void_p), _ptr(X),
                                 _ptr(out), _DT[X.dtype], int(bool(accumulate)), _stream(X.device))
    check(rc, "ttm_reorder")
    return out


def hosvd(X: torch.Tensor, J, with_evals: bool = False):
    """ttm_hosvd: the truncated HOSVD factors (J_n x I_n, float64) of a float64
    X, each mode's rows the leading left singular vectors of its unfolding;
    with_evals also returns each mode's Gram eigenvalues, decreasing."""
    _need_cuda(X)
    if X.dim() != 3 or X.dtype != torch.float64:
        raise ValueError("X must be a 3-way float64 tensor")
    I = tuple(X.shape)
    s = _lib.shape(I, J)
    lib = _lib.load()
    ws = torch.empty(max(int(lib.ttm_hosvd_workspace_size(ctypes.byref(s))), 1), dtype=torch.uint8,
                     device=X.device)
    fs = [torch.empty((int(J[n]), I[n]), dtype=torch.float64, device=X.device) for n in range(3)]
    ev = torch.empty(sum(I), dtype=torch.float64, device=X.device) if with_evals else None
    rc = lib.ttm_hosvd(ctypes.byref(s), _ptr(X), *[_ptr(f) for f in fs], _ptr(ev), _ptr(ws), ws.numel(),
                       _stream(X.device))
    check(rc, "ttm_hosvd")
    if not with_evals:
        return fs
    return fs, [ev[sum(I[:n]):sum(I[:n + 1])] for n in range(3)]
