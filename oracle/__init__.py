"""FP64 CPU oracle for the mode-n product chain Y = X x1 A x2 B x3 C.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_2411_13532_amd`` and neither imports the
other.  The arithmetic lives in ``ttm_oracle.c`` (plain loops, double
precision, fixed summation order); this module only marshals numpy arrays.

Definition followed (standard multilinear algebra; the paper's directional
operator of Sec. 4.2, Eq. (cfds), is a single mode product with the dense
matrix D = A_c^-1 B_c):

    Y[j1,j2,j3] = sum_{i1,i2,i3} A[j1,i1] B[j2,i2] C[j3,i3] X[i1,i2,i3]

Every input is converted to float64 before use, so a float32 or bfloat16
stored tensor is consumed at its exact stored value.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ttm_oracle.c")
_LIB = os.path.join(_HERE, "libttm_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.ttmo_num_threads.restype = ctypes.c_int
        for name in ("ttmo_mode_product", "ttmo_mode_product_xf32"):
            getattr(lib, name).argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P]
            getattr(lib, name).restype = None
        for name in ("ttmo_chain_ordered", "ttmo_chain_ordered_xf32"):
            getattr(lib, name).argtypes = [P] * 8
            getattr(lib, name).restype = ctypes.c_int
        lib.ttmo_chain.argtypes = [P] * 7
        lib.ttmo_chain.restype = ctypes.c_int
        lib.ttmo_brute.argtypes = [P] * 7
        lib.ttmo_brute.restype = None
        lib.ttmo_loss.argtypes = [P] * 7
        lib.ttmo_loss.restype = ctypes.c_double
        lib.ttmo_backward.argtypes = [P] * 11
        lib.ttmo_backward.restype = ctypes.c_int
        lib.ttmo_batched.argtypes = [ctypes.c_int64] + [P] * 6
        lib.ttmo_compact6_apply.argtypes = [ctypes.c_int, P] + [ctypes.c_double] * 4 + [P, P]
        lib.ttmo_compact6_apply.restype = ctypes.c_int
        lib.ttmo_batched.restype = ctypes.c_int
        lib.ttmo_gram.argtypes = [P, ctypes.c_int, P, P]
        lib.ttmo_gram.restype = ctypes.c_int
        lib.ttmo_reorder.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int]
        lib.ttmo_reorder.restype = ctypes.c_int
        for name in ("ttmo_thomas", "ttmo_thomas_periodic"):
            getattr(lib, name).argtypes = [ctypes.c_int64] + [P] * 5
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    """Exact upcast to a contiguous float64 array (accepts torch tensors)."""
    if hasattr(a, "detach"):
        a = a.detach().cpu().float().numpy() if str(a.dtype) == "torch.bfloat16" else a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i64(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.int64))


def num_threads() -> int:
    return int(_load().ttmo_num_threads())


def mode_product(X, U, mode: int) -> np.ndarray:
    """X x_mode U for a 3-way X and U of shape (J_n, I_n)."""
    X = np.asarray(X)
    U = _f64(U)
    dims = _i64(X.shape)
    out_shape = list(X.shape)
    out_shape[mode - 1] = U.shape[0]
    assert U.shape[1] == X.shape[mode - 1]
    out = np.empty(out_shape, dtype=np.float64)
    lib = _load()
    if X.dtype == np.float32:
        Xc = np.ascontiguousarray(X)
        lib.ttmo_mode_product_xf32(mode, _ptr(dims), U.shape[0], _ptr(Xc), _ptr(U), _ptr(out))
    else:
        Xc = _f64(X)
        lib.ttmo_mode_product(mode, _ptr(dims), U.shape[0], _ptr(Xc), _ptr(U), _ptr(out))
    return out


def chain(X, A, B, C, order=(1, 2, 3)) -> np.ndarray:
    """Y = X x1 A x2 B x3 C, applying the mode products in ``order``.

    A float32 X is read as float32 and upcast element by element (no float64
    copy of X is made); any other X is converted to float64 first.
    """
    A, B, C = _f64(A), _f64(B), _f64(C)
    if hasattr(X, "detach"):
        X = X.detach().cpu()
        X = X.float().numpy() if str(X.dtype) == "torch.bfloat16" else X.numpy()
    X = np.asarray(X)
    I = _i64(X.shape)
    J = _i64([A.shape[0], B.shape[0], C.shape[0]])
    assert A.shape[1] == I[0] and B.shape[1] == I[1] and C.shape[1] == I[2]
    ordv = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    Y = np.empty(tuple(J), dtype=np.float64)
    lib = _load()
    if X.dtype == np.float32:
        Xc = np.ascontiguousarray(X)
        rc = lib.ttmo_chain_ordered_xf32(_ptr(ordv), _ptr(I), _ptr(J), _ptr(Xc), _ptr(A), _ptr(B), _ptr(C), _ptr(Y))
    else:
        Xc = _f64(X)
        rc = lib.ttmo_chain_ordered(_ptr(ordv), _ptr(I), _ptr(J), _ptr(Xc), _ptr(A), _ptr(B), _ptr(C), _ptr(Y))
    if rc != 0:
        raise RuntimeError(f"oracle chain failed ({rc})")
    return Y


def brute(X, A, B, C) -> np.ndarray:
    """The six-fold sum of the definition (tiny shapes only)."""
    X, A, B, C = _f64(X), _f64(A), _f64(B), _f64(C)
    I = _i64(X.shape)
    J = _i64([A.shape[0], B.shape[0], C.shape[0]])
    Y = np.empty(tuple(J), dtype=np.float64)
    _load().ttmo_brute(_ptr(I), _ptr(J), _ptr(X), _ptr(A), _ptr(B), _ptr(C), _ptr(Y))
    return Y


def loss(X, A, B, C, T) -> float:
    """L = 1/2 ||X x1 A x2 B x3 C - T||_F^2."""
    X, A, B, C, T = _f64(X), _f64(A), _f64(B), _f64(C), _f64(T)
    I = _i64(X.shape)
    J = _i64([A.shape[0], B.shape[0], C.shape[0]])
    return float(_load().ttmo_loss(_ptr(I), _ptr(J), _ptr(X), _ptr(A), _ptr(B), _ptr(C), _ptr(T)))


def backward(G, X, A, B, C):
    """(dX, dA, dB, dC) of <G, X x1 A x2 B x3 C> with respect to each input."""
    G, X, A, B, C = _f64(G), _f64(X), _f64(A), _f64(B), _f64(C)
    I = _i64(X.shape)
    J = _i64([A.shape[0], B.shape[0], C.shape[0]])
    dX = np.empty(X.shape, dtype=np.float64)
    dA = np.empty(A.shape, dtype=np.float64)
    dB = np.empty(B.shape, dtype=np.float64)
    dC = np.empty(C.shape, dtype=np.float64)
    rc = _load().ttmo_backward(_ptr(I), _ptr(J), _ptr(G), _ptr(X), _ptr(A), _ptr(B), _ptr(C),
                               _ptr(dX), _ptr(dA), _ptr(dB), _ptr(dC))
    if rc != 0:
        raise RuntimeError(f"oracle backward failed ({rc})")
    return dX, dA, dB, dC


def batched(dims, X, A, B, C) -> np.ndarray:
    """Chain over cuboids stored back to back; dims is (count, 6) = (I1,I2,I3,J1,J2,J3)."""
    dims = _i64(dims).reshape(-1, 6)
    X, A, B, C = _f64(X).ravel(), _f64(A).ravel(), _f64(B).ravel(), _f64(C).ravel()
    ny = int(np.sum(dims[:, 3] * dims[:, 4] * dims[:, 5]))
    Y = np.empty(ny, dtype=np.float64)
    rc = _load().ttmo_batched(dims.shape[0], _ptr(dims), _ptr(X), _ptr(A), _ptr(B), _ptr(C), _ptr(Y))
    if rc != 0:
        raise RuntimeError(f"oracle batched chain failed ({rc})")
    return Y


def thomas(a, b, c, d, periodic: bool = False) -> np.ndarray:
    """Solve one tridiagonal (or cyclic tridiagonal) system, Sec. 2.1."""
    a, b, c, d = _f64(a), _f64(b), _f64(c), _f64(d)
    u = np.empty_like(d)
    fn = _load().ttmo_thomas_periodic if periodic else _load().ttmo_thomas
    rc = fn(d.shape[0], _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(u))
    if rc != 0:
        raise RuntimeError("thomas failed")
    return u


def compact6_apply(X, mode: int, alpha: float, a: float, b: float, h: float) -> np.ndarray:
    """The compact scheme of Sec. 4.2 Eq. (cfds) on a periodic grid, applied along
    mode `mode` of X (right-hand side built per fiber, periodic Thomas solve)."""
    Xc = _f64(X)
    if Xc.ndim != 3:
        raise ValueError("X must be 3-way")
    out = np.empty_like(Xc)
    rc = _load().ttmo_compact6_apply(int(mode), _ptr(_i64(Xc.shape)), float(alpha), float(a), float(b),
                                     float(h), _ptr(Xc), _ptr(out))
    if rc != 0:
        raise ValueError("compact6_apply needs mode in 1..3 and at least 3 points along it")
    return out


def reorder(X, perm, Y=None) -> np.ndarray:
    """X (3-way, float32 or float64) with its axes permuted, Y's axis k being
    X's axis perm[k] (Sec. 4.1's move between directional layouts), moved as
    bytes; with Y given, Y + that in X's dtype (returned as a new array)."""
    X = np.ascontiguousarray(X)
    if X.ndim != 3 or X.dtype not in (np.float32, np.float64):
        raise ValueError("X must be a 3-way float32 or float64 array")
    p = np.ascontiguousarray(np.asarray(perm, dtype=np.int32))
    if sorted(int(k) for k in p) != [0, 1, 2]:
        raise ValueError("perm must be a permutation of (0, 1, 2)")
    yshape = tuple(X.shape[int(k)] for k in p)
    if Y is None:
        out = np.empty(yshape, dtype=X.dtype)
        acc = 0
    else:
        out = np.array(Y, dtype=X.dtype, copy=True, order="C")
        if out.shape != yshape:
            raise ValueError("Y has the wrong shape")
        acc = 1
    rc = _load().ttmo_reorder(_ptr(_i64(X.shape)), _ptr(p), _ptr(X), _ptr(out), X.dtype.itemsize, acc)
    if rc != 0:
        raise ValueError("perm must be a permutation of (0, 1, 2)")
    return out


def gram(X, mode: int) -> np.ndarray:
    """G = X_(mode) X_(mode)^T in float64 (plain loops)."""
    Xc = _f64(X)
    n = Xc.shape[mode - 1]
    G = np.empty((n, n), dtype=np.float64)
    if _load().ttmo_gram(_ptr(_i64(Xc.shape)), int(mode), _ptr(Xc), _ptr(G)) != 0:
        raise ValueError("mode must be 1, 2 or 3")
    return G


def sign_fixed_rows(U: np.ndarray) -> np.ndarray:
    """Each row multiplied by +-1 so that its entry of largest magnitude (the
    first such) is positive: the sign convention that makes singular vectors
    of a simple singular value unique."""
    U = np.array(U, dtype=np.float64, copy=True)
    for r in range(U.shape[0]):
        k = int(np.argmax(np.abs(U[r])))
        if U[r, k] < 0:
            U[r] = -U[r]
    return U


def hosvd_factors(X, J):
    """Truncated HOSVD (the Tucker factors): for each mode n, the J_n leading
    eigenvectors of the Gram matrix of the mode-n unfolding (its leading left
    singular vectors), as the rows of a J_n x I_n factor, by decreasing
    eigenvalue, sign-fixed; also the eigenvalues (squared singular values) in
    decreasing order.  The symmetric eigensolver is numpy's (a library step)."""
    factors, evals = [], []
    for mode in (1, 2, 3):
        w, V = np.linalg.eigh(gram(X, mode))
        order = np.argsort(-w, kind="stable")
        evals.append(w[order])
        factors.append(sign_fixed_rows(V[:, order[:J[mode - 1]]].T))
    return factors, evals
