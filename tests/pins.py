"""Independent checks ("pins") of a chain implementation.

Each pin takes ``chain_fn(X, A, B, C) -> Y`` (float64 numpy result) and
raises ``AssertionError`` when the implementation breaks a fact fixed by the
mathematics or by the paper.  None of them re-types the oracle's loop nest:
they use closed forms, textbook identities, brute force on tiny inputs,
exact integer arithmetic, and the paper's compact finite-difference scheme.
The same pins run against the oracle (must pass) and against deliberately
broken variants of it (must fail), which shows that each pin has teeth.
"""
from __future__ import annotations

import itertools
import json
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_fro(y, ref) -> float:
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm((y - ref).ravel())
    n = np.linalg.norm(ref.ravel())
    return float(d / n) if n > 0 else float(d)


# ---------------------------------------------------------------------------
# The paper's compact scheme (Sec. 4.2, Eq. (cfds))
# ---------------------------------------------------------------------------
def compact6_coefficients():
    with open(os.path.join(GOLDEN, "compact6_first_derivative.json")) as f:
        g = json.load(f)
    return tuple(float(Fraction(*g[k])) for k in ("alpha", "a", "b"))


def compact6_periodic_matrices(n: int, h: float):
    """Circulant LHS A_c (1 on the diagonal, alpha beside it) and RHS stencil B_c
    so that A_c u' = B_c u is Eq. (cfds) on a periodic grid of n points."""
    alpha, a, b = compact6_coefficients()
    Ac = np.zeros((n, n))
    Bc = np.zeros((n, n))
    for i in range(n):
        Ac[i, i] = 1.0
        Ac[i, (i - 1) % n] += alpha
        Ac[i, (i + 1) % n] += alpha
        Bc[i, (i + 1) % n] += a / (2 * h)
        Bc[i, (i - 1) % n] -= a / (2 * h)
        Bc[i, (i + 2) % n] += b / (4 * h)
        Bc[i, (i - 2) % n] -= b / (4 * h)
    return Ac, Bc


def compact6_derivative_matrix(n: int) -> np.ndarray:
    """Dense D = A_c^-1 B_c on the periodic grid x_i = i*2*pi/n."""
    h = 2 * np.pi / n
    Ac, Bc = compact6_periodic_matrices(n, h)
    return np.linalg.solve(Ac, Bc)


def compact6_modified_wavenumber(m: int, n: int) -> float:
    """Exact eigenvalue relation of the periodic scheme: applying D to sin(m x)
    gives k'(m) cos(m x) with
        k'(m) = [a sin(mh) + (b/2) sin(2mh)] / (h [1 + 2 alpha cos(mh)]),
    obtained by substituting the Fourier mode into both sides of Eq. (cfds)."""
    alpha, a, b = compact6_coefficients()
    h = 2 * np.pi / n
    return (a * np.sin(m * h) + 0.5 * b * np.sin(2 * m * h)) / (h * (1.0 + 2 * alpha * np.cos(m * h)))


def compact6_nonperiodic_matrices(n: int, h: float):
    """Eq. (cfds) on a non-periodic grid.  The paper gives no boundary closure;
    this reading uses identity rows for the first and last LHS rows and drops
    stencil entries that fall outside the grid."""
    alpha, a, b = compact6_coefficients()
    Ac = np.eye(n)
    Bc = np.zeros((n, n))
    for i in range(n):
        if 0 < i < n - 1:
            Ac[i, i - 1] = alpha
            Ac[i, i + 1] = alpha
        for off, w in ((1, a / (2 * h)), (-1, -a / (2 * h)), (2, b / (4 * h)), (-2, -b / (4 * h))):
            if 0 <= i + off < n:
                Bc[i, i + off] += w
    return Ac, Bc


# ---------------------------------------------------------------------------
# Pins
# ---------------------------------------------------------------------------
def pin_bruteforce(chain_fn, brute_fn, seed=11):
    """P1a: chain equals the six-fold definition on tiny non-cubic shapes."""
    rng = np.random.default_rng(seed)
    for I, J in (((3, 4, 5), (2, 3, 6)), ((1, 2, 3), (1, 1, 1)), ((5, 1, 2), (4, 3, 1)), ((2, 3, 2), (3, 2, 4))):
        X = rng.standard_normal(I)
        A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
        err = rel_fro(chain_fn(X, A, B, C), brute_fn(X, A, B, C))
        assert err < 1e-14, (I, J, err)


def pin_kronecker(chain_fn, seed=12):
    """P1b: row-major vec(Y) = (A kron B kron C) vec(X)."""
    rng = np.random.default_rng(seed)
    I, J = (3, 5, 4), (4, 2, 3)
    X = rng.standard_normal(I)
    A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
    ref = (np.kron(A, np.kron(B, C)) @ X.ravel()).reshape(J)
    err = rel_fro(chain_fn(X, A, B, C), ref)
    assert err < 1e-14, err


def pin_einsum(chain_fn, seed=13):
    """P1c: a library contraction as a third opinion."""
    rng = np.random.default_rng(seed)
    I, J = (7, 6, 9), (5, 8, 3)
    X = rng.standard_normal(I)
    A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
    ref = np.einsum("abc,ia,jb,kc->ijk", X, A, B, C, optimize=False)
    err = rel_fro(chain_fn(X, A, B, C), ref)
    assert err < 1e-13, err


def pin_identity(chain_fn, seed=14):
    """P3: identity factors return X bit for bit."""
    rng = np.random.default_rng(seed)
    I = (6, 7, 5)
    X = rng.standard_normal(I)
    Y = chain_fn(X, np.eye(I[0]), np.eye(I[1]), np.eye(I[2]))
    assert np.array_equal(Y, X)


def pin_rank1(chain_fn, seed=15):
    """P4: X = u o v o w gives Y = (Au) o (Bv) o (Cw); distinct sizes per mode
    catch a factor applied to the wrong mode or transposed."""
    rng = np.random.default_rng(seed)
    I, J = (4, 6, 5), (3, 7, 2)
    u, v, w = (rng.standard_normal(I[n]) for n in range(3))
    X = np.einsum("a,b,c->abc", u, v, w)
    A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
    ref = np.einsum("a,b,c->abc", A @ u, B @ v, C @ w)
    err = rel_fro(chain_fn(X, A, B, C), ref)
    assert err < 1e-14, err


def pin_orthogonal_norm(chain_fn, seed=16):
    """P5: square orthogonal factors preserve the Frobenius norm; factors with
    orthonormal rows give ||Y|| <= ||X|| and re-applying the transposed
    factors then the factors returns Y (projection)."""
    rng = np.random.default_rng(seed)
    I = (8, 9, 10)
    X = rng.standard_normal(I)
    Qs = [np.linalg.qr(rng.standard_normal((n, n)))[0] for n in I]
    Y = chain_fn(X, *Qs)
    assert abs(np.linalg.norm(Y) - np.linalg.norm(X)) / np.linalg.norm(X) < 1e-14
    J = (3, 4, 5)
    R = [np.linalg.qr(rng.standard_normal((I[n], J[n])))[0].T for n in range(3)]
    Y = chain_fn(X, *R)
    assert np.linalg.norm(Y) <= np.linalg.norm(X) * (1 + 1e-14)
    back = chain_fn(Y, R[0].T, R[1].T, R[2].T)
    again = chain_fn(back, *R)
    assert rel_fro(again, Y) < 1e-14


def pin_compact6_closed_form(chain_fn, sizes=(16, 24, 32), modes=(3, 5, 2)):
    """P6: with D_n = A_c^-1 B_c of Eq. (cfds) on periodic grids, the field
    sin(m1 x) sin(m2 y) sin(m3 z) maps to k'(m1) k'(m2) k'(m3) cos cos cos."""
    Ds = [compact6_derivative_matrix(n) for n in sizes]
    xs = [np.arange(n) * (2 * np.pi / n) for n in sizes]
    X = np.einsum("a,b,c->abc", *[np.sin(m * x) for m, x in zip(modes, xs)])
    kap = np.prod([compact6_modified_wavenumber(m, n) for m, n in zip(modes, sizes)])
    ref = kap * np.einsum("a,b,c->abc", *[np.cos(m * x) for m, x in zip(modes, xs)])
    err = rel_fro(chain_fn(X, *Ds), ref)
    assert err < 1e-12, err


def pin_exact_integers(chain_fn, seed=17):
    """P9: small-integer data are summed exactly; compare with int64 einsum."""
    rng = np.random.default_rng(seed)
    I, J = (6, 5, 7), (4, 6, 3)
    X = rng.integers(-4, 5, size=I)
    A, B, C = (rng.integers(-4, 5, size=(J[n], I[n])) for n in range(3))
    ref = np.einsum("abc,ia,jb,kc->ijk", X, A, B, C)  # int64, exact
    Y = chain_fn(X.astype(np.float64), A.astype(np.float64), B.astype(np.float64), C.astype(np.float64))
    assert np.array_equal(Y, ref.astype(np.float64))


def pin_mode_order(chain_ordered_fn, seed=18):
    """P2: the six orders of applying the three mode products agree."""
    rng = np.random.default_rng(seed)
    I, J = (9, 7, 8), (4, 6, 5)
    X = rng.standard_normal(I)
    A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
    ys = [chain_ordered_fn(X, A, B, C, order) for order in itertools.permutations((1, 2, 3))]
    for y in ys[1:]:
        assert rel_fro(y, ys[0]) < 1e-14


ALL_CHAIN_PINS = (pin_kronecker, pin_einsum, pin_identity, pin_rank1, pin_orthogonal_norm,
                  pin_compact6_closed_form, pin_exact_integers)


# ---------------------------------------------------------------------------
# Pins of the compact scheme applied along one mode without forming D
# (apply_fn(X, mode, alpha, a, b, h) -> Y, same shape as X)
# ---------------------------------------------------------------------------
def pin_compact_apply_closed_form(apply_fn, shape=(16, 24, 32), ms=(3, 5, 2), rtol=1e-12):
    """P6 on a 3-way periodic field: with X = sin(m1 x) sin(m2 y) sin(m3 z) on
    x_i = i 2 pi / n, applying the scheme along mode k replaces sin(m_k .) by
    k'(m_k) cos(m_k .) exactly (the Fourier mode is an eigenvector)."""
    alpha, a, b = compact6_coefficients()
    grids = [np.arange(n) * 2 * np.pi / n for n in shape]
    sins = [np.sin(m * g) for m, g in zip(ms, grids)]
    X = np.einsum("i,j,k->ijk", *sins)
    for mode in (1, 2, 3):
        n, m = shape[mode - 1], ms[mode - 1]
        parts = list(sins)
        parts[mode - 1] = compact6_modified_wavenumber(m, n) * np.cos(m * grids[mode - 1])
        ref = np.einsum("i,j,k->ijk", *parts)
        out = apply_fn(X, mode, alpha, a, b, 2 * np.pi / n)
        err = rel_fro(out, ref)
        assert err <= rtol, (mode, err)


def pin_compact_apply_dense(apply_fn, shapes=((7, 9, 11), (5, 3, 4), (12, 6, 5)), seed=21, rtol=1e-12):
    """The same operator as the dense mode product with D = A_c^-1 B_c (solved
    densely), on random fields, every mode, a grid spacing not tied to n."""
    alpha, a, b = compact6_coefficients()
    r = np.random.default_rng(seed)
    for shape in shapes:
        X = r.standard_normal(shape)
        for mode in (1, 2, 3):
            n = shape[mode - 1]
            h = 0.37 / n
            Ac, Bc = compact6_periodic_matrices(n, h)
            D = np.linalg.solve(Ac, Bc)
            ref = np.moveaxis(np.tensordot(D, X, axes=([1], [mode - 1])), 0, mode - 1)
            out = apply_fn(X, mode, alpha, a, b, h)
            err = rel_fro(out, ref)
            assert err <= rtol, (shape, mode, err)


ALL_COMPACT_PINS = (pin_compact_apply_closed_form, pin_compact_apply_dense)
