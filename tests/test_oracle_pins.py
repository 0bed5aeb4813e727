"""The FP64 oracle checked against facts that do not come from the oracle itself."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2411_13532_amd import workloads
from tests import pins


def chain(X, A, B, C):
    return oracle.chain(X, A, B, C)


def chain_ordered(X, A, B, C, order):
    return oracle.chain(X, A, B, C, order=order)


@pytest.mark.parametrize("pin", pins.ALL_CHAIN_PINS, ids=lambda p: p.__name__)
def test_oracle_chain_pins(pin):
    pin(chain)


def test_oracle_bruteforce_pin():
    pins.pin_bruteforce(chain, oracle.brute)


def test_oracle_brute_is_the_definition():
    # the C six-fold sum against Python loops written from the definition
    rng = np.random.default_rng(1)
    I, J = (2, 3, 2), (2, 2, 3)
    X = rng.standard_normal(I)
    A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
    ref = np.zeros(J)
    for j1, j2, j3 in itertools.product(*(range(j) for j in J)):
        for i1, i2, i3 in itertools.product(*(range(i) for i in I)):
            ref[j1, j2, j3] += A[j1, i1] * B[j2, i2] * C[j3, i3] * X[i1, i2, i3]
    np.testing.assert_allclose(oracle.brute(X, A, B, C), ref, rtol=1e-14, atol=1e-15)


def test_oracle_mode_order_pin():
    pins.pin_mode_order(chain_ordered)


def test_oracle_float32_input_is_exact_upcast():
    p = workloads.random_problem((9, 10, 11), (3, 4, 5), seed=3, dtype=np.float32)
    y32 = oracle.chain(p["X"], p["A"], p["B"], p["C"])
    y64 = oracle.chain(p["X"].astype(np.float64), p["A"], p["B"], p["C"])
    assert np.array_equal(y32, y64)
    for order in itertools.permutations((1, 2, 3)):
        y = oracle.chain(p["X"], p["A"], p["B"], p["C"], order=order)
        assert pins.rel_fro(y, y64) < 1e-14


def test_oracle_single_mode_product_matches_matrix_product():
    # X x_n U is U @ (mode-n unfolding); numpy moveaxis builds the unfolding
    rng = np.random.default_rng(4)
    X = rng.standard_normal((4, 5, 6))
    for mode, n in ((1, 4), (2, 5), (3, 6)):
        U = rng.standard_normal((3, n))
        out = oracle.mode_product(X, U, mode)
        ref = np.moveaxis(np.tensordot(U, X, axes=([1], [mode - 1])), 0, mode - 1)
        np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------------------
# Planted mistakes: each broken chain must fail at least one pin.
# ---------------------------------------------------------------------------
def _mut_transposed_A(X, A, B, C):
    # uses A^T where A is square, or fails on shape otherwise
    if A.shape[0] != A.shape[1]:
        A = np.resize(A.T, A.shape)
    else:
        A = A.T
    return np.einsum("abc,ia,jb,kc->ijk", X, A, B, C)


def _mut_reversed_index(X, A, B, C):
    # contracts mode 3 against C with its column index reversed
    return np.einsum("abc,ia,jb,kc->ijk", X, A, B, C[:, ::-1])


def _mut_dropped_last_term(X, A, B, C):
    return np.einsum("abc,ia,jb,kc->ijk", X[:, :, :-1], A, B, C[:, :-1])


def _mut_sign(X, A, B, C):
    Y = np.einsum("abc,ia,jb,kc->ijk", X, A, B, C)
    Y[..., -1] *= -1
    return Y


def _mut_float32_intermediate(X, A, B, C):
    t = np.einsum("abc,kc->abk", X, C).astype(np.float32).astype(np.float64)
    return np.einsum("abk,ia,jb->ijk", t, A, B)


@pytest.mark.parametrize("mutant", [_mut_transposed_A, _mut_reversed_index, _mut_dropped_last_term,
                                    _mut_sign, _mut_float32_intermediate],
                         ids=lambda m: m.__name__)
def test_planted_mistakes_are_caught(mutant):
    failures = 0
    for pin in pins.ALL_CHAIN_PINS:
        try:
            pin(mutant)
        except AssertionError:
            failures += 1
    assert failures > 0, f"{mutant.__name__} passed every pin"


# ---------------------------------------------------------------------------
# Thomas algorithm (Sec. 2.1) and the paper's compact scheme as a mode product
# ---------------------------------------------------------------------------
def test_thomas_matches_dense_solve():
    rng = np.random.default_rng(5)
    for n in (1, 2, 5, 33):
        a, c = rng.standard_normal(n), rng.standard_normal(n)
        b = 4.0 + np.abs(rng.standard_normal(n))
        d = rng.standard_normal(n)
        M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        np.testing.assert_allclose(oracle.thomas(a, b, c, d), np.linalg.solve(M, d), rtol=1e-12, atol=1e-14)


def test_periodic_thomas_matches_dense_solve():
    rng = np.random.default_rng(6)
    for n in (3, 4, 17):
        a, c = rng.standard_normal(n), rng.standard_normal(n)
        b = 4.0 + np.abs(rng.standard_normal(n))
        d = rng.standard_normal(n)
        M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        M[0, n - 1] = a[0]
        M[n - 1, 0] = c[n - 1]
        np.testing.assert_allclose(oracle.thomas(a, b, c, d, periodic=True), np.linalg.solve(M, d),
                                   rtol=1e-12, atol=1e-14)


def test_compact6_eigen_relation_1d():
    # D sin(m x) = k'(m) cos(m x) on periodic grids (Eq. (cfds))
    for n in (16, 32, 64):
        D = pins.compact6_derivative_matrix(n)
        x = np.arange(n) * 2 * np.pi / n
        for m in (1, 3, n // 4):
            lhs = D @ np.sin(m * x)
            rhs = pins.compact6_modified_wavenumber(m, n) * np.cos(m * x)
            assert np.max(np.abs(lhs - rhs)) < 1e-12 * max(1.0, np.max(np.abs(rhs)))
    # low modes approach the exact derivative (sixth-order accuracy)
    n = 64
    assert abs(pins.compact6_modified_wavenumber(1, n) - 1.0) < 1e-9


def test_periodic_thomas_applies_compact6_along_fibers():
    # the paper's solver (periodic Thomas on A_c u' = B_c u) per mode-2 fiber
    # equals the dense mode product with D = A_c^-1 B_c
    n = 24
    h = 2 * np.pi / n
    alpha, _, _ = pins.compact6_coefficients()
    Ac, Bc = pins.compact6_periodic_matrices(n, h)
    D = np.linalg.solve(Ac, Bc)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((5, n, 6))
    ref = oracle.mode_product(X, D, 2)
    out = np.empty_like(X)
    band = np.full(n, alpha)
    ones = np.ones(n)
    for i1 in range(X.shape[0]):
        for i3 in range(X.shape[2]):
            out[i1, :, i3] = oracle.thomas(band, ones, band, Bc @ X[i1, :, i3], periodic=True)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_thomas_applies_nonperiodic_compact6_along_mode1():
    n = 20
    h = 1.0 / (n - 1)
    Ac, Bc = pins.compact6_nonperiodic_matrices(n, h)
    D = np.linalg.solve(Ac, Bc)
    a = np.concatenate([[0.0], np.diag(Ac, -1)])
    c = np.concatenate([np.diag(Ac, 1), [0.0]])
    b = np.diag(Ac).copy()
    rng = np.random.default_rng(8)
    X = rng.standard_normal((n, 4, 3))
    ref = oracle.mode_product(X, D, 1)
    out = np.empty_like(X)
    for i2 in range(4):
        for i3 in range(3):
            out[:, i2, i3] = oracle.thomas(a, b, c, Bc @ X[:, i2, i3])
    np.testing.assert_allclose(out, ref, rtol=1e-11, atol=1e-10)


# ---------------------------------------------------------------------------
# Backward oracle
# ---------------------------------------------------------------------------
def test_adjoint_identity():
    rng = np.random.default_rng(9)
    I, J = (6, 7, 8), (3, 5, 4)
    X = rng.standard_normal(I)
    A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
    G = rng.standard_normal(J)
    dX, _, _, _ = oracle.backward(G, X, A, B, C)
    lhs = float(np.sum(oracle.chain(X, A, B, C) * G))
    rhs = float(np.sum(X * dX))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-13


def test_backward_matches_einsum_gradients():
    rng = np.random.default_rng(10)
    I, J = (5, 6, 4), (3, 2, 4)
    X = rng.standard_normal(I)
    A, B, C = (rng.standard_normal((J[n], I[n])) for n in range(3))
    G = rng.standard_normal(J)
    dX, dA, dB, dC = oracle.backward(G, X, A, B, C)
    np.testing.assert_allclose(dX, np.einsum("ijk,ia,jb,kc->abc", G, A, B, C), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(dA, np.einsum("ijk,abc,jb,kc->ia", G, X, B, C), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(dB, np.einsum("ijk,abc,ia,kc->jb", G, X, A, C), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(dC, np.einsum("ijk,abc,ia,jb->kc", G, X, A, B), rtol=1e-12, atol=1e-13)


def test_backward_central_differences_fd_variant():
    """Full central-difference gradient of L = 1/2||Y-T||^2 on the 16^3 variant.
    L is quadratic along every single coordinate, so the central difference has
    no truncation error, only rounding (about eps*L/h)."""
    p = workloads.fd_variant()
    X, A, B, C, T = p["X"], p["A"], p["B"], p["C"], p["T"]
    G = oracle.chain(X, A, B, C) - T
    grads = oracle.backward(G, X, A, B, C)
    h = 1e-6
    L0 = oracle.loss(X, A, B, C, T)
    args = [X, A, B, C]
    for which, g in enumerate(grads):
        base = args[which]
        fd = np.empty(base.size)
        flat = base.ravel()
        for k in range(base.size):
            old = flat[k]
            flat[k] = old + h
            lp = oracle.loss(*args, T)
            flat[k] = old - h
            lm = oracle.loss(*args, T)
            flat[k] = old
            fd[k] = (lp - lm) / (2 * h)
        err = np.linalg.norm(fd - g.ravel()) / np.linalg.norm(g.ravel())
        assert err < 1e-6, (which, err, L0)


# ---------------------------------------------------------------------------
# Batched oracle
# ---------------------------------------------------------------------------
def test_batched_oracle_matches_per_cuboid_brute():
    dims = [(2, 3, 4, 3, 2, 1), (1, 1, 1, 1, 1, 1), (3, 3, 3, 3, 3, 3), (4, 2, 1, 2, 5, 3)]
    p = workloads.random_batched(dims, seed=11)
    Y = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    ox = oa = ob = oc = oy = 0
    for d in dims:
        I1, I2, I3, J1, J2, J3 = d
        X = p["X"][ox:ox + I1 * I2 * I3].reshape(I1, I2, I3)
        A = p["A"][oa:oa + J1 * I1].reshape(J1, I1)
        B = p["B"][ob:ob + J2 * I2].reshape(J2, I2)
        C = p["C"][oc:oc + J3 * I3].reshape(J3, I3)
        ref = oracle.brute(X, A, B, C)
        got = Y[oy:oy + J1 * J2 * J3].reshape(J1, J2, J3)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)
        ox += I1 * I2 * I3; oa += J1 * I1; ob += J2 * I2; oc += J3 * I3; oy += J1 * J2 * J3
    assert oy == Y.size


# ---------------------------------------------------------------------------
# Workload generators (no arithmetic of the method; shapes and statistics)
# ---------------------------------------------------------------------------
def test_workload_c1_shapes_and_determinism():
    p = workloads.dense("c1_f64_64_16")
    q = workloads.dense("c1_f64_64_16")
    assert p["X"].shape == (64, 64, 64) and p["A"].shape == (16, 64)
    assert np.array_equal(p["X"], q["X"]) and np.array_equal(p["C"], q["C"])
    # N(0, 1/64): standard deviation 1/8
    assert abs(np.std(np.concatenate([p["A"].ravel(), p["B"].ravel(), p["C"].ravel()])) - 0.125) < 0.01


def test_orthonormal_rows_generator():
    rng = np.random.default_rng(0)
    Q = workloads.orthonormal_rows(rng, 8, 40)
    np.testing.assert_allclose(Q @ Q.T, np.eye(8), atol=1e-14)


def test_c1_oracle_gaussian_statistics():
    # For X ~ N(0,1) i.i.d. and factors with N(0,1/I) entries, E[Y^2] = product of
    # the squared row norms' expectation, i.e. about 1; the sample mean square of
    # 16^3 entries is 1 within a few percent.
    p = workloads.dense("c1_f64_64_16")
    Y = oracle.chain(p["X"], p["A"], p["B"], p["C"])
    assert Y.shape == (16, 16, 16)
    ms = float(np.mean(Y ** 2))
    expected = float(np.mean(np.sum(p["A"] ** 2, 1))) * float(np.mean(np.sum(p["B"] ** 2, 1))) \
        * float(np.mean(np.sum(p["C"] ** 2, 1)))
    assert abs(ms / expected - 1.0) < 0.25


# ---------------------------------------------------------------------------
# The compact scheme applied along a mode without forming D (Sec. 4.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pin", pins.ALL_COMPACT_PINS, ids=lambda p: p.__name__)
def test_oracle_compact_apply_pins(pin):
    pin(oracle.compact6_apply)


def _dense_apply(X, mode, D):
    return np.moveaxis(np.tensordot(D, X, axes=([1], [mode - 1])), 0, mode - 1)


def _cmut_b_sign(X, mode, alpha, a, b, h):
    Ac, Bc = pins.compact6_periodic_matrices(X.shape[mode - 1], h)
    _, Bm = pins.compact6_periodic_matrices(X.shape[mode - 1], h)
    n = X.shape[mode - 1]
    for i in range(n):   # flip the sign of the two-point-wide term only
        Bm[i, (i + 2) % n] -= 2 * b / (4 * h)
        Bm[i, (i - 2) % n] += 2 * b / (4 * h)
    return _dense_apply(X, mode, np.linalg.solve(Ac, Bm))


def _cmut_alpha_sign(X, mode, alpha, a, b, h):
    n = X.shape[mode - 1]
    Ac, Bc = pins.compact6_periodic_matrices(n, h)
    Am = 2 * np.eye(n) - Ac          # alpha -> -alpha, diagonal kept
    return _dense_apply(X, mode, np.linalg.solve(Am, Bc))


def _cmut_no_wrap(X, mode, alpha, a, b, h):
    n = X.shape[mode - 1]
    Ac, Bc = pins.compact6_periodic_matrices(n, h)
    for i in range(n):
        for j in range(n):
            if abs(i - j) > 2:
                Ac[i, j] = 0.0
                Bc[i, j] = 0.0
    return _dense_apply(X, mode, np.linalg.solve(Ac, Bc))


def _cmut_transposed(X, mode, alpha, a, b, h):
    n = X.shape[mode - 1]
    Ac, Bc = pins.compact6_periodic_matrices(n, h)
    return _dense_apply(X, mode, np.linalg.solve(Ac, Bc).T)


def _cmut_h_twice(X, mode, alpha, a, b, h):
    n = X.shape[mode - 1]
    Ac, Bc = pins.compact6_periodic_matrices(n, 2 * h)
    return _dense_apply(X, mode, np.linalg.solve(Ac, Bc))


def _cmut_wrong_mode(X, mode, alpha, a, b, h):
    other = 1 + mode % 3
    return oracle.compact6_apply(X, other, alpha, a, b, h) if X.shape[other - 1] == X.shape[mode - 1] else \
        np.zeros_like(X)


@pytest.mark.parametrize("mutant", [_cmut_b_sign, _cmut_alpha_sign, _cmut_no_wrap, _cmut_transposed, _cmut_h_twice,
                                    _cmut_wrong_mode], ids=lambda m: m.__name__)
def test_compact_planted_mistakes_are_caught(mutant):
    failures = 0
    for pin in pins.ALL_COMPACT_PINS:
        try:
            pin(mutant)
        except AssertionError:
            failures += 1
    assert failures > 0, f"{mutant.__name__} passed every pin"


def test_oracle_compact_apply_rejects_short_fibers():
    with pytest.raises(ValueError):
        oracle.compact6_apply(np.zeros((2, 4, 4)), 1, 1 / 3, 14 / 9, 1 / 9, 0.1)


# ---------------------------------------------------------------------------
# Reordering between directional layouts (Sec. 4.1) and accumulation
# ---------------------------------------------------------------------------
import itertools

PERMS = list(itertools.permutations(range(3)))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_reorder_matches_numpy_transpose(dtype):
    rng = np.random.default_rng(61)
    X = rng.standard_normal((5, 7, 9)).astype(dtype)
    for perm in PERMS:
        Y = oracle.reorder(X, perm)
        assert Y.dtype == dtype and Y.shape == tuple(X.shape[k] for k in perm)
        assert np.array_equal(Y.view(np.uint8), np.ascontiguousarray(np.transpose(X, perm)).view(np.uint8)), perm


def test_reorder_inverse_and_composition_bitwise():
    rng = np.random.default_rng(62)
    X = rng.standard_normal((4, 6, 3))
    for p in PERMS:
        inv = tuple(int(i) for i in np.argsort(p))
        assert np.array_equal(oracle.reorder(oracle.reorder(X, p), inv), X)
        for q in PERMS:
            # Y = reorder(X, p) has axis k = X axis p[k]; reordering Y by q
            # gives axis k = Y axis q[k] = X axis p[q[k]]
            pq = tuple(p[q[k]] for k in range(3))
            assert np.array_equal(oracle.reorder(oracle.reorder(X, p), q), oracle.reorder(X, pq))


def test_reorder_keeps_nan_and_signed_zero_bits():
    X = np.array([np.nan, -0.0, np.inf, 1.0, -np.inf, 0.0], dtype=np.float32).reshape(1, 2, 3)
    Y = oracle.reorder(X, (2, 0, 1))
    assert np.array_equal(Y.view(np.uint32), np.transpose(X, (2, 0, 1)).copy().view(np.uint32))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_accumulate_is_the_rounded_sum(dtype):
    rng = np.random.default_rng(63)
    X = rng.standard_normal((3, 8, 5)).astype(dtype)
    for perm in PERMS:
        Y0 = rng.standard_normal(tuple(X.shape[k] for k in perm)).astype(dtype)
        Y = oracle.reorder(X, perm, Y=Y0)
        # the sum in the element type (numpy adds float32 arrays in float32)
        assert np.array_equal(Y, Y0 + np.transpose(X, perm)), perm


def test_reorder_rejects_bad_perm():
    X = np.zeros((2, 2, 2))
    for bad in [(0, 0, 1), (0, 1, 3), (-1, 1, 2)]:
        with pytest.raises(ValueError):
            oracle.reorder(X, bad)


# ---------------------------------------------------------------------------
# Gram matrices of the unfoldings and the truncated HOSVD factors
# ---------------------------------------------------------------------------
def unfold(X, mode):
    return np.moveaxis(np.asarray(X, dtype=np.float64), mode - 1, 0).reshape(X.shape[mode - 1], -1)


def test_gram_matches_unfolding_product():
    rng = np.random.default_rng(71)
    X = rng.standard_normal((5, 7, 6))
    for mode in (1, 2, 3):
        U = unfold(X, mode)
        np.testing.assert_allclose(oracle.gram(X, mode), U @ U.T, rtol=1e-13, atol=1e-12)


def test_hosvd_factors_match_svd_of_the_unfoldings():
    """Eigenvectors of the Gram matrices (the oracle's route) against the left
    singular vectors of the unfoldings (numpy's SVD): same subspaces, and the
    same vectors after the sign convention where singular values are simple."""
    rng = np.random.default_rng(72)
    X = rng.standard_normal((6, 8, 7))
    J = (3, 4, 5)
    fs, ev = oracle.hosvd_factors(X, J)
    for mode in (1, 2, 3):
        Usvd, sv, _ = np.linalg.svd(unfold(X, mode), full_matrices=False)
        np.testing.assert_allclose(ev[mode - 1][: len(sv)], sv ** 2, rtol=1e-10, atol=1e-10)
        ref = oracle.sign_fixed_rows(Usvd[:, : J[mode - 1]].T)
        np.testing.assert_allclose(fs[mode - 1], ref, atol=1e-10)
        np.testing.assert_allclose(fs[mode - 1] @ fs[mode - 1].T, np.eye(J[mode - 1]), atol=1e-13)


def test_hosvd_recovers_a_low_multilinear_rank_tensor():
    """X = G x1 P x2 Q x3 R with orthonormal-column P, Q, R of ranks (2, 3, 2):
    the truncated factors span exactly those column spaces, and the chain with
    the factors and back with their transposes returns X."""
    rng = np.random.default_rng(73)
    I, r = (9, 10, 8), (2, 3, 2)
    core = rng.standard_normal(r)
    Ps = [np.linalg.qr(rng.standard_normal((I[n], r[n])))[0] for n in range(3)]
    X = oracle.chain(core, *Ps)
    fs, ev = oracle.hosvd_factors(X, r)
    for n in range(3):
        np.testing.assert_allclose(fs[n].T @ fs[n], Ps[n] @ Ps[n].T, atol=1e-11)
        assert np.all(np.abs(ev[n][r[n]:]) < 1e-13 * ev[n][0])   # rounding level of the eigensolver
    G = oracle.chain(X, *fs)
    back = oracle.chain(G, *(f.T for f in fs))
    np.testing.assert_allclose(back, X, atol=1e-12)
