"""Parity of the HIP chain (ttm_chain) against the FP64 oracle.

Tolerances (relative Frobenius error against the FP64 oracle on the exact
stored inputs): 1e-12 for f64, 1e-5 for f32 and bf16x3, 2e-2 for plain bf16.
Bitwise checks where the arithmetic is exact (identity factors, small
integers).  The full-size workloads compare every output element with the
oracle's result on the same stored inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_13532_amd import chain, workloads
from tests import pins

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-5, "bf16": 2e-2}
DEV = "cuda:0"


def to_dev(a, dtype):
    if isinstance(a, torch.Tensor):
        return a.to(DEV).to(dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype).contiguous()


def int_chain(X, A, B, C):
    """Exact integer chain (int64 tensordot per mode) for integer-valued data."""
    Y = np.tensordot(X.astype(np.int64), C.astype(np.int64), axes=([2], [1]))      # [i1][i2][j3]
    Y = np.tensordot(Y, B.astype(np.int64), axes=([1], [1]))                        # [i1][j3][j2]
    Y = np.tensordot(Y, A.astype(np.int64), axes=([0], [1]))                        # [j3][j2][j1]
    return np.transpose(Y, (2, 1, 0)).astype(np.float64)


def run(X, A, B, C, math, xdtype=None):
    fdt = torch.float64 if math == "f64" else torch.float32
    xdt = xdtype or fdt
    Xd = to_dev(X, xdt)
    Y = chain(Xd, to_dev(A, fdt), to_dev(B, fdt), to_dev(C, fdt), math=math)
    torch.cuda.synchronize()
    return Y.double().cpu().numpy(), Xd


def stored(Xd):
    """The exact values the GPU consumed, as a float64/float32 numpy array."""
    if Xd.dtype == torch.bfloat16:
        return Xd.float().cpu().numpy()
    return Xd.cpu().numpy()


def check_vs_oracle(p, math, xdtype=None, tol=None):
    Y, Xd = run(p["X"], p["A"], p["B"], p["C"], math, xdtype)
    fdt = np.float64 if math == "f64" else np.float32
    ref = oracle.chain(stored(Xd), *(np.asarray(p[k], dtype=fdt) for k in "ABC"))
    err = pins.rel_fro(Y, ref)
    print(f"[{math} x={xdtype} I={np.shape(p['X'])} J={ref.shape}] rel err {err:.3e}", flush=True)
    assert err <= (tol if tol is not None else TOL[math]), err
    return Y, ref


FORMS = [("f64", None), ("f32", None), ("f32", torch.bfloat16), ("bf16", torch.bfloat16),
         ("bf16", None), ("bf16x3", torch.bfloat16), ("bf16x3", None)]
FORM_IDS = [f"{m}-x{'bf16' if x is torch.bfloat16 else 'native'}" for m, x in FORMS]

# shapes spanning several row tiles and k chunks with ragged tails, the
# unaligned (scalar-load) path, wide J (column and j2 tiling), size-1 modes,
# and (last) factors whose shapes need no padding, read in place by the
# float and double forms
SHAPES = [
    ((37, 150, 200), (20, 35, 70)),
    ((3, 260, 136), (130, 140, 150)),
    ((5, 7, 13), (3, 4, 5)),
    ((2, 129, 72), (17, 1, 33)),
    ((1, 1, 1), (1, 1, 1)),
    ((4, 5, 6), (7, 8, 9)),
    ((16, 300, 24), (2, 260, 16)),
    ((64, 128, 96), (16, 32, 32)),
]


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"I{s[0]}J{s[1]}")
def test_chain_ragged_shapes(form, shape):
    math, xdt = form
    I, J = shape
    p = workloads.random_problem(I, J, seed=sum(I) + 7 * sum(J))
    check_vs_oracle(p, math, xdt)


def test_c1_fp64():
    p = workloads.dense("c1_f64_64_16")
    check_vs_oracle(p, "f64")


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_identity_factors_bitwise(form):
    math, xdt = form
    rng = np.random.default_rng(3)
    I = (9, 140, 70)
    X = rng.standard_normal(I)
    if math in ("bf16", "bf16x3"):
        X = torch.from_numpy(X.astype(np.float32)).to(torch.bfloat16).float().numpy()  # exactly bf16
    eye = [np.eye(n) for n in I]
    Y, Xd = run(X, *eye, math, xdt)
    assert np.array_equal(Y, stored(Xd).astype(np.float64))


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_exact_integers_bitwise(form):
    """Small integers: every partial sum is exact on every path (values in
    {-1,0,1}, I <= 6 keeps plain-bf16 intermediates within 256)."""
    math, xdt = form
    rng = np.random.default_rng(5)
    I, J = (6, 5, 6), (4, 6, 3)
    X = rng.integers(-1, 2, size=I).astype(np.float64)
    A, B, C = (rng.integers(-1, 2, size=(J[n], I[n])).astype(np.float64) for n in range(3))
    Y, _ = run(X, A, B, C, math, xdt)
    assert np.array_equal(Y, int_chain(X, A, B, C))


@pytest.mark.parametrize("math", ["f32", "bf16x3", "f64"])
def test_exact_integers_one_mode_larger(math):
    """One nontrivial mode at a time with integer data over several tiles:
    bitwise on f32/f64 (sums < 2^24) and bf16x3 (intermediates < 2^16)."""
    rng = np.random.default_rng(6)
    I = (20, 150, 200)
    X = rng.integers(-4, 5, size=I).astype(np.float64)
    for mode in range(3):
        fs = [np.eye(n) for n in I]
        fs[mode] = rng.integers(-4, 5, size=(17, I[mode])).astype(np.float64)
        Y, _ = run(X, *fs, math)
        assert np.array_equal(Y, int_chain(X, *fs)), mode


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_rank1_closed_form(form):
    math, xdt = form
    rng = np.random.default_rng(7)
    I, J = (33, 140, 90), (12, 40, 70)
    u, v, w = (rng.standard_normal(I[n]) for n in range(3))
    X = np.einsum("a,b,c->abc", u, v, w)
    fs = [rng.standard_normal((J[n], I[n])) / np.sqrt(I[n]) for n in range(3)]
    Y, Xd = run(X, *fs, math, xdt)
    # reference from the closed form on the values the GPU consumed
    fdt = np.float64 if math == "f64" else np.float32
    fs_st = [f.astype(fdt).astype(np.float64) for f in fs]
    ref = oracle.chain(stored(Xd), *fs_st)
    closed = np.einsum("a,b,c->abc", fs_st[0] @ u, fs_st[1] @ v, fs_st[2] @ w)
    if math == "f64":
        assert pins.rel_fro(ref, closed) < 1e-13
    assert pins.rel_fro(Y, ref) <= TOL[math]


@pytest.mark.parametrize("n", [8, 12, 13, 64])
@pytest.mark.parametrize("math", ["f64", "f32", "bf16x3"])
def test_compact6_closed_form(n, math):
    """Factors D = A_c^-1 B_c of the paper's compact scheme on periodic grids:
    sin sin sin maps to k'k'k' cos cos cos exactly.  In f64 the GPU result is
    compared with the closed form itself; in f32 and bf16x3 with the oracle on
    the rounded inputs (rounding D to float moves the exact answer by more
    than the arithmetic tolerance, since D amplifies high wavenumbers)."""
    sizes = (n, n + 3, n + 5) if n < 64 else (64, 64, 64)
    modes = (1, 2, 3) if n < 64 else (5, 9, 13)
    Ds = [pins.compact6_derivative_matrix(k) for k in sizes]
    xs = [np.arange(k) * (2 * np.pi / k) for k in sizes]
    X = np.einsum("a,b,c->abc", *[np.sin(m * x) for m, x in zip(modes, xs)])
    kap = np.prod([pins.compact6_modified_wavenumber(m, k) for m, k in zip(modes, sizes)])
    closed = kap * np.einsum("a,b,c->abc", *[np.cos(m * x) for m, x in zip(modes, xs)])
    Y, Xd = run(X, *Ds, math)
    if math == "f64":
        assert pins.rel_fro(Y, closed) <= 1e-12
    else:
        # Reference: the oracle on the rounded factors.  f32 meets the general
        # 1e-5.  bf16x3 keeps about 16 significant bits per operand, so its
        # error is about 2^-17 times the condition number of these sums, which
        # cancel heavily (D amplifies high wavenumbers while Y is smooth):
        # cond = ||chain(|X|, |D|, ..)|| / ||Y|| is 10-34 for these sizes and
        # 3.7e-5 was measured at n = 64.  The fixed cap 1e-4 still fails a
        # tenfold loss of accuracy.
        Ds32 = [D.astype(np.float32) for D in Ds]
        ref = oracle.chain(stored(Xd), *Ds32)
        cond = np.linalg.norm(oracle.chain(np.abs(stored(Xd)), *(np.abs(D) for D in Ds32))) / np.linalg.norm(ref)
        err = pins.rel_fro(Y, ref)
        print(f"[compact6 {math} n={n}] rel err {err:.3e}, cond {cond:.1f}", flush=True)
        assert err <= {"f32": TOL["f32"], "bf16x3": 1e-4}[math]


@pytest.mark.parametrize("math", ["f32", "bf16x3", "bf16", "f64"])
def test_deterministic(math):
    p = workloads.random_problem((40, 300, 96), (30, 50, 70), seed=9)
    Y1, _ = run(p["X"], p["A"], p["B"], p["C"], math)
    Y2, _ = run(p["X"], p["A"], p["B"], p["C"], math)
    assert np.array_equal(Y1, Y2)


def test_mode_order_free_operator():
    """Y computed for (X, A, B, C) equals the chain of the permuted problem
    (X transposed, factors permuted) transposed back: the library's internal
    contraction order does not change the operator."""
    p = workloads.random_problem((20, 36, 50), (8, 9, 10), seed=13)
    Y, _ = run(p["X"], p["A"], p["B"], p["C"], "f64")
    Xp = np.ascontiguousarray(np.transpose(p["X"], (2, 0, 1)))
    Yp, _ = run(Xp, p["C"], p["A"], p["B"], "f64")
    assert pins.rel_fro(np.transpose(Yp, (1, 2, 0)), Y) < 1e-13


# ---------------------------------------------------------------------------
# Full-size workloads: every element of Y against the oracle
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c2_inputs():
    p = workloads.dense("c2_f32_512_64")
    dev = [to_dev(p[k], torch.float32) for k in "XABC"]
    ref = oracle.chain(p["X"], *(p[k].astype(np.float64) for k in "ABC"))
    return dev, ref


@pytest.mark.parametrize("math", ["f32", "bf16x3"])
def test_c2_full_size(c2_inputs, math):
    (Xd, Ad, Bd, Cd), ref = c2_inputs
    Y = chain(Xd, Ad, Bd, Cd, math=math)
    err = pins.rel_fro(Y.double().cpu().numpy(), ref)
    print(f"[c2 {math}] rel err {err:.3e}", flush=True)
    assert err <= TOL[math]
    # orthonormal rows and Gaussian X: entries of Y are N(0,1)
    var = float(Y.double().var().cpu())
    assert abs(var - 1.0) < 0.02


@pytest.fixture(scope="module")
def c3_inputs():
    p = workloads.dense("c3_bf16_1024_128")
    Xd = p["X"].to(DEV)
    fs = [to_dev(p[k], torch.float32) for k in "ABC"]
    X_np = p["X"].float().numpy()          # the stored bf16 values, exactly
    ref = oracle.chain(X_np, *(p[k].astype(np.float64) for k in "ABC"))
    del X_np
    return Xd, fs, ref


@pytest.mark.parametrize("math", ["bf16x3", "bf16", "f32"])
def test_c3_full_size(c3_inputs, math):
    Xd, fs, ref = c3_inputs
    Y = chain(Xd, *fs, math=math)
    err = pins.rel_fro(Y.double().cpu().numpy(), ref)
    print(f"[c3 {math}] rel err {err:.3e}", flush=True)
    assert err <= TOL[math]


# ---------------------------------------------------------------------------
# The automatic selection on bf16 X with ragged multi-tile row ranges: several
# 256-row tiles per workgroup with a partial last tile, 384-row ranges over
# two splits, and one or two 64-value chunks per row (the short-row preamble).
# The last three cover the mode-2 step's B staging with one column block per
# wave and eight j2 blocks (three phase buffers in bf16x3), two j2 blocks
# with two column blocks, and a single j2 block (B fragments from L2).
# ---------------------------------------------------------------------------
LC_SHAPES = [((1024, 300, 64), (24, 40, 100)), ((512, 600, 128), (33, 40, 70)), ((1024, 600, 64), (16, 20, 48)),
             ((512, 300, 128), (10, 120, 50)), ((512, 280, 64), (10, 30, 80)), ((512, 300, 128), (5, 16, 100))]


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("shape", LC_SHAPES, ids=lambda s: f"I{s[0]}J{s[1]}")
def test_chain_multi_tile_ranges(form, shape):
    math, xdt = form
    I, J = shape
    p = workloads.random_problem(I, J, seed=sum(I) + 3 * sum(J))
    check_vs_oracle(p, math, xdt)


# ---------------------------------------------------------------------------
# Every slab kernel (direct-to-LDS variants and register-staged) on shapes
# where the direct-to-LDS ones apply: whole 128 or 256-byte chunks along i3,
# ragged i2 ranges, one, two and four column waves.
# ---------------------------------------------------------------------------
DMA_SHAPES = [((7, 300, 256), (20, 35, 70)), ((3, 129, 128), (16, 130, 128)), ((2, 513, 512), (64, 64, 64)),
              ((5, 40, 1024), (128, 128, 128)), ((4, 517, 192), (9, 33, 100)), ((6, 70, 320), (5, 31, 24)),
              ((2, 260, 64), (3, 12, 12))]


@pytest.fixture
def slab_kernel_mode():
    from paper_2411_13532_amd import set_slab_kernel
    yield set_slab_kernel
    set_slab_kernel(0)


@pytest.mark.parametrize("mode", [0, 1, 2, 3], ids=["auto", "staged", "dma256", "ldsc"])
@pytest.mark.parametrize("form", [("f64", None), ("f32", None), ("bf16", torch.bfloat16), ("bf16x3", torch.bfloat16)],
                         ids=["f64", "f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("shape", DMA_SHAPES, ids=lambda s: f"I{s[0]}J{s[1]}")
def test_slab_kernels_agree_with_oracle(shape, form, mode, slab_kernel_mode):
    slab_kernel_mode(mode)
    math, xdt = form
    I, J = shape
    p = workloads.random_problem(I, J, seed=sum(I) + sum(J))
    check_vs_oracle(p, math, xdt)


@pytest.mark.parametrize("form", [("f32", None), ("bf16x3", torch.bfloat16)], ids=["f32", "bf16x3"])
def test_slab_kernels_identity_bitwise(form, slab_kernel_mode):
    math, xdt = form
    rng = np.random.default_rng(31)
    I = (3, 200, 256)
    X = torch.from_numpy(rng.standard_normal(I).astype(np.float32)).to(torch.bfloat16).float().numpy()
    outs = []
    for mode in (0, 1, 2, 3):
        slab_kernel_mode(mode)
        Y, Xd = run(X, *[np.eye(n) for n in I], math, xdt)
        assert np.array_equal(Y, stored(Xd).astype(np.float64))
        outs.append(Y)
    assert np.array_equal(outs[0], outs[1])
