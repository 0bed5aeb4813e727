"""Parity of the adjoint (ttm_chain_backward, TTMChain autograd) against the
FP64 oracle gradient and FP64 central differences."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_13532_amd import TTMChain, chain, chain_backward, workloads
from tests import pins

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt)


def gpu_grads(G, X, A, B, C, dt, math):
    outs = chain_backward(*(dev(t, dt) for t in (G, X, A, B, C)), math=math)
    torch.cuda.synchronize()
    return [o.double().cpu().numpy() for o in outs]


SHAPES = [((6, 7, 8), (3, 5, 4)), ((37, 70, 65), (20, 9, 33)), ((1, 1, 1), (1, 1, 1)),
          ((100, 3, 130), (1, 70, 2)),
          # float32 with J3 <= 32 (a multiple of 4) and I3 a multiple of 64:
          # the streaming kernels for W, dX and dC (ragged row counts, a
          # partial last group of 256 columns, J3 below 16)
          ((5, 70, 128), (6, 9, 32)), ((3, 33, 192), (4, 5, 12)), ((2, 1, 64), (3, 2, 4)),
          ((300, 7, 320), (2, 3, 20)),
          # ... and J2 <= 32 with I2 a multiple of 64: V and R on streaming kernels too
          ((5, 64, 128), (6, 9, 32)), ((3, 192, 64), (4, 32, 12)),
          # float32 with J <= 32, I3 in {256, 512}, I2 a multiple of 4: the
          # fused kernels (two and one 16-row blocks per chunk; ragged last
          # chunks, a single chunk, many slabs, padded J); I3 = 64 and 128 take
          # the product sequence
          ((3, 40, 256), (5, 7, 30)), ((2, 100, 512), (32, 32, 32)), ((4, 132, 256), (1, 17, 3)),
          ((1, 4, 256), (2, 2, 2)), ((7, 256, 256), (32, 32, 32)), ((300, 8, 512), (3, 4, 5)),
          ((2, 100, 64), (32, 32, 32)), ((4, 132, 128), (1, 17, 3))]

FUSED_SHAPES = [((3, 40, 256), (5, 7, 30)), ((2, 100, 512), (32, 32, 32)), ((4, 132, 256), (1, 17, 3))]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"I{s[0]}J{s[1]}")
@pytest.mark.parametrize("math,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_backward_vs_oracle(shape, math, tol):
    I, J = shape
    rng = np.random.default_rng(sum(I) + sum(J))
    p = workloads.random_problem(I, J, seed=sum(I))
    G = rng.standard_normal(J)
    fdt = np.float64 if math == "f64" else np.float32
    ins = [np.asarray(t, dtype=fdt) for t in (G, p["X"], p["A"], p["B"], p["C"])]
    got = gpu_grads(*ins, torch.float64 if math == "f64" else torch.float32, math)
    ref = oracle.backward(*ins)
    for name, g, r in zip(("dX", "dA", "dB", "dC"), got, ref):
        err = pins.rel_fro(g, r)
        assert err <= tol, (name, err)


def test_partial_gradients_only():
    p = workloads.random_problem((9, 10, 11), (4, 5, 6), seed=3)
    G = np.random.default_rng(4).standard_normal((4, 5, 6))
    ref = oracle.backward(G, p["X"], p["A"], p["B"], p["C"])
    for k in range(4):
        need = [i == k for i in range(4)]
        outs = chain_backward(*(dev(t) for t in (G, p["X"], p["A"], p["B"], p["C"])), math="f64", need=need)
        for i, o in enumerate(outs):
            if i == k:
                assert pins.rel_fro(o.cpu().numpy(), ref[i]) <= 1e-12
            else:
                assert o is None


@pytest.mark.parametrize("shape", FUSED_SHAPES, ids=lambda s: f"I{s[0]}J{s[1]}")
def test_fused_partial_gradients_and_determinism(shape):
    """Each gradient alone through the fused float32 kernels, and two runs of
    all four bit for bit equal (every sum has a fixed order)."""
    I, J = shape
    p = workloads.random_problem(I, J, seed=11, dtype=np.float32)
    G = np.random.default_rng(12).standard_normal(J).astype(np.float32)
    ins = (G, p["X"], p["A"], p["B"], p["C"])
    ref = oracle.backward(*ins)
    args = [dev(t, torch.float32) for t in ins]
    for k in range(4):
        need = [i == k for i in range(4)]
        outs = chain_backward(*args, math="f32", need=need)
        for i, o in enumerate(outs):
            if i == k:
                assert pins.rel_fro(o.double().cpu().numpy(), ref[i]) <= 1e-5, (i, shape)
            else:
                assert o is None
    a = chain_backward(*args, math="f32")
    b = chain_backward(*args, math="f32")
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_adjoint_identity_gpu():
    p = workloads.random_problem((30, 40, 50), (7, 8, 9), seed=5)
    G = np.random.default_rng(6).standard_normal((7, 8, 9))
    Xd, Ad, Bd, Cd, Gd = (dev(t) for t in (p["X"], p["A"], p["B"], p["C"], G))
    Y = chain(Xd, Ad, Bd, Cd, math="f64")
    dX, _, _, _ = chain_backward(Gd, Xd, Ad, Bd, Cd, math="f64", need=(True, False, False, False))
    lhs = float((Y * Gd).sum())
    rhs = float((Xd * dX).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_fd_variant_central_differences():
    """16^3 variant: GPU f64 gradient vs central differences of the oracle's loss
    (L is quadratic along each coordinate: no truncation error)."""
    p = workloads.fd_variant()
    X, A, B, C, T = p["X"], p["A"], p["B"], p["C"], p["T"]
    Xd, Ad, Bd, Cd = (dev(t) for t in (X, A, B, C))
    Y = chain(Xd, Ad, Bd, Cd, math="f64")
    G = Y - dev(T)
    grads = [g.cpu().numpy() for g in chain_backward(G, Xd, Ad, Bd, Cd, math="f64")]
    h = 1e-6
    args = [X, A, B, C]
    for which, g in enumerate(grads):
        flat = args[which].ravel()
        fd = np.empty(flat.size)
        for k in range(flat.size):
            old = flat[k]
            flat[k] = old + h
            lp = oracle.loss(*args, T)
            flat[k] = old - h
            lm = oracle.loss(*args, T)
            flat[k] = old
            fd[k] = (lp - lm) / (2 * h)
        err = np.linalg.norm(fd - g.ravel()) / np.linalg.norm(g.ravel())
        assert err < 1e-6, (which, err)


def test_autograd_function_matches_library():
    p = workloads.random_problem((12, 14, 16), (5, 6, 7), seed=8, dtype=np.float32)
    T = np.random.default_rng(9).standard_normal((5, 6, 7)).astype(np.float32)
    leaves = [dev(p[k], torch.float32).requires_grad_(True) for k in "XABC"]
    Y = TTMChain.apply(*leaves, "f32")
    loss = 0.5 * ((Y - dev(T, torch.float32)) ** 2).sum()
    loss.backward()
    G = (Y.detach() - dev(T, torch.float32))
    ref = oracle.backward(G.double().cpu().numpy(), *(p[k] for k in "XABC"))
    for leaf, r in zip(leaves, ref):
        assert pins.rel_fro(leaf.grad.double().cpu().numpy(), r) <= 1e-5


def test_c5_full_size():
    """X 256^3, factors 32 x 256 N(0,1/256), T 32^3: forward and all four
    gradients of L = 1/2||Y - T||^2 against the FP64 oracle."""
    p = workloads.dense("c5_f32_256_32")
    Xd, Ad, Bd, Cd = (dev(p[k], torch.float32) for k in "XABC")
    Y = chain(Xd, Ad, Bd, Cd, math="f32")
    G = Y - dev(p["T"], torch.float32)
    grads = chain_backward(G, Xd, Ad, Bd, Cd, math="f32")
    torch.cuda.synchronize()
    Gn = G.double().cpu().numpy()
    Yref = oracle.chain(p["X"], p["A"], p["B"], p["C"])
    assert pins.rel_fro(Y.double().cpu().numpy(), Yref) <= 1e-5
    ref = oracle.backward(Gn, p["X"], p["A"], p["B"], p["C"])
    for name, g, r in zip(("dX", "dA", "dB", "dC"), grads, ref):
        err = pins.rel_fro(g.double().cpu().numpy(), r)
        print(f"[c5 {name}] rel err {err:.3e}", flush=True)
        assert err <= 1e-5, (name, err)
