"""The FP64 HOSVD factors (Gram matrices on the matrix cores, Jacobi
eigensolver in one workgroup) against the oracle's (plain-loop Gram
matrices, numpy's symmetric eigensolver).  Test tensors have simple leading
eigenvalues (a decaying core), so the sign-fixed vectors are unique."""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_13532_amd import chain, hosvd, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def structured(I, r, seed, noise=1e-3):
    """A decaying Tucker core of multilinear rank r plus small noise."""
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(r) * np.einsum("a,b,c->abc", *[0.7 ** np.arange(k) for k in r])
    Ps = [np.linalg.qr(rng.standard_normal((I[n], r[n])))[0] for n in range(3)]
    return oracle.chain(core, *Ps) + noise * rng.standard_normal(I)


@pytest.mark.parametrize("I,J", [((8, 9, 10), (3, 4, 5)), ((64, 64, 64), (16, 16, 16)),
                                 ((33, 128, 17), (6, 10, 4)), ((100, 7, 128), (12, 7, 9))],
                         ids=lambda v: "x".join(map(str, v)))
def test_hosvd_factors_match_oracle(I, J):
    X = structured(I, tuple(min(2 * j, i) for j, i in zip(J, I)), seed=sum(I))
    fs, ev = hosvd(torch.from_numpy(X).to(DEV), J, with_evals=True)
    ref, ref_ev = oracle.hosvd_factors(X, J)
    for n in range(3):
        U = fs[n].cpu().numpy()
        np.testing.assert_allclose(U @ U.T, np.eye(J[n]), atol=1e-12)
        np.testing.assert_allclose(U, ref[n], atol=1e-9)
        e = ev[n].cpu().numpy()
        np.testing.assert_allclose(e, ref_ev[n], rtol=1e-10, atol=1e-10 * ref_ev[n][0])


def test_hosvd_on_the_small_workload_and_tucker_core():
    """The 64^3 float64 workload: the factors give the core X x1 U1 x2 U2 x3 U3
    through the chain, and the core's norm is the captured energy (the sum of
    the leading squared singular values of any one mode bounds it)."""
    p = workloads.dense("c1_f64_64_16")
    X = p["X"]
    Xd = torch.from_numpy(X).to(DEV)
    fs, ev = hosvd(Xd, (16, 16, 16), with_evals=True)
    ref, _ = oracle.hosvd_factors(X, (16, 16, 16))
    for n in range(3):
        # Gaussian data: compare subspaces (projectors), robust to near-ties
        U = fs[n].cpu().numpy()
        np.testing.assert_allclose(U.T @ U, ref[n].T @ ref[n], atol=1e-8)
    core = chain(Xd, *fs, math="f64").cpu().numpy()
    np.testing.assert_allclose(core, oracle.chain(X, *(f.cpu().numpy() for f in fs)), atol=1e-12)
    for n in range(3):
        assert np.sum(core ** 2) <= ev[n][:16].sum().item() * (1 + 1e-12)


def test_hosvd_rejects_long_modes():
    from paper_2411_13532_amd._lib import TTMError
    X = torch.zeros((129, 4, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(TTMError):
        hosvd(X, (4, 4, 4))
