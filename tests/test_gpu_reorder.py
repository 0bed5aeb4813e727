"""The layout reorder and accumulate kernels (ttm_reorder) against the
oracle, bit for bit: every permutation of the three axes, float32 and
float64, the 16-byte path and the element path, tiles with ragged edges."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2411_13532_amd import reorder

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PERMS = list(itertools.permutations(range(3)))
SHAPES = [(3, 130, 200), (70, 65, 64), (1, 1, 1), (2, 64, 129), (17, 1, 257), (128, 128, 128)]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_reorder_bitwise(shape, dtype):
    rng = np.random.default_rng(sum(shape))
    X = rng.standard_normal(shape).astype(dtype)
    Xd = torch.from_numpy(X).to(DEV)
    for perm in PERMS:
        Y = reorder(Xd, perm).cpu().numpy()
        assert np.array_equal(Y.view(np.uint8), oracle.reorder(X, perm).view(np.uint8)), perm


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(3, 130, 200), (70, 65, 64), (5, 9, 7)], ids=lambda s: "x".join(map(str, s)))
def test_accumulate_bitwise(shape, dtype):
    rng = np.random.default_rng(7 + sum(shape))
    X = rng.standard_normal(shape).astype(dtype)
    Xd = torch.from_numpy(X).to(DEV)
    for perm in PERMS:
        Y0 = rng.standard_normal(tuple(shape[k] for k in perm)).astype(dtype)
        Yd = torch.from_numpy(Y0.copy()).to(DEV)
        reorder(Xd, perm, out=Yd, accumulate=True)
        assert np.array_equal(Yd.cpu().numpy(), oracle.reorder(X, perm, Y=Y0)), perm


def test_reorder_unaligned_views_take_the_element_path():
    """A tensor starting 4 bytes past a 16-byte boundary is valid input (element
    alignment only); the result is still bit-exact."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 64, 128)).astype(np.float32)
    big = torch.empty(X.size + 1, dtype=torch.float32, device=DEV)
    Xd = big[1:].view(X.shape)
    Xd.copy_(torch.from_numpy(X))
    for perm in PERMS:
        Y = reorder(Xd, perm).cpu().numpy()
        assert np.array_equal(Y, oracle.reorder(X, perm)), perm


def test_reorder_rejects_overlap_and_bad_perm():
    from paper_2411_13532_amd._lib import TTMError
    X = torch.zeros((4, 4, 4), device=DEV)
    with pytest.raises(TTMError):
        reorder(X, (1, 0, 2), out=X.view(4, 4, 4))
    with pytest.raises(ValueError):
        reorder(X, (0, 0, 1))
