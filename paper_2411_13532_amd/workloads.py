"""Seeded synthetic inputs for the mode-n product chain.

This module only draws random numbers and arranges them into arrays.  It holds
none of the chain's arithmetic, so both the HIP path and the FP64 oracle may
take their inputs from it.

Recipe (one numpy ``default_rng(seed)`` per workload, draws in the order
listed, every normal drawn in float64 with ``standard_normal`` and then cast
with round-to-nearest-even):

* ``N(0, s2)`` means mean 0 and *variance* s2 (standard deviation sqrt(s2)).
* Orthonormal-row factors: draw G of shape (I, J), take the reduced QR
  ``Q, _ = numpy.linalg.qr(G)`` and use Q^T (J x I), cast to float32.
* Cubic dense chain sizes: X is I x I x I, every factor is J x I.
"""
from __future__ import annotations

import numpy as np

# Workload table: name -> (seed, I, J, storage of X, description)
DENSE = {
    "c1_f64_64_16": dict(seed=0, I=64, J=16, x_dtype="f64", factors="gauss"),
    "c2_f32_512_64": dict(seed=1, I=512, J=64, x_dtype="f32", factors="orth"),
    "c3_bf16_1024_128": dict(seed=2, I=1024, J=128, x_dtype="bf16", factors="orth"),
    "c5_f32_256_32": dict(seed=4, I=256, J=32, x_dtype="f32", factors="gauss"),
}

BATCHED_COUNT = 20000
BATCHED_NMIN, BATCHED_NMAX = 5, 13
BATCHED_SEED = 3


def _normals(rng: np.random.Generator, shape, chunk: int = 1 << 26) -> np.ndarray:
    """float64 N(0,1) draws filled in chunks (same stream as one big call)."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = rng.standard_normal(e - s)
    return out.reshape(shape)


def _normals_f32(rng: np.random.Generator, shape, chunk: int = 1 << 26) -> np.ndarray:
    """float64 N(0,1) draws cast chunk by chunk to float32 (no float64 copy of the whole)."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = rng.standard_normal(e - s).astype(np.float32)
    return out.reshape(shape)


def orthonormal_rows(rng: np.random.Generator, J: int, I: int) -> np.ndarray:
    """J x I float64 matrix with orthonormal rows (Q^T of a reduced QR)."""
    g = rng.standard_normal((I, J))
    q, _ = np.linalg.qr(g)
    return np.ascontiguousarray(q.T)


def to_bf16(x32: np.ndarray):
    """Round a float32 array to bfloat16 (round to nearest even) as a CPU torch tensor."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(x32)).to(torch.bfloat16)


def dense(name: str) -> dict:
    """Inputs of one dense workload.

    Returns a dict with X (numpy float64/float32, or a CPU torch bfloat16
    tensor for the BF16-stored workload), A, B, C (float64 for the FP64
    workload, else float32), and T for the differentiation workload.
    """
    cfg = DENSE[name]
    rng = np.random.default_rng(cfg["seed"])
    I, J = cfg["I"], cfg["J"]
    if cfg["x_dtype"] == "f64":
        X = _normals(rng, (I, I, I))
    else:
        X = _normals_f32(rng, (I, I, I))
    fs = []
    for _ in range(3):
        if cfg["factors"] == "orth":
            fs.append(orthonormal_rows(rng, J, I))
        else:
            fs.append(rng.standard_normal((J, I)) * (1.0 / np.sqrt(I)))
    out = dict(name=name, I=I, J=J)
    if cfg["x_dtype"] == "f64":
        out.update(X=X, A=fs[0], B=fs[1], C=fs[2])
    else:
        out.update(A=fs[0].astype(np.float32), B=fs[1].astype(np.float32), C=fs[2].astype(np.float32))
        out["X"] = to_bf16(X) if cfg["x_dtype"] == "bf16" else X
    if name.startswith("c5"):
        out["T"] = rng.standard_normal((J, J, J)).astype(np.float32)
    return out


def fd_variant(seed: int = 4, I: int = 16, J: int = 4) -> dict:
    """Small float64 variant of the differentiation workload for finite differences:
    X I^3 N(0,1), factors J x I N(0, 1/I), target T J^3 N(0,1)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((I, I, I))
    A, B, C = (rng.standard_normal((J, I)) / np.sqrt(I) for _ in range(3))
    T = rng.standard_normal((J, J, J))
    return dict(X=X, A=A, B=B, C=C, T=T)


def batched(count: int = BATCHED_COUNT, seed: int = BATCHED_SEED,
            nmin: int = BATCHED_NMIN, nmax: int = BATCHED_NMAX,
            dtype=np.float32) -> dict:
    """Ragged batch of cubic cuboids n_k^3 with square n_k x n_k factors.

    n_k ~ uniform{nmin..nmax}; then per cuboid, in index order, X_k N(0,1),
    A_k, B_k, C_k N(0, 1/n_k).  Buffers are concatenated in cuboid order.
    """
    rng = np.random.default_rng(seed)
    n = rng.integers(nmin, nmax + 1, size=count)
    xs, as_, bs, cs = [], [], [], []
    for k in range(count):
        nk = int(n[k])
        xs.append(rng.standard_normal(nk * nk * nk))
        s = 1.0 / np.sqrt(nk)
        as_.append(rng.standard_normal(nk * nk) * s)
        bs.append(rng.standard_normal(nk * nk) * s)
        cs.append(rng.standard_normal(nk * nk) * s)
    dims = np.stack([n, n, n, n, n, n], axis=1).astype(np.int64)
    cat = lambda parts: np.concatenate(parts).astype(dtype)
    return dict(dims=dims, X=cat(xs), A=cat(as_), B=cat(bs), C=cat(cs))


def random_problem(I, J, seed: int, dtype=np.float64, fscale: float | None = None) -> dict:
    """Generic problem for tests: X N(0,1) of shape I, factors J_n x I_n N(0, 1/I_n)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(tuple(I))
    fs = [rng.standard_normal((J[n], I[n])) * (fscale if fscale is not None else 1.0 / np.sqrt(I[n]))
          for n in range(3)]
    return dict(X=X.astype(dtype), A=fs[0].astype(dtype), B=fs[1].astype(dtype), C=fs[2].astype(dtype))


def random_batched(dims, seed: int, dtype=np.float64) -> dict:
    """Generic ragged batch for tests with arbitrary (I1,I2,I3,J1,J2,J3) per cuboid."""
    rng = np.random.default_rng(seed)
    dims = np.asarray(dims, dtype=np.int64).reshape(-1, 6)
    xs, as_, bs, cs = [], [], [], []
    for d in dims:
        I1, I2, I3, J1, J2, J3 = (int(v) for v in d)
        xs.append(rng.standard_normal(I1 * I2 * I3))
        as_.append(rng.standard_normal(J1 * I1) / np.sqrt(I1))
        bs.append(rng.standard_normal(J2 * I2) / np.sqrt(I2))
        cs.append(rng.standard_normal(J3 * I3) / np.sqrt(I3))
    cat = lambda parts: np.concatenate(parts).astype(dtype)
    return dict(dims=dims, X=cat(xs), A=cat(as_), B=cat(bs), C=cat(cs))
