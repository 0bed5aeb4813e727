"""Parity of the ragged batched chain (one persistent launch, graph replay,
per-cuboid launch loop) against the FP64 oracle."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2411_13532_amd import BatchedPlan, workloads
from tests import pins

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt)


def run_plan(p, dtype, mode="persistent", plan=None):
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    plan = plan or BatchedPlan(p["dims"], dtype=tdt)
    bufs = [dev(p[k], tdt) for k in "XABC"]
    Y = plan.run(*bufs, mode=mode)
    torch.cuda.synchronize()
    return Y.double().cpu().numpy(), plan, bufs


def ragged_dims(rng, count, lo=1, hi=16, square=False):
    if square:
        n = rng.integers(lo, hi + 1, size=count)
        return np.stack([n] * 6, axis=1)
    return rng.integers(lo, hi + 1, size=(count, 6))


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
@pytest.mark.parametrize("mode", ["persistent", "graph", "loop"])
def test_ragged_nonsquare(dtype, tol, mode):
    rng = np.random.default_rng(21)
    dims = ragged_dims(rng, 300)
    p = workloads.random_batched(dims, seed=22, dtype=dtype)
    Y, _, _ = run_plan(p, dtype, mode)
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    assert pins.rel_fro(Y, ref) <= tol


@pytest.mark.parametrize("dims", [
    [(1, 1, 1, 1, 1, 1)],
    [(13, 13, 13, 13, 13, 13)],
    [(16, 16, 16, 16, 16, 16)] * 3,
    [(5, 5, 5, 5, 5, 5)] * 500,
    [(16, 1, 16, 1, 16, 1), (1, 16, 1, 16, 1, 16)],
], ids=["single-1", "single-13", "max-16", "all-5", "skinny"])
def test_edge_batches(dims):
    p = workloads.random_batched(dims, seed=23, dtype=np.float64)
    Y, _, _ = run_plan(p, np.float64)
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    assert pins.rel_fro(Y, ref) <= 1e-12


def test_exact_integers_bitwise():
    rng = np.random.default_rng(24)
    dims = ragged_dims(rng, 200, 1, 8)
    p = workloads.random_batched(dims, seed=25, dtype=np.float64)
    for k in "XABC":
        p[k] = np.round(p[k] * 2.0).clip(-3, 3)
    Y, _, _ = run_plan(p, np.float32)
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    assert np.array_equal(Y, ref)


def test_graph_replays_match_eager():
    rng = np.random.default_rng(26)
    dims = ragged_dims(rng, 1000, 3, 13, square=True)
    p = workloads.random_batched(dims, seed=27, dtype=np.float32)
    Y0, plan, bufs = run_plan(p, np.float32)
    for rep in range(4):
        # eager work between replays
        _ = (bufs[0] * 2.0).sum().item()
        Y = plan.run(*bufs, mode="graph")
        torch.cuda.synchronize()
        assert np.array_equal(Y.double().cpu().numpy(), Y0), rep
    # new output buffer: the graph node is updated in place
    Y2 = torch.full_like(bufs[0][: plan.totals[4]], float("nan"))
    plan.run(*bufs, Y=Y2, mode="graph")
    torch.cuda.synchronize()
    assert np.array_equal(Y2.double().cpu().numpy(), Y0)


def test_deterministic_and_autotune(tmp_path):
    rng = np.random.default_rng(28)
    dims = ragged_dims(rng, 3000, 5, 13, square=True)
    p = workloads.random_batched(dims, seed=29, dtype=np.float32)
    cache = str(tmp_path / "tune.json")
    tdt = torch.float32
    plan = BatchedPlan(p["dims"], dtype=tdt, tune_cache=cache)
    bufs = [dev(p[k], tdt) for k in "XABC"]
    Y0 = plan.run(*bufs).cpu().numpy()
    Y1 = plan.run(*bufs).cpu().numpy()
    assert np.array_equal(Y0, Y1)
    best = plan.autotune(*bufs, reps=3)
    assert best > 0
    cfg = plan.config()
    assert cfg["threads"] in (64, 128, 256) and cfg["blocks_per_cu"] >= 1
    Y2 = plan.run(*bufs).cpu().numpy()
    if cfg["variant"] in (0, 1, 2):
        assert np.array_equal(Y0, Y2)   # the launch shape does not change the arithmetic
    else:                               # matrix cores: another order of the terms
        ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
        assert pins.rel_fro(Y2.astype(np.float64), ref) <= 1e-5
    assert os.path.exists(cache)
    plan2 = BatchedPlan(p["dims"], dtype=tdt, tune_cache=cache)
    assert plan2.config()["threads"] == cfg["threads"]
    assert plan2.config()["blocks_per_cu"] == cfg["blocks_per_cu"]


def test_autotune_double():
    """float64 has one kernel: the autotuner only picks the launch shape, and
    the result stays bit for bit."""
    rng = np.random.default_rng(36)
    dims = ragged_dims(rng, 400, 1, 16)
    p = workloads.random_batched(dims, seed=37, dtype=np.float64)
    Y0, plan, bufs = run_plan(p, np.float64)
    best = plan.autotune(*bufs, reps=1)
    assert best > 0 and plan.config()["variant"] == 0
    Y1 = plan.run(*bufs).cpu().numpy()
    assert np.array_equal(Y1, Y0)
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    assert pins.rel_fro(Y1, ref) <= 1e-12


def test_c4_full_workload():
    """20000 cuboids n ~ U{5..13}, square factors N(0, 1/n), float32."""
    p = workloads.batched()
    Y, plan, bufs = run_plan(p, np.float32)
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    err = pins.rel_fro(Y, ref)
    # worst single cuboid
    worst = 0.0
    off = 0
    for d in p["dims"]:
        n = int(d[3] * d[4] * d[5])
        worst = max(worst, pins.rel_fro(Y[off:off + n], ref[off:off + n]))
        off += n
    print(f"[c4] rel err {err:.3e}, worst cuboid {worst:.3e}", flush=True)
    assert err <= 1e-5 and worst <= 1e-5
    Yg = plan.run(*bufs, mode="graph")
    torch.cuda.synchronize()
    assert np.array_equal(Yg.double().cpu().numpy(), Y)


VECTOR_VARIANTS = (0, 1, 2)     # mode products on the vector units
MATRIX_VARIANTS = (3, 4)        # mode products on the matrix cores


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4],
                         ids=["occ2-prefetch", "occ3", "occ4", "mfma-occ3-prefetch", "mfma-occ4"])
@pytest.mark.parametrize("threads", [64, 256])
def test_every_launch_variant(variant, threads):
    """Every kernel variant and block size gives the oracle's result to 1e-5
    on ragged sizes up to 16 (four passes of 64 fibers, sixteen tiles of 16),
    and the result of every other variant of its arithmetic (vector units:
    the default shape; matrix cores: variant 3 at 256 threads) bit for bit."""
    rng = np.random.default_rng(30)
    dims = ragged_dims(rng, 700, 1, 16)
    p = workloads.random_batched(dims, seed=31, dtype=np.float32)
    tdt = torch.float32
    plan = BatchedPlan(p["dims"], dtype=tdt)
    bufs = [dev(p[k], tdt) for k in "XABC"]
    if variant in MATRIX_VARIANTS:
        plan.set_config(256, 1, 3)
    Y0 = plan.run(*bufs).cpu().numpy()
    plan.set_config(threads, 1, variant)
    cfg = plan.config()
    assert cfg["threads"] == threads and cfg["blocks_per_cu"] == 1 and cfg["variant"] == variant
    Y = plan.run(*bufs).cpu().numpy()
    assert np.array_equal(Y, Y0)
    Yg = plan.run(*bufs, mode="graph").cpu().numpy()
    assert np.array_equal(Yg, Y0)
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    assert pins.rel_fro(Y.astype(np.float64), ref) <= 1e-5
    with pytest.raises(RuntimeError):
        plan.set_config(96, 1, variant)
    with pytest.raises(RuntimeError):
        plan.set_config(threads, 1, 5)


@pytest.mark.parametrize("variant", MATRIX_VARIANTS, ids=["mfma-occ3-prefetch", "mfma-occ4"])
@pytest.mark.parametrize("dims", [
    [(1, 1, 1, 1, 1, 1)],
    [(13, 13, 13, 13, 13, 13)],
    [(16, 16, 16, 16, 16, 16)] * 3,
    [(5, 5, 5, 5, 5, 5)] * 500,
    [(16, 1, 16, 1, 16, 1), (1, 16, 1, 16, 1, 16)],
    [(3, 16, 7, 16, 2, 9), (16, 2, 5, 1, 16, 16), (9, 9, 16, 4, 13, 1)],
], ids=["single-1", "single-13", "max-16", "all-5", "skinny", "mixed-ragged"])
def test_matrix_core_variant_edges(variant, dims):
    """The matrix-core variants on single elements, the largest cuboids (16
    tiles, four k steps), many equal small ones, skinny and mixed shapes
    (fibers and outputs that end inside a tile, k slots past the fiber)."""
    p = workloads.random_batched(dims, seed=33, dtype=np.float32)
    tdt = torch.float32
    plan = BatchedPlan(p["dims"], dtype=tdt)
    plan.set_config(256 if len(dims) > 8 else 64, 1, variant)
    bufs = [dev(p[k], tdt) for k in "XABC"]
    Y = plan.run(*bufs).double().cpu().numpy()
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    assert pins.rel_fro(Y, ref) <= 1e-5


@pytest.mark.parametrize("variant", MATRIX_VARIANTS, ids=["mfma-occ3-prefetch", "mfma-occ4"])
def test_matrix_core_exact_integers_bitwise(variant):
    rng = np.random.default_rng(34)
    dims = ragged_dims(rng, 200, 1, 16)
    p = workloads.random_batched(dims, seed=35, dtype=np.float64)
    for k in "XABC":
        p[k] = np.round(p[k] * 2.0).clip(-3, 3)
    tdt = torch.float32
    plan = BatchedPlan(p["dims"], dtype=tdt)
    plan.set_config(256, 1, variant)
    bufs = [dev(p[k], tdt) for k in "XABC"]
    Y = plan.run(*bufs).double().cpu().numpy()
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    assert np.array_equal(Y, ref)


def test_c4_full_workload_matrix_cores():
    """The c4 batch through the matrix-core variant, every cuboid to 1e-5."""
    p = workloads.batched()
    tdt = torch.float32
    plan = BatchedPlan(p["dims"], dtype=tdt)
    plan.set_config(256, 1, 4)
    Y, _, bufs = run_plan(p, np.float32, plan=plan)
    ref = oracle.batched(p["dims"], p["X"], p["A"], p["B"], p["C"])
    off = 0
    worst = 0.0
    for d in p["dims"]:
        n = int(d[3] * d[4] * d[5])
        worst = max(worst, pins.rel_fro(Y[off:off + n], ref[off:off + n]))
        off += n
    print(f"[c4 matrix cores] rel err {pins.rel_fro(Y, ref):.3e}, worst cuboid {worst:.3e}", flush=True)
    assert pins.rel_fro(Y, ref) <= 1e-5 and worst <= 1e-5
