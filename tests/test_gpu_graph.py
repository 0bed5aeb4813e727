"""Stream capture of ttm_chain and ttm_chain_backward into a HIP graph.

The compute calls neither allocate nor synchronise, so a caller may capture
them.  Each captured graph is replayed several times, with eager library
work and synchronisations between replays, and every replay must reproduce
the eager result bit for bit (the same kernels in the same order).  The
output buffers are overwritten with NaN before each replay, so a replay that
skipped a kernel would show.
"""
import numpy as np
import pytest
import torch

from paper_2411_13532_amd import chain, chain_backward, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (math, X storage): the 1024 x 256 x 64 shape takes the slab kernel with C in
# LDS for the bf16 forms and the split mode-1 reduction
CASES = [("f32", torch.float32), ("bf16x3", torch.bfloat16), ("bf16", torch.bfloat16), ("f64", torch.float64)]


def _inputs(I, J, math, xdt, seed):
    p = workloads.random_problem(I, J, seed=seed)
    fdt = torch.float64 if math == "f64" else torch.float32
    X = torch.from_numpy(p["X"]).to(DEV).to(xdt).contiguous()
    fs = [torch.from_numpy(p[k]).to(DEV).to(fdt).contiguous() for k in "ABC"]
    return X, fs


@pytest.mark.parametrize("math,xdt", CASES, ids=[c[0] for c in CASES])
def test_chain_graph_replay_bitwise(math, xdt):
    I, J = (1024, 256, 64), (20, 36, 48)
    X, (A, B, C) = _inputs(I, J, math, xdt, seed=41)
    X2, (A2, B2, C2) = _inputs(I, J, math, xdt, seed=42)
    eager = chain(X, A, B, C, math=math).clone()
    eager2 = chain(X2, A2, B2, C2, math=math).clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            chain(X, A, B, C, math=math)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        Yg = chain(X, A, B, C, math=math)
    for rep in range(4):
        Yg.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Yg, eager), rep
        # eager work between replays, on other buffers
        Ye = chain(X2, A2, B2, C2, math=math)
        torch.cuda.synchronize()
        assert torch.equal(Ye, eager2), rep
    del g


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_backward_graph_replay_bitwise(dtype):
    math = "f64" if dtype == torch.float64 else "f32"
    I, J = (64, 128, 128), (16, 24, 32)
    X, (A, B, C) = _inputs(I, J, math, dtype, seed=43)
    G = torch.from_numpy(np.random.default_rng(44).standard_normal(J)).to(DEV).to(dtype)
    eager = [t.clone() for t in chain_backward(G, X, A, B, C, math=math)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            chain_backward(G, X, A, B, C, math=math)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = chain_backward(G, X, A, B, C, math=math)
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for k, (o, e) in enumerate(zip(outs, eager)):
            assert torch.equal(o, e), (rep, "dX dA dB dC".split()[k])
        chain(X, A, B, C, math=math)     # eager work between replays
        torch.cuda.synchronize()
    del g
