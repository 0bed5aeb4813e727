"""Throughput of the TTM chain on one MI355X, printed as one JSON line.

Default workload (the precision form of the chain):
  X 1024 x 1024 x 1024 stored bfloat16 (seeded N(0,1) float32, rounded to
  nearest even), factors A, B, C 128 x 1024 float32 with orthonormal rows,
  Y = X x1 A x2 B x3 C computed with split-precision bf16x3 matrix-core
  products.  The same inputs are also run in plain float32 and plain bfloat16;
  the line reports each form's time, its relative Frobenius error against the
  FP64 oracle (run on the whole step, which is also the CPU baseline), and
  the bf16x3 / float32 speedup.

A step is one full chain (factor preparation, the fused mode-3/mode-2 slab
kernel, the mode-1 kernel) on inputs already resident in HBM.  `value` is the
useful GFLOP/s, 2 (J I^3 + J^2 I^2 + J^3 I) per chain; split-precision extra
products are not counted.  `roofline` is for the dominant kernel (the slab
kernel), timed with HIP events recorded by the library on the launch stream
in a second pass after the timed steps.  Step times are medians over the
timed steps (one HIP event after each step on the stream).

Other workloads: --workload c2 (X 512^3 float32, J = 64, float32),
c4 (20000 ragged cuboids), c5 (X 256^3 float32, J = 32, forward + adjoint),
c6 (compact sixth-order derivative sweeps along each mode of a 512^3
float64 field), reorder (moves of a 512^3 float64 field between
directional layouts), hosvd (the FP64 HOSVD factors of a 128^3 tensor).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
MFMA_BF16_TFLOPS = 2516.6      # dense bf16 matrix cores
F32_TFLOPS = 157.3             # fp32 (matrix and vector)
PROFILES = os.path.join(ROOT, "profiles")


def chain_flops(I, J):
    return 2.0 * (J * I ** 3 + J * J * I * I + J ** 3 * I)


# the sources the chain kernels (the slab kernel among them) are built from,
# and those of the batched kernel
CHAIN_SOURCES = ("ttm_chain.hip", "ttm_device.hpp", "ttm_host.hpp")
BATCHED_SOURCES = ("ttm_batched.hip", "ttm_device.hpp", "ttm_host.hpp")


def kernel_src_sha(sources=CHAIN_SOURCES):
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_13532_amd", "csrc")
    for name in sources:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(tag, per_launch_units=1.0, sources=CHAIN_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernels changed since it was taken."""
    path = os.path.join(PROFILES, f"{tag}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_src_sha") != kernel_src_sha(sources):
        return None
    return float(t["bytes_per_launch"]) * per_launch_units


def timed(fn, steps, warmup, torch):
    """`warmup` untimed calls, then `steps` timed ones with a HIP event on the
    current stream after each call (no synchronisation inside the loop).
    Returns the median, mean and minimum ms per call and the wall seconds."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return {"median": float(np.median(per)), "mean": float(per.mean()), "min": float(per.min()), "wall": wall}


def kernel_times(fn, steps, torch, ttm):
    """Second pass, separate from the timed steps: the library's per-launch
    HIP events (recorded on each kernel's own launch stream) over `steps`
    calls.  Returns {kernel: (launches per call, average ms per launch)}."""
    torch.cuda.synchronize()
    ttm.timing_enable(True)
    ttm.timing_collect()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t = ttm.timing_collect()
    ttm.timing_enable(False)
    return {k: (v[0] / steps, v[1] / v[0]) for k, v in t.items()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def rel_err(y, ref):
    return float(np.linalg.norm((y - ref).ravel()) / np.linalg.norm(ref.ravel()))


def bench_dense_precision(args, torch, ttm):
    from paper_2411_13532_amd import workloads
    I, J = 1024, 128
    t_gen = time.perf_counter()
    p = workloads.dense("c3_bf16_1024_128")
    print(f"# inputs generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    dev = "cuda:0"
    X = p["X"].to(dev)
    fs = [torch.from_numpy(p[k]).to(dev) for k in "ABC"]
    flops = chain_flops(I, J)
    forms = {}
    Ys = {}
    kt = {}
    plan = [f for f in ("bf16x3", "f32", "bf16") if f in args.forms.split(",")]
    for math in plan:
        wsm = torch.empty(ttm.chain_workspace_size((I,) * 3, (J,) * 3, torch.bfloat16, math), dtype=torch.uint8,
                          device=dev)
        Y = torch.empty((J, J, J), dtype=torch.float32, device=dev)
        fn = lambda: ttm.chain(X, *fs, math=math, out=Y, workspace=wsm)
        t = timed(fn, args.steps, args.warmup, torch)
        kt[math] = kernel_times(fn, args.steps, torch, ttm)
        forms[math] = {"ms_per_step": t["median"], "ms_mean": t["mean"], "ms_min": t["min"],
                       "gflops": flops / (t["median"] * 1e-3) / 1e9, "steps": args.steps,
                       "kernel_ms": {k: round(v[1], 4) for k, v in kt[math].items()}}
        Ys[math] = Y.clone()
        print(f"# {math}: {t['median']:.3f} ms/step (median), kernels {forms[math]['kernel_ms']}",
              file=sys.stderr, flush=True)
    # the oracle on the whole step (every output, X read as float32 and
    # widened element by element, float64 arithmetic): the CPU baseline and
    # the accuracy of every form
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        X_np = p["X"].float().numpy()
        A64, B64, C64 = (p[k].astype(np.float64) for k in "ABC")
        t0 = time.perf_counter()
        ref = oracle.chain(X_np, A64, B64, C64, order=(3, 2, 1))
        dt = time.perf_counter() - t0
        cpu = {"value": round(flops / dt / 1e9, 2), "unit": "GFLOP/s", "cores": oracle.num_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"the whole 1024^3 -> 128^3 step (all of Y, mode-3 product first), "
                         f"{flops / 1e9:.1f} GFLOP in {dt:.1f} s"}
        for math, Y in Ys.items():
            forms[math]["rel_err_vs_oracle"] = rel_err(Y.double().cpu().numpy(), ref)
        del X_np
    # dominant kernel: the slab kernel (modes 3 and 2).  Algorithmic bytes of
    # the step: X (bf16) read once, Y (float) written once, the three stored
    # float factors read once; the slab kernel is the one that moves them
    # (the V partial it writes and the mode-1 kernel reads is the
    # implementation's own intermediate and shows up under `traffic`).
    # MFMA flops issued in bf16x3: two products for mode 3 (X is exact
    # bf16), three for modes 2 and 1.
    ms = forms["bf16x3"]["ms_per_step"]
    slab_ms = kt["bf16x3"]["ttm_slab"][1]
    alg_bytes = I ** 3 * 2 + J ** 3 * 4 + 3 * J * I * 4
    mfma = 2 * (2.0 * J * I ** 3) + 3 * (2.0 * J * J * I * I) + 3 * (2.0 * J ** 3 * I)
    t_hbm = alg_bytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = mfma / (MFMA_BF16_TFLOPS * 1e12)
    gbs = alg_bytes / (slab_ms * 1e-3) / 1e9
    if t_hbm >= t_mfma:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        tf = mfma / (slab_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(tf, 1), "peak": MFMA_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / MFMA_BF16_TFLOPS, 4)}
    roof["traffic"] = measured_traffic("ttm_slab_c3_bf16x3")
    roof["kernel"] = "ttm_slab (k_slab_lc<bf16x3>)"
    roof["kernel_ms"] = round(slab_ms, 4)
    roof["algorithmic_bytes"] = alg_bytes
    roof["mfma_flops"] = mfma
    roof["mfma_frac"] = round(mfma / (slab_ms * 1e-3) / 1e12 / MFMA_BF16_TFLOPS, 4)
    roof["step_frac"] = round(max(t_hbm, t_mfma) / (ms * 1e-3), 4)
    roof["copy_ceiling_gbs"] = round(copy_gbs(torch, ttm, 1 << 30, 10), 1)
    speedup = (round(forms["f32"]["ms_per_step"] / forms["bf16x3"]["ms_per_step"], 3)
               if "f32" in forms and "bf16x3" in forms else None)
    line = {
        "metric": "TTM-chain GFLOP/s + % roofline; bf16x3 vs FP32 speedup at rel err<=1e-5",
        "value": round(flops / (ms * 1e-3) / 1e9, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3", "data": "synthetic",
        "config": {"workload": "X 1024^3 bfloat16 N(0,1) seed 2; A,B,C 128x1024 float32 orthonormal rows; "
                               "Y = X x1 A x2 B x3 C, split-precision bf16x3",
                   "I": I, "J": J, "x_dtype": "bf16", "math": "bf16x3", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in forms.items()},
        "bf16x3_vs_f32_speedup": speedup,
    }
    return line


def copy_gbs(torch, ttm, nbytes, reps):
    """Practical HBM ceiling: read + write bytes per second of the library's copy kernel."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    t = timed(lambda: ttm.stream_copy(dst, src), reps, 2, torch)
    return 2 * nbytes / (t["median"] * 1e-3) / 1e9


def bench_copy(args, torch, ttm):
    nbytes = 1 << 30
    gbs = copy_gbs(torch, ttm, nbytes, args.steps)
    return {"metric": "device copy GB/s (read + write)", "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 2, "ms_per_step": round(2 * nbytes / gbs / 1e6, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "copy of 1 GiB (ttm_stream_copy)", "bytes": nbytes},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}}


def bench_c2(args, torch, ttm):
    from paper_2411_13532_amd import workloads
    I, J = 512, 64
    p = workloads.dense("c2_f32_512_64")
    dev = "cuda:0"
    X = torch.from_numpy(p["X"]).to(dev)
    fs = [torch.from_numpy(p[k]).to(dev) for k in "ABC"]
    res = {}
    for math in ("f32", "bf16x3"):
        ws = torch.empty(ttm.chain_workspace_size((I,) * 3, (J,) * 3, torch.float32, math), dtype=torch.uint8, device=dev)
        Y = torch.empty((J, J, J), dtype=torch.float32, device=dev)
        fn = lambda: ttm.chain(X, *fs, math=math, out=Y, workspace=ws)
        ms = timed(fn, args.steps, args.warmup, torch)["median"]
        kt = {k: round(v[1], 4) for k, v in kernel_times(fn, args.steps, torch, ttm).items()}
        res[math] = {"ms_per_step": ms, "gflops": chain_flops(I, J) / (ms * 1e-3) / 1e9, "kernel_ms": kt}
    ms = res["f32"]["ms_per_step"]
    slab = res["f32"]["kernel_ms"]["ttm_slab"]
    slab_flops = 2.0 * J * I ** 3 + 2.0 * J * J * I * I
    tf = slab_flops / (slab * 1e-3) / 1e12
    return {"metric": "TTM-chain GFLOP/s + % roofline", "value": round(chain_flops(I, J) / (ms * 1e-3) / 1e9, 1),
            "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "X 512^3 float32 N(0,1) seed 1; A,B,C 64x512 orthonormal rows; float32",
                       "I": I, "J": J},
            "roofline": {"bound": "mfma", "achieved": round(tf, 1), "peak": F32_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / F32_TFLOPS, 4), "traffic": None, "kernel": "ttm_slab", "kernel_ms": slab},
            "forms": res}


def c4_traffic(variant):
    """The batched kernel's measured HBM bytes per launch, when the launch
    runs the variant the counters were taken on."""
    path = os.path.join(PROFILES, "ttm_batched_c4_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        if json.load(f).get("variant") != variant:
            return None
    return measured_traffic("ttm_batched_c4", sources=BATCHED_SOURCES)


def bench_c4(args, torch, ttm):
    from paper_2411_13532_amd import BatchedPlan, workloads
    p = workloads.batched()
    dev = "cuda:0"
    bufs = [torch.from_numpy(p[k]).to(dev) for k in "XABC"]
    plan = BatchedPlan(p["dims"], dtype=torch.float32)
    Y = plan.empty_output()
    flops = float(np.sum(6.0 * p["dims"][:, 0].astype(np.float64) ** 4))
    nbytes = 4.0 * sum(b.numel() for b in bufs) + 4.0 * Y.numel()
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    if args.c4_config:
        # a pinned launch shape (for counter runs of one kernel shape)
        threads, bpc, variant = (int(v) for v in args.c4_config.split(","))
        plan.set_config(threads, bpc, variant)
        best = None
    else:
        best = plan.autotune(*bufs, Y=Y, reps=5)

    def cold(mode):
        flush.fill_(1)   # evict the 256 MB last-level cache between steps
        plan.run(*bufs, Y=Y, mode=mode)

    res = {}
    for mode in ("persistent", "graph"):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        per = []
        for _ in range(args.warmup):
            cold(mode)
        for _ in range(args.steps):
            flush.fill_(1)
            e0.record()
            plan.run(*bufs, Y=Y, mode=mode)
            e1.record()
            torch.cuda.synchronize()
            per.append(e0.elapsed_time(e1))
        res[mode] = float(np.median(per))
    ms_loop = timed(lambda: plan.run(*bufs, Y=Y, mode="loop"), 2, 1, torch)["median"]
    ms = res["graph"]
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"metric": "batched TTM-chain GFLOP/s + % roofline", "value": round(flops / (ms * 1e-3) / 1e9, 1),
            "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "20000 cuboids n^3, n ~ U{5..13} seed 3, square factors N(0,1/n); float32",
                       "count": 20000, "config": plan.config(), "autotune_best_ms": best},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": c4_traffic(plan.config()["variant"]),
                         "kernel": "ttm_batched"},
            "persistent_ms": round(res["persistent"], 5), "graph_ms": round(res["graph"], 5),
            "per_cuboid_loop_ms": round(ms_loop, 3), "loop_over_graph": round(ms_loop / ms, 1)}


def bench_c5(args, torch, ttm):
    from paper_2411_13532_amd import workloads
    I, J = 256, 32
    p = workloads.dense("c5_f32_256_32")
    dev = "cuda:0"
    X, A, B, C, T = (torch.from_numpy(p[k]).to(dev) for k in "XABCT")
    Y = torch.empty((J, J, J), dtype=torch.float32, device=dev)
    fwd = lambda: ttm.chain(X, A, B, C, math="f32", out=Y)
    ms_f = timed(fwd, args.steps, args.warmup, torch)["median"]
    G = Y - T
    bwd = lambda: ttm.chain_backward(G, X, A, B, C, math="f32")
    # the step time without per-kernel events (their host cost would show in
    # short launches), then the kernel breakdown
    ms_b = timed(bwd, args.steps, args.warmup, torch)["median"]
    kt_b = {k: n * v for k, (n, v) in kernel_times(bwd, args.steps, torch, ttm).items()}
    fl_f = chain_flops(I, J)
    # dominant kernel of the step: the adjoint's X pass, which does the whole
    # backward but the fixed-order sums of the dB and dC shares.  Algorithmic
    # work of the backward: dX = G x1 A^T x2 B^T x3 C^T (the chain with J and
    # I swapped), Z = X x2 B x3 C for dA, the dB path, and the three small
    # GEMMs of dA, dB, dC; bytes: X read, dX written, G and the factors read,
    # dA, dB, dC written
    bwd_flops = chain_flops(I, J) + 2.0 * (J * I ** 3 + J * J * I * I) + 2.0 * J * J * I * I + 3 * 2.0 * J ** 3 * I
    bwd_bytes = 2 * I ** 3 * 4 + J ** 3 * 4 + 2 * 3 * J * I * 4
    roof = None
    if "ttm_bwd_xpass" in kt_b:
        xms = kt_b["ttm_bwd_xpass"]
        gbs = bwd_bytes / (xms * 1e-3) / 1e9
        tf = bwd_flops / (xms * 1e-3) / 1e12
        if bwd_bytes / (HBM_PEAK_GBS * 1e9) >= bwd_flops / (F32_TFLOPS * 1e12):
            roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4)}
        else:
            roof = {"bound": "mfma", "achieved": round(tf, 2), "peak": F32_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / F32_TFLOPS, 4)}
        roof.update({"traffic": None, "kernel": "ttm_bwd_xpass (k_bwd_xpass_f32)", "kernel_ms": round(xms, 4),
                     "algorithmic_bytes": bwd_bytes, "flops": bwd_flops,
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "mfma_frac": round(tf / F32_TFLOPS, 4)})
    return {"metric": "TTM-chain forward+adjoint GFLOP/s", "value": round(fl_f / ((ms_f) * 1e-3) / 1e9, 1),
            "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_f + ms_b, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "X 256^3 float32, factors 32x256 N(0,1/256), L = 1/2||Y - T||^2", "I": I, "J": J},
            "roofline": roof,
            "forward_ms": round(ms_f, 4), "backward_ms": round(ms_b, 4),
            "backward_kernels_ms": {k: round(v, 4) for k, v in kt_b.items()}}


def bench_c6(args, torch, ttm):
    """The compact scheme of Sec. 4.2 Eq. (cfds) along each mode of a 512^3
    float64 field (the paper's benchmarks are double precision, 512 points per
    system in its bandwidth table)."""
    I = 512
    dev = "cuda:0"
    g = torch.Generator(device=dev)
    g.manual_seed(6)
    X = torch.randn((I, I, I), dtype=torch.float64, device=dev, generator=g)
    Y = torch.empty_like(X)
    ws = torch.empty(4096 * 8, dtype=torch.uint8, device=dev)
    nbytes = 2.0 * X.numel() * 8           # algorithmic: read X once, write Y once
    per_mode = {}
    for mode in (1, 2, 3):
        # the coefficients are prepared once per operator (as the paper's
        # preprocessing step), outside the timed sweeps
        ttm.compact_apply(X, mode, out=Y, workspace=ws)
        fn = lambda: ttm.compact_apply(X, mode, out=Y, workspace=ws, prepared=True)
        ms = timed(fn, args.steps, args.warmup, torch)["median"]
        kms = kernel_times(fn, args.steps, torch, ttm)["ttm_compact"][1]
        per_mode[mode] = {"ms": round(ms, 4), "kernel_ms": round(kms, 4),
                          "gbs": round(nbytes / (kms * 1e-3) / 1e9, 1)}
    ms = sum(v["ms"] for v in per_mode.values())
    kms = max(per_mode.values(), key=lambda v: v["kernel_ms"])
    worst = [m for m, v in per_mode.items() if v is kms][0]
    gbs = nbytes / (kms["kernel_ms"] * 1e-3) / 1e9
    points = 3.0 * X.numel()
    return {"metric": "compact-scheme sweep Gpoints/s (three directions)", "value": round(points / (ms * 1e-3) / 1e9, 2),
            "unit": "Gpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "X 512^3 float64 N(0,1); Eq. (cfds) periodic, alpha 1/3, a 14/9, b 1/9, "
                                   "h 2 pi / 512, applied along mode 1, 2 and 3", "I": I},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": f"ttm_compact (mode {worst}, the slowest)", "kernel_ms": kms["kernel_ms"]},
            "per_mode": per_mode}


def bench_reorder(args, torch, ttm):
    """Moves of a 512^3 float64 field between directional layouts (Sec. 4.1)
    and the accumulating form; algorithmic bytes: read X and write Y once
    (accumulate: also read Y)."""
    I = 512
    dev = "cuda:0"
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    X = torch.randn((I, I, I), dtype=torch.float64, device=dev, generator=g)
    Y = torch.empty_like(X)
    nb = X.numel() * 8
    res = {}
    for name, perm, acc in (("xy_swap_inner", (0, 2, 1), False), ("xz_swap", (2, 1, 0), False),
                            ("outer_swap", (1, 0, 2), False), ("cycle", (1, 2, 0), False),
                            ("xz_swap_accumulate", (2, 1, 0), True)):
        fn = lambda: ttm.reorder(X, perm, out=Y, accumulate=acc)
        ms = timed(fn, args.steps, args.warmup, torch)["median"]
        kms = kernel_times(fn, args.steps, torch, ttm)["ttm_reorder"][1]
        bytes_ = (3 if acc else 2) * nb
        res[name] = {"perm": perm, "accumulate": acc, "ms": round(ms, 4), "kernel_ms": round(kms, 4),
                     "gbs": round(bytes_ / (kms * 1e-3) / 1e9, 1)}
    worst = min(res.values(), key=lambda v: v["gbs"])
    copy = copy_gbs(torch, ttm, 1 << 30, 10)
    main = res["xz_swap"]
    return {"metric": "layout reorder GB/s (read + write)", "value": main["gbs"], "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": main["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "X 512^3 float64 N(0,1); Y = X with axes 0 and 2 exchanged (perm (2, 1, 0))",
                       "I": I},
            "roofline": {"bound": "hbm", "achieved": main["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(main["gbs"] / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "ttm_reorder",
                         "kernel_ms": main["kernel_ms"], "copy_ceiling_gbs": round(copy, 1),
                         "slowest_perm_gbs": worst["gbs"]},
            "per_perm": res}


def bench_hosvd(args, torch, ttm):
    """Truncated HOSVD factors of X 128^3 float64 (ranks 16): three Gram
    matrices on the FP64 matrix cores and three Jacobi eigensolves."""
    I, J = 128, 16
    dev = "cuda:0"
    g = torch.Generator(device=dev)
    g.manual_seed(8)
    X = torch.randn((I, I, I), dtype=torch.float64, device=dev, generator=g)
    fn = lambda: ttm.hosvd(X, (J, J, J))
    ms = timed(fn, args.steps, args.warmup, torch)["median"]
    kt = kernel_times(fn, args.steps, torch, ttm)
    gram_ms = kt["ttm_gram"][0] * kt["ttm_gram"][1] + (kt["ttm_gram_sum"][0] * kt["ttm_gram_sum"][1]
                                                       if "ttm_gram_sum" in kt else 0.0)
    gram_flops = 3 * 2.0 * I * I * I ** 3 / I
    tf = gram_flops / (gram_ms * 1e-3) / 1e12
    return {"metric": "HOSVD factors ms (3 modes)", "value": round(ms, 4), "unit": "ms", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "X 128^3 float64 N(0,1); ranks (16, 16, 16)", "I": I, "J": J},
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 78.6, "unit": "TFLOP/s",
                         "frac": round(tf / 78.6, 4), "traffic": None, "kernel": "ttm_gram (FP64 Gram matrices)",
                         "kernel_ms": round(gram_ms, 4)},
            # the step's time is the eigensolve: three workgroups (one per
            # mode) of rotation rounds, each round a few LDS passes over the
            # Gram matrix between barriers -- latency-bound, with no roofline
            # of the chip's units to quote
            "dominant_kernel": "ttm_sym_jacobi",
            "kernels_ms": {k: round(v[0] * v[1], 4) for k, v in kt.items()}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c4", "c5", "c6", "copy", "reorder", "hosvd"])
    ap.add_argument("--forms", default="bf16x3,f32,bf16",
                    help="c3: arithmetic forms to run (bf16x3 is the headline and must be included)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c4-config", default="",
                    help="c4: threads,blocks_per_cu,variant of the batched launch instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2411_13532_amd as ttm
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.init()
    fn = {"c3": bench_dense_precision, "c2": bench_c2, "c4": bench_c4, "c5": bench_c5, "c6": bench_c6, "copy": bench_copy,
          "reorder": bench_reorder, "hosvd": bench_hosvd}[args.workload]
    line = fn(args, torch, ttm)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
