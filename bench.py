"""Benchmark of the bandlimited NFFT-like transform (Algorithm 4.2) on one MI355X.

One step = steps 1-3 of Algorithm 4.2 (deconvolution + zero-padding, oversampled iFFT,
regularized Shannon short sums) for one batch of synthetic input already resident in
HBM, with the nodes bound (binned) beforehand; binning time is reported as plan time.

Default workload: d=2, M=512, L=1024, m=5, N=1e6 uniform nodes, fhat complex normal
scaled by 1/(1+|k|^2), FP32 with compensated short sums ("f32c").  The FP64 path is
timed beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node evals/sec at rel err 1e-6 (FP32c) vs 1e-12 (FP64); % HBM roofline"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="d2_M512_L1024_m5_N1M")
    ap.add_argument("--precision", default="f32c", choices=["f32c", "f32", "f64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-nodes", type=int, default=100_000,
                    help="nodes of the oracle's step-3 sample for the CPU baseline")
    return ap.parse_args()


def gather_flops_per_node(d: int, m: int) -> int:
    """Algorithmic flops of one node's short sum: (2m)^d terms, each a real weight times
    a complex sample accumulated (2 FMA = 4 flops).  Weight evaluation is not counted."""
    return 4 * (2 * m) ** d


def algorithmic_bytes(p, csize: int, rsize: int) -> dict:
    """Bytes one step must move at least: read fhat, write + read the L^d grid of samples
    (every FFT pass reads and writes its pruned lines once), read nodes, write f."""
    d, M, L, N = p.d, p.M, p.L, p.N
    fft = 0
    for axis in range(d - 1, -1, -1):
        lines_in = M ** (axis + 1) * L ** (d - 1 - axis)
        lines_out = M ** axis * L ** (d - axis)
        fft += (lines_in + lines_out) * csize
    gather = L ** d * csize + N * d * rsize + N * csize + N * 4  # grid, nodes, f, perm
    return {"fft": fft, "gather": gather, "total": fft + gather}


def time_calls(torch, fn, steps: int, warmup: int, stream) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def run_gpu(name: str, prec: str, steps: int, warmup: int):
    import numpy as np
    import torch

    import workloads as W
    from paper_2502_07155_amd import Plan

    p = W.make_problem(name, precision="f32" if prec != "f64" else "f64")
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    x = torch.from_numpy(p.x).to(rdt).cuda()
    fhat = torch.from_numpy(p.fhat).to(cdt).cuda()
    plan = Plan(p.d, p.M, p.L, p.m, precision=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.set_nodes(x)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    out = torch.empty(p.N, dtype=cdt, device="cuda")
    stream = plan.stream
    ms = time_calls(torch, lambda: plan.forward(fhat, out=out), steps, warmup, stream)
    theta = plan.theta()
    gout = torch.empty_like(out)
    gms = time_calls(torch, lambda: plan.interpolate(theta, out=gout), steps, warmup, stream)
    f = out.cpu().numpy().astype(np.complex128)
    return p, plan, f, ms, gms, plan_ms


def accuracy(p, f, sample: int = 20000):
    import numpy as np

    import oracle as O
    import workloads as W
    beta = O.default_beta(p.M, p.L, p.m)
    theta = O.inverse_fft_step(O.deconvolve_pad(p.fhat, p.L, p.m, beta))
    idx = np.sort(W.rng_for(17).choice(p.N, size=min(sample, p.N), replace=False))
    ref = O.gather_shannon(theta, p.x[idx], p.L, p.m, beta)
    return O.rel_err_inf(f[idx], ref), O.rel_err_l2(f[idx], ref)


def cpu_baseline(name: str, nodes: int):
    """The oracle as it stands (numpy FP64), steps 1-3: full grid steps 1-2 plus step 3 on
    a seeded node sample, the step-3 time scaled to the full node count."""
    import numpy as np

    import oracle as O
    import workloads as W
    p = W.make_problem(name, precision="f32")
    n = min(nodes, p.N)
    beta = O.default_beta(p.M, p.L, p.m)
    t0 = time.perf_counter()
    theta = O.inverse_fft_step(O.deconvolve_pad(p.fhat, p.L, p.m, beta))
    t1 = time.perf_counter()
    O.gather_shannon(theta, p.x[:n], p.L, p.m, beta)
    t2 = time.perf_counter()
    t_full = (t1 - t0) + (t2 - t1) * (p.N / n)
    return {"value": p.N / t_full, "unit": "node evals/s", "cores": 1, "kind": "oracle",
            "sample": f"numpy FP64 oracle: steps 1-2 on the full {p.L}^{p.d} grid "
                      f"({t1 - t0:.2f} s) + step 3 on {n} of {p.N} nodes ({t2 - t1:.2f} s), "
                      f"step-3 time scaled by {p.N / n:.1f}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import workloads as W

    prec = args.precision
    p, plan, f, ms, gms, plan_ms = run_gpu(args.workload, prec, args.steps, args.warmup)
    err_inf, err_l2 = accuracy(p, f)
    csize, rsize = (16, 8) if prec == "f64" else (8, 4)
    ab = algorithmic_bytes(p, csize, rsize)
    flops = gather_flops_per_node(p.d, p.m) * p.N
    peak = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    gather_tflops = flops / (gms * 1e-3) / 1e12
    fft_ms = max(ms - gms, 1e-9)
    rec = {
        "metric": METRIC,
        "value": p.N / (ms * 1e-3),
        "unit": "node evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "d": p.d, "M": p.M, "L": p.L, "m": p.m,
                   "N": p.N, "precision": prec, "method": "shannon (Algorithm 4.2)",
                   "parallelism": "single GPU"},
        "rel_err_inf": err_inf,
        "rel_err_l2": err_l2,
        "plan_ms": plan_ms,
        "stage_ms": {"deconv_fft": fft_ms, "gather": gms},
        "roofline": {"bound": "alu", "kernel": "k_gather (step 3 short sums)",
                     "achieved": gather_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": gather_tflops / peak, "traffic": None,
                     "per_node_flops": gather_flops_per_node(p.d, p.m)},
        "hbm": {"algorithmic_bytes": ab, "deconv_fft_GBs": ab["fft"] / (fft_ms * 1e-3) / 1e9,
                "gather_GBs": ab["gather"] / (gms * 1e-3) / 1e9, "peak_GBs": HBM_PEAK_GBS},
    }
    if not args.no_fp64 and prec != "f64":
        p64, _, f64, ms64, gms64, _ = run_gpu(args.workload, "f64", max(5, args.steps // 2), 2)
        e64, _ = accuracy(p64, f64)
        rec["f64"] = {"value": p64.N / (ms64 * 1e-3), "ms_per_step": ms64, "gather_ms": gms64,
                      "rel_err_inf": e64}
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_nodes)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
