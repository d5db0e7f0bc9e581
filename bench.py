"""Benchmark of the bandlimited NFFT-like transform (Algorithm 4.2) on one MI355X.

One step = steps 1-3 of Algorithm 4.2 (deconvolution + zero-padding, oversampled iFFT,
regularized Shannon short sums) for one batch of synthetic input already resident in
HBM, with the nodes bound (binned) beforehand; binning time is reported as plan time.

Headline workload: d=2, M=512, L=1024, m=5, N=1e6 uniform nodes, fhat complex normal
scaled by 1/(1+|k|^2), FP32 with compensated short sums ("f32c").  Beside it, unless
--headline-only: the same workload in FP64 and with the classical NFFT (Algorithm 2.1),
and the other workloads (d=1 FP64, d=3 clustered nodes, 512 batched d=1 instances, d=2
forward + backward).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node evals/sec at rel err 1e-6 (FP32c) vs 1e-12 (FP64); % HBM roofline"
HBM_PEAK_GBS = 8000.0
# Vector FP32 without packed instructions (the library is built without them) issues like
# FP64: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 78.6
FP64_PEAK_TFLOPS = 78.6
GATHER_SOURCES = ["paper_2502_07155_amd/csrc/gather.hip", "paper_2502_07155_amd/csrc/device_math.h"]
TRAFFIC_FILE = "profiles/k_gather_d2_M512_L1024_m5_N1M_f32c_traffic.txt"
HEADLINE = "d2_M512_L1024_m5_N1M"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--precision", default="f32c", choices=["f32c", "f32", "f64"])
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline workload only (no other legs, no CPU baseline)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-nodes", type=int, default=1_000_000,
                    help="nodes of the oracle's step-3 sample for the CPU baseline")
    ap.add_argument("--leg", choices=["batched", "fwd_bwd", "nfft"],
                    help="run only this leg (batched d=1 instances, d=2 forward + backward, or "
                         "Algorithm 2.1 on the headline workload) and print its JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy five times (for counter scaling)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print a per-kernel summary of a rocprofv3 --kernel-trace --stats "
                         "csv output directory and exit (no GPU use)")
    ap.add_argument("--summarize-traffic", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="print the gather's HBM traffic per launch from four rocprofv3 --pmc "
                         "csv output directories and exit (no GPU use)")
    return ap.parse_args()


def gather_flops_per_node(d: int, m: int) -> int:
    """Algorithmic flops of one node's short sum: (2m)^d terms, each a real weight times
    a complex sample accumulated (2 FMA = 4 flops).  Weight evaluation is not counted."""
    return 4 * (2 * m) ** d


def algorithmic_bytes(d, M, L, N, csize: int, rsize: int) -> dict:
    """Bytes one step must move at least: read fhat, write + read the L^d grid of samples
    (every FFT pass reads and writes its pruned lines once), read nodes, write f."""
    fft = 0
    for axis in range(d - 1, -1, -1):
        lines_in = M ** (axis + 1) * L ** (d - 1 - axis)
        lines_out = M ** axis * L ** (d - axis)
        fft += (lines_in + lines_out) * csize
    gather = L ** d * csize + N * d * rsize + N * csize + N * 4  # grid, nodes, f, perm
    return {"fft": fft, "gather": gather, "total": fft + gather}


def time_calls(torch, fn, steps: int, warmup: int, stream) -> float:
    """Average ms per call between HIP events recorded on `stream` (the stream the
    library launches on)."""
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


def source_digest(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the gather from the committed counter summary, if it was
    taken on the current gather sources; else None."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = re.search(r"^source_sha256:\s*(\w+)", text, re.M)
    val = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not sha or not val or sha.group(1) != source_digest(GATHER_SOURCES):
        return None
    return float(val.group(1))


# ---------------------------------------------------------------- legs
def run_plan(name: str, prec: str, steps: int, warmup: int, method: str = "shannon", beta: float = 0.0):
    import numpy as np
    import torch

    import workloads as W
    from paper_2502_07155_amd import Plan

    p = W.make_problem(name, precision="f32" if prec != "f64" else "f64")
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    x = torch.from_numpy(p.x).to(rdt).cuda()
    fhat = torch.from_numpy(p.fhat).to(cdt).cuda()
    plan = Plan(p.d, p.M, p.L, p.m, precision=prec, method=method, beta=beta)
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


def accuracy(p, f, sample: int = 20000, method: str = "shannon", beta=None):
    """Normwise relative errors against the oracle's fast form on a node sample."""
    import numpy as np

    import oracle as O
    import workloads as W
    idx = np.sort(W.rng_for(17).choice(p.N, size=min(sample, p.N), replace=False))
    if method == "shannon":
        ref = O.forward_shannon(p.fhat, p.x[idx], p.L, p.m, beta)
    else:
        ref = O.forward_nfft(p.fhat, p.x[idx], p.L, p.m, beta)
    return O.rel_err_inf(f[idx], ref), O.rel_err_l2(f[idx], ref), idx


def leg_nfft(steps, warmup, f_shannon, p_shannon):
    """Algorithm 2.1 on the headline workload with the same m, both beta readings; both
    methods' error against the direct sum on truncated-domain sample nodes."""
    import numpy as np

    import oracle as O
    import workloads as W
    out = {}
    idx_all = np.sort(W.rng_for(18).choice(p_shannon.N, 2000, replace=False))
    mask = O.in_truncated_domain(p_shannon.x[idx_all], p_shannon.L, p_shannon.m)
    idx = idx_all[mask]
    direct = O.direct_sum(p_shannon.fhat, p_shannon.x[idx])
    out["shannon_vs_direct_sum"] = O.rel_err_inf(f_shannon[idx], direct)
    for label, beta in (("nfft_beta_standard", 0.0),
                        ("nfft_beta_shannon", O.default_beta(p_shannon.M, p_shannon.L, p_shannon.m))):
        p, plan, f, ms, gms, _ = run_plan(HEADLINE, "f32c", steps, warmup, "nfft", beta)
        err, _, _ = accuracy(p, f, 5000, "nfft", beta if beta > 0 else None)
        out[label] = {"value": p.N / (ms * 1e-3), "ms_per_step": ms, "gather_ms": gms,
                      "beta": plan.stats()["beta"], "rel_err_inf_vs_oracle": err,
                      "rel_err_inf_vs_direct_sum": O.rel_err_inf(f[idx], direct)}
        plan.close()
    out["direct_sum_nodes"] = int(idx.size)
    return out


def leg_plan(name, prec, steps, warmup, sample=5000):
    p, plan, f, ms, gms, plan_ms = run_plan(name, prec, steps, warmup)
    err, _, _ = accuracy(p, f, sample)
    plan.close()
    return {"value": p.N / (ms * 1e-3), "ms_per_step": ms, "gather_ms": gms, "plan_ms": plan_ms,
            "precision": prec, "rel_err_inf": err}


def leg_batched(steps, warmup):
    """512 independent d=1 instances, one graph launch per step, FP32."""
    import numpy as np
    import torch

    import oracle as O
    import workloads as W
    from paper_2502_07155_amd import BatchPlan
    insts = W.batched_instances()
    bp = BatchPlan([i.M for i in insts], [i.L for i in insts], [i.m for i in insts],
                   [i.x.size for i in insts], precision="f32")
    x = torch.from_numpy(np.concatenate([i.x for i in insts]).astype(np.float32)).cuda()
    fhat = torch.from_numpy(np.concatenate([i.fhat for i in insts]).astype(np.complex64)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bp.set_nodes(x)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    out = torch.empty(bp.total_N, dtype=torch.complex64, device="cuda")
    ms = time_calls(torch, lambda: bp.forward(fhat, out), steps, warmup, bp.stream)
    f = out.cpu().numpy().astype(np.complex128)
    rng = W.rng_for(19)
    worst = 0.0
    for i in rng.choice(len(insts), 32, replace=False):
        inst = insts[i]
        idx = rng.choice(inst.x.size, min(32, inst.x.size), replace=False)
        ref = O.forward_shannon(inst.fhat, inst.x[idx, None], inst.L, inst.m)
        got = f[bp.node_offsets[i]:bp.node_offsets[i + 1]][idx]
        worst = max(worst, O.rel_err_inf(got, ref))
    bp.close()
    return {"value": bp.total_N / (ms * 1e-3), "ms_per_step": ms, "plan_ms": plan_ms,
            "instances": len(insts), "total_nodes": bp.total_N, "precision": "f32",
            "rel_err_inf_worst_of_32_sampled_instances": worst}


def leg_differentiation(steps, warmup):
    """d=2, M=256, L=512, m=6, N=2e5: FP32 forward + hand-written backward (grad fhat and
    grad x) of sum |f - y|^2 through torch.autograd."""
    import torch

    import workloads as W
    from paper_2502_07155_amd import Plan, bandlimited_nfft
    p = W.make_problem("d2_M256_L512_m6_N200k", precision="f32", with_targets=True)
    plan = Plan(p.d, p.M, p.L, p.m, precision="f32")
    fhat = torch.from_numpy(p.fhat).to(torch.complex64).cuda().requires_grad_(True)
    x = torch.from_numpy(p.x).to(torch.float32).cuda().requires_grad_(True)
    y = torch.from_numpy(p.y).to(torch.complex64).cuda()

    def step():
        fhat.grad = None
        x.grad = None
        loss = (bandlimited_nfft(fhat, x, plan) - y).abs().pow(2).sum()
        loss.backward()

    ms = time_calls(torch, step, steps, warmup, plan.stream)
    plan.close()
    return {"value": p.N / (ms * 1e-3), "ms_per_step": ms, "precision": "f32",
            "step": "forward + backward (grad fhat, grad x)"}


def cpu_baseline(name: str, nodes: int):
    """The oracle as it stands (numpy FP64), steps 1-3: full grid steps 1-2 plus step 3 on
    a seeded node sample, the step-3 time scaled to the full node count."""
    from threadpoolctl import threadpool_limits

    import oracle as O
    import workloads as W
    p = W.make_problem(name, precision="f32")
    n = min(nodes, p.N)
    beta = O.default_beta(p.M, p.L, p.m)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        theta = O.inverse_fft_step(O.deconvolve_pad(p.fhat, p.L, p.m, beta))
        t1 = time.perf_counter()
        O.gather_shannon(theta, p.x[:n], p.L, p.m, beta)
        t2 = time.perf_counter()
    t_full = (t1 - t0) + (t2 - t1) * (p.N / n)
    return {"value": p.N / t_full, "unit": "node evals/s", "cores": 1, "kind": "oracle",
            "sample": f"numpy FP64 oracle, one thread: steps 1-2 on the full {p.L}^{p.d} grid "
                      f"({t1 - t0:.2f} s) + step 3 on {n} of {p.N} nodes ({t2 - t1:.2f} s), "
                      f"step-3 time scaled by {p.N / n:.1f}"}


def _csv_rows(directory: str, suffix: str):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(path) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def summarize_trace(directory: str) -> str:
    rows = _csv_rows(directory, "kernel_stats.csv")
    lines = [f"{'calls':>6} {'avg_us':>10} {'total_%':>8}  kernel"]
    for r in rows:
        lines.append(f"{int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>10.2f} "
                     f"{float(r['Percentage']):>8.2f}  {r['Name'][:150]}")
    return "\n".join(lines)


def _counter_per_dispatch(directory: str, keep):
    vals = [float(r["Counter_Value"]) for r in _csv_rows(directory, "counter_collection.csv")
            if keep(r["Kernel_Name"])]
    return (sum(vals) / len(vals), len(vals)) if vals else (float("nan"), 0)


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir) -> str:
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the gather, each divided by the
    counter-to-bytes factor of a 1 GiB device copy (which reads and writes 1 GiB)."""
    def gather(name):
        return "k_gather<" in name

    def copy(name):
        return True   # the calibration run launches nothing but the copies

    fetch, nf = _counter_per_dispatch(fetch_dir, gather)
    write, nw = _counter_per_dispatch(write_dir, gather)
    cf, ncf = _counter_per_dispatch(copy_fetch_dir, copy)
    cw, ncw = _counter_per_dispatch(copy_write_dir, copy)
    gib_kib = float(1 << 20)
    ff, fw = cf / gib_kib, cw / gib_kib
    traffic = (fetch / ff + write / fw) * 1024.0
    return "\n".join([
        f"gather_fetch_kib_per_dispatch: {fetch:.1f}  (dispatches: {nf})",
        f"gather_write_kib_per_dispatch: {write:.1f}  (dispatches: {nw})",
        f"copy_fetch_kib_per_GiB_copy: {cf:.1f}  (dispatches: {ncf}); factor {ff:.4f}",
        f"copy_write_kib_per_GiB_copy: {cw:.1f}  (dispatches: {ncw}); factor {fw:.4f}",
        f"traffic_bytes_per_launch: {traffic:.6e}",
        f"source_sha256: {source_digest(GATHER_SOURCES)}",
    ])


def copy_calibration():
    """A plain device copy of 1 GiB, five times: the reference for scaling the FETCH_SIZE
    and WRITE_SIZE counters (each copy reads and writes exactly 1 GiB).  The source is left
    uninitialized so that the copies are the only kernels of the run."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 5}))


def main():
    args = parse()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_traffic:
        print(summarize_traffic(*args.summarize_traffic))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "bench.py needs a GPU"}))
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.leg == "batched":
        print(json.dumps(leg_batched(args.steps, args.warmup)))
        return
    if args.leg == "fwd_bwd":
        print(json.dumps(leg_differentiation(args.steps, args.warmup)))
        return
    if args.leg == "nfft":
        p, plan, f, _, _, _ = run_plan(HEADLINE, "f32c", 2, 1)
        plan.close()
        print(json.dumps(leg_nfft(args.steps, args.warmup, f, p)))
        return

    prec = args.precision
    p, plan, f, ms, gms, plan_ms = run_plan(args.workload, prec, args.steps, args.warmup)
    err_inf, err_l2, _ = accuracy(p, f)
    csize, rsize = (16, 8) if prec == "f64" else (8, 4)
    ab = algorithmic_bytes(p.d, p.M, p.L, p.N, csize, rsize)
    flops = gather_flops_per_node(p.d, p.m) * p.N
    peak = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    gather_tflops = flops / (gms * 1e-3) / 1e12
    fft_ms = max(ms - gms, 1e-9)
    traffic = measured_traffic() if (args.workload == HEADLINE and prec == "f32c") else None
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
                     "frac": gather_tflops / peak, "traffic": traffic,
                     "algorithmic_flops_per_launch": flops,
                     "per_node_flops": gather_flops_per_node(p.d, p.m)},
        "hbm": {"algorithmic_bytes": ab, "deconv_fft_GBs": ab["fft"] / (fft_ms * 1e-3) / 1e9,
                "gather_GBs": ab["gather"] / (gms * 1e-3) / 1e9, "peak_GBs": HBM_PEAK_GBS},
    }
    plan.close()
    if not args.headline_only and args.workload == HEADLINE and prec != "f64":
        legs = {}
        short = max(5, args.steps // 5)
        legs["d2_M512_L1024_m5_N1M_f64"] = leg_plan(HEADLINE, "f64", short, 2)
        legs["d2_M512_L1024_m5_N1M_nfft"] = leg_nfft(short, 2, f, p)
        legs["d1_M256_L512_m6_N1k_f64"] = leg_plan("d1_M256_L512_m6_N1k", "f64", short, 2, 1000)
        legs["d3_M128_L256_m4_N2M_f32c"] = leg_plan("d3_M128_L256_m4_N2M", "f32c", short, 2, 3000)
        legs["d3_M128_L256_m4_N2M_f64"] = leg_plan("d3_M128_L256_m4_N2M", "f64", short, 2, 3000)
        legs["batched_512_d1_f32"] = leg_batched(short, 2)
        legs["d2_M256_L512_m6_N200k_fwd_bwd_f32"] = leg_differentiation(short, 2)
        rec["legs"] = legs
    if not args.no_cpu and not args.headline_only:
        rec["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_nodes)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
