"""Benchmark of the bandlimited NFFT-like transform (Algorithm 4.2) on one MI355X.

One step = steps 1-3 of Algorithm 4.2 (deconvolution + zero-padding, oversampled iFFT,
regularized Shannon short sums) for one batch of synthetic input already resident in
HBM, with the nodes bound (binned) beforehand; binning time is reported as plan time.

Headline workload: d=2, M=512, L=1024, m=5, N=1e6 uniform nodes, fhat complex normal
scaled by 1/(1+|k|^2), FP32 with compensated short sums ("f32c").  Beside it, unless
--headline-only: the same workload in FP64 and with the classical NFFT (Algorithm 2.1),
and the other workloads (d=1 FP64, d=3 clustered nodes, 512 batched d=1 instances, d=2
forward + backward, the Example 5.1 sweep).  Prints one JSON line.

The GPU legs keep seeded samples of their outputs; the oracle leg at the end (the only
part of this file that calls the oracle) times the oracle for cpu_baseline and fills in
each leg's error against it.  --headline-only and --no-cpu skip it.
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
# FP64: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s.  The
# published vector FP32 figure, 157.3 TFLOP/s, counts packed (two-wide) FP32 FMAs.
FP32_PEAK_TFLOPS = 78.6
FP64_PEAK_TFLOPS = 78.6
FP32_PUBLISHED_TFLOPS = 157.3
PEAK_BASIS = ("alu peak from unit counts and clock: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) "
              "x 2.4 GHz = 78.6 TFLOP/s, the non-packed FP32 (and FP64) vector rate; packed FP32 "
              "instructions are disabled in this build, so the published 157.3 TFLOP/s (packed "
              "FP32) is out of reach by construction; frac_vs_published divides by it")
GATHER_SOURCES = ["paper_2502_07155_amd/csrc/gather.hip", "paper_2502_07155_amd/csrc/device_math.h"]
TRAFFIC_FILE = "profiles/k_gather_d2_M512_L1024_m5_N1M_f32c_traffic.txt"
HEADLINE = "d2_M512_L1024_m5_N1M"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--precision", default="f32c", choices=["f32c", "f32d", "f32", "f64"])
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline workload only (no other legs, no CPU baseline)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (CPU baseline and the error checks against the oracle)")
    ap.add_argument("--cpu-nodes", type=int, default=1_000_000,
                    help="nodes of the oracle's step-3 sample for the CPU baseline")
    ap.add_argument("--leg", choices=["batched", "fwd_bwd", "nfft", "example51", "fig51", "adjoint"],
                    help="run only this leg (batched d=1 instances, d=2 forward + backward, "
                         "Algorithm 2.1 on the headline workload, the Example 5.1 sweep, the "
                         "Figure 5.1 sweep, or the adjoint on --workload at --precision) "
                         "and print its JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy five times (for counter scaling)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print a per-kernel summary of a rocprofv3 --kernel-trace --stats "
                         "csv output directory and exit (no GPU use)")
    ap.add_argument("--summarize-traffic", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="print a kernel's HBM traffic per launch from four rocprofv3 --pmc "
                         "csv output directories and exit (no GPU use)")
    ap.add_argument("--traffic-kernel", default="gather", choices=["gather", "fft", "spread", "merge"],
                    help="with --summarize-traffic: the gather, the FFT passes of a transform, or the "
                         "adjoint's spreading or box-merge kernel")
    ap.add_argument("--traffic-passes", type=int, default=1,
                    help="with --summarize-traffic: dispatches per launch (FFT: one per dimension)")
    return ap.parse_args()


WEIGHT_EVAL_FLOPS = 25   # one window weight psi(x - l/L): sinc, sqrt, sinh/exp, products


def mac_flops_per_node(d: int, m: int) -> int:
    """The contraction of one node's short sum: (2m)^d terms, each a real weight times a
    complex sample accumulated (2 FMA = 4 flops)."""
    return 4 * (2 * m) ** d


def gather_flops_per_node(d: int, m: int) -> int:
    """Algorithmic flops of one node's short sum: the contraction plus its d x 2m weight
    evaluations at WEIGHT_EVAL_FLOPS each (the compensated FP32C outer sum is not counted
    as extra work)."""
    return mac_flops_per_node(d, m) + WEIGHT_EVAL_FLOPS * d * 2 * m


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


def pass_bytes(d, M, L, csize):
    """(read, written) bytes of each pruned forward pass, in pass order (last axis first)."""
    out = []
    for axis in range(d - 1, -1, -1):
        out.append((M ** (axis + 1) * L ** (d - 1 - axis) * csize, M ** axis * L ** (d - axis) * csize))
    return out


def copy_floor_ms(torch, passes) -> float:
    """Time of plain device copies that move the same bytes as the FFT passes (one copy of
    (read + written) / 2 bytes per pass, each launched on its own): the latency and bandwidth
    floor a pass kernel of that traffic is compared with."""
    total = 0.0
    for rd, wr in passes:
        n = (rd + wr) // 2
        a = torch.empty(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        total += time_calls(torch, lambda: b.copy_(a), 50, 5, torch.cuda.current_stream())
        del a, b
    return total


def copy_bandwidth(torch, nbytes: int = 1 << 28, reps: int = 20) -> float:
    """Measured HBM bandwidth of a plain device copy (bytes read + written per second, GB/s),
    the achievable figure beside the nominal peak."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = time_calls(torch, lambda: b.copy_(a), reps, 3, torch.cuda.current_stream())
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


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


FFT_SOURCES = ["paper_2502_07155_amd/csrc/fft.hip", "paper_2502_07155_amd/csrc/stockham.h"]
SPREAD_SOURCES = ["paper_2502_07155_amd/csrc/spread.hip", "paper_2502_07155_amd/csrc/device_math.h"]


def measured_fft_traffic(workload: str, prec: str):
    """HBM bytes per transform (all passes) from the committed counter summary of this
    workload and precision, if it was taken on the current FFT sources; else None."""
    path = os.path.join(ROOT, f"profiles/k_fft_pass_{workload}_{prec}_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = re.search(r"^source_sha256:\s*(\w+)", text, re.M)
    val = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not sha or not val or sha.group(1) != source_digest(FFT_SOURCES):
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
    # steps 1-2 alone (the FFT passes), for the transform's own roofline entry
    fms = time_calls(torch, lambda: plan.samples(fhat), steps, warmup, stream)
    plan.forward(fhat, out=out)   # the plan's samples are those of this forward again
    f = out.cpu().numpy().astype(np.complex128)
    plan.fft_ms = fms
    return p, plan, f, ms, gms, plan_ms


def accuracy_check(rec: dict, p, f, sample: int = 20000, method: str = "shannon",
                   beta: float = 0.0, key: str = "rel_err", l2: bool = False):
    """Keep f on a seeded node sample; the returned check (run by the oracle leg) writes
    the normwise relative error against the oracle's fast form into rec[key + '_inf']."""
    import numpy as np

    import workloads as W
    idx = np.sort(W.rng_for(17).choice(p.N, size=min(sample, p.N), replace=False))
    got, x, fhat, L, m = f[idx].copy(), p.x[idx].copy(), p.fhat, p.L, p.m

    def check(O):
        b = beta if beta > 0 else None
        ref = (O.forward_shannon if method == "shannon" else O.forward_nfft)(fhat, x, L, m, b)
        rec[key + "_inf"] = O.rel_err_inf(got, ref)
        if l2:
            rec[key + "_l2"] = O.rel_err_l2(got, ref)
    return check


def leg_nfft(steps, warmup, f_shannon, p_shannon, checks: list):
    """Algorithm 2.1 on the headline workload with the same m, both beta readings; both
    methods' error against the direct sum on truncated-domain sample nodes (oracle leg)."""
    import numpy as np

    import workloads as W
    from paper_2502_07155_amd import Plan
    out = {}
    idx_all = np.sort(W.rng_for(18).choice(p_shannon.N, 2000, replace=False))
    probe = Plan(p_shannon.d, p_shannon.M, p_shannon.L, p_shannon.m, precision="f32c")
    beta_shannon = probe.stats()["beta"]   # the library's default beta of Algorithm 4.2
    probe.close()
    samples = {"shannon": f_shannon[idx_all].copy()}
    for label, beta in (("nfft_beta_standard", 0.0), ("nfft_beta_shannon", beta_shannon)):
        p, plan, f, ms, gms, _ = run_plan(HEADLINE, "f32c", steps, warmup, "nfft", beta)
        out[label] = {"value": p.N / (ms * 1e-3), "ms_per_step": ms, "gather_ms": gms,
                      "beta": plan.stats()["beta"]}
        checks.append(accuracy_check(out[label], p, f, 5000, "nfft", beta, key="rel_err_vs_oracle"))
        samples[label] = f[idx_all].copy()
        plan.close()
    x, fhat, L, m = p_shannon.x[idx_all], p_shannon.fhat, p_shannon.L, p_shannon.m

    def check(O):
        mask = O.in_truncated_domain(x, L, m)
        direct = O.direct_sum(fhat, x[mask])
        out["shannon_vs_direct_sum"] = O.rel_err_inf(samples["shannon"][mask], direct)
        for label in ("nfft_beta_standard", "nfft_beta_shannon"):
            out[label]["rel_err_inf_vs_direct_sum"] = O.rel_err_inf(samples[label][mask], direct)
        out["direct_sum_nodes"] = int(mask.sum())
    checks.append(check)
    return out


def plan_shape(plan) -> dict:
    """Launch shapes the plan runs with (tile edge, chunk capacity, FFT lines per workgroup)
    and how they were chosen (0 built-in rule, 1 timed, 2 tuning cache)."""
    st = plan.stats()
    return {"tile": st["tile"][:plan.d], "chunk_cap": st["chunk_cap"], "chunks": st["n_chunks"],
            "fft_lines_forward": st["fft_lines"][0][:plan.d], "fft_lines_adjoint": st["fft_lines"][1][:plan.d],
            "fft_radix_forward": st["fft_radix"][0][:plan.d], "fft_radix_adjoint": st["fft_radix"][1][:plan.d],
            "tuned": st["tuned"]}


def reference_check(rec: dict, p, f, kind: str):
    """The workload's own reference, applied to the GPU output by the oracle leg: the direct
    trigonometric sum on the truncated-domain nodes (boundary nodes reported apart), or, for
    fhat = 1 on the band, the Dirichlet product prod_t D_M(x_t) on 20000 sampled nodes
    (relative to max |D| = M^d).  Bound: d e^{-beta}, beta = pi m (L - M) / L."""
    import numpy as np

    import workloads as W
    if kind == "direct_sum":
        got, x = f.copy(), p.x.copy()
    else:
        idx = np.sort(W.rng_for(23).choice(p.N, size=min(20000, p.N), replace=False))
        got, x = f[idx].copy(), p.x[idx].copy()
    fhat, d, M, L, m = p.fhat, p.d, p.M, p.L, p.m

    def check(O):
        inside = O.in_truncated_domain(x, L, m)
        rec["reference_bound_d_exp_minus_beta"] = d * float(np.exp(-O.default_beta(M, L, m)))
        if kind == "direct_sum":
            ref = O.direct_sum(fhat, x)
            rec["rel_err_inf_vs_direct_sum_truncated_domain"] = O.rel_err_inf(got[inside], ref[inside])
            if (~inside).any():
                rec["rel_err_inf_vs_direct_sum_boundary_nodes"] = float(
                    np.max(np.abs(got[~inside] - ref[~inside])) / np.max(np.abs(ref[inside])))
            rec["truncated_domain_nodes"] = int(inside.sum())
        else:
            D = O.dirichlet(x[inside], M)
            rec["err_vs_dirichlet_product_rel_M_pow_d"] = float(np.max(np.abs(got[inside] - D)) / float(M) ** d)
            rec["dirichlet_sampled_nodes"] = int(inside.sum())
    return check


def leg_plan(name, prec, steps, warmup, checks: list, sample=5000, reference: str | None = None):
    p, plan, f, ms, gms, plan_ms = run_plan(name, prec, steps, warmup)
    shape = plan_shape(plan)
    plan.close()
    ab = algorithmic_bytes(p.d, p.M, p.L, p.N, 16 if prec == "f64" else 8, 8 if prec == "f64" else 4)
    rec = {"value": p.N / (ms * 1e-3), "ms_per_step": ms, "gather_ms": gms, "fft_ms": plan.fft_ms,
           "fft_GBs": ab["fft"] / (plan.fft_ms * 1e-3) / 1e9,
           "fft_frac_of_hbm_peak": ab["fft"] / (plan.fft_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "plan_ms": plan_ms, "precision": prec, "shape": shape}
    checks.append(accuracy_check(rec, p, f, sample))
    if reference:
        checks.append(reference_check(rec, p, f, reference))
    return rec


# Example 5.1 (Section 5): f(x) = sinc^2(M pi x / 2) with the triangle fhat, N = M/2
# Chebyshev nodes (5.6), m = 5, L = 2M, error max_j |f_j - f(x_j)| (5.5).
EXAMPLE51_M_PAPER = list(range(20, 1001, 20))   # M in {20, 40, ..., 1000}, Example 5.1


def example51_inputs(M: int, m: int = 5):
    import numpy as np

    import workloads as W
    L = 2 * M
    x = W.chebyshev_nodes(M // 2, L, m)
    exact = np.sinc(0.5 * M * x) ** 2   # numpy's sinc is sin(pi t)/(pi t)
    return L, x, W.triangle_fhat(M), exact


def leg_example51(checks: list):
    """Example 5.1 on the GPU at the paper's M = 20, 40, ..., 1000 (L = 2M, steps 1-2 by the
    chirp-z passes where L is not a power of two): per-plan FP64 for Algorithm 4.2 and
    Algorithm 2.1 with both beta readings (the same beta as Algorithm 4.2, and the standard
    NFFT beta), and the batched FP32 path for Algorithm 4.2.  Parity of every run with the
    oracle is filled in by the oracle leg; the 50-row table goes to stderr."""
    import numpy as np
    import torch

    from paper_2502_07155_amd import BatchPlan, Plan
    m = 5
    out = {"m": m, "M_values": EXAMPLE51_M_PAPER, "per_plan_f64": {}, "batched_f32": {}}
    for M in EXAMPLE51_M_PAPER:
        L, x, fhat, exact = example51_inputs(M, m)
        row = {"L": L}
        runs = (("alg4_2", "shannon", 0.0), ("alg2_1_same_beta", "nfft", None),
                ("alg2_1_standard_beta", "nfft", 0.0))
        beta_shannon = None
        for label, method, beta in runs:
            b = beta_shannon if beta is None else beta
            plan = Plan(1, M, L, m, precision="f64", method=method, beta=b)
            if method == "shannon":
                beta_shannon = plan.stats()["beta"]
            plan.set_nodes(torch.from_numpy(x[:, None]).cuda())
            f = plan.forward(torch.from_numpy(fhat).cuda()).cpu().numpy()
            used_beta = plan.stats()["beta"]
            plan.close()
            row[label] = {"max_err_vs_f": float(np.max(np.abs(f - exact))), "beta": used_beta}

            def check(O, rec=row[label], f=f, x=x, fhat=fhat, L=L, method=method, beta=used_beta):
                fn = O.forward_shannon if method == "shannon" else O.forward_nfft
                rec["rel_err_vs_oracle"] = O.rel_err_inf(f, fn(fhat, x[:, None], L, m, beta))
            checks.append(check)
        out["per_plan_f64"][str(M)] = row
        print(f"example 5.1  M={M:5d} L={L:5d}  alg 4.2 {row['alg4_2']['max_err_vs_f']:.3e}  "
              f"alg 2.1 same beta {row['alg2_1_same_beta']['max_err_vs_f']:.3e}  "
              f"alg 2.1 standard beta {row['alg2_1_standard_beta']['max_err_vs_f']:.3e}",
              file=sys.stderr)
    Ms = EXAMPLE51_M_PAPER
    ins = []
    for M in Ms:   # FP32 inputs; the exact f and the oracle see the same rounded values
        L, x, fhat, _ = example51_inputs(M, m)
        x = x.astype(np.float32).astype(np.float64)
        fhat = fhat.astype(np.complex64).astype(np.complex128)
        ins.append((L, x, fhat, np.sinc(0.5 * M * x) ** 2))
    bp = BatchPlan(Ms, [i[0] for i in ins], [m] * len(Ms), [M // 2 for M in Ms], precision="f32")
    bp.set_nodes(torch.from_numpy(np.concatenate([i[1] for i in ins]).astype(np.float32)).cuda())
    fhat_all = torch.from_numpy(np.concatenate([i[2] for i in ins]).astype(np.complex64)).cuda()
    fb = torch.empty(bp.total_N, dtype=torch.complex64, device="cuda")
    bp.forward(fhat_all, fb)
    fb = fb.cpu().numpy().astype(np.complex128)
    for k, M in enumerate(Ms):
        L, x, fhat, exact = ins[k]
        f = fb[bp.node_offsets[k]:bp.node_offsets[k + 1]]
        rec = {"L": L, "max_err_vs_f": float(np.max(np.abs(f - exact)))}
        out["batched_f32"][str(M)] = rec

        def check(O, rec=rec, f=f, x=x, fhat=fhat, L=L):
            rec["rel_err_vs_oracle"] = O.rel_err_inf(f, O.forward_shannon(fhat, x[:, None], L, m))
        checks.append(check)
    bp.close()
    return out


def leg_fig51(checks: list):
    """Figure 5.1 (Section 5): e(v) = max_p |e^{2 pi i v x_p} - h(x_p)| (5.3) at P = 1e5
    equispaced x_p, for v_s of (5.4) with S = 32, M = 20, L = 40, m = 5 (sinh window), on
    [-1/2, 1/2) and on the truncated interval.  h is (5.2), the short sums of Algorithm 4.2
    on the samples e^{2 pi i v l/L}, or (5.1), the periodic window sums of Algorithm 2.1 on
    those samples divided by L phihat(v), with the same beta and with the standard one.
    Every h is one bl_interpolate call of an FP64 plan (L = 40 needs no FFT)."""
    import numpy as np
    import torch

    from paper_2502_07155_amd import Plan, window_transform
    M, L, m, S, P = 20, 40, 5, 32, 100_000
    vs = -M / 2 - m + np.arange(S * (M + 2 * m) + 1) / S
    inband = np.abs(vs) <= M / 2
    integer = np.abs(vs - np.rint(vs)) < 1e-12
    ell = np.arange(L) - L // 2
    a, b = -0.5 + m / L, 0.5 - m / L
    intervals = {"full": -0.5 + np.arange(P) / P, "truncated": a + np.arange(P) * (b - a) / P}
    v_pick = set(range(0, vs.size, 37))         # parity sample: every 37th frequency
    out = {"M": M, "L": L, "m": m, "S": S, "P": P, "frequencies": int(vs.size)}
    t_all = time.perf_counter()
    calls = 0
    for iname, x in intervals.items():
        xd = torch.from_numpy(x[:, None]).cuda()
        node_pick = np.sort(np.random.default_rng(51).choice(P, 2000, replace=False))
        for label, method, beta_arg in (("eq5_2_alg4_2", "shannon", 0.0),
                                        ("eq5_1_alg2_1_same_beta", "nfft", None),
                                        ("eq5_1_alg2_1_standard_beta", "nfft", 0.0)):
            if beta_arg is None:
                probe = Plan(1, M, L, m, precision="f64")
                beta_arg = probe.stats()["beta"]
                probe.close()
            plan = Plan(1, M, L, m, precision="f64", method=method, beta=beta_arg)
            plan.set_nodes(xd)
            beta = plan.stats()["beta"]
            fac = np.ones(vs.size)
            if method == "nfft":
                fac = 1.0 / (L * window_transform(vs, M, L, m, beta, "sinh", "nfft"))
            theta = torch.from_numpy(np.exp(2j * np.pi * np.outer(vs, ell) / L) * fac[:, None]).cuda()
            h = torch.empty(P, dtype=torch.complex128, device="cuda")
            err = np.empty(vs.size)
            picked = {}
            for i, v in enumerate(vs):
                plan.interpolate(theta[i], out=h)
                calls += 1
                e = (h - torch.exp(2j * np.pi * v * xd[:, 0])).abs().max()
                err[i] = float(e)
                if i in v_pick:
                    picked[i] = h[torch.from_numpy(node_pick).cuda()].cpu().numpy()
            plan.close()
            rec = {"beta": beta,
                   "max_e_in_band": float(err[inband].max()),
                   "max_e_in_band_integer_v": float(err[inband & integer].max()),
                   "max_e_in_band_noninteger_v": float(err[inband & ~integer].max()),
                   "min_e_beyond_band_plus_1": float(err[np.abs(vs) >= M / 2 + 1].min()),
                   "e_at_v": {f"{vs[i]:g}": float(err[i]) for i in range(0, vs.size, S * 5)}}
            out[f"{iname}/{label}"] = rec

            def check(O, rec=rec, picked=picked, x=x[node_pick], method=method, beta=beta):
                fn = O.exp_approx_shannon if method == "shannon" else O.exp_approx_nfft
                rec["rel_err_vs_oracle"] = max(O.rel_err_inf(hv, fn(vs[i], x, L, m, beta))
                                               for i, hv in picked.items())
            checks.append(check)
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t_all
    out["interpolate_calls"] = calls
    return out


def leg_precomputed_weights(steps, warmup, checks: list):
    """Algorithm 4.2 step 0b with stored weights on the headline workload (FP32C): the
    d x 2m weights of every node are read from HBM by the short sums instead of being
    evaluated.  Reports both short-sum times, the one-time weight pass and the bytes."""
    import torch

    import workloads as W
    from paper_2502_07155_amd import Plan
    p = W.make_problem(HEADLINE, precision="f32")
    x = torch.from_numpy(p.x).to(torch.float32).cuda()
    fhat = torch.from_numpy(p.fhat).to(torch.complex64).cuda()
    plan = Plan(p.d, p.M, p.L, p.m, precision="f32c")
    plan.set_nodes(x)
    out = torch.empty(p.N, dtype=torch.complex64, device="cuda")
    plan.forward(fhat, out=out)
    theta = plan.theta()
    g_fly = time_calls(torch, lambda: plan.interpolate(theta, out=out), steps, warmup, plan.stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.precompute_weights(True)
    torch.cuda.synchronize()
    pre_ms = (time.perf_counter() - t0) * 1e3
    ms = time_calls(torch, lambda: plan.forward(fhat, out=out), steps, warmup, plan.stream)
    g_pre = time_calls(torch, lambda: plan.interpolate(theta, out=out), steps, warmup, plan.stream)
    f = out.cpu().numpy().astype("complex128")
    plan.close()
    rec = {"value": p.N / (ms * 1e-3), "ms_per_step": ms, "gather_ms_precomputed": g_pre,
           "gather_ms_on_the_fly": g_fly, "precompute_ms": pre_ms,
           "weight_bytes": p.N * p.d * 2 * p.m * 4, "precision": "f32c"}
    checks.append(accuracy_check(rec, p, f, 5000))
    return rec


def leg_two_streams(steps, warmup, checks: list):
    """Serving throughput of independent headline transforms (FP32C): two plans with the same
    nodes on two streams (default priority), transforms alternating between them, so that one
    transform's FFT passes (which leave most CUs idle) overlap the other's short sums.  Every
    transform runs in full; the time per transform is the host-clock span of all of them,
    bracketed by device synchronization, divided by their number."""
    import torch

    import workloads as W
    from paper_2502_07155_amd import Plan
    p = W.make_problem(HEADLINE, precision="f32")
    x = torch.from_numpy(p.x).to(torch.float32).cuda()
    fhat = torch.from_numpy(p.fhat).to(torch.complex64).cuda()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    plans = [Plan(p.d, p.M, p.L, p.m, precision="f32c", stream=st) for st in streams]
    outs = [torch.empty(p.N, dtype=torch.complex64, device="cuda") for _ in plans]
    for pl in plans:
        pl.set_nodes(x)
    for _ in range(max(warmup, 1)):
        for pl, o in zip(plans, outs):
            pl.forward(fhat, out=o)   # also captures each plan's graph for these buffers
    torch.cuda.synchronize()
    # issue through the C entry point with resolved pointers, so that host-side argument
    # checks do not limit the issue rate (every status is still checked)
    import ctypes
    calls = [(pl._lib.bl_forward, pl.handle, ctypes.c_void_p(fhat.data_ptr()),
              ctypes.c_void_p(o.data_ptr())) for pl, o in zip(plans, outs)]
    n = 2 * steps
    status = []
    t0 = time.perf_counter()
    for k in range(n):
        fn, h, a, b = calls[k % 2]
        status.append(fn(h, a, b))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / n
    if any(st != 0 for st in status):
        raise RuntimeError(f"bl_forward failed in the two-stream leg: {set(status)}")
    f = outs[1].cpu().numpy().astype("complex128")
    for pl in plans:
        pl.close()
    rec = {"value": p.N / (ms * 1e-3), "ms_per_transform": ms, "transforms": n, "streams": 2,
           "precision": "f32c"}
    checks.append(accuracy_check(rec, p, f, 5000))
    return rec


def leg_batched(steps, warmup, checks: list):
    """512 independent d=1 instances, one graph launch per step, FP32."""
    import numpy as np
    import torch

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
    # a second batch of the same shapes reads its tile edge from the tuning cache
    bp2 = BatchPlan([i.M for i in insts], [i.L for i in insts], [i.m for i in insts],
                    [i.x.size for i in insts], precision="f32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bp2.set_nodes(x)
    torch.cuda.synchronize()
    plan_ms_cached = (time.perf_counter() - t0) * 1e3
    bp2.close()
    rng = W.rng_for(19)
    picks = []
    for i in rng.choice(len(insts), 32, replace=False):
        inst = insts[i]
        idx = rng.choice(inst.x.size, min(32, inst.x.size), replace=False)
        picks.append((inst, idx, f[bp.node_offsets[i]:bp.node_offsets[i + 1]][idx].copy()))
    bp.close()
    rec = {"value": bp.total_N / (ms * 1e-3), "ms_per_step": ms, "plan_ms": plan_ms,
           "plan_ms_cached_tuning": plan_ms_cached,
           "instances": len(insts), "total_nodes": bp.total_N, "precision": "f32"}

    def check(O):
        rec["rel_err_inf_worst_of_32_sampled_instances"] = max(
            O.rel_err_inf(got, O.forward_shannon(inst.fhat, inst.x[idx, None], inst.L, inst.m))
            for inst, idx, got in picks)
    checks.append(check)
    return rec


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


def leg_adjoint(name, prec, steps, warmup, checks: list, nk=4):
    """The adjoint A^H g (spreading, forward DFT passes, truncation and deconvolution) on a
    named workload with seeded random g; the deferred check compares nk sampled
    frequencies, including the band's two corners, with the oracle's entry-by-entry
    adjoint."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2502_07155_amd import Plan
    p = W.make_problem(name, precision="f64" if prec == "f64" else "f32")
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    rdt = torch.float64 if prec == "f64" else torch.float32
    rng = W.rng_for(91)
    g = rng.standard_normal(p.N) + 1j * rng.standard_normal(p.N)
    if prec != "f64":
        g = g.astype(np.complex64).astype(np.complex128)
    plan = Plan(p.d, p.M, p.L, p.m, precision=prec)
    plan.set_nodes(torch.from_numpy(p.x).to(rdt).cuda())
    gd = torch.from_numpy(g).to(cdt).cuda()
    out = plan.adjoint(gd)
    ms = time_calls(torch, lambda: plan.adjoint(gd, out), steps, warmup, plan.stream)
    a = out.cpu().numpy().astype(np.complex128)
    stats = plan.stats()
    plan.close()
    h = p.M // 2
    ks = np.concatenate([np.array([[-h] * p.d, [h - 1] * p.d]), rng.integers(-h, h, size=(nk - 2, p.d))])
    rec = {"value": p.N / (ms * 1e-3), "unit": "nodes/s", "ms_per_step": ms, "precision": prec,
           "chunks": stats["n_chunks"], "tile": stats["tile"],
           "step": "adjoint: spreading + forward DFT passes + truncation and deconvolution"}

    def check(O):
        ref = O.adjoint_at(g, p.x, p.M, p.L, p.m, ks)
        rec["rel_err_inf_vs_oracle_sampled_k"] = O.rel_err_inf(a[tuple((ks + h).T)], ref)
        rec["sampled_k"] = int(len(ks))
    checks.append(check)
    return rec


def oracle_checks(checks: list) -> None:
    """Run the GPU legs' deferred error checks against the oracle."""
    import oracle as O
    for check in checks:
        check(O)


def oracle_leg(checks: list, name: str, nodes: int) -> dict:
    """The oracle leg, the only part of this file that uses the oracle: the deferred error
    checks, then the CPU baseline."""
    oracle_checks(checks)
    return cpu_baseline(name, nodes)


def cpu_baseline(name: str, nodes: int, runs: int = 5, direct_nodes: int = 4000):
    """The oracle as it stands (numpy FP64) on every host core this process may use:
    steps 1-2 on the full grid with the BLAS/FFT threads of numpy, then step 3 over node
    chunks in a thread pool (numpy releases the interpreter lock inside its array
    operations), the median of `runs` runs; `nodes` caps the step-3 sample (its time is
    scaled to the full node count).  The direct O(N M^d) sum, the target both algorithms
    approximate, is timed on `direct_nodes` nodes and extrapolated to N."""
    import statistics
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    import workloads as W
    p = W.make_problem(name, precision="f32")
    n = min(nodes, p.N)
    cores = len(os.sched_getaffinity(0))
    beta = O.default_beta(p.M, p.L, p.m)
    chunks = np.array_split(np.arange(n), 4 * cores)
    t12, t3 = [], []
    for _ in range(runs):
        with threadpool_limits(limits=cores):
            t0 = time.perf_counter()
            theta = O.inverse_fft_step(O.deconvolve_pad(p.fhat, p.L, p.m, beta))
            t1 = time.perf_counter()
        with threadpool_limits(limits=1), ThreadPoolExecutor(cores) as ex:
            t2 = time.perf_counter()
            list(ex.map(lambda c: O.gather_shannon(theta, p.x[c], p.L, p.m, beta), chunks))
            t3.append(time.perf_counter() - t2)
        t12.append(t1 - t0)
    t_full = statistics.median(t12) + statistics.median(t3) * (p.N / n)
    nd = min(direct_nodes, p.N)
    dchunks = np.array_split(np.arange(nd), cores)
    with threadpool_limits(limits=1), ThreadPoolExecutor(cores) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda c: O.direct_sum(p.fhat, p.x[c]), dchunks))
        t_direct = (time.perf_counter() - t0) * (p.N / nd)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": p.N / t_full, "unit": "node evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model, "runs": runs,
            "sample": f"numpy FP64 oracle on {cores} host threads, median of {runs} runs: steps 1-2 "
                      f"on the full {p.L}^{p.d} grid ({statistics.median(t12):.3f} s) + step 3 on "
                      f"{n} of {p.N} nodes in {len(chunks)} chunks ({statistics.median(t3):.3f} s)"
                      + (f", step-3 time scaled by {p.N / n:.1f}" if n < p.N else ""),
            "direct_sum": {"value_extrapolated": p.N / t_direct, "unit": "node evals/s",
                           "sample": f"direct O(N M^d) sum on {nd} nodes, {cores} threads, "
                                     f"time extrapolated to {p.N} nodes ({t_direct:.1f} s)"}}


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


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, kernel: str = "gather",
                      per_launch: int = 1) -> str:
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the gather (kernel "gather"), of the
    FFT passes (kernel "fft": per_launch passes per transform, summed) or of the adjoint's
    spreading ("spread") or box-merge ("merge") kernel, each divided by the counter-to-bytes
    factor of a 1 GiB device copy (which reads and writes 1 GiB)."""
    marks = {"gather": ("k_gather<",), "fft": ("k_fft_pass<", "k_czt_pass<"),
             "spread": ("k_spread",), "merge": ("k_box_merge",)}[kernel]

    def pick(name):
        return any(k in name for k in marks)

    def copy(name):
        return True   # the calibration run launches nothing but the copies

    fetch, nf = _counter_per_dispatch(fetch_dir, pick)
    write, nw = _counter_per_dispatch(write_dir, pick)
    cf, ncf = _counter_per_dispatch(copy_fetch_dir, copy)
    cw, ncw = _counter_per_dispatch(copy_write_dir, copy)
    gib_kib = float(1 << 20)
    ff, fw = cf / gib_kib, cw / gib_kib
    traffic = (fetch / ff + write / fw) * 1024.0 * per_launch
    sources = {"gather": GATHER_SOURCES, "fft": FFT_SOURCES}.get(kernel, SPREAD_SOURCES)
    return "\n".join([
        f"{kernel}_fetch_kib_per_dispatch: {fetch:.1f}  (dispatches: {nf})",
        f"{kernel}_write_kib_per_dispatch: {write:.1f}  (dispatches: {nw})",
        f"dispatches_per_launch: {per_launch}",
        f"copy_fetch_kib_per_GiB_copy: {cf:.1f}  (dispatches: {ncf}); factor {ff:.4f}",
        f"copy_write_kib_per_GiB_copy: {cw:.1f}  (dispatches: {ncw}); factor {fw:.4f}",
        f"traffic_bytes_per_launch: {traffic:.6e}",
        f"source_sha256: {source_digest(sources)}",
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
        print(summarize_traffic(*args.summarize_traffic, kernel=args.traffic_kernel,
                                per_launch=args.traffic_passes))
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
    checks: list = []
    if args.leg == "batched":
        rec = leg_batched(args.steps, args.warmup, checks)
        if not args.no_cpu:
            oracle_checks(checks)
        print(json.dumps(rec))
        return
    if args.leg == "fwd_bwd":
        print(json.dumps(leg_differentiation(args.steps, args.warmup)))
        return
    if args.leg == "nfft":
        p, plan, f, _, _, _ = run_plan(HEADLINE, "f32c", 2, 1)
        plan.close()
        rec = leg_nfft(args.steps, args.warmup, f, p, checks)
        if not args.no_cpu:
            oracle_checks(checks)
        print(json.dumps(rec))
        return
    if args.leg == "adjoint":
        rec = leg_adjoint(args.workload, args.precision, args.steps, args.warmup, checks)
        if not args.no_cpu:
            oracle_checks(checks)
        print(json.dumps(rec))
        return
    if args.leg == "fig51":
        rec = leg_fig51(checks)
        if not args.no_cpu:
            oracle_checks(checks)
        print(json.dumps(rec))
        return
    if args.leg == "example51":
        rec = leg_example51(checks)
        if not args.no_cpu:
            oracle_checks(checks)
        print(json.dumps(rec))
        return

    prec = args.precision
    p, plan, f, ms, gms, plan_ms = run_plan(args.workload, prec, args.steps, args.warmup)
    csize, rsize = (16, 8) if prec == "f64" else (8, 4)
    ab = algorithmic_bytes(p.d, p.M, p.L, p.N, csize, rsize)
    flops = gather_flops_per_node(p.d, p.m) * p.N
    peak = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    published = 78.6 if prec == "f64" else FP32_PUBLISHED_TFLOPS
    gather_tflops = flops / (gms * 1e-3) / 1e12
    fft_ms = plan.fft_ms
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
        "rel_err_inf": None,
        "rel_err_l2": None,
        "plan_ms": plan_ms,
        "stage_ms": {"deconv_fft": fft_ms, "gather": gms},
        "roofline": {"bound": "alu", "kernel": "k_gather (step 3 short sums)",
                     "achieved": gather_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": gather_tflops / peak, "traffic": traffic,
                     "peak_basis": PEAK_BASIS, "peak_published": published,
                     "frac_vs_published": gather_tflops / published,
                     "algorithmic_flops_per_launch": flops,
                     "per_node_flops": gather_flops_per_node(p.d, p.m),
                     "per_node_flops_contraction_only": mac_flops_per_node(p.d, p.m),
                     "frac_contraction_only": mac_flops_per_node(p.d, p.m) * p.N / (gms * 1e-3) / 1e12 / peak},
        "roofline_fft": {"bound": "hbm", "kernel": "k_fft_pass (steps 1-2: deconvolution, zero-padding, "
                                                  f"{p.d} pruned passes)",
                         "achieved": ab["fft"] / (fft_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ab["fft"] / (fft_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "traffic": measured_fft_traffic(args.workload, prec),
                         "algorithmic_bytes_per_launch": ab["fft"],
                         "ms_per_launch": fft_ms,
                         "copy_floor_ms": None if args.headline_only else copy_floor_ms(
                             torch, pass_bytes(p.d, p.M, p.L, csize)),
                         "note": "all passes of one transform between HIP events on the plan's stream "
                                 "(bl_samples); algorithmic bytes: every pruned pass reads and writes "
                                 "its lines once in the data type; copy_floor_ms: plain device copies "
                                 "moving the same bytes, one per pass"},
        "hbm": {"algorithmic_bytes": ab, "deconv_fft_GBs": ab["fft"] / (fft_ms * 1e-3) / 1e9,
                "gather_GBs": ab["gather"] / (gms * 1e-3) / 1e9, "peak_GBs": HBM_PEAK_GBS,
                "copy_GBs": None if args.headline_only else copy_bandwidth(torch),
                "copy_note": "device-to-device copy of 256 MiB, read + write bytes per second "
                             "(full runs only, so that profiles of --headline-only stay clean)"},
    }
    # steady-state rebinding of the same nodes (a training loop that moves x pays this per step)
    xr = torch.from_numpy(p.x).to(torch.float64 if prec == "f64" else torch.float32).cuda()
    plan.set_nodes(xr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.set_nodes(xr)
    torch.cuda.synchronize()
    rec["rebind_ms"] = (time.perf_counter() - t0) * 1e3 / 5
    rec["shape"] = plan_shape(plan)
    plan.close()
    checks.append(accuracy_check(rec, p, f, key="rel_err", l2=True))
    if not args.headline_only and args.workload == HEADLINE and prec != "f64":
        legs = {}
        short = max(5, args.steps // 5)
        legs["d2_M512_L1024_m5_N1M_f64"] = leg_plan(HEADLINE, "f64", short, 2, checks)
        legs["d2_M512_L1024_m5_N1M_f32d"] = leg_plan(HEADLINE, "f32d", short, 2, checks)
        legs["d2_M512_L1024_m5_N1M_f32"] = leg_plan(HEADLINE, "f32", short, 2, checks)
        legs["d2_M512_L1024_m5_N1M_nfft"] = leg_nfft(short, 2, f, p, checks)
        legs["d1_M256_L512_m6_N1k_f64"] = leg_plan("d1_M256_L512_m6_N1k", "f64", short, 2, checks, 1000,
                                                   reference="direct_sum")
        legs["d3_M128_L256_m4_N2M_f32c"] = leg_plan("d3_M128_L256_m4_N2M", "f32c", short, 2, checks, 3000,
                                                    reference="dirichlet")
        legs["d3_M128_L256_m4_N2M_f32d"] = leg_plan("d3_M128_L256_m4_N2M", "f32d", short, 2, checks, 3000)
        legs["d3_M128_L256_m4_N2M_f64"] = leg_plan("d3_M128_L256_m4_N2M", "f64", short, 2, checks, 3000,
                                                   reference="dirichlet")
        legs["batched_512_d1_f32"] = leg_batched(short, 2, checks)
        legs["d2_M256_L512_m6_N200k_fwd_bwd_f32"] = leg_differentiation(short, 2)
        legs["d2_M512_L1024_m5_N1M_adjoint_f32c"] = leg_adjoint(HEADLINE, "f32c", short, 2, checks)
        legs["d3_M128_L256_m4_N2M_adjoint_f32c"] = leg_adjoint("d3_M128_L256_m4_N2M", "f32c", short, 2, checks)
        legs["d2_M512_L1024_m5_N1M_precomputed_weights"] = leg_precomputed_weights(short, 2, checks)
        legs["d2_M512_L1024_m5_N1M_two_streams"] = leg_two_streams(args.steps, args.warmup, checks)
        legs["example_5_1"] = leg_example51(checks)
        legs["figure_5_1"] = leg_fig51(checks)
        rec["legs"] = legs
    if not args.no_cpu and not args.headline_only:
        rec["cpu_baseline"] = oracle_leg(checks, args.workload, args.cpu_nodes)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
