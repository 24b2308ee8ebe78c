"""Benchmark of the dSMC smoother on one MI355X.

Workload: stochastic-volatility model (mu = -1, rho = 0.95, sigma = 0.3),
K = 4096 time points (T = 4096 in the configs' notation), N = 1024 particles,
fp32 pair weights, data simulated from the model with a fixed seed.  One step
is one whole smoother run (leaves, 12 tree levels, output) on resident inputs,
through the C ABI.

Output: one JSON line.  `value` = algorithmic pair evaluations per second,
(K-1) N^2 per step.  `roofline` prices the dominant kernel (the pair-row
kernel) against the VALU issue rate of the chip; `cpu_baseline` times the fp64
oracle on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.32e12 lane-instructions/s
# for single-rate VALU work (fp32 add/sub/fma without packed math).
LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# VALU issue slots per pair evaluation in the pair-row kernel (d_x = 1):
# v_sub, v_fma, v_add at one slot each, plus v_exp_f32 at TRANS_SLOTS slots
# (v_exp_f32 issues at half the rate of v_fma_f32 on gfx950 and does not
# co-issue with it: measured 1.85e13 vs 3.5e13 lane-instructions/s).
TRANS_SLOTS = 2.0
SLOTS_PER_PAIR = 3.0 + TRANS_SLOTS


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--K", type=int, default=4096)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="wall-clock budget of the oracle baseline sample (0 = skip)")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the steps without per-kernel HIP events")
    ap.add_argument("--workload", choices=("sv", "batch"), default="sv",
                    help="sv: one long stochastic-volatility series (default); batch: "
                         "B linear-Gaussian series of uneven length, packed vs one at a time")
    ap.add_argument("--B", type=int, default=512)
    return ap.parse_args()


def cpu_baseline(spec, N: int, budget_s: float) -> dict:
    """The fp64 oracle's combine (Algorithm 1) on level-0 nodes of the same
    workload, one after another until the time budget is spent."""
    import numpy as np

    from oracle import dsmc as D
    from oracle import philox as P
    t_wall0, t_cpu0 = time.perf_counter(), time.process_time()
    nodes = 0
    seed = 1
    c = 1
    while time.perf_counter() - t_wall0 < budget_s and c < spec.K:
        sub = spec.truncated(c + 1)
        xs = []
        for t in (c - 1, c):
            z = P.leaf_normals(seed, t, N, 1)
            xs.append(sub.q_mean[t][None, :] + z @ sub.q_chol[t].T)
        lws = [D.normalise(D.leaf_logweights(sub, t, x))[0] for t, x in zip((c - 1, c), xs)]
        u1, u2 = P.combine_uniforms(seed, c, N)
        D.combine(sub, c, xs[0], xs[1], lws[0], lws[1], u1, u2)
        nodes += 1
        c += 2
    wall = time.perf_counter() - t_wall0
    cpu = time.process_time() - t_cpu0
    pairs = nodes * N * N
    return {"value": pairs / wall, "unit": "pair-evals/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"{nodes} level-0 combines (leaf draws, weights, N x N pair weights, "
                      f"{N} two-stage draws each) of the same workload, fp64 numpy, "
                      f"{wall:.1f} s wall"}


def bench_batch(args):
    """B independent 1-D linear-Gaussian series (A ~ U[0.5, 0.99], Q, R ~ U[0.1, 2],
    K ~ U{64..8192}), N = 256: dsmc_smooth_batch (every level of every series
    in shared launches) against dsmc_smooth called once per series (one set of
    launches per level per series).  Results are bit-identical between the two."""
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    N = 256 if args.N == 1024 else args.N
    specs = W.lg1d_batch(args.B)
    Ks = [s.K for s in specs]
    models = [G.Model(s) for s in specs]
    plan = G.Plan(N, 1, max(Ks), max_total_K=sum(Ks), profile=not args.no_kernel_events)
    outs = [G.alloc_output(plan, K) for K in Ks]
    seeds = list(range(1, args.B + 1))
    for _ in range(max(1, args.warmup)):
        G.dsmc_smooth_batch(plan, models, seeds, outs)
    torch.cuda.synchronize()
    if not args.no_kernel_events:
        G.dsmc_plan_profile(plan)
    steps = max(1, min(args.steps, 5))
    t0 = time.perf_counter()
    for _ in range(steps):
        G.dsmc_smooth_batch(plan, models, seeds, outs)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / steps
    prof = G.dsmc_plan_profile(plan) if not args.no_kernel_events else None
    # plain: one series at a time
    plan1 = G.Plan(N, 1, max(Ks))
    out1 = G.alloc_output(plan1, max(Ks))
    outs1 = [G.Output(traj=out1.traj[:, :K], logw=out1.logw, log_Z=out1.log_Z,
                      status=out1.status) for K in Ks]
    for m, s, o in zip(models[:8], seeds, outs1):
        G.dsmc_smooth(plan1, m, s, o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m, s, o in zip(models, seeds, outs1):
        G.dsmc_smooth(plan1, m, s, o)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    pairs = sum((K - 1) * N * N for K in Ks)
    res = {"metric": "smoothers/sec", "value": args.B / dt_b, "unit": "smoothers/s",
           "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": dt_b * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{args.B} linear-Gaussian series, K ~ U{{64..8192}} "
                                  f"(sum {sum(Ks)}), N={N}, one batch per step",
                      "B": args.B, "N": N, "sum_K": sum(Ks)},
           "plain_smoothers_per_sec": args.B / dt_p, "plain_ms_per_batch": dt_p * 1e3,
           "speedup_vs_plain": dt_p / dt_b, "pair_evals_per_sec": pairs / dt_b}
    if prof:
        ms_rows = prof["ms"]["rows"]
        peak = LANE_OPS_PER_S / SLOTS_PER_PAIR
        res["roofline"] = {"bound": "alu", "kernel": "k_rows<float,1,RPL>",
                           "achieved": prof["pairs"] / (ms_rows * 1e-3) / 1e9,
                           "peak": peak / 1e9, "unit": "Gpair/s",
                           "frac": prof["pairs"] / (ms_rows * 1e-3) / peak, "traffic": None}
        res["kernel_ms_per_step"] = {k: v / steps for k, v in prof["ms"].items()}
    print(json.dumps(res))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W

    torch.cuda.set_device(0)
    K, N = args.K, args.N
    spec = W.sv(K)
    model = G.Model(spec)
    plan = G.Plan(N, 1, K, profile=not args.no_kernel_events)
    out = G.alloc_output(plan, K)
    for s in range(args.warmup):
        G.dsmc_smooth(plan, model, 1000 + s, out)
    torch.cuda.synchronize()
    if not args.no_kernel_events:
        G.dsmc_plan_profile(plan)  # drop the warm-up records
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        G.dsmc_smooth(plan, model, s + 1, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    status = int(out.status.item())
    if status:
        raise RuntimeError(f"device status {status}")
    pairs = (K - 1) * N * N
    res = {
        "metric": "pair-evals/sec",
        "value": pairs / dt,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"stochastic volatility, K={K} time points, N={N} particles, "
                               "one smoother per step", "K": K, "N": N, "d_x": 1,
                   "precision": "fp32 pair weights, fp64 sums and CDFs",
                   "weighting": spec.weighting, "data_seed": W.DATA_SEED},
        "smoothers_per_sec": 1.0 / dt,
        "pair_evals_T_log2T_N2_per_sec": K * math.log2(K) * N * N / dt,
    }
    if not args.no_kernel_events:
        prof = G.dsmc_plan_profile(plan)
        n_rows = prof["launches"]["rows"]
        ms_rows = prof["ms"]["rows"]
        achieved = prof["pairs"] / (ms_rows * 1e-3)
        peak = LANE_OPS_PER_S / SLOTS_PER_PAIR
        res["roofline"] = {"bound": "alu", "kernel": "k_rows<float,1,RPL>",
                           "achieved": achieved / 1e9, "peak": peak / 1e9, "unit": "Gpair/s",
                           "frac": achieved / peak, "traffic": None,
                           "avg_launch_ms": ms_rows / max(1, n_rows),
                           "pairs_per_launch": prof["pairs"] / max(1, n_rows)}
        res["kernel_ms_per_step"] = {k: v / args.steps for k, v in prof["ms"].items()}
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(spec, N, args.cpu_seconds)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
