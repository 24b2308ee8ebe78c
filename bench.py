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
    ap.add_argument("--workload", choices=("sv", "batch", "serve"), default="sv",
                    help="sv: one long stochastic-volatility series (default); batch: "
                         "B linear-Gaussian series of uneven length, packed vs one at a time")
    ap.add_argument("--B", type=int, default=512)
    ap.add_argument("--jobs", type=int, default=600, help="serving: jobs per arrival run")
    ap.add_argument("--rates", type=str, default="0.25,0.5,0.75,0.9,1.1",
                    help="serving: Poisson arrival rates as fractions of the saturated rate")
    ap.add_argument("--serve-mem-gib", type=int, default=72)
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


def _pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q)) if len(a) else float("nan")


def bench_serve(args):
    """Serving: a seeded stream of jobs (half stochastic-volatility, half 4-D
    linear-Gaussian, K ~ lognormal(median 512, sigma_log 1) clipped to
    [2, 16384], N uniform over {256, 1024, 4096}, fp32) through dsmc_submit /
    dsmc_poll.  First all jobs at once (saturated throughput), then Poisson
    arrivals at fractions of that rate (p50/p99 latency from submission to
    completion as the engine observes it).  Models and output buffers are on
    the device before the clock starts.  Against it: the same jobs through
    dsmc_smooth one after another (one set of launches per level per job)."""
    import numpy as np
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    t_gen = time.perf_counter()
    jobs = W.serving_jobs(args.jobs)
    models = [G.Model(s) for s, _, _ in jobs]
    outs = [G.alloc_job_output(N, s.d_x, s.K) for s, N, _ in jobs]
    torch.cuda.synchronize()
    print(f"# serve: {len(jobs)} jobs generated and uploaded in "
          f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    pairs = sum((s.K - 1) * N * N for s, N, _ in jobs)
    srv = G.Server(mem_budget=args.serve_mem_gib << 30, max_jobs=1024, max_classes=6)

    def run(order, gaps=None):
        ids = []
        t0 = time.monotonic()
        t_next = t0
        for k in order:
            spec, N, seed = jobs[k]
            if gaps is not None:
                t_next += gaps[len(ids)]
                while True:
                    d = t_next - time.monotonic()
                    if d <= 0:
                        break
                    if d > 1e-3:
                        time.sleep(d - 5e-4)
            ids.append(G.dsmc_submit(srv, models[k], N, seed, outs[k]))
        pending = set(ids)
        while pending:
            for i in list(pending):
                rc, _ = G.dsmc_poll(srv, i)
                if rc != G.DSMC_EAGAIN:
                    if rc != 0:
                        raise RuntimeError(f"serving job {i} failed with code {rc}")
                    pending.discard(i)
            time.sleep(2e-4)
        ts = np.array([G.dsmc_job_times(srv, i) for i in ids])
        lat = (ts[:, 2] - ts[:, 0]) * 1e3
        span = ts[:, 2].max() - ts[:, 0].min()
        return {"jobs_per_sec": len(ids) / span, "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
                "mean_ms": float(lat.mean()), "span_s": float(span),
                "pair_evals_per_sec": sum((jobs[k][0].K - 1) * jobs[k][1] ** 2 for k in order) / span}

    warm = list(range(min(len(jobs), 48)))
    run(warm)  # creates the class pools
    sat = run(range(len(jobs)))
    print(f"# serve saturated: {sat['jobs_per_sec']:.1f} jobs/s", file=sys.stderr, flush=True)
    # the same jobs alone through dsmc_smooth, compared with the served results
    served = {k: outs[k].traj.cpu() for k in range(0, len(jobs), 37)}
    plans = {}
    for spec, N, _ in jobs:
        key = (N, spec.d_x)
        plans[key] = max(plans.get(key, 0), spec.K)
    plans = {k: G.Plan(k[0], k[1], K) for k, K in plans.items()}
    for k in warm[:8]:
        spec, N, seed = jobs[k]
        G.dsmc_smooth(plans[(N, spec.d_x)], models[k], seed, outs[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (spec, N, seed) in enumerate(jobs):
        G.dsmc_smooth(plans[(N, spec.d_x)], models[k], seed, outs[k])
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    same = all(torch.equal(served[k], outs[k].traj.cpu()) for k in served)
    print(f"# serve plain: {len(jobs) / dt_plain:.1f} jobs/s, served == alone: {same}",
          file=sys.stderr, flush=True)
    g = np.random.default_rng(7)
    sweep = []
    for f in [float(x) for x in args.rates.split(",") if x]:
        rate = f * sat["jobs_per_sec"]
        gaps = g.exponential(1.0 / rate, len(jobs))
        r = run(range(len(jobs)), gaps)
        r.update({"offered_jobs_per_sec": rate, "fraction_of_saturation": f})
        sweep.append(r)
        print(f"# serve rate {rate:.1f}/s: {r['jobs_per_sec']:.1f} jobs/s p50 {r['p50_ms']:.2f} ms "
              f"p99 {r['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    srv.close()
    Ks = np.array([s.K for s, _, _ in jobs])
    res = {"metric": "jobs/sec (serving, continuous batching)", "value": sat["jobs_per_sec"],
           "unit": "jobs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": sat["span_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(jobs)} jobs, SV / 4-D LG 50/50, K ~ lognormal(median 512, "
                                  f"sigma 1) in [2, 16384] (median {int(np.median(Ks))}, max "
                                  f"{int(Ks.max())}), N in {{256, 1024, 4096}}, fp32",
                      "jobs": len(jobs), "sum_pairs": pairs},
           "saturated": sat, "plain_jobs_per_sec": len(jobs) / dt_plain,
           "speedup_vs_plain": sat["jobs_per_sec"] * dt_plain / len(jobs),
           "served_equals_alone": same, "sweep": sweep}
    print(json.dumps(res))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "serve":
        return bench_serve(args)
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
