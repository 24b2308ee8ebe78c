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
# bf16 matrix-core pair rows (d_x = 16, 32): the dot products run on the
# matrix cores; per pair the VALU issues the accumulator start (one v_sub),
# v_exp_f32 (TRANS_SLOTS) and the chunk-sum add.
SLOTS_PER_PAIR_MFMA = 2.0 + TRANS_SLOTS
# dense bf16 matrix-core peak of MI355X, and flops per pair at d_x = 32
BF16_MFMA_PEAK = 2.5e15
# HBM traffic of one pair-row launch of the default workload (K = 4096,
# N = 1024), averaged over the 12 levels: rocprofv3 FETCH_SIZE / WRITE_SIZE,
# each scaled by the same counter's reading for a 256 MiB device copy (see
# profiles/k_rows_sv_K4096_N1024.md).  Reset to None when k_rows changes.
K_ROWS_SV_TRAFFIC_MIB = {"read": 21.89, "write": 89.85}
# Lazy resampling kernel (k_sample_lazy<float, 1>): VALU instructions per
# proposal in its Metropolis-Hastings loop, counted in the gfx950 assembly of
# this source (half a Philox4x64-10 block, pair weight, fp64 exponential: 395
# per loop trip of two proposals); each is priced at one issue slot, so the
# derived peak is an upper bound.
LAZY_VALU_PER_PROPOSAL = 198
# HBM traffic of one k_sample_lazy launch (MH, B = 32) of the default
# workload: rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by the copy calibration
# (see profiles/k_sample_lazy_mh_sv_K4096_N1024.md).  Reset to None when
# k_sample_lazy changes.
LAZY_MH_SV_TRAFFIC_MIB = {"read": 14.00, "write": 8.01}


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
    ap.add_argument("--workload", choices=("sv", "batch", "serve", "highdim", "pgibbs", "lazy"),
                    default="sv",
                    help="sv: one long stochastic-volatility series (default); batch: "
                         "B linear-Gaussian series of uneven length, packed vs one at a time; "
                         "pgibbs: particle Gibbs sweeps of conditional dSMC on the sv series; "
                         "lazy: lazy resampling (MH, rejection) vs exact on the sv series")
    ap.add_argument("--B", type=int, default=512)
    ap.add_argument("--schemes", type=str, default="exact,mh_B8,mh_B32,rs",
                    help="lazy: which runs (exact, mh_B8, mh_B32, rs)")
    ap.add_argument("--model", choices=("sv", "crw"), default="sv",
                    help="lazy: stochastic volatility, or the constrained random walk "
                         "(uniform proposals on [-1, 1], box potential)")
    ap.add_argument("--sigma", type=float, default=0.5, help="lazy --model crw: walk noise")
    ap.add_argument("--jobs", type=int, default=600, help="serving: jobs per arrival run")
    ap.add_argument("--rates", type=str, default="0.25,0.5,0.75,0.9,1.1",
                    help="serving: Poisson arrival rates as fractions of the saturated rate")
    ap.add_argument("--serve-mem-gib", type=int, default=192)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 10 device copies of 256 MiB (HBM counter calibration)")
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
            z = P.leaf_normals(seed, t, N, spec.d_x)
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
    in shared launches, replayed as one hipGraph) against dsmc_smooth called
    once per series (one set of launches per level per series).  Results are
    bit-identical between the two."""
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    N = 256 if args.N == 1024 else args.N
    specs = W.lg1d_batch(args.B)
    Ks = [s.K for s in specs]
    models = [G.Model(s) for s in specs]
    # timed: one hipGraph replay per batch (warm-up: eager + tile tuning, then capture)
    plan = G.Plan(N, 1, max(Ks), max_total_K=sum(Ks), graph=True)
    outs = [G.alloc_output(plan, K) for K in Ks]
    seeds = list(range(1, args.B + 1))
    for _ in range(max(2, args.warmup)):
        G.dsmc_smooth_batch(plan, models, seeds, outs)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 5))
    t0 = time.perf_counter()
    for _ in range(steps):
        G.dsmc_smooth_batch(plan, models, seeds, outs)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / steps
    prof = None
    if not args.no_kernel_events:  # kernel durations: the same batch eagerly with HIP events
        plan_p = G.Plan(N, 1, max(Ks), max_total_K=sum(Ks), profile=True)
        G.dsmc_smooth_batch(plan_p, models, seeds, outs)
        torch.cuda.synchronize()
        G.dsmc_plan_profile(plan_p)
        for _ in range(steps):
            G.dsmc_smooth_batch(plan_p, models, seeds, outs)
        torch.cuda.synchronize()
        prof = G.dsmc_plan_profile(plan_p)
        del plan_p
    # plain: one series at a time
    plan1 = G.Plan(N, 1, max(Ks))
    out1 = G.alloc_output(plan1, max(Ks))
    outs1 = [G.Output(traj=out1.traj[:, :K], logw=out1.logw, log_Z=out1.log_Z,
                      status=out1.status) for K in Ks]
    # one untimed pass: the plan tunes its tile for every level size on first use
    for m, s, o in zip(models, seeds, outs1):
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
    # one untimed pass: each plan tunes its tile for every level size on first use
    for k, (spec, N, seed) in enumerate(jobs):
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


def bench_highdim(args):
    """d_x = 32 linear-Gaussian model (A = 0.95 orth, Q = 0.1 I, d_y = 8,
    R = 0.5 I, RTS proposals), K = 2048, N = 4096: the bf16 matrix-core
    pair-row path (DSMC_BF16), with the fp32 VALU path on the same model
    beside it."""
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    K = 2048 if args.K == 4096 else args.K
    N = 4096 if args.N == 1024 else args.N
    spec = W.lg_highdim(K=K)
    model = G.Model(spec)
    pairs = (K - 1) * N * N
    runs = {}
    for name, prec, steps in (("bf16", G.DSMC_BF16, max(1, min(args.steps, 10))),
                              ("fp32", G.DSMC_FP32, max(1, min(args.steps, 3)))):
        plan = G.Plan(N, spec.d_x, K, precision=prec, profile=not args.no_kernel_events)
        out = G.alloc_output(plan, K)
        for s in range(max(1, args.warmup)):
            G.dsmc_smooth(plan, model, 1000 + s, out)
        torch.cuda.synchronize()
        if not args.no_kernel_events:
            G.dsmc_plan_profile(plan)
        t0 = time.perf_counter()
        for s in range(steps):
            G.dsmc_smooth(plan, model, s + 1, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        status = int(out.status.item())
        if status:
            raise RuntimeError(f"{name}: device status {status}")
        r = {"ms_per_step": dt * 1e3, "pair_evals_per_sec": pairs / dt, "steps": steps,
             "log_Z_last": float(out.log_Z.item())}
        if not args.no_kernel_events:
            prof = G.dsmc_plan_profile(plan)
            r["kernel_ms_per_step"] = {k: v / steps for k, v in prof["ms"].items()}
            r["rows_pairs_per_sec"] = prof["pairs"] / (prof["ms"]["rows"] * 1e-3)
            r["rows_launches"] = prof["launches"]["rows"]
            r["rows_pairs"] = prof["pairs"]
            r["rescued_rows_per_step"] = prof["rescued_rows"] / steps
        runs[name] = r
        print(f"# highdim {name}: {dt * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
        del plan, out
        torch.cuda.empty_cache()
    b = runs["bf16"]
    res = {"metric": "pair-evals/sec", "value": b["pair_evals_per_sec"], "unit": "pair-evals/s",
           "n_gpus": 1, "steps": b["steps"], "warmup": args.warmup, "ms_per_step": b["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": f"linear-Gaussian d_x=32 (d_y=8, A=0.95 orth, Q=0.1I, R=0.5I, "
                                  f"RTS proposals), K={K}, N={N}, one smoother per step",
                      "K": K, "N": N, "d_x": 32,
                      "precision": "bf16 matrix-core dot products, fp32 accumulation and "
                                   "exponentials, fp64 row sums and CDFs"},
           "smoothers_per_sec": 1e3 / b["ms_per_step"], "fp32_valu": runs["fp32"],
           "speedup_vs_fp32": runs["fp32"]["ms_per_step"] / b["ms_per_step"]}
    if "rows_pairs_per_sec" in b:
        ach = b["rows_pairs_per_sec"]
        peak = LANE_OPS_PER_S / SLOTS_PER_PAIR_MFMA
        ms_rows = b["kernel_ms_per_step"]["rows"] * b["steps"]
        res["roofline"] = {"bound": "alu", "kernel": "k_rows_mfma<32,MB>", "achieved": ach / 1e9,
                           "peak": peak / 1e9, "unit": "Gpair/s", "frac": ach / peak,
                           "traffic": None, "avg_launch_ms": ms_rows / max(1, b["rows_launches"]),
                           "pairs_per_launch": b["rows_pairs"] / max(1, b["rows_launches"]),
                           "mfma_utilisation": ach * 2 * spec.d_x / BF16_MFMA_PEAK}
        res["kernel_ms_per_step"] = b["kernel_ms_per_step"]
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(spec, N, args.cpu_seconds)
    print(json.dumps(res))


def bench_pgibbs(args):
    """Particle Gibbs sweeps (Section 3.2) on the stochastic-volatility
    workload: each step is one conditional smoother run (Algorithm 4 at every
    node) with the previous sweep's star in slot 0, then the next star is an
    output trajectory picked uniformly (a device copy).  The model is fixed
    (no parameter update between sweeps).  Beside it: the unconditional
    smoother on the same plan."""
    import numpy as np
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    torch.cuda.set_device(0)
    K, N = args.K, args.N
    spec = W.sv(K)
    model = G.Model(spec)
    plan = G.Plan(N, 1, K, graph=True)
    out = G.alloc_output(plan, K)
    star = torch.tensor(spec.x_true.T.copy(), dtype=torch.float32, device="cuda")
    pick = np.random.default_rng(7)

    def sweep(seed):
        G.dsmc_smooth_conditional(plan, model, seed, star, out)
        j = int(pick.integers(N))
        star.copy_(out.traj[:, :, j])

    for s in range(max(2, args.warmup)):
        sweep(1000 + s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        sweep(s + 1)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    status = int(out.status.item())
    if status:
        raise RuntimeError(f"device status {status}")
    # one more sweep with a known star: it must come back in slot 0
    before = star.clone()
    G.dsmc_smooth_conditional(plan, model, 77, star, out)
    torch.cuda.synchronize()
    if not torch.equal(out.traj[:, :, 0], before):
        raise RuntimeError("star trajectory not kept in slot 0")
    for s in range(max(2, args.warmup)):
        G.dsmc_smooth(plan, model, 1000 + s, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(args.steps):
        G.dsmc_smooth(plan, model, s + 1, out)
    torch.cuda.synchronize()
    dt_plain = (time.perf_counter() - t1) / args.steps
    pairs = (K - 1) * N * N
    res = {"metric": "pair-evals/sec", "value": pairs / dt, "unit": "pair-evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"particle Gibbs sweeps of conditional dSMC, stochastic "
                                  f"volatility, K={K}, N={N}, fixed parameters",
                      "K": K, "N": N, "d_x": 1},
           "sweeps_per_sec": 1.0 / dt, "unconditional_ms_per_step": dt_plain * 1e3,
           "conditional_overhead": dt / dt_plain - 1.0}
    print(json.dumps(res))


def bench_lazy(args):
    """Lazy resampling (Section 4.2) on the stochastic-volatility workload:
    whole smoother runs with Algorithm 7 (Metropolis-Hastings, B steps per
    draw) or Algorithm 8 (rejection) in every combine, beside the exact
    multinomial draw of Algorithm 1.  Lazy runs estimate no log L^N."""
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    torch.cuda.set_device(0)
    K, N = args.K, args.N
    spec = W.sv(K) if args.model == "sv" else W.constrained_rw(K, sigma=args.sigma)
    model = G.Model(spec)
    runs = {}
    wanted = set(args.schemes.split(","))
    for name, scheme, param, steps in (("exact", G.DSMC_RESAMPLE_EXACT, 0, args.steps),
                                       ("mh_B8", G.DSMC_RESAMPLE_MH, 8, args.steps),
                                       ("mh_B32", G.DSMC_RESAMPLE_MH, 32, args.steps),
                                       ("rs", G.DSMC_RESAMPLE_RS, 0,
                                        args.steps if args.model == "crw"
                                        else max(1, min(args.steps, 3)))):
        if name not in wanted:
            continue
        plan = G.Plan(N, 1, K, graph=True, resampling=scheme, lazy_param=param)
        out = G.alloc_output(plan, K)
        for s in range(2):
            G.dsmc_smooth(plan, model, 1000 + s, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            G.dsmc_smooth(plan, model, s + 1, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        runs[name] = {"ms_per_step": dt * 1e3, "steps": steps,
                      "status": int(out.status.item())}
        print(f"# lazy {name}: {dt * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        del plan, out
    if args.model == "crw":  # the rejection run is the one reported
        rs = runs["rs"]
        res = {"metric": "smoothers/sec", "value": 1e3 / rs["ms_per_step"], "unit": "smoothers/s",
               "n_gpus": 1, "steps": rs["steps"], "warmup": 2, "ms_per_step": rs["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic",
               "config": {"workload": f"rejection lazy resampling, constrained random walk "
                                      f"(sigma={args.sigma}, uniform proposals on [-1, 1]), "
                                      f"K={K}, N={N}", "K": K, "N": N, "d_x": 1},
               "runs": runs}
        if "exact" in runs:
            res["speedup_vs_exact"] = runs["exact"]["ms_per_step"] / rs["ms_per_step"]
        print(json.dumps(res))
        return
    mh = runs["mh_B32"]
    res = {"metric": "smoothers/sec", "value": 1e3 / mh["ms_per_step"], "unit": "smoothers/s",
           "n_gpus": 1, "steps": mh["steps"], "warmup": 2, "ms_per_step": mh["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"lazy resampling (Metropolis-Hastings, B=32), stochastic "
                                  f"volatility, K={K}, N={N}", "K": K, "N": N, "d_x": 1},
           "runs": runs}
    if not args.no_kernel_events:
        # the B = 32 run once more, eagerly, with HIP events around every launch
        plan = G.Plan(N, 1, K, profile=True, resampling=G.DSMC_RESAMPLE_MH, lazy_param=32)
        out = G.alloc_output(plan, K)
        for s in range(2):
            G.dsmc_smooth(plan, model, 1000 + s, out)
        torch.cuda.synchronize()
        G.dsmc_plan_profile(plan)
        for s in range(args.steps):
            G.dsmc_smooth(plan, model, s + 1, out)
        prof = G.dsmc_plan_profile(plan)
        launches = prof["launches"]["sample"]
        ms = prof["ms"]["sample"]
        proposals = args.steps * (K - 1) * N * 32
        achieved = proposals / (ms * 1e-3)
        peak = LANE_OPS_PER_S / LAZY_VALU_PER_PROPOSAL
        traffic = None
        if LAZY_MH_SV_TRAFFIC_MIB and (K, N) == (4096, 1024):
            traffic = (LAZY_MH_SV_TRAFFIC_MIB["read"] + LAZY_MH_SV_TRAFFIC_MIB["write"]) * 2 ** 20
        res["roofline"] = {"bound": "alu", "kernel": "k_sample_lazy<float,1>",
                           "achieved": achieved / 1e9, "peak": peak / 1e9,
                           "unit": "Gproposal/s", "frac": achieved / peak, "traffic": traffic,
                           "avg_launch_ms": ms / max(1, launches),
                           "proposals_per_launch": proposals / max(1, launches)}
        res["kernel_ms_per_step"] = {k: v / args.steps for k, v in prof["ms"].items()}
    print(json.dumps(res))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the smoother runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        import torch
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 2 * x.numel() * 4, "launches": 10}))
        return
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "highdim":
        return bench_highdim(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "pgibbs":
        return bench_pgibbs(args)
    if args.workload == "lazy":
        return bench_lazy(args)
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W

    torch.cuda.set_device(0)
    K, N = args.K, args.N
    spec = W.sv(K)
    model = G.Model(spec)
    # timed steps: the plan replays one hipGraph per step (first warm-up call
    # runs eagerly and tunes the tiles, the second captures)
    plan = G.Plan(N, 1, K, graph=True)
    out = G.alloc_output(plan, K)
    for s in range(max(2, args.warmup)):
        G.dsmc_smooth(plan, model, 1000 + s, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        G.dsmc_smooth(plan, model, s + 1, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    status = int(out.status.item())
    if status:
        raise RuntimeError(f"device status {status}")
    prof = None
    if not args.no_kernel_events:
        # the same steps once more, eagerly, with HIP events around every launch
        plan_p = G.Plan(N, 1, K, profile=True)
        for s in range(max(1, args.warmup)):
            G.dsmc_smooth(plan_p, model, 1000 + s, out)
        torch.cuda.synchronize()
        G.dsmc_plan_profile(plan_p)  # drop the warm-up records
        t1 = time.perf_counter()
        for s in range(args.steps):
            G.dsmc_smooth(plan_p, model, s + 1, out)
        torch.cuda.synchronize()
        dt_ev = (time.perf_counter() - t1) / args.steps
        prof = G.dsmc_plan_profile(plan_p)
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
    if prof is not None:
        res["ms_per_step_with_kernel_events"] = dt_ev * 1e3
        n_rows = prof["launches"]["rows"]
        ms_rows = prof["ms"]["rows"]
        achieved = prof["pairs"] / (ms_rows * 1e-3)
        peak = LANE_OPS_PER_S / SLOTS_PER_PAIR
        traffic = None
        if K_ROWS_SV_TRAFFIC_MIB and (K, N) == (4096, 1024):
            traffic = (K_ROWS_SV_TRAFFIC_MIB["read"] + K_ROWS_SV_TRAFFIC_MIB["write"]) * 2 ** 20
        nodes = K - 1
        Npad = (N + 31) // 32 * 32
        algo_bytes = nodes * (Npad * 2 * 4 + Npad * 4 + N * ((Npad // 32 + 3) // 4 * 4) * 4
                              + N * 8) / max(1, n_rows / args.steps)
        res["roofline"] = {"bound": "alu", "kernel": "k_rows<float,1,RPL>",
                           "achieved": achieved / 1e9, "peak": peak / 1e9, "unit": "Gpair/s",
                           "frac": achieved / peak, "traffic": traffic,
                           "traffic_algorithmic": algo_bytes,
                           "avg_launch_ms": ms_rows / max(1, n_rows),
                           "pairs_per_launch": prof["pairs"] / max(1, n_rows)}
        res["kernel_ms_per_step"] = {k: v / args.steps for k, v in prof["ms"].items()}
        res["rescued_rows_per_step"] = prof["rescued_rows"] / args.steps
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(spec, N, args.cpu_seconds)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
