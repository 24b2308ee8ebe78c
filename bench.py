"""Benchmark of the dSMC smoother on one MI355X.

Default run (`python bench.py`): the headline workload, stochastic-volatility
model (mu = -1, rho = 0.95, sigma = 0.3), K = 4096 time points (T = 4096 in
the configs' notation), N = 1024 particles, fp32 pair weights, data simulated
from the model with a fixed seed.  One step is one whole smoother run (leaves,
12 tree levels, output) on resident inputs, through the C ABI.  The same JSON
line carries, under "workloads", shorter runs of the other configurations:
the 512-series batch, the d_x = 32 bf16 matrix-core precision workload, the
serving mix, and rejection lazy resampling on the constrained random walk.

Output: one JSON line.  `value` = algorithmic pair evaluations per second,
(K-1) N^2 per step.  `roofline` prices the dominant kernel (the pair-row
kernel) against the VALU issue rate of the chip; `cpu_baseline` times the fp64
oracle on a bounded sample of the same workload on the host cores (one core,
then all cores of the process's CPU share).

`--workload X` runs one configuration alone in more detail; `--issue-rates`
runs the VALU issue-rate microbenchmark behind the roofline's pricing.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.32e12 lane-instructions/s
# for single-rate VALU work (fp32 add/sub/fma without packed math): one wave64
# instruction per SIMD every four cycles.
LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# VALU issue slots per pair evaluation in the pair-row kernel (d_x = 1):
# v_sub, v_fma, v_add at one slot each, plus v_exp_f32 at TRANS_SLOTS slots.
# v_exp_f32 issues at half the rate of v_fma_f32 on gfx950 and does not
# co-issue with it (paper_2202_02264_amd/microbench/issue_rates.hip, run by
# `bench.py --issue-rates`; profiles/valu_issue_rates.md).  The line also
# reports the fraction with every instruction at one slot (4 per pair).
TRANS_SLOTS = 2.0
SLOTS_PER_PAIR = 3.0 + TRANS_SLOTS
SLOTS_PER_PAIR_SINGLE = 4.0
# bf16 matrix-core pair rows (d_x = 16, 32): the dot products run on the
# matrix cores; per pair the VALU issues the accumulator start (one v_sub),
# v_exp_f32 (TRANS_SLOTS) and the chunk-sum add.
SLOTS_PER_PAIR_MFMA = 2.0 + TRANS_SLOTS
# dense bf16 matrix-core peak of MI355X
BF16_MFMA_PEAK = 2.5e15
# HBM traffic of one pair-row launch of the headline workload (K = 4096,
# N = 1024), averaged over the 12 levels: rocprofv3 FETCH_SIZE / WRITE_SIZE,
# each scaled by the same counter's reading for a 256 MiB device copy
# (profiles/k_rows_sv_K4096_N1024.md).  `src` is the sha256 prefix of the
# kernel source the counters were taken on; when the source differs the
# figure is reported as null.
K_ROWS_SV_TRAFFIC = {"src": "ab4d91511ce3b5d6", "read_MiB": 10.01, "write_MiB": 57.04}
# Lazy resampling kernel (k_sample_lazy<float, 1>): VALU instructions per
# proposal in its Metropolis-Hastings loop, counted in the gfx950 assembly of
# this source (half a Philox4x64-10 block, pair weight, fp64 exponential: 395
# per loop trip of two proposals); each is priced at one issue slot, so the
# derived peak is an upper bound.
LAZY_VALU_PER_PROPOSAL = 198
KERNEL_SOURCES = ("paper_2202_02264_amd/csrc/dsmc_kernels_impl.h",
                  "paper_2202_02264_amd/csrc/dsmc_device.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--K", type=int, default=4096)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="wall-clock budget of each oracle baseline sample, per core count "
                         "(0 = skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the other configurations")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the steps without per-kernel HIP events")
    ap.add_argument("--workload", choices=("sv", "batch", "serve", "highdim", "pgibbs", "lazy"),
                    default="sv",
                    help="sv: the headline series (default, with the other configurations "
                         "under 'workloads'); batch: 512 linear-Gaussian series packed vs one at "
                         "a time; highdim: d_x = 32 bf16 matrix-core pair rows; serve: "
                         "continuous-batching server; pgibbs: particle Gibbs sweeps of "
                         "conditional dSMC; lazy: lazy resampling vs exact")
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
    ap.add_argument("--issue-rates", action="store_true",
                    help="only run the VALU issue-rate microbenchmark")
    return ap.parse_args()


# ----------------------------------------------------------------- CPU baseline

def host_cores() -> int:
    """Cores of this process's CPU share (at most 16, a GPU machine's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _oracle_worker(job):
    """Oracle combines (Algorithm 1 with Algorithm 2's leaves) on the boundaries
    c = first, first + stride, ... of the spec until `budget` seconds pass,
    single-threaded.  Returns (pairs, wall seconds, combines)."""
    spec, N, first, stride, budget = job
    from threadpoolctl import threadpool_limits

    from oracle import dsmc as D
    from oracle import philox as P
    from oracle import ssm
    with threadpool_limits(1):
        t0 = time.perf_counter()
        done = 0
        c = first
        while time.perf_counter() - t0 < budget and c < spec.K:
            xs = [ssm.proposal_draw(spec, t, P.leaf_normals(1, t, N, spec.d_x)) for t in (c - 1, c)]
            lws = [D.normalise(D.leaf_logweights(spec, t, x))[0] for t, x in zip((c - 1, c), xs)]
            u1, u2 = P.combine_uniforms(1, c, N)
            D.combine(spec, c, xs[0], xs[1], lws[0], lws[1], u1, u2)
            done += 1
            c += stride
        wall = time.perf_counter() - t0
    return done * N * N, wall, done


def cpu_baseline(spec, N: int, budget_s: float, label: str) -> dict:
    """The fp64 oracle's combine on level-0 boundaries of the workload: one
    single-threaded process, then one single-threaded process per host core on
    disjoint boundaries, each for `budget_s` seconds (pair-evals/s = all pairs
    done / the longest wall time)."""
    import multiprocessing as mp
    cores = host_cores()
    single = _oracle_worker((spec, N, 1, 2, budget_s))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(spec, N, 1 + 2 * i, 2 * cores, budget_s)
                                        for i in range(cores)])
    pairs = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return {"value": pairs / wall, "unit": "pair-evals/s", "cores": cores, "kind": "oracle",
            "host_cpus": os.cpu_count(),
            "sample": f"{sum(r[2] for r in res)} level-0 combines of {label} (leaf draws and "
                      f"weights of both times, N x N pair weights, N = {N} two-stage draws "
                      f"each), fp64 numpy, one single-threaded process per core, "
                      f"{wall:.1f} s wall",
            "single_core": {"value": single[0] / single[1], "cores": 1,
                            "sample": f"{single[2]} combines, {single[1]:.1f} s wall"}}


# ------------------------------------------------------------------ helpers

def _pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q)) if len(a) else float("nan")


def _timed(G, torch, plan, model, out, steps, warmup, seed0=1):
    for s in range(warmup):
        G.dsmc_smooth(plan, model, 1000 + s, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        G.dsmc_smooth(plan, model, seed0 + s, out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _rows_roofline(prof, steps, slots, kernel, single_slots=None, extra=None):
    """Pair-row kernel against the VALU issue rate: achieved pairs/s over its
    launches (HIP events), peak = lane-instructions/s / slots per pair."""
    n_rows = prof["launches"]["rows"]
    ms_rows = prof["ms"]["rows"]
    achieved = prof["pairs"] / (ms_rows * 1e-3)
    peak = LANE_OPS_PER_S / slots
    r = {"bound": "alu", "kernel": kernel, "achieved": achieved / 1e9, "peak": peak / 1e9,
         "unit": "Gpair/s", "frac": achieved / peak, "traffic": None,
         "avg_launch_ms": ms_rows / max(1, n_rows),
         "pairs_per_launch": prof["pairs"] / max(1, n_rows),
         "slots_per_pair": slots}
    if single_slots:
        r["frac_one_slot_per_instruction"] = achieved / (LANE_OPS_PER_S / single_slots)
    if extra:
        r.update(extra)
    return r


def _profile_run(G, torch, N, dx, K, model, steps, warmup, **plan_kw):
    """The same steps eagerly with HIP events around every launch."""
    plan = G.Plan(N, dx, K, profile=True, **plan_kw)
    out = G.alloc_output(plan, K)
    for s in range(max(1, warmup)):
        G.dsmc_smooth(plan, model, 1000 + s, out)
    torch.cuda.synchronize()
    G.dsmc_plan_profile(plan)  # drop the warm-up records
    t0 = time.perf_counter()
    for s in range(steps):
        G.dsmc_smooth(plan, model, s + 1, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = G.dsmc_plan_profile(plan)
    return prof, dt


# ----------------------------------------------------------------- headline

def bench_sv(args) -> dict:
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
    dt = _timed(G, torch, plan, model, out, args.steps, max(2, args.warmup))
    status = int(out.status.item())
    if status:
        raise RuntimeError(f"device status {status}")
    pairs = (K - 1) * N * N
    res = {
        "metric": "pair-evals/sec", "value": pairs / dt, "unit": "pair-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"stochastic volatility, K={K} time points, N={N} particles, "
                               "one smoother per step", "K": K, "N": N, "d_x": 1,
                   "precision": "fp32 pair weights, fp64 sums and CDFs",
                   "weighting": spec.weighting, "data_seed": W.DATA_SEED},
        "smoothers_per_sec": 1.0 / dt,
        "pair_evals_T_log2T_N2_per_sec": K * math.log2(K) * N * N / dt,
    }
    if not args.no_kernel_events:
        ev_steps = min(args.steps, 20)
        prof, dt_ev = _profile_run(G, torch, N, 1, K, model, ev_steps, args.warmup)
        n_rows = prof["launches"]["rows"]
        nodes = K - 1
        Npad = (N + 31) // 32 * 32
        NcP = (Npad // 32 + 7) // 8 * 8
        algo_bytes = nodes * (Npad * 2 * 4 + Npad * 4 + N * NcP * 4 + N * 8) / max(1, n_rows / ev_steps)
        src = kernel_source_hash()
        traffic = None
        if (K, N) == (4096, 1024) and K_ROWS_SV_TRAFFIC["src"] == src:
            traffic = (K_ROWS_SV_TRAFFIC["read_MiB"] + K_ROWS_SV_TRAFFIC["write_MiB"]) * 2 ** 20
        res["ms_per_step_with_kernel_events"] = dt_ev * 1e3
        res["roofline"] = _rows_roofline(
            prof, ev_steps, SLOTS_PER_PAIR, "k_rows<float,1,RPL>", SLOTS_PER_PAIR_SINGLE,
            {"traffic": traffic, "traffic_algorithmic": algo_bytes, "kernel_source": src,
             "traffic_source": K_ROWS_SV_TRAFFIC["src"]})
        res["kernel_ms_per_step"] = {k: v / ev_steps for k, v in prof["ms"].items()}
        ms_comb = (prof["ms"]["rows"] + prof["ms"]["sample"]) / ev_steps
        res["combine"] = {
            "ms_per_step": ms_comb, "pairs_per_sec": pairs / (ms_comb * 1e-3),
            "frac": pairs / (ms_comb * 1e-3) / (LANE_OPS_PER_S / SLOTS_PER_PAIR),
            "frac_one_slot_per_instruction":
                pairs / (ms_comb * 1e-3) / (LANE_OPS_PER_S / SLOTS_PER_PAIR_SINGLE),
            "note": "pair rows + sampling kernels of every level against the pair-row roofline"}
        draws = nodes * N
        ms_s = prof["ms"]["sample"] / ev_steps
        res["sample_kernel"] = {"ms_per_step": ms_s, "draws_per_sec": draws / (ms_s * 1e-3),
                                "launches_per_step": prof["launches"]["sample"] / ev_steps}
        res["rescued_rows_per_step"] = prof["rescued_rows"] / ev_steps
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(spec, N, args.cpu_seconds, "the same workload")
    return res


# ------------------------------------------------------------------- batch

def bench_batch(args, quick=False) -> dict:
    """B independent 1-D linear-Gaussian series (A ~ U[0.5, 0.99], Q, R ~ U[0.1, 2],
    K ~ U{64..8192}), N = 256: dsmc_smooth_batch (every level of every series
    in shared launches, replayed as one hipGraph) against dsmc_smooth called
    once per series (one set of launches per level per series).  Results are
    bit-identical between the two."""
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    N = 256 if (quick or args.N == 1024) else args.N
    specs = W.lg1d_batch(args.B)
    Ks = [s.K for s in specs]
    models = [G.Model(s) for s in specs]
    plan = G.Plan(N, 1, max(Ks), max_total_K=sum(Ks), graph=True)
    outs = [G.alloc_output(plan, K) for K in Ks]
    seeds = list(range(1, args.B + 1))
    for _ in range(5):  # eager, capture, replays: the timed calls all replay the graph
        G.dsmc_smooth_batch(plan, models, seeds, outs)
    torch.cuda.synchronize()
    steps = 8
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
        for _ in range(2):
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
           "n_gpus": 1, "steps": steps, "warmup": 5, "ms_per_step": dt_b * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{args.B} linear-Gaussian series, K ~ U{{64..8192}} "
                                  f"(sum {sum(Ks)}), N={N}, one batch per step",
                      "B": args.B, "N": N, "sum_K": sum(Ks)},
           "plain_smoothers_per_sec": args.B / dt_p, "plain_ms_per_batch": dt_p * 1e3,
           "speedup_vs_plain": dt_p / dt_b, "pair_evals_per_sec": pairs / dt_b}
    if prof:
        res["roofline"] = _rows_roofline(prof, 2, SLOTS_PER_PAIR, "k_rows<float,1,RPL>",
                                         SLOTS_PER_PAIR_SINGLE)
        res["kernel_ms_per_step"] = {k: v / 2 for k, v in prof["ms"].items()}
    if args.cpu_seconds > 0:
        long = specs[max(range(len(specs)), key=lambda i: Ks[i])]
        res["cpu_baseline"] = cpu_baseline(long, N, min(args.cpu_seconds, 3.0),
                                           f"the longest series (K={long.K})")
    return res


# ------------------------------------------------------------------ serving

def bench_serve(args, quick=False) -> dict:
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
        for i in ids:
            G.dsmc_job_release(srv, i)
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
    rates = [0.5] if quick else [float(x) for x in args.rates.split(",") if x]
    for f in rates:
        rate = f * sat["jobs_per_sec"]
        gaps = g.exponential(1.0 / rate, len(jobs))
        r = run(range(len(jobs)), gaps)
        r.update({"offered_jobs_per_sec": rate, "fraction_of_saturation": f})
        sweep.append(r)
        print(f"# serve rate {rate:.1f}/s: {r['jobs_per_sec']:.1f} jobs/s p50 {r['p50_ms']:.2f} ms "
              f"p99 {r['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    srv.close()
    Ks = np.array([s.K for s, _, _ in jobs])
    return {"metric": "jobs/sec (serving, continuous batching)", "value": sat["jobs_per_sec"],
            "unit": "jobs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": sat["span_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{len(jobs)} jobs, SV / 4-D LG 50/50, K ~ lognormal(median "
                                   f"512, sigma 1) in [2, 16384] (median {int(np.median(Ks))}, "
                                   f"max {int(Ks.max())}), N in {{256, 1024, 4096}}, fp32",
                       "jobs": len(jobs), "sum_pairs": pairs},
            "saturated": sat, "plain_jobs_per_sec": len(jobs) / dt_plain,
            "speedup_vs_plain": sat["jobs_per_sec"] * dt_plain / len(jobs),
            "served_equals_alone": same, "sweep": sweep}


# ------------------------------------------------------------- precision

def bench_highdim(args, quick=False) -> dict:
    """d_x = 32 linear-Gaussian model (A = 0.95 orth, Q = 0.1 I, d_y = 8,
    R = 0.5 I), K = 2048, N = 4096: each step computes the RTS proposals on the
    device (Algorithm 5: parallel-in-time Kalman filter and RTS smoother) and
    runs the smoother with the bf16 matrix-core pair rows (DSMC_BF16); the fp32
    VALU path on the same model beside it."""
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    K = 2048 if (quick or args.K == 4096) else args.K
    N = 4096 if (quick or args.N == 1024) else args.N
    spec = W.lg_highdim(K=K)
    model = G.Model(spec)
    pairs = (K - 1) * N * N
    # Algorithm 5 on the device: every step recomputes the RTS proposals with
    # the parallel-in-time Kalman filter and smoother before the smoother run
    stream = torch.cuda.current_stream()
    G.dsmc_model_gaussian_proposals(model, stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(3):
        G.dsmc_model_gaussian_proposals(model, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    pit_ms = ev0.elapsed_time(ev1) / 3
    runs = {}
    for name, prec, steps in (("bf16", G.DSMC_BF16, 5 if quick else 10),
                              ("fp32", G.DSMC_FP32, 2 if quick else 3)):
        plan = G.Plan(N, spec.d_x, K, precision=prec, graph=True)
        out = G.alloc_output(plan, K)
        for s in range(2):
            G.dsmc_model_gaussian_proposals(model, stream)
            G.dsmc_smooth(plan, model, 1000 + s, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            G.dsmc_model_gaussian_proposals(model, stream)
            G.dsmc_smooth(plan, model, s + 1, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        status = int(out.status.item())
        if status:
            raise RuntimeError(f"{name}: device status {status}")
        r = {"ms_per_step": dt * 1e3, "pair_evals_per_sec": pairs / dt, "steps": steps,
             "log_Z_last": float(out.log_Z.item())}
        del plan, out
        if not args.no_kernel_events:
            prof, _ = _profile_run(G, torch, N, spec.d_x, K, model, 2, 1, precision=prec)
            r["kernel_ms_per_step"] = {k: v / 2 for k, v in prof["ms"].items()}
            r["prof"] = prof
            r["rescued_rows_per_step"] = prof["rescued_rows"] / 2
        runs[name] = r
        print(f"# highdim {name}: {dt * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    b = runs["bf16"]
    res = {"metric": "pair-evals/sec", "value": b["pair_evals_per_sec"], "unit": "pair-evals/s",
           "n_gpus": 1, "steps": b["steps"], "warmup": 2, "ms_per_step": b["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": f"linear-Gaussian d_x=32 (d_y=8, A=0.95 orth, Q=0.1I, R=0.5I, "
                                  f"RTS proposals), K={K}, N={N}, one smoother per step",
                      "K": K, "N": N, "d_x": 32,
                      "precision": "bf16 matrix-core dot products, fp32 accumulation and "
                                   "exponentials, fp64 row sums and CDFs"},
           "smoothers_per_sec": 1e3 / b["ms_per_step"],
           "speedup_vs_fp32": runs["fp32"]["ms_per_step"] / b["ms_per_step"],
           "proposals_ms_per_step": pit_ms,
           "proposals": "RTS smoothing marginals recomputed every step on the device by the "
                        "parallel-in-time Kalman filter and RTS smoother (Algorithm 5), "
                        "included in ms_per_step"}
    if "prof" in b:
        prof = b.pop("prof")
        ach = prof["pairs"] / (prof["ms"]["rows"] * 1e-3)
        res["roofline"] = _rows_roofline(
            prof, 2, SLOTS_PER_PAIR_MFMA, "k_rows_mfma<32,MB>", None,
            {"mfma_utilisation": ach * 2 * spec.d_x / BF16_MFMA_PEAK})
        res["kernel_ms_per_step"] = b["kernel_ms_per_step"]
        f = runs["fp32"].pop("prof")
        runs["fp32"]["roofline"] = _rows_roofline(f, 2, 2.0 * 32 + 2.0 + TRANS_SLOTS,
                                                  "k_rows<float,32,RPL>")
    res["fp32_valu"] = runs["fp32"]
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(spec, N, min(args.cpu_seconds, 3.0),
                                           "the same workload")
    return res


# ------------------------------------------------------------ particle Gibbs

def bench_pgibbs(args) -> dict:
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
    dt_plain = _timed(G, torch, plan, model, out, args.steps, max(2, args.warmup))
    pairs = (K - 1) * N * N
    return {"metric": "pair-evals/sec", "value": pairs / dt, "unit": "pair-evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"particle Gibbs sweeps of conditional dSMC, stochastic "
                                   f"volatility, K={K}, N={N}, fixed parameters",
                       "K": K, "N": N, "d_x": 1},
            "sweeps_per_sec": 1.0 / dt, "unconditional_ms_per_step": dt_plain * 1e3,
            "conditional_overhead": dt / dt_plain - 1.0}


# ------------------------------------------------------------------- lazy

def bench_lazy(args, quick=False) -> dict:
    """Lazy resampling (Section 4.2): whole smoother runs with Algorithm 7
    (Metropolis-Hastings, B steps per draw) or Algorithm 8 (rejection) in every
    combine, beside the exact multinomial draw of Algorithm 1.  Lazy runs
    estimate no log L^N.  Model: stochastic volatility, or the constrained
    random walk of Section 5.3 (uniform proposals, box potential)."""
    import torch

    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W
    torch.cuda.set_device(0)
    model_name = "crw" if quick else args.model
    K = args.K
    N = 4096 if quick else args.N
    spec = W.sv(K) if model_name == "sv" else W.constrained_rw(K, sigma=args.sigma)
    model = G.Model(spec)
    runs = {}
    wanted = {"exact", "rs"} if quick else set(args.schemes.split(","))
    steps_all = 5 if quick else args.steps
    for name, scheme, param, steps in (("exact", G.DSMC_RESAMPLE_EXACT, 0, steps_all),
                                       ("mh_B8", G.DSMC_RESAMPLE_MH, 8, steps_all),
                                       ("mh_B32", G.DSMC_RESAMPLE_MH, 32, steps_all),
                                       ("rs", G.DSMC_RESAMPLE_RS, 0,
                                        steps_all if model_name == "crw"
                                        else max(1, min(steps_all, 3)))):
        if name not in wanted:
            continue
        plan = G.Plan(N, 1, K, graph=True, resampling=scheme, lazy_param=param)
        out = G.alloc_output(plan, K)
        dt = _timed(G, torch, plan, model, out, steps, 2)
        runs[name] = {"ms_per_step": dt * 1e3, "steps": steps, "status": int(out.status.item())}
        print(f"# lazy {name}: {dt * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        del plan, out
    if model_name == "crw":  # the rejection run is the one reported
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
        return res
    mh = runs["mh_B32"]
    res = {"metric": "smoothers/sec", "value": 1e3 / mh["ms_per_step"], "unit": "smoothers/s",
           "n_gpus": 1, "steps": mh["steps"], "warmup": 2, "ms_per_step": mh["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"lazy resampling (Metropolis-Hastings, B=32), stochastic "
                                  f"volatility, K={K}, N={N}", "K": K, "N": N, "d_x": 1},
           "runs": runs}
    if not args.no_kernel_events:
        prof, _ = _profile_run(G, torch, N, 1, K, model, args.steps, 2,
                               resampling=G.DSMC_RESAMPLE_MH, lazy_param=32)
        launches = prof["launches"]["sample"]
        ms = prof["ms"]["sample"]
        proposals = args.steps * (K - 1) * N * 32
        achieved = proposals / (ms * 1e-3)
        peak = LANE_OPS_PER_S / LAZY_VALU_PER_PROPOSAL
        res["roofline"] = {"bound": "alu", "kernel": "k_sample_lazy<float,1>",
                           "achieved": achieved / 1e9, "peak": peak / 1e9,
                           "unit": "Gproposal/s", "frac": achieved / peak, "traffic": None,
                           "avg_launch_ms": ms / max(1, launches),
                           "proposals_per_launch": proposals / max(1, launches)}
        res["kernel_ms_per_step"] = {k: v / args.steps for k, v in prof["ms"].items()}
    return res


# --------------------------------------------------------------------- main

def issue_rates() -> dict:
    exe = os.path.join(ROOT, "paper_2202_02264_amd", "issue_rates")
    if not os.path.exists(exe):
        raise SystemExit(f"{exe} is not built; run __graft_entry__.build()")
    r = subprocess.run([exe], capture_output=True, text=True, check=True)
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.issue_rates:
        print(json.dumps(issue_rates()))
        return
    if args.copy_calibration:
        import torch
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 2 * x.numel() * 4, "launches": 10}))
        return
    single = {"serve": bench_serve, "highdim": bench_highdim, "batch": bench_batch,
              "pgibbs": bench_pgibbs, "lazy": bench_lazy}
    if args.workload in single:
        print(json.dumps(single[args.workload](args)))
        return
    res = bench_sv(args)
    if not args.no_extras:
        extras = {}
        for name, fn in (("batch", bench_batch), ("highdim", bench_highdim),
                         ("serve", bench_serve), ("lazy_crw", bench_lazy)):
            t0 = time.perf_counter()
            extras[name] = fn(args, quick=True)
            extras[name]["wall_s"] = time.perf_counter() - t0
            print(f"# {name} done in {extras[name]['wall_s']:.1f} s", file=sys.stderr, flush=True)
        res["workloads"] = extras
    print(json.dumps(res))


if __name__ == "__main__":
    main()
