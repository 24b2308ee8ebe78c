"""GPU parity: the HIP smoother (through the C ABI) against the fp64 oracle.

Tolerances: log-weights, row log-sums and increments within 1e-5 relative
(|d| <= 1e-5 max(1, |ref|)) for the fp32 path and 1e-10 for the fp64 path;
ancestry indices bit-exact except for draws whose uniform lies within 1e-6 of
a boundary of the oracle's CDF (the fraction is printed).  Comparisons are
teacher-forced: at each level the oracle gets the GPU's particles and weights.
"""
import numpy as np
import pytest

from oracle import dsmc as D
from paper_2202_02264_amd import workloads as W

from parity import TOL32, TOL64, check_leaves, log, run_gpu, teacher_forced

pytestmark = pytest.mark.gpu


def _lg_dx(dx, K, seed=5):
    g = np.random.Generator(np.random.Philox(seed))
    F = 0.8 * W.random_orthogonal(dx, g)
    return W.lg(K, F, 0.7 * np.eye(dx), np.eye(1, dx) + 0.3, np.eye(1) * 0.8, np.zeros(dx),
                np.eye(dx) * 1.5, seed=seed, proposal="prior", name=f"lg(d_x={dx},K={K})")


CASES = {
    # name: (spec builder, N)
    "sv_ragged": (lambda: W.sv(300, seed=11), 256),
    "sv_boundary_obs": (lambda: W.sv(129, seed=12, weighting="boundary_obs"), 128),
    "lg1d_n100": (lambda: W.lg1d(64, seed=13), 100),
    "lg1d_n33_k37": (lambda: W.lg1d(37, A=0.95, Q=0.3, R=2.0, seed=14), 33),
    "lg4d": (lambda: W.lg4d(40, seed=15), 128),
    "lg3d_padded": (lambda: _lg_dx(3, 21), 64),
    "lg2d_boundary": (lambda: _lg_dx(2, 50).with_weighting("boundary_obs"), 96),
    "sv_n1": (lambda: W.sv(17, seed=16), 1),
    "sv_n4096": (lambda: W.sv(5, seed=17), 4096),
    "sv_k2": (lambda: W.sv(2, seed=18), 512),
    # d_x >= 8: row sums relative to per-row shifts
    "lg8d": (lambda: _lg_dx(8, 24), 160),
    "lg32d_fp32": (lambda: W.lg_highdim(K=20, seed=19), 256),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_teacher_forced_parity(case):
    build, N = CASES[case]
    spec = build()
    seed = 1000 + len(case)
    g = run_gpu(spec, N, seed)
    assert g["status"][0] == 0
    check_leaves(spec, N, seed, g, TOL32)
    rep = teacher_forced(spec, N, seed, g, TOL32)
    log(f"{case}: {rep.summary()}")
    assert rep.mismatches_outside_band == 0, rep.worst[:5]


def test_fp64_end_to_end_correctness_workload():
    """LG-1D K = 32, N = 64 in fp64: the whole run equals the oracle's own
    (no teacher forcing): every index, the trajectories and log L^N."""
    spec = W.c1_lg1d()
    N, seed = 64, 7
    g = run_gpu(spec, N, seed, precision="fp64")
    ref = D.smooth(spec, N, seed)
    assert g["status"][0] == 0
    np.testing.assert_array_equal(g["ancestry"], ref.ancestry)
    np.testing.assert_array_equal(g["index"], ref.idx)
    np.testing.assert_allclose(g["traj"][0], ref.x[:, :, 0], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(g["logZ_inc"], ref.Zc, rtol=TOL64, atol=TOL64)
    assert abs(g["log_Z"][0] - ref.logZ) <= TOL64 * max(1.0, abs(ref.logZ))
    rep = teacher_forced(spec, N, seed, g, TOL64)
    assert rep.mismatches == 0


@pytest.mark.parametrize("weighting", ["leaf_obs", "boundary_obs"])
def test_fp64_end_to_end_many_seeds(weighting):
    """fp64, ragged K, several seeds: bit-exact ancestry against the oracle."""
    spec = W.sv(45, seed=3, weighting=weighting)
    for seed in (1, 2, 3):
        g = run_gpu(spec, 48, seed, precision="fp64")
        ref = D.smooth(spec, 48, seed)
        np.testing.assert_array_equal(g["ancestry"], ref.ancestry)
        assert abs(g["log_Z"][0] - ref.logZ) <= TOL64 * max(1.0, abs(ref.logZ))


def test_headline_workload_sampled():
    """The benchmarked workload (SV, K = 4096, N = 1024, fp32, bench's launch
    configuration): leaves in full, then teacher-forced parity on every node of
    the top five levels and 12 nodes of each lower level."""
    spec = W.c2_sv()
    N, seed = 1024, 1
    g = run_gpu(spec, N, seed)
    assert g["status"][0] == 0
    check_leaves(spec, N, seed, g, TOL32)
    rng = np.random.default_rng(0)
    chosen = set()
    for l, level in enumerate(D.schedule(spec.K)):
        cs = [c for (_, c, _) in level]
        if len(cs) <= 16:
            chosen.update(cs)
        else:
            chosen.update(int(v) for v in rng.choice(cs, 12, replace=False))
    rep = teacher_forced(spec, N, seed, g, TOL32, select=lambda a, c, b: c in chosen)
    log(f"headline: {rep.summary()}")
    assert rep.mismatches_outside_band == 0, rep.worst[:5]


def test_single_time_point():
    spec = W.sv(1, seed=4)
    g = run_gpu(spec, 300, 9)
    np.testing.assert_array_equal(g["traj"], g["leaf_x"])
    np.testing.assert_array_equal(g["logw"], g["leaf_logw"][0])
    assert g["log_Z"][0] == g["leaf_logL"][0]
    check_leaves(spec, 300, 9, g, TOL32)


@pytest.mark.parametrize("N", [64, 512])
def test_underflow_rescue_rows(N):
    """Consecutive proposal means two units apart with transition sd 0.1: every
    pair weight underflows fp32 (about -290 in log2 units), so every row goes
    through the rescue path (N = 512: more rows than one rescue pass takes);
    results still match the oracle."""
    K = 24 if N == 64 else 9
    qm = np.where(np.arange(K) % 2 == 0, 0.0, 2.0)[:, None]
    spec = W.lg1d(K, A=1.0, Q=0.01, R=1.0, seed=21)
    spec.q_mean = qm.astype(float)
    spec.q_chol = np.full((K, 1, 1), 0.05)
    g = run_gpu(spec, N, 5)
    assert g["status"][0] == 0
    rep = teacher_forced(spec, N, 5, g, TOL32)
    log(f"rescue: {rep.summary()}")
    assert rep.mismatches_outside_band == 0, rep.worst[:5]


@pytest.mark.parametrize("case", ["sv_ragged", "lg4d", "lg8d", "lg32d_fp32", "sv_n4096"])
def test_rescue_path_parity(case):
    """DSMC_PLAN_RESCUE_ALL sends every row through the path taken by rows whose
    sum leaves the fp32 range (exact row maximum, chunk sums recomputed into
    their own buffer, draws through them); results still match the oracle."""
    build, N = CASES[case]
    spec = build()
    seed = 2000 + len(case)
    g = run_gpu(spec, N, seed, rescue_all=True)
    assert g["status"][0] == 0
    rep = teacher_forced(spec, N, seed, g, TOL32)
    log(f"rescue-all {case}: {rep.summary()}")
    assert rep.mismatches_outside_band == 0, rep.worst[:5]


def test_rescue_path_fp64_end_to_end():
    spec = W.c1_lg1d()
    g = run_gpu(spec, 64, 7, precision="fp64", rescue_all=True)
    ref = D.smooth(spec, 64, 7)
    np.testing.assert_array_equal(g["ancestry"], ref.ancestry)
    assert abs(g["log_Z"][0] - ref.logZ) <= TOL64 * max(1.0, abs(ref.logZ))


def test_degenerate_leaf_flagged():
    spec = W.lg1d(20, seed=22)
    spec.y = spec.y.copy()
    spec.y[7, 0] = np.inf
    g = run_gpu(spec, 64, 3)
    assert g["status"][0] & 1
    assert g["log_Z"][0] == -np.inf
    assert np.all(np.isfinite(g["traj"]))
    assert g["ancestry"].min() >= 0 and g["ancestry"].max() < 64


def test_deterministic():
    spec = W.sv(200, seed=23)
    a = run_gpu(spec, 256, 77)
    b = run_gpu(spec, 256, 77)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_batch_equals_single():
    """dsmc_smooth_batch packs every level of every series into shared launches;
    each series' results equal its own dsmc_smooth run bit for bit."""
    import torch
    from paper_2202_02264_amd import dsmc as G
    specs = [W.lg1d(K, seed=30 + K) for K in (70, 1, 33, 128, 2)]
    seeds = [11, 12, 13, 14, 15]
    N = 128
    plan = G.Plan(N, 1, max_K=128, max_total_K=sum(s.K for s in specs))
    models = [G.Model(s) for s in specs]
    outs = [G.alloc_output(plan, s.K, diagnostics=True) for s in specs]
    log("gpu dsmc_smooth_batch of 5 series")
    G.dsmc_smooth_batch(plan, models, seeds, outs)
    torch.cuda.synchronize()
    for spec, m, o, seed in zip(specs, models, outs, seeds):
        single = run_gpu(spec, N, seed, model=m)
        for k in ("traj", "log_Z", "ancestry", "logZ_inc", "row_lse", "index", "leaf_x"):
            np.testing.assert_array_equal(getattr(o, k).cpu().numpy(), single[k])


def test_graph_replays_equal_eager():
    """DSMC_PLAN_GRAPH: the first call of a batch shape runs eagerly, the second
    captures a hipGraph, later calls replay it.  Every call, with new seeds and
    ordinary GPU work in between, equals an eager plan's result bit for bit;
    a new shape is captured afresh."""
    import torch
    from paper_2202_02264_amd import dsmc as G
    N = 128
    fields = ("traj", "log_Z", "status", "ancestry", "logZ_inc", "row_lse", "index", "leaf_x")
    shapes = [[70, 1, 33, 128, 2], [40, 64]]
    plan_e = G.Plan(N, 1, max_K=128, max_total_K=234)
    plan_g = G.Plan(N, 1, max_K=128, max_total_K=234, graph=True)
    for shape in shapes:
        specs = [W.lg1d(K, seed=40 + K) for K in shape]
        models = [G.Model(s) for s in specs]
        outs_e = [G.alloc_output(plan_e, s.K, diagnostics=True) for s in specs]
        outs_g = [G.alloc_output(plan_g, s.K, diagnostics=True) for s in specs]
        for rep in range(4):
            seeds = [100 * rep + i for i in range(len(specs))]
            log(f"graph shape {shape} call {rep}")
            G.dsmc_smooth_batch(plan_e, models, seeds, outs_e)
            torch.cuda.synchronize()
            junk = torch.randn(4096, device="cuda").cumsum(0)  # eager work between replays
            G.dsmc_smooth_batch(plan_g, models, seeds, outs_g)
            torch.cuda.synchronize()
            del junk
            for oe, og in zip(outs_e, outs_g):
                for f in fields:
                    assert torch.equal(getattr(oe, f), getattr(og, f)), (shape, rep, f)
    # a single series through dsmc_smooth on the graph plan
    spec = W.sv(100, seed=9)
    m = G.Model(spec)
    oe = G.alloc_output(plan_e, spec.K)
    og = G.alloc_output(plan_g, spec.K)
    for rep in range(3):
        G.dsmc_smooth(plan_e, m, rep, oe)
        G.dsmc_smooth(plan_g, m, rep, og)
        torch.cuda.synchronize()
        assert torch.equal(oe.traj, og.traj) and torch.equal(oe.log_Z, og.log_Z)
