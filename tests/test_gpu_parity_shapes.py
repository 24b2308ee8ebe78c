"""GPU parity against the oracle at the shapes of the batch, precision and
serving workloads, in the launch configurations the benchmark times.

Each run is compared teacher-forced (the oracle's combine on the GPU's own
inputs of that level) on a sample of combines: every combine of the top
levels and a few of each lower level, with the tolerances of the headline
parity tests (log-weights, row log-sums and increments within 1e-5 relative;
indices bit-exact outside the 1e-6 band of a CDF boundary).  Leaves are checked
at a sample of time points.
"""
import numpy as np
import pytest

from oracle import dsmc as D
from oracle import philox as Ph
from oracle import ssm
from paper_2202_02264_amd import workloads as W

from parity import TOL32, _rel, log, teacher_forced

pytestmark = pytest.mark.gpu


def _pick(K, per_level, top, seed=0, levels=None):
    """Boundaries of every combine of levels with <= `top` combines and of
    `per_level` combines of each other level (of the listed levels only, if
    `levels` is given)."""
    rng = np.random.default_rng(seed)
    chosen = set()
    for li, level in enumerate(D.schedule(K)):
        cs = [c for (_, c, _) in level]
        if len(cs) <= top:
            chosen.update(cs)
        elif levels is None or li in levels:
            chosen.update(int(v) for v in rng.choice(cs, per_level, replace=False))
    return chosen


def _check_leaves_at(spec, N, seed, g, times, tol=TOL32):
    """Leaf particles at the given times equal the oracle's draws rounded to
    fp32 (within one ulp); their log-weights and log L_t equal the oracle's on
    the stored particles."""
    d = spec.d_x
    for t in times:
        x = ssm.proposal_draw(spec, t, Ph.leaf_normals(seed, t, N, d))
        xr = x.astype(np.float32).astype(np.float64)
        xg = g["leaf_x"][:, t, :].T.astype(np.float64)
        ulp = np.spacing(np.abs(xr).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(xg - xr) <= ulp), t
        lw, lL = D.normalise(D.leaf_logweights(spec, t, xg))
        assert np.max(_rel(g["leaf_logw"][t], lw)) <= tol, t
        assert float(_rel(g["leaf_logL"][t], lL)) <= tol, t


def _numpy(out):
    res = {}
    for k in ("traj", "logw", "log_Z", "status", "leaf_x", "leaf_logw", "leaf_logL", "ancestry",
              "logZ_inc", "row_lse", "index"):
        res[k] = getattr(out, k).cpu().numpy()
    return res


@pytest.mark.parametrize("N,K", [(1024, 512), (4096, 256)])
def test_served_lg4d_oracle_parity(N, K):
    """The serving workload's 4-D linear-Gaussian class (RTS proposals) at
    N = 1024 and 4096, served through dsmc_submit / dsmc_poll next to
    stochastic-volatility jobs, compared with the oracle."""
    import time
    import torch
    from paper_2202_02264_amd import dsmc as G
    spec = W.lg4d(K, seed=W.DATA_SEED + 201, proposal="rts")
    others = [(W.sv(700, seed=31), N, 5), (W.lg4d(90, seed=32, proposal="rts"), N, 6)]
    srv = G.Server(mem_budget=16 << 30, max_jobs=8, max_classes=4)
    m = G.Model(spec)
    o = G.alloc_job_output(N, 4, K, diagnostics=True)
    keep = [(G.Model(s), G.alloc_job_output(n, s.d_x, s.K)) for s, n, _ in others]
    seed = 77
    log(f"serving lg4d K={K} N={N} with {len(others)} other jobs")
    ids = [G.dsmc_submit(srv, km, n, sd, ko) for (s, n, sd), (km, ko) in zip(others, keep)]
    ids.append(G.dsmc_submit(srv, m, N, seed, o))
    t0 = time.time()
    pending = set(ids)
    while pending and time.time() - t0 < 120:
        for i in list(pending):
            rc, _ = G.dsmc_poll(srv, i)
            if rc != G.DSMC_EAGAIN:
                assert rc == 0, rc
                pending.discard(i)
        time.sleep(0.002)
    assert not pending
    torch.cuda.synchronize()
    g = _numpy(o)
    srv.close()
    assert g["status"][0] == 0
    _check_leaves_at(spec, N, seed, g, [0, 1, K // 2, K - 1])
    chosen = _pick(K, 2, 4)
    rep = teacher_forced(spec, N, seed, g, TOL32, select=lambda a, c, b: c in chosen)
    log(f"served lg4d N={N}: {rep.summary()}")
    assert rep.mismatches_outside_band == 0, rep.worst[:5]


def test_batch_workload_oracle_parity():
    """The batch workload (512 1-D linear-Gaussian series, K ~ U{64..8192},
    N = 256) in the benchmark's launch configuration (dsmc_smooth_batch with a
    hipGraph replayed on the third call); the longest series and a short one
    are compared with the oracle."""
    import torch
    from paper_2202_02264_amd import dsmc as G
    specs = W.lg1d_batch(512)
    Ks = [s.K for s in specs]
    N = 256
    ilong = int(np.argmax(Ks))
    ishort = int(np.argmin(Ks))
    assert Ks[ilong] >= 4096
    plan = G.Plan(N, 1, max(Ks), max_total_K=sum(Ks), graph=True)
    models = [G.Model(s) for s in specs]
    outs = [G.alloc_output(plan, K, diagnostics=(i in (ilong, ishort))) for i, K in enumerate(Ks)]
    seeds = list(range(1, 513))
    for call in range(3):  # eager (tile tuning), capture, replay
        log(f"batch of 512 series, call {call}")
        G.dsmc_smooth_batch(plan, models, seeds, outs)
    torch.cuda.synchronize()
    for i in (ilong, ishort):
        spec, seed = specs[i], seeds[i]
        g = _numpy(outs[i])
        assert g["status"][0] == 0
        _check_leaves_at(spec, N, seed, g, [0, 1, spec.K // 3, spec.K - 1])
        chosen = _pick(spec.K, 6, 16)
        rep = teacher_forced(spec, N, seed, g, TOL32, select=lambda a, c, b: c in chosen)
        log(f"batch series K={spec.K}: {rep.summary()}")
        assert rep.mismatches_outside_band == 0, rep.worst[:5]


def test_highdim_fp32_full_size_oracle_parity():
    """The precision workload (d_x = 32 linear-Gaussian, K = 2048, N = 4096)
    on the fp32 VALU pair-row path: the full run, compared with the oracle on
    every combine of the top two levels and one combine of levels 0, 4 and 8
    (an oracle combine at this size takes several seconds)."""
    import torch
    from paper_2202_02264_amd import dsmc as G
    spec = W.lg_highdim(K=2048)
    N, seed = 4096, 3
    plan = G.Plan(N, 32, spec.K, precision=G.DSMC_FP32)
    model = G.Model(spec)
    out = G.alloc_output(plan, spec.K, diagnostics=True)
    log("highdim fp32 K=2048 N=4096")
    G.dsmc_smooth(plan, model, seed, out)
    torch.cuda.synchronize()
    g = _numpy(out)
    del out, plan
    torch.cuda.empty_cache()
    assert g["status"][0] == 0
    _check_leaves_at(spec, N, seed, g, [0, 1, 1024, 2047])
    chosen = _pick(spec.K, 1, 2, levels=(0, 4, 8))
    rep = teacher_forced(spec, N, seed, g, TOL32, select=lambda a, c, b: c in chosen)
    log(f"highdim fp32 full size: {rep.summary()}")
    assert rep.mismatches_outside_band == 0, rep.worst[:5]
