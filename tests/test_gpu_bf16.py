"""GPU: the bf16 matrix-core pair-row path (DSMC_BF16, d_x = 16 and 32).

Its results are not expected to equal the fp64 oracle to fp32 tolerance: the
pair weight's quadratic form is formed as ||u||^2 + ||v||^2 - 2 u.v with the
dot product from split bf16 operands (hi + remainder, about 16 significant
bits) and fp32 accumulation, so each pair's log weight moves by the dropped
remainder product and the cancellation of the expanded form.  The tests state
the errors (row log-sums, increments, index agreement; teacher-forced against
the oracle) and bound them: median row log-sum error at most 0.005 and maximum
at most 0.03 (natural log), at least 97 % of the index draws equal; everything
that does not depend on the pair weights (leaves, gather, ancestry
bookkeeping, log L = sum of the parts) is checked exactly.
"""
import numpy as np
import pytest

from oracle import kalman
from paper_2202_02264_amd import workloads as W

from parity import TOL32, check_leaves, log, run_gpu, teacher_forced

pytestmark = pytest.mark.gpu


def _errors(spec, N, seed, select=None, leaves=True):
    g = run_gpu(spec, N, seed, precision="bf16")
    assert g["status"][0] == 0
    if leaves:
        check_leaves(spec, N, seed, g, TOL32)
    rep = teacher_forced(spec, N, seed, g, None, select=select)
    er = np.concatenate(rep.abs_err_row)
    ez = np.array(rep.abs_err_Z)
    agree = 1.0 - rep.mismatches / max(1, rep.draws)
    log(f"bf16 {spec.name} N={N}: |d row_lse| median {np.median(er):.3g} p99 "
        f"{np.percentile(er, 99):.3g} max {er.max():.3g}; |d Z_c| median {np.median(ez):.3g} "
        f"max {ez.max():.3g}; index agreement {agree:.4f} over {rep.draws} draws")
    return er, ez, agree


def test_bf16_dx32_errors_vs_oracle():
    """d_x = 32 (the precision workload's model, K = 64, N = 512)."""
    er, ez, agree = _errors(W.lg_highdim(K=64, seed=31), 512, 5)
    assert np.median(er) <= 0.005 and er.max() <= 0.03
    assert ez.max() <= 0.03
    assert agree >= 0.97


def test_bf16_dx16_errors_vs_oracle():
    """d_x = 12, padded to 16 (one matrix-core instruction per 32 x 32 block)."""
    er, ez, agree = _errors(W.lg_highdim(K=40, d_x=12, d_y=4, seed=32), 256, 6)
    assert np.median(er) <= 0.005 and er.max() <= 0.03
    assert ez.max() <= 0.03
    assert agree >= 0.97


def test_bf16_smoothed_means_vs_rts():
    """d_x = 32, K = 16, N = 1024, 24 seeds: plain smoothed means (RTS proposals)
    against the Kalman/RTS smoother, as z-scores with the replicate standard
    error; the bf16 weights add a bias that must stay small against it."""
    import torch
    from paper_2202_02264_amd import dsmc as G
    spec = W.lg_highdim(K=16, seed=33)
    ms, _, _ = kalman.kalman_smoother(spec)
    N, R = 1024, 24
    plan = G.Plan(N, spec.d_x, spec.K, precision=G.DSMC_BF16)
    model = G.Model(spec)
    out = G.alloc_output(plan, spec.K)
    means = []
    log("bf16 RTS replicates")
    for s in range(1, R + 1):
        G.dsmc_smooth(plan, model, s, out)
        torch.cuda.synchronize()
        assert int(out.status.cpu()[0]) == 0
        means.append(out.traj.double().mean(dim=2).cpu().numpy().T)  # (K, d_x)
    means = np.array(means)
    z = (means.mean(0) - ms) / (means.std(0, ddof=1) / np.sqrt(R))
    log(f"bf16 RTS: mean z^2 {np.mean(z ** 2):.3f}, max |z| {np.abs(z).max():.2f} over {z.size}")
    assert np.mean(z ** 2) < 2.0
    assert np.abs(z).max() < 6.0


def test_bf16_precision_workload_sampled():
    """The full precision workload (d_x = 32, K = 2048, N = 4096, bf16): errors
    teacher-forced on a level-0 combine, a level-5 combine and the root."""
    spec = W.lg_highdim()
    chosen = {1, 32 * 33, 1024}
    er, ez, agree = _errors(spec, 4096, 1, select=lambda a, c, b: c in chosen, leaves=False)
    assert np.median(er) <= 0.005 and er.max() <= 0.03
    assert ez.max() <= 0.03
    assert agree >= 0.97


def test_bf16_rescue_paths():
    """DSMC_PLAN_RESCUE_ALL with bf16: the matrix-core kernel redoes every row
    with its exact maximum and the sampler recomputes every row; the errors
    against the oracle stay at the bf16 level."""
    spec = W.lg_highdim(K=24, seed=34)
    g = run_gpu(spec, 256, 8, precision="bf16", rescue_all=True)
    assert g["status"][0] == 0
    rep = teacher_forced(spec, 256, 8, g, None)
    er = np.concatenate(rep.abs_err_row)
    log(f"bf16 rescue-all: |d row_lse| median {np.median(er):.3g} max {er.max():.3g}")
    assert np.median(er) <= 0.005 and er.max() <= 0.03
