"""dsmc_smooth_static (the allocation-free entry point) through the C ABI: its
results equal dsmc_smooth's on a plan, bit for bit, over consecutive calls that
share the library's fixed workspace (each later call smaller than the one
before), in fp32 and fp64; a run larger than the workspace is refused before
any device work."""
import numpy as np
import pytest

from paper_2202_02264_amd import workloads as W

from parity import log

pytestmark = pytest.mark.gpu

FIELDS = ("traj", "logw", "log_Z", "status", "leaf_x", "leaf_logw", "leaf_logL", "ancestry",
          "logZ_inc", "row_lse", "index")


def _compare(G, spec, N, seed, precision):
    import torch
    model = G.Model(spec)
    plan = G.Plan(N, spec.d_x, spec.K, precision=precision)
    ref = G.alloc_output(plan, spec.K, diagnostics=True)
    got = G.alloc_output(plan, spec.K, diagnostics=True)
    for t in (got.traj, got.leaf_x, got.row_lse):
        t.fill_(-7.0)  # stale values must not survive
    log(f"static vs plan: {spec.name} N={N} precision={precision}")
    G.dsmc_smooth(plan, model, seed, ref)
    G.dsmc_smooth_static(model, N, seed, got, precision=precision)
    torch.cuda.synchronize()
    for f in FIELDS:
        a, b = getattr(ref, f).cpu().numpy(), getattr(got, f).cpu().numpy()
        np.testing.assert_array_equal(a, b, err_msg=f"{spec.name} {f}")
    assert int(got.status.item()) == 0


def test_static_equals_plan_consecutive_calls():
    from paper_2202_02264_amd import dsmc as G
    # the headline size, then smaller runs reusing the same workspace
    _compare(G, W.sv(4096, seed=3), 1024, 11, G.DSMC_FP32)
    _compare(G, W.sv(300, seed=4), 256, 12, G.DSMC_FP32)
    _compare(G, W.lg4d(40, seed=5), 64, 13, G.DSMC_FP32)
    _compare(G, W.lg1d(33, seed=6), 48, 14, G.DSMC_FP64)


def test_static_rejects_runs_beyond_the_workspace():
    import torch
    from paper_2202_02264_amd import dsmc as G
    spec = W.sv(4096, seed=7)
    model = G.Model(spec)
    out = G.alloc_job_output(4096, 1, spec.K)
    with pytest.raises(G.DsmcError) as e:
        G.dsmc_smooth_static(model, 4096, 1, out)
    assert e.value.code == G.DSMC_EUNSUPPORTED
    assert "static workspace" in str(e.value)
    with pytest.raises(G.DsmcError) as e:
        G.dsmc_smooth_static(model, 64, 1, out, precision=G.DSMC_BF16)
    assert e.value.code == G.DSMC_EUNSUPPORTED
    torch.cuda.synchronize()
