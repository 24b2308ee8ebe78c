"""dsmc_plan under device allocation failure: every workspace allocation that
fails gives DSMC_ENOMEM, frees what the call had allocated, and leaves the
library usable (the failure is injected with dsmc_debug_fail_allocation)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _plan_failing_at(G, k, **kw):
    G.dsmc_debug_fail_allocation(k)
    try:
        return G.Plan(**kw)
    finally:
        G.dsmc_debug_fail_allocation(-1)


@pytest.mark.parametrize("case", ["fp32_profiled_dx1", "bf16_dx32"])
def test_each_allocation_failure_is_clean(case):
    import torch

    from paper_2202_02264_amd import dsmc as G

    kw = (dict(N=256, d_x=1, max_K=64, precision=G.DSMC_FP32, profile=True)
          if case == "fp32_profiled_dx1" else
          dict(N=256, d_x=32, max_K=64, precision=G.DSMC_BF16))
    print(f"case {case}", flush=True)
    failed = 0
    while True:
        assert failed < 64, "dsmc_plan never succeeded"
        try:
            plan = _plan_failing_at(G, failed, **kw)
        except G.DsmcError as e:
            assert e.code == G.DSMC_ENOMEM, e
            assert "hipMalloc(" in str(e), e
            failed += 1
            continue
        break
    # the base workspace is 23 allocations; profiling adds one, bf16 eight
    assert failed == (24 if case == "fp32_profiled_dx1" else 31), failed
    del plan
    # the hook is off again: a plan and a run work as before
    plan = G.Plan(**kw)
    del plan
    torch.cuda.synchronize()


def test_failed_plans_leak_no_device_memory():
    """A large workspace (about 6.5 GiB) failing at its last allocation, four
    times after a first such failure: a leak of the allocations made before it
    would hold about 26 GiB more at the end (whatever the runtime keeps cached
    from the first attempt stays the same)."""
    import torch

    from paper_2202_02264_amd import dsmc as G

    kw = dict(N=4096, d_x=1, max_K=16384, precision=G.DSMC_FP32)

    def fail_at_last():
        with pytest.raises(G.DsmcError) as ei:
            _plan_failing_at(G, 22, **kw)  # the base workspace's last allocation
        assert ei.value.code == G.DSMC_ENOMEM

    fail_at_last()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(4):
        fail_at_last()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < (3 << 30), (free0, free1)


def test_library_usable_after_failures():
    """After injected failures, an fp64 run equals the oracle's run."""
    import torch

    from oracle import dsmc as D
    from paper_2202_02264_amd import dsmc as G
    from paper_2202_02264_amd import workloads as W

    for k in (0, 5, 22):
        with pytest.raises(G.DsmcError):
            _plan_failing_at(G, k, N=64, d_x=1, max_K=32, precision=G.DSMC_FP64)
    spec = W.c1_lg1d()
    out = G.smooth(spec, 64, seed=7, precision=G.DSMC_FP64, diagnostics=True)
    torch.cuda.synchronize()
    ref = D.smooth(spec, 64, 7)
    assert np.array_equal(out.ancestry.cpu().numpy(), ref.ancestry)
    assert abs(float(out.log_Z.item()) - ref.logZ) < 1e-10 * max(1.0, abs(ref.logZ))
