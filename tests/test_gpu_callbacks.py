"""A model created with host callbacks (checked against its device form by
dsmc_model_create) runs on the GPU exactly as the same model without them."""
import numpy as np
import pytest

from paper_2202_02264_amd import workloads as W

from parity import log
from test_model_callbacks import Callbacks

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["sv", "lg4d"])
def test_callback_model_runs_like_plain_model(name):
    import torch
    from paper_2202_02264_amd import dsmc as G
    spec = W.sv(200, seed=5) if name == "sv" else W.lg4d(60, seed=6, proposal="rts")
    cb = Callbacks(spec)
    log(f"callback model {name}")
    m_cb = G.Model(spec, cb.c)
    m = G.Model(spec)
    plan = G.Plan(128, spec.d_x, spec.K)
    a = G.alloc_output(plan, spec.K)
    b = G.alloc_output(plan, spec.K)
    G.dsmc_smooth(plan, m_cb, 9, a)
    G.dsmc_smooth(plan, m, 9, b)
    torch.cuda.synchronize()
    assert torch.equal(a.traj, b.traj) and torch.equal(a.log_Z, b.log_Z)
    bad = Callbacks(spec, fault="obs_sign")
    with pytest.raises(G.DsmcError) as e:
        G.Model(spec, bad.c)
    assert e.value.code == G.DSMC_EINVAL
