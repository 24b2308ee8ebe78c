"""Parallel-in-time Gaussian proposals (Section 4.1, Algorithm 5) on the GPU:
the associative-scan Kalman filter and RTS smoother of
dsmc_model_gaussian_proposals equal the oracle's sequential Kalman/RTS
smoother (the linear-Gaussian closed form) within 1e-9 relative, at
d_x = 1, 4 and 32 and K up to 16384; a smoother run with the device-computed
proposals equals one with the same proposals given from the host."""
import numpy as np
import pytest

from oracle import kalman
from paper_2202_02264_amd import workloads as W

from parity import log

pytestmark = pytest.mark.gpu


def _model(kind, K):
    if kind == "lg1d":
        return W.lg(K, np.array([[0.9]]), np.array([[0.7]]), np.array([[1.2]]), np.array([[0.8]]),
                    np.array([0.3]), np.array([[1.5]]), proposal="prior", f=np.array([0.05]),
                    h=np.array([-0.1]), name=f"lg1d(K={K})")
    if kind == "lg4d":
        g = np.random.Generator(np.random.Philox(5))
        F = 0.85 * W.random_orthogonal(4, g) + np.triu(0.1 * np.ones((4, 4)), 1)
        Qc = np.tril(0.1 * g.standard_normal((4, 4)), -1) + np.diag([0.6, 0.5, 0.7, 0.4])
        Rc = np.array([[0.8, 0, 0], [0.2, 0.6, 0], [-0.1, 0.1, 0.9]])
        return W.lg(K, F, Qc, g.standard_normal((3, 4)), Rc, np.zeros(4), np.eye(4),
                    proposal="prior", f=0.1 * g.standard_normal(4), h=0.1 * g.standard_normal(3),
                    name=f"lg4d(K={K})")
    return W.lg_highdim(K=K, seed=7)


@pytest.mark.parametrize("kind,K", [("lg1d", 1), ("lg1d", 2), ("lg1d", 37), ("lg1d", 16384),
                                    ("lg4d", 300), ("lg4d", 16384), ("lg32", 17), ("lg32", 2048)])
def test_pit_kalman_equals_sequential(kind, K):
    import torch
    from paper_2202_02264_amd import dsmc as G
    spec = _model(kind, K)
    log(f"pit kalman {spec.name}")
    ms, Ps, _ = kalman.kalman_smoother(spec)
    m = G.Model(spec)
    G.dsmc_model_gaussian_proposals(m)
    torch.cuda.synchronize()
    qm, qc = G.dsmc_model_read_proposals(m)
    P = qc @ np.swapaxes(qc, 1, 2)
    err_m = np.max(np.abs(qm - ms) / np.maximum(1.0, np.abs(ms)))
    err_P = np.max(np.abs(P - Ps) / np.maximum(1.0, np.abs(Ps).max(axis=(1, 2), keepdims=True)))
    log(f"  max rel err mean {err_m:.2e}, covariance {err_P:.2e}")
    assert err_m <= 1e-9 and err_P <= 1e-9
    # the factor is the lower Cholesky factor of P
    assert np.all(np.triu(qc, 1) == 0.0) and np.all(np.diagonal(qc, axis1=1, axis2=2) > 0)


def test_device_proposals_drive_the_smoother():
    """dsmc_smooth after dsmc_model_gaussian_proposals on the same stream equals
    dsmc_smooth on a model created with the read-back proposals (fp64 plan:
    every index equal)."""
    import torch
    from paper_2202_02264_amd import dsmc as G
    spec = _model("lg4d", 64)
    m = G.Model(spec)                     # created with prior-marginal proposals
    G.dsmc_model_gaussian_proposals(m)
    qm, qc = G.dsmc_model_read_proposals(m)
    spec2 = W.SSM(**{**spec.__dict__, "q_mean": qm, "q_chol": qc})
    m2 = G.Model(spec2)
    plan = G.Plan(128, 4, 64, precision=G.DSMC_FP64)
    a = G.alloc_output(plan, 64, diagnostics=True)
    b = G.alloc_output(plan, 64, diagnostics=True)
    G.dsmc_smooth(plan, m, 3, a)
    G.dsmc_smooth(plan, m2, 3, b)
    torch.cuda.synchronize()
    for f in ("traj", "ancestry", "log_Z", "leaf_x"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f
