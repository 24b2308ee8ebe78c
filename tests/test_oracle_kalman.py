"""Pins of the oracle's Kalman filter / RTS smoother against direct Gaussian
conditioning of the stacked (x, y) vector."""
import numpy as np
import pytest
from scipy import stats

from oracle import kalman
from paper_2202_02264_amd import workloads as W


@pytest.mark.parametrize("which", ["lg1d", "lg2d"])
def test_kalman_vs_joint_gaussian(which):
    if which == "lg1d":
        spec = W.lg1d(6, A=0.8, Q=0.6, R=0.9, m0=0.3, P0=1.5, seed=2)
    else:
        g = np.random.default_rng(0)
        F = np.array([[0.9, 0.2], [-0.1, 0.7]])
        spec = W.lg(5, F, np.array([[0.7, 0.0], [0.2, 0.5]]), np.array([[1.0, -0.5]]),
                    np.array([[0.8]]), np.array([0.1, -0.2]), np.array([[1.0, 0.0], [0.3, 0.9]]),
                    seed=4, proposal="prior")
    ms, Ps, ll = kalman.kalman_smoother(spec)
    mx, my, Cxx, Cxy, Cyy = kalman.joint_gaussian(spec)
    y = spec.y.reshape(-1)
    ll_direct = stats.multivariate_normal(my, Cyy).logpdf(y)
    assert abs(ll - ll_direct) < 1e-9 * max(1, abs(ll))
    mpost = mx + Cxy @ np.linalg.solve(Cyy, y - my)
    Cpost = Cxx - Cxy @ np.linalg.solve(Cyy, Cxy.T)
    dx = spec.d_x
    np.testing.assert_allclose(ms.reshape(-1), mpost, rtol=1e-9, atol=1e-10)
    for t in range(spec.K):
        np.testing.assert_allclose(Ps[t], Cpost[t * dx:(t + 1) * dx, t * dx:(t + 1) * dx],
                                   rtol=1e-9, atol=1e-10)


def test_proposal_builder_matches_oracle_rts():
    """The workload's RTS proposals (built for the d_x >= 2 configs) agree with the
    oracle's smoother; it only matters that they are valid proposals, but a match
    also shows the input builder is what it says."""
    g = np.random.default_rng(1)
    spec = W.lg(7, 0.8 * W.random_orthogonal(3, np.random.Generator(np.random.Philox(3))),
                0.5 * np.eye(3), np.ones((1, 3)) / 3, np.eye(1), np.zeros(3), np.eye(3), seed=5)
    ms, Ps, _ = kalman.kalman_smoother(spec)
    np.testing.assert_allclose(spec.q_mean, ms, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(spec.q_chol @ np.swapaxes(spec.q_chol, 1, 2), Ps, rtol=1e-8, atol=1e-10)
