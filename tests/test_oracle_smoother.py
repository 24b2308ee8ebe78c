"""Statistical pins of the whole oracle smoother against the Kalman/RTS closed form.

Replicate seeds are fixed, so every test is deterministic.

Two estimators are checked.  The plain smoothed mean (1/N) sum_n X_t^n is a
self-normalised estimate with an O(1/N) bias, which can exceed the Monte Carlo
standard error when the proposal is poor (prior proposals on the correctness
workload).  The L^N-weighted replicate mean sum_r L_r m_r / sum_r L_r has no
such bias: the extended target pi = (L^N / L) psi of Section 3.1 is a
probability measure under which an output trajectory is distributed as the
smoothing distribution, so E[L^N (1/N) sum_n phi(X^n)] = L Q(phi) at every N.
"""
import numpy as np
import pytest

from oracle import dsmc as D
from oracle import kalman
from paper_2202_02264_amd import workloads as W


def _replicates(spec, N, seeds):
    means, logZ = [], []
    for s in seeds:
        out = D.smooth(spec, N, s)
        means.append(out.x[:, :, 0].mean(axis=1))
        logZ.append(out.logZ)
    return np.array(means), np.array(logZ)


def _weighted_z(means, logZ, ll, ref):
    """z-scores of the L^N-weighted replicate mean (delta-method standard error)."""
    w = np.exp(logZ - ll)
    est = (w[:, None] * means).sum(0) / w.sum()
    se = np.sqrt(((w[:, None] * (means - est[None, :])) ** 2).sum(0)) / w.sum()
    return (est - ref) / se


def _plain_z(means, ref):
    R = means.shape[0]
    return (means.mean(0) - ref) / (means.std(0, ddof=1) / np.sqrt(R))


def _lg1d_rts(weighting):
    return W.lg(32, np.array([[0.9]]), np.array([[1.0]]), np.eye(1), np.eye(1), np.zeros(1),
                np.eye(1), proposal="rts", weighting=weighting)


@pytest.mark.slow
def test_correctness_workload_vs_kalman():
    """LG-1D, K = 32, N = 64, prior proposals, 100 seeds: the L^N-weighted
    smoothed means are within 3 standard errors of RTS at every t; L^N is
    unbiased (mean of L^N / L_KF within 1 +- 3 SE); by Jensen,
    mean log L^N <= log L_KF."""
    spec = W.c1_lg1d()
    ms, _, ll = kalman.kalman_smoother(spec)
    means, logZ = _replicates(spec, 64, range(1, 101))
    z = _weighted_z(means, logZ, ll, ms[:, 0])
    assert np.all(np.abs(z) < 3.0), z
    ratio = np.exp(logZ - ll)
    assert abs(ratio.mean() - 1.0) < 3.0 * ratio.std(ddof=1) / 10.0
    assert logZ.mean() <= ll + 3.0 * logZ.std(ddof=1) / 10.0


@pytest.mark.slow
@pytest.mark.parametrize("weighting", ["leaf_obs", "boundary_obs"])
def test_rts_proposals_vs_kalman(weighting):
    """LG-1D, K = 32, N = 64 with the exact smoothing marginals as proposals
    (Section 4.1): smoothed means within 3 standard errors of RTS at every t
    (plain means for leaf_obs; L^N-weighted for boundary_obs, whose plain means
    carry a visible O(1/N) bias at this N)."""
    spec = _lg1d_rts(weighting)
    ms, _, ll = kalman.kalman_smoother(spec)
    means, logZ = _replicates(spec, 64, range(1, 101))
    if weighting == "leaf_obs":
        z = _plain_z(means, ms[:, 0])
    else:
        z = _weighted_z(means, logZ, ll, ms[:, 0])
    assert np.all(np.abs(z) < 3.0), z


@pytest.mark.slow
def test_unbiasedness_small_model():
    """K = 8, N = 16, 3000 seeds: E[L^N] = L and E[L^N Q^N(phi)] = L Q(phi)
    (Section 3.1), checked for phi = x_t at every t."""
    spec = W.lg1d(8, A=0.9, Q=1.0, R=1.0, seed=31)
    ms, _, ll = kalman.kalman_smoother(spec)
    means, logZ = _replicates(spec, 16, range(1, 3001))
    ratio = np.exp(logZ - ll)
    assert abs(ratio.mean() - 1.0) < 3.0 * ratio.std(ddof=1) / np.sqrt(len(ratio))
    z = _weighted_z(means, logZ, ll, ms[:, 0])
    assert np.all(np.abs(z) < 3.0), z


@pytest.mark.slow
def test_error_rate_in_N():
    """Proposition 2.4: the L_p error of smoothed expectations falls like
    N^{-1/2}; quadrupling N halves the RMSE against RTS (ratio 2 +- 30%)."""
    spec = _lg1d_rts("leaf_obs").truncated(16)
    ms, _, _ = kalman.kalman_smoother(_lg1d_rts("leaf_obs"))
    rmse = []
    for N in (32, 128):
        means, _ = _replicates(spec, N, range(1, 61))
        rmse.append(np.sqrt(np.mean((means - ms[None, :16, 0]) ** 2)))
    assert 1.4 < rmse[0] / rmse[1] < 2.6, rmse


def test_single_time_point_is_importance_sampling():
    """K = 1: no combine; output = weighted leaf particles, log L = log L_0."""
    spec = W.lg1d(1, seed=5)
    out = D.smooth(spec, 500, seed=7)
    assert out.ancestry.shape == (0, 2, 500)
    np.testing.assert_array_equal(out.x, out.leaves.x)
    est = np.sum(np.exp(out.logw) * out.x[0, :, 0])
    ms, Ps, ll = kalman.kalman_smoother(spec)
    assert abs(est - ms[0, 0]) < 8 * np.sqrt(Ps[0, 0, 0] / 500)
    assert abs(out.logZ - ll) < 0.2


def test_deterministic_in_seed():
    spec = W.sv(13, seed=2)
    a = D.smooth(spec, 9, 5)
    b = D.smooth(spec, 9, 5)
    c = D.smooth(spec, 9, 6)
    np.testing.assert_array_equal(a.x, b.x)
    assert a.logZ == b.logZ
    assert not np.array_equal(a.ancestry, c.ancestry)
