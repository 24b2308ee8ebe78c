"""Pins of the oracle's constrained-random-walk model (Section 5.3): uniform
proposals on [-1, 1], the box-indicator potential, the Gaussian random-walk
transition, against scipy's densities; the K = 2 increment by brute force."""
import numpy as np
import pytest
from scipy import stats

from oracle import dsmc as D
from oracle import ssm
from paper_2202_02264_amd import workloads as W


def test_densities_match_scipy():
    spec = W.constrained_rw(4, sigma=0.4)
    x = np.linspace(-1.5, 1.5, 31)[:, None]
    np.testing.assert_allclose(ssm.log_proposal(spec, 2, x), stats.uniform(-1, 2).logpdf(x[:, 0]))
    ind = np.where(np.abs(x[:, 0]) <= 1.0, 0.0, -np.inf)
    np.testing.assert_array_equal(ssm.log_potential(spec, 1, x), ind)
    T = ssm.log_transition_pairs(spec, x[:5], x[5:9])
    np.testing.assert_allclose(T, stats.norm.logpdf(x[5:9, 0][None, :], x[:5, 0][:, None], 0.4),
                               rtol=1e-12)


def test_leaf_draws_are_uniform_on_the_box():
    spec = W.constrained_rw(3, sigma=0.5)
    lv = D.sample_leaves(spec, 4000, 17)
    for t in range(3):
        xs = lv.x[t, :, 0]
        assert xs.min() >= -1.0 and xs.max() < 1.0
        assert stats.kstest(xs, stats.uniform(-1, 2).cdf).pvalue > 1e-4
    # boundary weighting: leaf weights uniform for t >= 1, h_0 p_0 / q_0 at t = 0
    np.testing.assert_allclose(lv.logw[1], -np.log(4000))
    raw0 = stats.norm.logpdf(lv.x[0, :, 0]) + np.log(2.0)
    np.testing.assert_allclose(lv.raw[0], raw0, rtol=1e-12)


@pytest.mark.parametrize("sigma", [0.3, 0.5])
def test_increment_brute_force(sigma):
    spec = W.constrained_rw(2, sigma=sigma)
    N = 4
    res = D.smooth(spec, N, 5)
    x0, x1 = res.leaves.x[0, :, 0], res.leaves.x[1, :, 0]
    w0 = stats.norm.pdf(x0) * 2.0                  # h_0 p_0 / q_0
    W0 = w0 / w0.sum()
    Z = np.log(sum(W0[m] / N * stats.norm.pdf(x1[n], x0[m], sigma) * 2.0
                   for m in range(N) for n in range(N)))
    assert res.Zc[0] == pytest.approx(Z, rel=1e-12)
    assert res.logZ == pytest.approx(np.log(w0.mean()) + Z, rel=1e-12)
