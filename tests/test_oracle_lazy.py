"""Pins of the oracle's lazy resampling (Section 4.2, Algorithms 7 and 8).

* Algorithm 8 (rejection) draws pairs exactly from W for any valid bound:
  chi-square of pooled draws against W on a small weight matrix with a zero
  entry (never drawn).
* Algorithm 7 (Metropolis-Hastings, B steps from (n, n)) has the law of a
  Markov chain on the N^2 pairs whose kernel is enumerated here: move to
  s' != s with probability min(1, W(s')/W(s)) / N^2.  The pooled draws are
  checked against start-state rows of that kernel's B-th power; B = 0 is the
  identity.
* The rejection bound is at least every realised pair weight.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import dsmc as D
from paper_2202_02264_amd import workloads as W

with np.errstate(divide="ignore"):
    S_SMALL = np.log(np.array([[0.30, 0.05, 0.00],
                               [0.10, 0.20, 0.02],
                               [0.15, 0.08, 0.10]]))


def _pooled_counts(draw, seeds, N):
    counts = np.zeros(N * N)
    for seed in seeds:
        I, J = draw(seed)
        np.add.at(counts, I * N + J, 1)
    return counts


def _chi2_p(counts, probs):
    keep = probs > 0
    assert counts[~keep].sum() == 0          # zero-weight pairs are never drawn
    exp = probs[keep] * counts.sum()
    return stats.chisquare(counts[keep], exp).pvalue


@pytest.mark.parametrize("slack", [0.0, 0.7])
def test_rejection_law_is_W(slack):
    N = 3
    bound = float(np.max(S_SMALL)) + slack
    counts = _pooled_counts(lambda s: D.rs_resampling(S_SMALL, bound, s, 5, 10000)[:2],
                            range(2000), N)
    w = np.exp(S_SMALL).ravel()
    assert _chi2_p(counts, w / w.sum()) > 1e-4


def _mh_kernel(S):
    N = S.shape[0]
    w = np.exp(S).ravel()
    n2 = N * N
    P = np.zeros((n2, n2))
    with np.errstate(divide="ignore", invalid="ignore"):
        for s in range(n2):
            for t in range(n2):
                if t != s:
                    r = w[t] / w[s] if w[s] > 0 else (np.inf if w[t] > 0 else 0.0)
                    P[s, t] = min(1.0, r) / n2
            P[s, s] = 1.0 - P[s].sum()
    return P


@pytest.mark.parametrize("B", [0, 1, 3, 25])
def test_metropolis_law_matches_enumerated_chain(B):
    N = 3
    counts = _pooled_counts(lambda s: D.mh_resampling(S_SMALL, s, 7, B), range(1500), N)
    PB = np.linalg.matrix_power(_mh_kernel(S_SMALL), B)
    starts = [n * N + n for n in range(N)]
    law = PB[starts].mean(axis=0)        # chain n starts at (n, n); draws pooled over n
    if B == 0:
        assert np.array_equal(counts / counts.sum(), law)
    else:
        assert _chi2_p(counts, law) > 1e-4
    if B == 25:                           # close to W after many steps
        w = np.exp(S_SMALL).ravel()
        assert np.abs(law - w / w.sum()).max() < 1e-3


@pytest.mark.parametrize("make", [lambda: W.lg1d(6, seed=3), lambda: W.sv(5, seed=4),
                                  lambda: W.lg4d(4, seed=6),
                                  lambda: W.sv(5, seed=8, weighting="boundary_obs")])
def test_rejection_bound_covers_every_pair(make):
    spec = make()
    N = 64
    lv = D.sample_leaves(spec, N, 9)
    for c in range(1, spec.K):
        S = D.pair_logweights(spec, c, lv.x[c - 1], lv.x[c], lv.logw[c - 1], lv.logw[c])
        bound = D.rs_log_bound(spec, c, lv.x[c], lv.logw[c - 1], lv.logw[c])
        assert S.max() <= bound + 1e-12


@pytest.mark.parametrize("scheme,param", [("mh", 8), ("rs", 1 << 16)])
def test_lazy_smoother_runs(scheme, param):
    spec = W.sv(11, seed=2)
    N = 32
    res = D.smooth_lazy(spec, N, 5, scheme, param)
    assert res.ancestry.min() >= 0 and res.ancestry.max() < N
    assert not res.capped
    # the gather follows the ancestry exactly as in the exact smoother
    lv = res.leaves
    np.testing.assert_array_equal(res.x, np.take_along_axis(lv.x, res.idx[:, :, None], axis=1))
