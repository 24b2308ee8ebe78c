"""Pins of the oracle's tree (Algorithm 6), gather and whole-tree law."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import dsmc as D
from paper_2202_02264_amd import workloads as W


@pytest.mark.parametrize("K", [1, 2, 3, 5, 7, 64, 100, 4097])
def test_schedule_covers_every_boundary_once(K):
    levels = D.schedule(K)
    assert len(levels) == (0 if K == 1 else math.ceil(math.log2(K)))
    cs = [c for lv in levels for (_, c, _) in lv]
    assert sorted(cs) == list(range(1, K))            # K - 1 combines, each boundary once
    for l, lv in enumerate(levels):
        for (a, c, b) in lv:
            assert c - a == 2 ** l                     # left block is a full 2^l block
            assert 1 <= b - c <= 2 ** l                # right block may be ragged (padding trails)
            assert a % 2 ** (l + 1) == 0


@pytest.mark.parametrize("K", [2, 5, 8, 13])
def test_resampling_depth_uniform(K):
    """Every time step is resampled once per combine whose span contains it, at
    most ceil(log2 K) times (Section 3.2, degeneracy remark); for K a power of
    two, exactly log2 K times."""
    depth = np.zeros(K, dtype=int)
    for lv in D.schedule(K):
        for (a, c, b) in lv:
            depth[a:b] += 1
    assert depth.max() <= math.ceil(math.log2(K))
    if K & (K - 1) == 0:
        assert np.all(depth == int(math.log2(K)))


@pytest.mark.parametrize("K", [1, 2, 6, 9])
def test_output_structure(K):
    """Each merged trajectory is (left trajectory l_n) followed by (right
    trajectory r_n) (Algorithm 1); rebuild the output from the leaves and the
    ancestry and compare."""
    spec = W.sv(K, seed=5)
    N = 7
    out = D.smooth(spec, N, seed=3)
    idx = {t: np.arange(N)[None, :] for t in range(K)}
    for lv in D.schedule(K):
        for (a, c, b) in lv:
            l, r = out.ancestry[c - 1]
            assert l.min() >= 0 and l.max() < N and r.min() >= 0 and r.max() < N
            idx[a] = np.concatenate([idx[a][:, l], idx.pop(c)[:, r]], axis=0)
    np.testing.assert_array_equal(idx[0], out.idx)
    rebuilt = out.leaves.x[np.arange(K)[:, None], idx[0]]
    np.testing.assert_array_equal(rebuilt, out.x)
    if K == 1:
        np.testing.assert_array_equal(out.logw, out.leaves.logw[0])
        assert out.logZ == out.leaves.logL[0]
    else:
        np.testing.assert_allclose(out.logw, -np.log(N))
        assert abs(out.logZ - (out.leaves.logL.sum() + out.Zc.sum())) < 1e-10


def _w_matrix(spec, c, xL, xR, wL, wR):
    """Normalised product-form W (Section 2.2) from scipy densities, leaf_obs weighting."""
    om = (stats.norm.pdf(xR[None, :], spec.F[0, 0] * xL[:, None] + spec.f[0], spec.Q_chol[0, 0])
          / stats.norm.pdf(xR, spec.q_mean[c, 0], spec.q_chol[c, 0, 0])[None, :])
    un = wL[:, None] * wR[None, :] * om
    return un / un.sum()


@pytest.mark.slow
def test_exact_law_four_points_two_particles():
    """K = 4, N = 2, fixed leaves: enumerate every level-0 outcome to get the
    exact law of output trajectory 0 over the 16 leaf-index tuples, and compare
    with the oracle over many seeds (chi-square)."""
    spec = W.lg1d(4, A=0.8, Q=0.5, R=0.7, seed=8)
    N = 2
    lv = D.sample_leaves(spec, N, seed=1)
    x = lv.x[:, :, 0]
    w = np.exp(lv.logw)
    W1 = _w_matrix(spec, 1, x[0], x[1], w[0], w[1])
    W3 = _w_matrix(spec, 3, x[2], x[3], w[2], w[3])
    pairs = list(itertools.product(range(N), range(N)))
    law = {}
    for outs1 in itertools.product(pairs, repeat=N):          # N draws of combine c=1
        p1 = np.prod([W1[l, r] for (l, r) in outs1])
        for outs3 in itertools.product(pairs, repeat=N):      # N draws of combine c=3
            p3 = np.prod([W3[l, r] for (l, r) in outs3])
            xl = np.array([x[1, r] for (_, r) in outs1])        # time-1 particles of block [0,2)
            xr = np.array([x[2, l] for (l, _) in outs3])        # time-2 particles of block [2,4)
            W2 = _w_matrix(spec, 2, xl, xr, np.full(N, 1.0 / N), np.full(N, 1.0 / N))
            for (a, b) in pairs:
                key = (outs1[a][0], outs1[a][1], outs3[b][0], outs3[b][1])
                law[key] = law.get(key, 0.0) + p1 * p3 * W2[a, b]
    assert abs(sum(law.values()) - 1.0) < 1e-12
    M = 6000
    counts = {}
    for s in range(M):
        out = D.run_tree(spec, lv, seed=100 + s)
        key = tuple(int(v) for v in out.idx[:, 0])
        counts[key] = counts.get(key, 0) + 1
    keys = sorted(law)
    exp = np.array([law[k] * M for k in keys])
    obs = np.array([counts.get(k, 0) for k in keys])
    assert sum(counts.get(k, 0) for k in counts if k not in law) == 0
    keep = exp > 5
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    p = stats.chi2.sf(chi2, keep.sum() - 1)
    assert p > 1e-3, (chi2, p)


def test_single_particle_closed_form():
    """N = 1: every index is 0, the output is the leaf path and L^N is the
    importance weight of that path: p_0 h_0 / q_0 (x_0) prod_t h_t p_t / q_t."""
    for weighting in ("leaf_obs", "boundary_obs"):
        spec = W.lg1d(11, seed=6, weighting=weighting)
        out = D.smooth(spec, 1, seed=2)
        assert np.all(out.ancestry == 0)
        x = out.leaves.x[:, 0, 0]
        np.testing.assert_array_equal(out.x[:, 0, 0], x)
        lw = (stats.norm.logpdf(x[0], spec.m0[0], spec.P0_chol[0, 0])
              - stats.norm.logpdf(x[0], spec.q_mean[0, 0], spec.q_chol[0, 0, 0]))
        for t in range(11):
            lw += stats.norm.logpdf(spec.y[t, 0], x[t], spec.R_chol[0, 0])
            if t:
                lw += (stats.norm.logpdf(x[t], spec.F[0, 0] * x[t - 1], spec.Q_chol[0, 0])
                       - stats.norm.logpdf(x[t], spec.q_mean[t, 0], spec.q_chol[t, 0, 0]))
        assert abs(out.logZ - lw) < 1e-10 * max(1, abs(lw))


def test_independence_model_increments_vanish():
    """If p_c(x | x') = q_c(x) (transition independent of the past and equal to
    the proposal), omega = p / q = 1 under leaf_obs, so every increment is
    log sum W_L W_R = 0 and W = W_L x W_R."""
    spec = W.sv(9, seed=3)
    spec.F = np.zeros((1, 1))
    spec.f = spec.q_mean[0].copy()
    spec.Q_chol = spec.q_chol[0].copy()
    out = D.smooth(spec, 16, seed=4)
    assert np.max(np.abs(out.Zc)) < 1e-12
    assert abs(out.logZ - out.leaves.logL.sum()) < 1e-11


def test_nan_raises():
    spec = W.sv(4, seed=1)
    spec.y = spec.y.copy()
    spec.y[2, 0] = np.nan
    with pytest.raises(FloatingPointError):
        D.smooth(spec, 8, seed=1)


def test_zero_leaf_weights_degenerate():
    """A time point where every leaf weight is zero: L_t = 0, uniform weights,
    log L = -inf and the run is flagged degenerate."""
    spec = W.sv(5, seed=1)
    spec.y = spec.y.copy()
    spec.y[3, 0] = np.inf
    out = D.smooth(spec, 8, seed=2)
    assert out.degenerate and out.logZ == -np.inf
    assert out.leaves.logL[3] == -np.inf
    np.testing.assert_allclose(out.leaves.logw[3], -np.log(8))
