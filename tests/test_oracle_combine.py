"""Pins of the oracle's combine (Algorithm 1) and leaves (Algorithm 2).

The references here are written independently of the oracle: densities come
from scipy.stats and weights are formed as products of densities, following
the normalised-weights equation of Section 2.2 and Proposition 2.3 directly.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import dsmc as D
from oracle import philox as P
from paper_2202_02264_amd import workloads as W


def _pdf_prior(spec, x):
    return stats.norm.pdf(x, spec.m0[0], spec.P0_chol[0, 0])


def _pdf_trans(spec, x1, x0):
    return stats.norm.pdf(x1, spec.F[0, 0] * x0 + spec.f[0], spec.Q_chol[0, 0])


def _pdf_q(spec, t, x):
    return stats.norm.pdf(x, spec.q_mean[t, 0], spec.q_chol[t, 0, 0])


def _pdf_h(spec, t, x):
    y = spec.y[t, 0]
    if spec.obs == "sv":
        return stats.norm.pdf(y, 0.0, np.exp(0.5 * x))
    return stats.norm.pdf(y, spec.H[0, 0] * x + spec.h[0], spec.R_chol[0, 0])


MODELS = {
    "lg1d": lambda w: W.lg1d(2, A=0.7, Q=0.8, R=0.6, seed=3, weighting=w),
    "sv": lambda w: W.sv(2, seed=4, weighting=w),
}


def _explicit_W(spec, x0, x1):
    """W^{mn} proportional to w_0^m w_1^n omega_1(x0^m, x1^n) at K = 2, with
    w_0 = h_0 dP_0/dq_0 (Proposition 2.2) and, per weighting,
    leaf_obs:      w_1 = h_1,  omega_1 = p_1 / q_1
    boundary_obs:  w_1 = 1,    omega_1 = p_1 h_1 / q_1     (Proposition 2.3)."""
    w0 = _pdf_h(spec, 0, x0) * _pdf_prior(spec, x0) / _pdf_q(spec, 0, x0)
    if spec.weighting == "leaf_obs":
        w1 = _pdf_h(spec, 1, x1)
        om = _pdf_trans(spec, x1[None, :], x0[:, None]) / _pdf_q(spec, 1, x1)[None, :]
    else:
        w1 = np.ones_like(x1)
        om = (_pdf_trans(spec, x1[None, :], x0[:, None]) * _pdf_h(spec, 1, x1)[None, :]
              / _pdf_q(spec, 1, x1)[None, :])
    un = (w0 / w0.sum())[:, None] * (w1 / w1.sum())[None, :] * om
    return un, w0, w1


@pytest.mark.parametrize("model", sorted(MODELS))
@pytest.mark.parametrize("weighting", ["leaf_obs", "boundary_obs"])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_brute_force_two_points(model, weighting, N):
    spec = MODELS[model](weighting)
    lv = D.sample_leaves(spec, N, seed=9)
    x0, x1 = lv.x[0, :, 0], lv.x[1, :, 0]
    un, w0, w1 = _explicit_W(spec, x0, x1)
    u1, u2 = P.combine_uniforms(9, 1, N)
    res = D.combine(spec, 1, lv.x[0], lv.x[1], lv.logw[0], lv.logw[1], u1, u2, keep_S=True)
    Wn = np.exp(res.S - res.Z)
    assert abs(Wn.sum() - 1.0) < 1e-12
    np.testing.assert_allclose(Wn, un / un.sum(), rtol=1e-10, atol=1e-300)
    np.testing.assert_allclose(res.row_lse, np.log(np.exp(res.S).sum(1)), rtol=1e-12, atol=1e-12)
    # the whole-smoother estimate at K = 2 is the plain importance-sampling sum
    # over all N^2 pairs, whatever the weighting (Section 2.2, equation for L_{a:b})
    L_explicit = np.sum(w0[:, None] * _pdf_h(spec, 1, x1)[None, :]
                        * _pdf_trans(spec, x1[None, :], x0[:, None])
                        / _pdf_q(spec, 1, x1)[None, :]) / N ** 2
    out = D.smooth(spec, N, seed=9)
    assert abs(out.logZ - np.log(L_explicit)) < 1e-11 * max(1.0, abs(out.logZ))
    # the indices follow the flat multinomial on W read by the (row, column)
    # inverse CDF: row by the cumulated row sums, column inside the row
    for n in range(N):
        rows = np.cumsum(un.sum(1))
        m = int(np.argmax(u1[n] * rows[-1] < rows))
        cols = np.cumsum(un[m])
        j = int(np.argmax(u2[n] * cols[-1] < cols))
        assert (res.l[n], res.r[n]) == (m, j)


@pytest.mark.parametrize("weighting", ["leaf_obs", "boundary_obs"])
def test_draw_frequencies_match_W(weighting):
    """Chi-square of many combine draws against the explicit W (N = 4)."""
    spec = MODELS["sv"](weighting)
    N, rep = 4, 100
    lv = D.sample_leaves(spec, N, seed=21)
    x0, x1 = lv.x[0, :, 0], lv.x[1, :, 0]
    un, _, _ = _explicit_W(spec, x0, x1)
    Wn = un / un.sum()
    # replicate each particle `rep` times: the draws of (l mod N, r mod N) then
    # follow W over the N original particles
    xL = np.repeat(lv.x[0], rep, axis=0)
    xR = np.repeat(lv.x[1], rep, axis=0)
    lwL = np.repeat(lv.logw[0], rep) - np.log(rep)
    lwR = np.repeat(lv.logw[1], rep) - np.log(rep)
    counts = np.zeros((N, N))
    for s in range(100):
        u1, u2 = P.combine_uniforms(1000 + s, 1, N * rep)
        res = D.combine(spec, 1, xL, xR, lwL, lwR, u1, u2)
        np.add.at(counts, (res.l // rep, res.r // rep), 1)
    total = counts.sum()
    exp = Wn * total
    keep = exp > 5
    chi2 = np.sum((counts[keep] - exp[keep]) ** 2 / exp[keep])
    p = stats.chi2.sf(chi2, keep.sum() - 1)
    assert p > 1e-3, (chi2, p)


def test_inverse_cdf_edges():
    w = np.array([0.0, 1.0, 0.0, 0.0, 2.0, 0.0])
    assert D.inverse_cdf(w, 0.0) == 1
    assert D.inverse_cdf(w, 1.0 / 3.0 - 1e-12) == 1
    assert D.inverse_cdf(w, 1.0 / 3.0) == 4          # boundary goes right (strict <)
    assert D.inverse_cdf(w, 1.0 - 2.0 ** -53) == 4
    assert D.inverse_cdf(w, 1.0) == 4                # u * total == total: last positive bin
    assert D.inverse_cdf(np.array([5.0]), 0.7) == 0


def test_leaf_weights_explicit():
    """Algorithm 2 with Proposition 2.2: w_0 = h_0 p_0 / q_0, w_t = h_t (leaf_obs)."""
    spec = W.sv(6, seed=2)
    N = 50
    lv = D.sample_leaves(spec, N, seed=5)
    for t in range(6):
        x = lv.x[t, :, 0]
        w = _pdf_h(spec, t, x) * (_pdf_prior(spec, x) / _pdf_q(spec, t, x) if t == 0 else 1.0)
        np.testing.assert_allclose(np.exp(lv.logw[t]), w / w.sum(), rtol=1e-12)
        assert abs(lv.logL[t] - np.log(w.mean())) < 1e-12
    # the particles are q_t draws built from the Philox normals
    z = P.leaf_normals(5, 3, N, 1)[:, 0]
    np.testing.assert_allclose(lv.x[3, :, 0], spec.q_mean[3, 0] + spec.q_chol[3, 0, 0] * z, rtol=1e-15)


def test_degenerate_combine():
    """All pair weights zero: increment -inf, uniform indices, degenerate flag."""
    spec = W.lg1d(2, seed=1)
    N = 8
    xL = np.zeros((N, 1))
    xR = np.zeros((N, 1))
    lwL = np.full(N, -np.inf)
    lwR = np.full(N, -np.log(N))
    u1, u2 = P.combine_uniforms(3, 1, N)
    res = D.combine(spec, 1, xL, xR, lwL, lwR, u1, u2)
    assert res.degenerate and res.Z == -np.inf
    np.testing.assert_array_equal(res.l, np.floor(u1 * N).astype(int))
    np.testing.assert_array_equal(res.r, np.floor(u2 * N).astype(int))


def test_zero_weight_particles_never_drawn():
    spec = W.lg1d(2, seed=1)
    N = 16
    lv = D.sample_leaves(spec, N, seed=4)
    lwL = lv.logw[0].copy()
    lwL[::2] = -np.inf
    lwL -= D.logsumexp(lwL)
    lwR = lv.logw[1].copy()
    lwR[1::2] = -np.inf
    lwR -= D.logsumexp(lwR)
    u1, u2 = P.combine_uniforms(4, 1, N)
    res = D.combine(spec, 1, lv.x[0], lv.x[1], lwL, lwR, u1, u2)
    assert np.all(res.l % 2 == 1) and np.all(res.r % 2 == 0)
