"""Log densities of the state-space model family, in fp64.

TEST INFRASTRUCTURE: part of the fp64 CPU oracle; see oracle/__init__.py.

The model is the Feynman-Kac form of the paper (Section 1): prior P_0,
transitions P_t(dx_t | x_{t-1}) with density p_t, potentials h_t and the
independent proposals q_t of Algorithm 2.  ``spec`` is any object carrying the
fields of ``paper_2202_02264_amd.workloads.SSM`` (duck-typed; this module does
not import the GPU package).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

LOG2PI = float(np.log(2.0 * np.pi))


def gauss_logpdf(x: np.ndarray, mean: np.ndarray, chol: np.ndarray) -> np.ndarray:
    """log N(x; mean, chol chol^T) along the last axis; x and mean broadcast."""
    x = np.asarray(x, dtype=np.float64)
    d = chol.shape[0]
    diff = np.broadcast_to(x - mean, np.broadcast_shapes(np.shape(x), np.shape(mean)))
    flat = diff.reshape(-1, d)
    z = solve_triangular(chol, flat.T, lower=True).T
    quad = np.sum(z * z, axis=-1).reshape(diff.shape[:-1])
    return -0.5 * quad - np.sum(np.log(np.diag(chol))) - 0.5 * d * LOG2PI


def log_prior(spec, x: np.ndarray) -> np.ndarray:
    """log p_0(x) of P_0 = N(m0, P0); x shape (..., d_x)."""
    return gauss_logpdf(x, spec.m0, spec.P0_chol)


def log_potential(spec, t: int, x: np.ndarray) -> np.ndarray:
    """log h_t(x) = log density of y_t given x_t = x; for the "box" kind the
    indicator of lo <= x <= hi with y_t = (lo, hi) (the constrained random
    walk of Section 5.3)."""
    y = spec.y[t]
    if spec.obs == "box":
        d = spec.d_x
        inside = np.all((x >= y[:d]) & (x <= y[d:]), axis=-1)
        return np.where(inside, 0.0, -np.inf)
    if spec.obs == "sv":
        v = x[..., 0]
        return -0.5 * LOG2PI - 0.5 * v - 0.5 * y[0] * y[0] * np.exp(-v)
    mean = x @ spec.H.T + spec.h
    return gauss_logpdf(y, mean, spec.R_chol)


def _half_widths(spec, t: int) -> np.ndarray:
    return np.diag(spec.q_chol[t])


def log_proposal(spec, t: int, x: np.ndarray) -> np.ndarray:
    """log q_t(x): Gaussian N(q_mean[t], q_chol[t] q_chol[t]^T), or for a
    "uniform" proposal the uniform density on the box q_mean[t] +- the
    diagonal of q_chol[t]."""
    if getattr(spec, "proposal", "gaussian") == "uniform":
        hw = _half_widths(spec, t)
        inside = np.all(np.abs(x - spec.q_mean[t]) <= hw, axis=-1)
        return np.where(inside, -np.sum(np.log(2.0 * hw)), -np.inf)
    return gauss_logpdf(x, spec.q_mean[t], spec.q_chol[t])


def proposal_draw(spec, t: int, z: np.ndarray) -> np.ndarray:
    """x = q_mean[t] + q_chol[t] z for standard normals z of shape (N, d_x)
    (Gaussian proposals), or x = q_mean[t] + hw (2 z - 1) for uniforms z in
    [0, 1) (uniform proposals, hw the box half-widths)."""
    if getattr(spec, "proposal", "gaussian") == "uniform":
        return spec.q_mean[t][None, :] + _half_widths(spec, t)[None, :] * (2.0 * z - 1.0)
    return spec.q_mean[t][None, :] + z @ spec.q_chol[t].T


def log_transition_pairs(spec, xL: np.ndarray, xR: np.ndarray) -> np.ndarray:
    """Matrix T[m, n] = log p(x_c = xR[n] | x_{c-1} = xL[m]) for the
    Gaussian transition N(F x + f, Q); xL, xR shape (N, d_x).  Row blocks keep
    the (rows, N, d_x) temporary bounded."""
    NL, NR, d = xL.shape[0], xR.shape[0], xL.shape[1]
    mean = xL @ spec.F.T + spec.f
    out = np.empty((NL, NR))
    step = max(1, int(2_000_000 // max(1, NR * d)))
    for m0 in range(0, NL, step):
        m1 = min(NL, m0 + step)
        out[m0:m1] = gauss_logpdf(xR[None, :, :], mean[m0:m1, None, :], spec.Q_chol)
    return out
