"""Kalman filter, RTS smoother and exact log-likelihood of a linear-Gaussian model.

TEST INFRASTRUCTURE: part of the fp64 CPU oracle; see oracle/__init__.py.

The linear-Gaussian state-space model has closed-form smoothing marginals and
normalising constant (the paper's introduction names LGSSMs as the closed-form
case); these pin the Monte Carlo smoother.  Observations y_t exist for
t = 0..K-1, the transition acts for t >= 1.
"""
from __future__ import annotations

import numpy as np


def kalman_smoother(spec):
    """Returns (smoothed means (K, d_x), smoothed covariances (K, d_x, d_x),
    log p(y_{0:K-1}))."""
    K, dx = spec.K, spec.d_x
    F, f, H, h = spec.F, spec.f, spec.H, spec.h
    Q = spec.Q_chol @ spec.Q_chol.T
    R = spec.R_chol @ spec.R_chol.T
    mf = np.zeros((K, dx)); Pf = np.zeros((K, dx, dx))
    mp = np.zeros((K, dx)); Pp = np.zeros((K, dx, dx))
    m = np.array(spec.m0, dtype=np.float64)
    P = spec.P0_chol @ spec.P0_chol.T
    loglik = 0.0
    for t in range(K):
        if t > 0:
            m = F @ m + f
            P = F @ P @ F.T + Q
        mp[t], Pp[t] = m, P
        S = H @ P @ H.T + R
        v = spec.y[t] - (H @ m + h)
        sign, logdet = np.linalg.slogdet(2.0 * np.pi * S)
        loglik += -0.5 * (logdet + v @ np.linalg.solve(S, v))
        G = P @ H.T @ np.linalg.inv(S)
        m = m + G @ v
        P = P - G @ S @ G.T
        mf[t], Pf[t] = m, P
    ms, Ps = mf.copy(), Pf.copy()
    for t in range(K - 2, -1, -1):
        C = Pf[t] @ F.T @ np.linalg.inv(Pp[t + 1])
        ms[t] = mf[t] + C @ (ms[t + 1] - mp[t + 1])
        Ps[t] = Pf[t] + C @ (Ps[t + 1] - Pp[t + 1]) @ C.T
    return ms, Ps, float(loglik)


def joint_gaussian(spec):
    """Mean and covariance of the stacked (x_{0:K-1}, y_{0:K-1}) under the model,
    built directly from the model equations; a brute-force check of the
    Kalman recursions for small K."""
    K, dx, dy = spec.K, spec.d_x, spec.d_y
    Q = spec.Q_chol @ spec.Q_chol.T
    R = spec.R_chol @ spec.R_chol.T
    # x_t = F^t x_0 + sum_{s=1}^t F^{t-s} (f + e_s)
    mx = np.zeros((K, dx))
    mx[0] = spec.m0
    for t in range(1, K):
        mx[t] = spec.F @ mx[t - 1] + spec.f
    Fp = [np.eye(dx)]
    for _ in range(K):
        Fp.append(spec.F @ Fp[-1])
    P0 = spec.P0_chol @ spec.P0_chol.T
    Cxx = np.zeros((K * dx, K * dx))
    for t in range(K):
        for u in range(K):
            c = Fp[t] @ P0 @ Fp[u].T
            for s in range(1, min(t, u) + 1):
                c = c + Fp[t - s] @ Q @ Fp[u - s].T
            Cxx[t * dx:(t + 1) * dx, u * dx:(u + 1) * dx] = c
    Hb = np.kron(np.eye(K), spec.H)
    my = (mx @ spec.H.T + spec.h).reshape(-1)
    Cyy = Hb @ Cxx @ Hb.T + np.kron(np.eye(K), R)
    Cxy = Cxx @ Hb.T
    return mx.reshape(-1), my, Cxx, Cxy, Cyy
