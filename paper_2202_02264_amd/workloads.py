"""Seeded synthetic state-space models and data for the dSMC smoother.

This module only builds inputs: model parameters and observations simulated
from the model with numpy's Philox generator.  It holds none of the smoother's
arithmetic and is shared by the GPU binding, the tests, ``bench.py`` and the
oracle's tests.

Model family (paper, Section 1, the Feynman-Kac form of the state-space model):

* prior        P_0 = N(m0, P0)                       (P0 = P0_chol P0_chol^T)
* transition   P_t(x_t | x_{t-1}) = N(F x_{t-1} + f, Q)   for t >= 1
* potential    h_t(x_t) = density of y_t given x_t, either
               "lg":  y_t ~ N(H x_t + h, R)
               "sv":  y_t ~ N(0, exp(x_t))                (d_x = d_y = 1)
* proposal     q_t = N(q_mean[t], q_chol[t] q_chol[t]^T), independent over t
               (the independent proposals dSMC needs, Section 4).

``weighting`` selects the auxiliary measures nu_t of Definition 2.1:
"leaf_obs" takes nu_t proportional to h_t q_t (the potential is applied at
the leaves); "boundary_obs" takes nu_t = q_t, as in the paper's experiments
(the potential enters the stitching weight omega_c of Proposition 2.3).

Time points are t = 0..K-1 (the paper's t = 0..T with K = T + 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

DATA_SEED = 20220204


@dataclass
class SSM:
    d_x: int
    d_y: int
    m0: np.ndarray
    P0_chol: np.ndarray
    F: np.ndarray
    f: np.ndarray
    Q_chol: np.ndarray
    obs: str
    y: np.ndarray
    q_mean: np.ndarray
    q_chol: np.ndarray
    H: Optional[np.ndarray] = None
    h: Optional[np.ndarray] = None
    R_chol: Optional[np.ndarray] = None
    weighting: str = "leaf_obs"
    name: str = ""
    proposal: str = "gaussian"   # or "uniform": q_t uniform on q_mean[t] +- diag(q_chol[t])
    x_true: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def K(self) -> int:
        return int(self.y.shape[0])

    def with_weighting(self, weighting: str) -> "SSM":
        return replace(self, weighting=weighting)

    def truncated(self, K: int) -> "SSM":
        """The same model restricted to the first K time points."""
        return replace(self, y=self.y[:K].copy(), q_mean=self.q_mean[:K].copy(),
                       q_chol=self.q_chol[:K].copy(),
                       x_true=None if self.x_true is None else self.x_true[:K].copy())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed) & ((1 << 64) - 1)))


def _as2(a) -> np.ndarray:
    return np.atleast_2d(np.asarray(a, dtype=np.float64))


def simulate(spec: SSM, K: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Draw (x_{0:K-1}, y_{0:K-1}) from the model."""
    g = _rng(seed)
    dx = spec.d_x
    x = np.empty((K, dx))
    x[0] = spec.m0 + spec.P0_chol @ g.standard_normal(dx)
    if dx == 1:
        from scipy.signal import lfilter
        e = spec.f[0] + spec.Q_chol[0, 0] * g.standard_normal(K - 1)
        a = spec.F[0, 0]
        if K > 1:
            x[1:, 0] = lfilter([1.0], [1.0, -a], e, zi=[a * x[0, 0]])[0]
    else:
        for t in range(1, K):
            x[t] = spec.F @ x[t - 1] + spec.f + spec.Q_chol @ g.standard_normal(dx)
    if spec.obs == "sv":
        y = (np.exp(0.5 * x[:, 0]) * g.standard_normal(K))[:, None]
    else:
        dy = spec.d_y
        y = x @ spec.H.T + spec.h + g.standard_normal((K, dy)) @ spec.R_chol.T
    return x, y


def _finish(spec: SSM, K: int, seed: int) -> SSM:
    x, y = simulate(spec, K, seed)
    spec.y = y
    spec.x_true = x
    return spec


def lg1d(K: int, A: float = 0.9, Q: float = 1.0, R: float = 1.0, m0: float = 0.0,
         P0: float = 1.0, seed: int = DATA_SEED, proposal: str = "prior",
         weighting: str = "leaf_obs") -> SSM:
    """1-D linear-Gaussian model x_t = A x_{t-1} + N(0, Q), y_t = x_t + N(0, R).

    proposal="prior": q_t is the prior marginal of X_t, N(mean_t, P_t) with
    P_t = A^2 P_{t-1} + Q (an independent proposal, the closest independent
    analogue of a bootstrap proposal).
    """
    tt = np.arange(K)
    means = m0 * A ** tt
    a2t = (A * A) ** tt
    var = a2t * P0 + (Q * tt if A * A == 1.0 else Q * (1.0 - a2t) / (1.0 - A * A))
    spec = SSM(d_x=1, d_y=1, m0=np.array([m0]), P0_chol=np.array([[np.sqrt(P0)]]),
               F=np.array([[A]]), f=np.zeros(1), Q_chol=np.array([[np.sqrt(Q)]]),
               obs="lg", H=np.eye(1), h=np.zeros(1), R_chol=np.array([[np.sqrt(R)]]),
               y=np.zeros((K, 1)), q_mean=means[:, None].copy(),
               q_chol=np.sqrt(var)[:, None, None].copy(), weighting=weighting,
               name=f"lg1d(K={K},A={A},Q={Q},R={R})")
    if proposal != "prior":
        raise ValueError(proposal)
    return _finish(spec, K, seed)


def sv(K: int, mu: float = -1.0, rho: float = 0.95, sigma: float = 0.3,
       seed: int = DATA_SEED, weighting: str = "leaf_obs") -> SSM:
    """Stochastic volatility: x_t = mu + rho (x_{t-1} - mu) + sigma e_t, y_t ~ N(0, exp(x_t)).

    Prior and proposals are the stationary law N(mu, sigma^2 / (1 - rho^2)), as the
    paper does for its Poisson model with the same latent dynamics (Section 5.1).
    """
    s2 = sigma * sigma / (1.0 - rho * rho)
    sd = np.sqrt(s2)
    spec = SSM(d_x=1, d_y=1, m0=np.array([mu]), P0_chol=np.array([[sd]]),
               F=np.array([[rho]]), f=np.array([mu * (1.0 - rho)]),
               Q_chol=np.array([[sigma]]), obs="sv", y=np.zeros((K, 1)),
               q_mean=np.full((K, 1), mu), q_chol=np.full((K, 1, 1), sd),
               weighting=weighting, name=f"sv(K={K},mu={mu},rho={rho},sigma={sigma})")
    return _finish(spec, K, seed)


def lg(K: int, F: np.ndarray, Q_chol: np.ndarray, H: np.ndarray, R_chol: np.ndarray,
       m0: np.ndarray, P0_chol: np.ndarray, seed: int = DATA_SEED,
       proposal: str = "rts", weighting: str = "leaf_obs", name: str = "lg",
       f: Optional[np.ndarray] = None, h: Optional[np.ndarray] = None) -> SSM:
    """General linear-Gaussian model x_t = F x_{t-1} + f + N(0, Q),
    y_t = H x_t + h + N(0, R) (f, h default to zero); proposal "rts" = exact
    smoothing marginals (the Gaussian-approximation proposals of Section 4.1,
    exact for this model), "prior" = prior marginals."""
    dx, dy = F.shape[0], H.shape[0]
    spec = SSM(d_x=dx, d_y=dy, m0=np.asarray(m0, float), P0_chol=_as2(P0_chol),
               F=_as2(F), f=np.zeros(dx) if f is None else np.asarray(f, float).reshape(dx),
               Q_chol=_as2(Q_chol), obs="lg", H=_as2(H),
               h=np.zeros(dy) if h is None else np.asarray(h, float).reshape(dy),
               R_chol=_as2(R_chol), y=np.zeros((K, dy)),
               q_mean=np.zeros((K, dx)), q_chol=np.zeros((K, dx, dx)),
               weighting=weighting, name=name)
    _finish(spec, K, seed)
    if proposal == "rts":
        means, covs = _rts_for_proposal(spec)
    elif proposal == "prior":
        means, covs = _prior_marginals(spec, K)
    else:
        raise ValueError(proposal)
    spec.q_mean = means
    spec.q_chol = np.linalg.cholesky(covs)
    return spec


def _prior_marginals(spec: SSM, K: int):
    dx = spec.d_x
    means = np.zeros((K, dx))
    covs = np.zeros((K, dx, dx))
    means[0] = spec.m0
    covs[0] = spec.P0_chol @ spec.P0_chol.T
    Q = spec.Q_chol @ spec.Q_chol.T
    for t in range(1, K):
        means[t] = spec.F @ means[t - 1] + spec.f
        covs[t] = spec.F @ covs[t - 1] @ spec.F.T + Q
    return means, 0.5 * (covs + np.swapaxes(covs, 1, 2))


def _rts_for_proposal(spec: SSM):
    """Sequential Kalman filter + RTS smoother used only to build proposals."""
    K, dx = spec.K, spec.d_x
    Q = spec.Q_chol @ spec.Q_chol.T
    R = spec.R_chol @ spec.R_chol.T
    H, F = spec.H, spec.F
    mf = np.zeros((K, dx)); Pf = np.zeros((K, dx, dx))
    mp = np.zeros((K, dx)); Pp = np.zeros((K, dx, dx))
    m, P = spec.m0.copy(), spec.P0_chol @ spec.P0_chol.T
    for t in range(K):
        if t > 0:
            m, P = F @ m + spec.f, F @ P @ F.T + Q
        mp[t], Pp[t] = m, P
        S = H @ P @ H.T + R
        G = np.linalg.solve(S, H @ P).T
        m = m + G @ (spec.y[t] - H @ m - spec.h)
        P = P - G @ S @ G.T
        P = 0.5 * (P + P.T)
        mf[t], Pf[t] = m, P
    ms, Ps = mf.copy(), Pf.copy()
    for t in range(K - 2, -1, -1):
        C = np.linalg.solve(Pp[t + 1], F @ Pf[t]).T
        ms[t] = mf[t] + C @ (ms[t + 1] - mp[t + 1])
        Ps[t] = Pf[t] + C @ (Ps[t + 1] - Pp[t + 1]) @ C.T
        Ps[t] = 0.5 * (Ps[t] + Ps[t].T)
    return ms, Ps


def random_orthogonal(d: int, g: np.random.Generator) -> np.ndarray:
    a = g.standard_normal((d, d))
    qm, r = np.linalg.qr(a)
    return qm * np.sign(np.diag(r))[None, :]


def lg_highdim(K: int = 2048, d_x: int = 32, d_y: int = 8, a: float = 0.95,
               q: float = 0.1, r: float = 0.5, seed: int = DATA_SEED,
               weighting: str = "leaf_obs") -> SSM:
    """d_x-dimensional linear-Gaussian model: A = a * random orthogonal, Q = q I,
    y_t = C x_t + N(0, r I) with C a d_y x d_x Gaussian matrix / sqrt(d_x);
    x_0 ~ stationary law; proposals = smoothing marginals."""
    g = _rng(seed + 1)
    F = a * random_orthogonal(d_x, g)
    H = g.standard_normal((d_y, d_x)) / np.sqrt(d_x)
    # stationary covariance of x_t = F x_{t-1} + N(0, qI) with F = a * orthogonal
    P0 = np.eye(d_x) * q / (1.0 - a * a)
    return lg(K, F, np.sqrt(q) * np.eye(d_x), H, np.sqrt(r) * np.eye(d_y), np.zeros(d_x),
              np.linalg.cholesky(P0), seed=seed, proposal="rts", weighting=weighting,
              name=f"lg(K={K},d_x={d_x},d_y={d_y})")


def lg1d_batch(B: int = 512, K_lo: int = 64, K_hi: int = 8192, seed: int = DATA_SEED,
               weighting: str = "leaf_obs") -> list[SSM]:
    """B independent 1-D linear-Gaussian series: A ~ U[0.5, 0.99], Q, R ~ U[0.1, 2],
    K ~ U{K_lo..K_hi}, x_0 from the stationary law, prior-marginal proposals."""
    g = _rng(seed + 7)
    out = []
    for i in range(B):
        A = float(g.uniform(0.5, 0.99))
        Q = float(g.uniform(0.1, 2.0))
        R = float(g.uniform(0.1, 2.0))
        K = int(g.integers(K_lo, K_hi + 1))
        P0 = Q / (1.0 - A * A)
        out.append(lg1d(K, A=A, Q=Q, R=R, m0=0.0, P0=P0, seed=seed + 1000 + i,
                        weighting=weighting))
    return out


def lg4d(K: int, seed: int = DATA_SEED, weighting: str = "leaf_obs",
         proposal: str = "prior") -> SSM:
    """4-D linear-Gaussian model: A = 0.9 * random orthogonal, Q = 0.5 I, H = I, R = I,
    x_0 stationary; prior-marginal ("prior") or RTS smoothing-marginal ("rts")
    proposals."""
    g = _rng(seed + 3)
    F = 0.9 * random_orthogonal(4, g)
    P0 = np.eye(4) * 0.5 / (1.0 - 0.81)
    return lg(K, F, np.sqrt(0.5) * np.eye(4), np.eye(4), np.eye(4), np.zeros(4),
              np.linalg.cholesky(P0), seed=seed, proposal=proposal, weighting=weighting,
              name=f"lg4d(K={K})")


def c1_lg1d() -> SSM:
    """Correctness workload: 1-D LG, A = 0.9, Q = R = 1, x_0 ~ N(0, 1), K = 32."""
    return lg1d(32)


def c2_sv() -> SSM:
    """Headline workload: stochastic volatility, K = 4096 time points."""
    return sv(4096)


def serving_jobs(J: int, seed: int = DATA_SEED, K_median: float = 512.0, sigma_log: float = 1.0,
                 K_cap: int = 16384, Ns=(256, 1024, 4096), bases: int = 4):
    """A seeded stream of J smoothing jobs: half stochastic-volatility, half
    4-D linear-Gaussian (RTS proposals); K = floor(lognormal(log K_median,
    sigma_log)) clipped to [2, K_cap]; N uniform over Ns.  Each job's model is
    the first K points of one of `bases` long series per model family.
    Returns (spec, N, seed) triples."""
    g = _rng(seed + 11)
    sv_b = [sv(K_cap, seed=seed + 100 + i) for i in range(bases)]
    lg_b = [lg4d(K_cap, seed=seed + 200 + i, proposal="rts") for i in range(bases)]
    jobs = []
    for j in range(J):
        K = int(np.clip(np.floor(np.exp(np.log(K_median) + sigma_log * g.standard_normal())),
                        2, K_cap))
        fam = sv_b if g.random() < 0.5 else lg_b
        base = fam[int(g.integers(bases))]
        N = int(Ns[int(g.integers(len(Ns)))])
        jobs.append((base.truncated(K), N, 1 + j))
    return jobs


def constrained_rw(K: int, sigma: float = 0.5, weighting: str = "boundary_obs") -> SSM:
    """Constrained random walk (the lazy-resampling experiment, Section 5.3):
    x_0 ~ N(0, 1), x_t = x_{t-1} + sigma eps_t, potential the indicator of
    -1 <= x_t <= 1 (y_t holds the bounds), proposals q_t = U([-1, 1])."""
    spec = SSM(d_x=1, d_y=2, m0=np.zeros(1), P0_chol=np.eye(1), F=np.eye(1), f=np.zeros(1),
               Q_chol=np.array([[sigma]]), obs="box", y=np.tile([-1.0, 1.0], (K, 1)),
               q_mean=np.zeros((K, 1)), q_chol=np.ones((K, 1, 1)), weighting=weighting,
               name=f"crw(K={K},sigma={sigma})", proposal="uniform")
    return spec
