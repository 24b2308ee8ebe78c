"""Test harness: run the HIP smoother through the C ABI and compare it with the
oracle, level by level, on the GPU's own inputs (teacher forcing).

A draw is *near a boundary* when its uniform lies within BAND of a boundary of
the oracle's normalised CDF (the row marginal for the left index; the chosen
row for the right index).  Index parity is bit-exact outside that band.
"""
from __future__ import annotations

import os
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from oracle import dsmc as D
from oracle import philox as P

BAND = 1e-6
TOL32 = 1e-5
TOL64 = 1e-10


def log(msg: str) -> None:
    """Print a progress / result line; also append it to $DSMC_PARITY_LOG if set."""
    line = f"[{time.strftime('%H:%M:%S')}] {msg}"
    print(line, flush=True)
    sys.stdout.flush()
    path = os.environ.get("DSMC_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")


def run_gpu(spec, N: int, seed: int, precision: str = "fp32", plan=None, model=None,
            rescue_all: bool = False, star=None):
    """dsmc_smooth (dsmc_smooth_conditional if ``star`` (K, d_x) is given) with
    every diagnostic output; returns numpy arrays."""
    import torch
    from paper_2202_02264_amd import dsmc as G
    prec = {"fp64": G.DSMC_FP64, "fp32": G.DSMC_FP32, "bf16": G.DSMC_BF16}[precision]
    log(f"gpu dsmc_smooth {spec.name} weighting={spec.weighting} N={N} seed={seed} {precision}")
    model = model or G.Model(spec)
    plan = plan or G.Plan(N, spec.d_x, spec.K, precision=prec, rescue_all=rescue_all)
    out = G.alloc_output(plan, spec.K, diagnostics=True)
    if star is None:
        G.dsmc_smooth(plan, model, seed, out)
    else:
        st = torch.tensor(np.ascontiguousarray(np.asarray(star, np.float64).reshape(spec.K, -1).T),
                          dtype=plan.dtype, device="cuda")
        G.dsmc_smooth_conditional(plan, model, seed, st, out)
    torch.cuda.synchronize()
    res = {}
    for k in ("traj", "logw", "log_Z", "status", "leaf_x", "leaf_logw", "leaf_logL", "ancestry",
              "logZ_inc", "row_lse", "index"):
        res[k] = getattr(out, k).cpu().numpy()
    log("gpu done")
    return res


def _dist_to_boundary(u: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Distance of each u to the nearest inner boundary of the normalised CDF of w."""
    cum = np.cumsum(w)
    cdf = cum[:-1] / cum[-1]
    if cdf.size == 0:
        return np.full(np.shape(u), np.inf)
    i = np.searchsorted(cdf, u)
    lo = np.abs(u - cdf[np.clip(i - 1, 0, cdf.size - 1)])
    hi = np.abs(u - cdf[np.clip(i, 0, cdf.size - 1)])
    return np.minimum(lo, hi)


@dataclass
class ParityReport:
    nodes: int = 0
    draws: int = 0
    near: int = 0
    mismatches: int = 0
    mismatches_outside_band: int = 0
    max_rel_err_Z: float = 0.0
    max_rel_err_row: float = 0.0
    worst: list = field(default_factory=list)
    abs_err_Z: list = field(default_factory=list)    # filled when tol is None
    abs_err_row: list = field(default_factory=list)  # arrays, filled when tol is None

    def summary(self) -> str:
        f = self.near / max(1, self.draws)
        return (f"nodes={self.nodes} draws={self.draws} near-boundary={self.near} ({f:.2e}) "
                f"mismatches={self.mismatches} outside-band={self.mismatches_outside_band} "
                f"max|dZ|rel={self.max_rel_err_Z:.2e} max|drow|rel={self.max_rel_err_row:.2e}")


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    both_inf = (a == b)
    err = np.abs(a - b) / np.maximum(1.0, np.abs(b))
    return np.where(both_inf, 0.0, err)


def check_leaves(spec, N: int, seed: int, g: dict, tol: float, star=None) -> None:
    """Leaf particles equal the oracle's draws rounded to the stored type; leaf
    log-weights and log L_t equal the oracle's on the stored particles.  With
    ``star`` (already in the stored type) the conditional leaves are checked."""
    K, dx = spec.K, spec.d_x
    xg = np.moveaxis(g["leaf_x"], 0, -1).astype(np.float64)  # (K, N, dx)
    ref = (D.sample_leaves(spec, N, seed) if star is None
           else D.sample_leaves_conditional(spec, N, seed, star))
    xr = ref.x.astype(g["leaf_x"].dtype).astype(np.float64)
    diff = np.abs(xg - xr)
    ulp = np.spacing(np.abs(xr).astype(g["leaf_x"].dtype)).astype(np.float64)
    assert np.all(diff <= ulp), float(np.max(diff / np.maximum(ulp, 1e-300)))
    assert np.mean(diff > 0) < 1e-3
    lv = D.sample_leaves(spec, N, seed, x=xg)
    e_w = _rel(g["leaf_logw"], lv.logw)
    e_L = _rel(g["leaf_logL"], lv.logL)
    assert np.max(e_w) <= tol, np.max(e_w)
    assert np.max(e_L) <= tol, np.max(e_L)


def teacher_forced(spec, N: int, seed: int, g: dict, tol, select=None,
                   conditional: bool = False) -> ParityReport:
    """Replay the GPU's ancestry; at every selected node run the oracle's combine
    on the GPU's inputs of that level and compare increments, row log-sums and
    indices (Algorithm 4's with ``conditional``).  Also checks the gather:
    final index and trajectories.  With tol=None the absolute errors are
    collected instead of asserted."""
    K, dx = spec.K, spec.d_x
    rep = ParityReport()
    leaf_x = g["leaf_x"].astype(np.float64)            # (dx, K, N)
    sig = np.tile(np.arange(N), (K, 1))
    logN = np.log(N)
    for level in D.schedule(K):
        for (a, c, b) in level:
            lg, rg = g["ancestry"][c - 1]
            assert lg.min() >= 0 and lg.max() < N and rg.min() >= 0 and rg.max() < N
            if select is None or select(a, c, b):
                xL = leaf_x[:, c - 1, sig[c - 1]].T
                xR = leaf_x[:, c, sig[c]].T
                lwL = g["leaf_logw"][c - 1].astype(np.float64) if c - a == 1 else np.full(N, -logN)
                lwR = g["leaf_logw"][c].astype(np.float64) if b - c == 1 else np.full(N, -logN)
                u1, u2 = P.combine_uniforms(seed, c, N)
                step = D.conditional_combine if conditional else D.combine
                res = step(spec, c, xL, xR, lwL, lwR, u1, u2, keep_S=True)
                rep.nodes += 1
                ez = float(_rel(g["logZ_inc"][c - 1], res.Z))
                rep.max_rel_err_Z = max(rep.max_rel_err_Z, ez)
                fin = np.isfinite(res.row_lse)
                er = _rel(g["row_lse"][c - 1][fin], res.row_lse[fin])
                if tol is None:
                    rep.abs_err_Z.append(abs(float(g["logZ_inc"][c - 1]) - float(res.Z)))
                    rep.abs_err_row.append(np.abs(g["row_lse"][c - 1][fin] - res.row_lse[fin]))
                else:
                    assert ez <= tol, (c, g["logZ_inc"][c - 1], res.Z)
                if er.size:
                    rep.max_rel_err_row = max(rep.max_rel_err_row, float(er.max()))
                    if tol is not None:
                        assert er.max() <= tol, (c, int(np.argmax(er)), er.max())
                if res.degenerate:
                    continue
                row_w = np.exp(res.row_lse - res.row_lse.max())
                d1 = _dist_to_boundary(u1, row_w)
                for n in range(N):
                    near = d1[n] < BAND
                    if res.l[n] == lg[n]:
                        row = res.S[res.l[n]]
                        d2 = _dist_to_boundary(np.array([u2[n]]), np.exp(row - row.max()))[0]
                        near = near or d2 < BAND
                        ok = res.r[n] == rg[n]
                    else:
                        ok = False
                    rep.draws += 1
                    rep.near += int(near)
                    if not ok:
                        rep.mismatches += 1
                        if not near:
                            rep.mismatches_outside_band += 1
                            rep.worst.append((c, n, int(res.l[n]), int(lg[n]), int(res.r[n]),
                                              int(rg[n]), float(d1[n])))
            sig[a:c] = sig[a:c][:, lg]
            sig[c:b] = sig[c:b][:, rg]
    np.testing.assert_array_equal(g["index"], sig)
    gathered = np.take_along_axis(g["leaf_x"], sig[None, :, :], axis=2)
    np.testing.assert_array_equal(g["traj"], gathered)
    total = float(g["leaf_logL"].sum() + g["logZ_inc"].sum())
    assert abs(float(g["log_Z"][0]) - total) <= 1e-9 * max(1.0, abs(total))
    return rep


def lazy_teacher_forced(spec, N: int, seed: int, g: dict, scheme: str, param: int,
                        band: float, conditional: bool = False) -> ParityReport:
    """Teacher-forced parity of a lazy-resampling run (Algorithms 7 and 8): at
    every node the oracle's lazy combine runs on the GPU's inputs of that
    level.  A draw is near a boundary when one of its chain's accept/reject
    decisions lies within ``band`` (relative to the log terms) of flipping;
    indices must agree outside that band."""
    K = spec.K
    rep = ParityReport()
    leaf_x = g["leaf_x"].astype(np.float64)
    sig = np.tile(np.arange(N), (K, 1))
    logN = np.log(N)
    for level in D.schedule(K):
        for (a, c, b) in level:
            lg, rg = g["ancestry"][c - 1]
            assert lg.min() >= 0 and lg.max() < N and rg.min() >= 0 and rg.max() < N
            xL = leaf_x[:, c - 1, sig[c - 1]].T
            xR = leaf_x[:, c, sig[c]].T
            lwL = g["leaf_logw"][c - 1].astype(np.float64) if c - a == 1 else np.full(N, -logN)
            lwR = g["leaf_logw"][c].astype(np.float64) if b - c == 1 else np.full(N, -logN)
            res = D.lazy_combine(spec, c, xL, xR, lwL, lwR, seed, scheme, param, margins=True)
            l, r = res.l.copy(), res.r.copy()
            if conditional:
                l[0] = r[0] = 0
            assert np.isnan(g["logZ_inc"][c - 1])
            rep.nodes += 1
            for n in range(N):
                near = bool(res.margin[n] < band)
                ok = l[n] == lg[n] and r[n] == rg[n]
                rep.draws += 1
                rep.near += int(near)
                if not ok:
                    rep.mismatches += 1
                    if not near:
                        rep.mismatches_outside_band += 1
                        rep.worst.append((c, n, int(l[n]), int(lg[n]), int(r[n]), int(rg[n]),
                                          float(res.margin[n])))
            sig[a:c] = sig[a:c][:, lg]
            sig[c:b] = sig[c:b][:, rg]
    np.testing.assert_array_equal(g["index"], sig)
    gathered = np.take_along_axis(g["leaf_x"], sig[None, :, :], axis=2)
    np.testing.assert_array_equal(g["traj"], gathered)
    return rep
