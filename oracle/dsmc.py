"""dSMC (de-Sequentialized Monte Carlo) smoother, plain fp64 CPU version.

TEST INFRASTRUCTURE: part of the fp64 CPU oracle; see oracle/__init__.py.

Steps, in the paper's order:

* ``sample_leaves``   Algorithm 2 (smoother initialisation) with the t = 0
                      reweighting of Proposition 2.2.
* ``combine``         Algorithm 1 (block combination): the product-form weights
                      W_c^{mn} (Section 2.2, normalised-weights equation), the
                      normalising-constant increment (equation for L_{a:b}),
                      multinomial resampling of N index pairs, and the gather.
* ``schedule``        Algorithm 6 (parallel combination by array reshaping):
                      the balanced tree actually executed.
* ``smooth``          leaves, then the tree, then the output.
* ``mh_resampling`` / ``rs_resampling``  the lazy resampling of Section 4.2,
                      Algorithms 7 (Metropolis-Hastings, B steps) and 8
                      (rejection), which replace the multinomial draw of
                      Algorithm 1; ``smooth_lazy`` runs the tree with them.
* ``smooth_conditional``  conditional dSMC (Section 3.1): the initialisation of
                      Algorithm 2 with a star trajectory put in front of the
                      proposal draws, and Algorithm 4 (conditional block
                      combination) at every node.

Readings of the paper this file takes:

* Time points are t = 0..K-1.
* Weights are carried normalised, with a separate log L per block (Algorithm 2
  returns both; Algorithm 1's return value is consistent with it).  A merged
  block carries uniform weights -log N.
* Algorithm 1 writes the pair measure with the roles of x_{c-1} and x_c
  swapped and the increment equation writes omega_c(X_{c-1}, X_{c-1}); here
  m indexes the left block (time c-1) and n the right block (time c), as in
  the normalised-weights equation.
* weighting "leaf_obs": nu_t proportional to h_t q_t, so the leaf log-weight
  is log h_t (t >= 1) and log omega_c = log p_c - log q_c up to the constant
  that the leaf L_t estimates; "boundary_obs": nu_t = q_t, leaf weight 1 for
  t >= 1 and log omega_c = log p_c + log h_c - log q_c.  At t = 0 both use
  log h_0 + log p_0 - log q_0 (Proposition 2.2 and Algorithm 2).
* Multinomial resampling (the scheme Proposition 2.4 assumes) realised in two
  stages: the row index from the row marginal with u1, then the column from the
  chosen row with u2; both by inverse CDF with the strict rule
  "first index whose cumulative sum exceeds u * total", on unnormalised fp64
  cumulative sums, so zero-weight entries are never drawn.
* If every pair weight of a combine is zero the increment is -inf, the status
  is "degenerate" and indices are drawn uniformly: l = floor(u1 N), r = floor(u2 N).
* Lazy resampling targets the product-form weight W_c^{mn} (its log is the
  pair matrix S), which is Algorithms 7 and 8's omega_c when the block weights
  are uniform.  Proposals 2j and 2j + 1 of chain n come from Philox block
  (n, c, 4 (MH) or 5 (RS), j) (see philox.lazy_proposals).  The rejection bound is
  max_m a_m + max_n b_n + max log p_c, a bound of every realised pair weight.
  The rejection loop stops after `cap` proposals (the last one is kept and the
  run flagged).  No increment is estimated: Z_c is NaN.
* Conditional runs: the star trajectory takes slot 0 (the paper's slot 1) and
  slot n >= 1 holds the proposal draw an unconditional run puts there; the N - 1
  draws of Algorithm 4 are those of slots 1..N-1 (uniforms of counter n), and
  slot 0 keeps the index pair (0, 0), degenerate combines included.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import philox
from .ssm import log_potential, log_prior, log_proposal, log_transition_pairs, proposal_draw


def logsumexp(v: np.ndarray, axis=None) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    m = np.max(v, axis=axis, keepdims=True)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        s = np.log(np.sum(np.exp(v - m_safe), axis=axis, keepdims=True)) + m_safe
    if axis is None:
        return s.reshape(())[()]
    return np.squeeze(s, axis=axis)


# --------------------------------------------------------------------------
# Leaves: Algorithm 2 and Proposition 2.2
# --------------------------------------------------------------------------

@dataclass
class Leaves:
    x: np.ndarray        # (K, N, d_x) particles X_t^n ~ q_t
    logw: np.ndarray     # (K, N) normalised log-weights
    logL: np.ndarray     # (K,) log L_t = log (1/N sum_n w_t^n)
    raw: np.ndarray      # (K, N) unnormalised log-weights

    @property
    def degenerate(self) -> bool:
        return bool(np.any(self.logL == -np.inf))


def leaf_logweights(spec, t: int, x: np.ndarray) -> np.ndarray:
    """Unnormalised leaf log-weights log w_t^n of Algorithm 2 for particles x (N, d_x)."""
    if t == 0:
        # nu_0 proportional to h_0 P_0 (Proposition 2.2): w = h_0 dP_0/dq_0
        return log_potential(spec, 0, x) + log_prior(spec, x) - log_proposal(spec, 0, x)
    if spec.weighting == "leaf_obs":
        return log_potential(spec, t, x)       # d nu_t / d q_t  with nu_t ~ h_t q_t
    if spec.weighting == "boundary_obs":
        return np.zeros(x.shape[0])            # nu_t = q_t
    raise ValueError(spec.weighting)


def normalise(raw: np.ndarray):
    """(normalised log-weights, log L) with L = mean of the weights (Algorithm 2).
    If every weight is zero, L = 0 and the weights are taken uniform (the run
    is then flagged degenerate)."""
    lse = logsumexp(raw)
    if lse == -np.inf:
        return np.full(raw.shape[0], -np.log(raw.shape[0])), -np.inf
    return raw - lse, lse - np.log(raw.shape[0])


def _leaf_variates(spec, seed: int, t: int, N: int, d: int) -> np.ndarray:
    """The proposal's base variates: normals, or uniforms for a uniform proposal."""
    if getattr(spec, "proposal", "gaussian") == "uniform":
        return philox.leaf_uniforms(seed, t, N, d)
    return philox.leaf_normals(seed, t, N, d)


def sample_leaves(spec, N: int, seed: int, x: np.ndarray | None = None) -> Leaves:
    """Algorithm 2.  If ``x`` (K, N, d_x) is given those particles are weighted
    instead of drawing new ones (used to feed the oracle another path's inputs)."""
    K, d = spec.K, spec.d_x
    if x is None:
        x = np.empty((K, N, d))
        for t in range(K):
            x[t] = proposal_draw(spec, t, _leaf_variates(spec, seed, t, N, d))
    x = np.asarray(x, dtype=np.float64)
    raw = np.empty((K, N))
    logw = np.empty((K, N))
    logL = np.empty(K)
    for t in range(K):
        raw[t] = leaf_logweights(spec, t, x[t])
        logw[t], logL[t] = normalise(raw[t])
    return Leaves(x=x, logw=logw, logL=logL, raw=raw)


# --------------------------------------------------------------------------
# Combine: Algorithm 1
# --------------------------------------------------------------------------

@dataclass
class CombineResult:
    l: np.ndarray            # (N,) left indices l_n
    r: np.ndarray            # (N,) right indices r_n
    row_lse: np.ndarray      # (N,) r_m = log sum_n exp S[m, n]
    Z: float                 # log of the normalising-constant increment
    degenerate: bool
    S: np.ndarray | None = None
    capped: bool = False     # lazy rejection: some chain hit its proposal cap


def pair_logweights(spec, c: int, xL, xR, lwL, lwR) -> np.ndarray:
    """S[m, n] = log( w_{c-1}^m w_c^n omega_c(X_{c-1}^m, X_c^n) ), the log of the
    unnormalised product-form weight (normalised-weights equation, Section 2.2)
    with omega_c of Proposition 2.3 for the chosen nu_c."""
    b = lwR - log_proposal(spec, c, xR)
    if spec.weighting == "boundary_obs":
        b = b + log_potential(spec, c, xR)
    return lwL[:, None] + b[None, :] + log_transition_pairs(spec, xL, xR)


def inverse_cdf(weights: np.ndarray, u: float) -> int:
    """First index i with u * total < cumsum(weights)[i] (fp64, sequential sums)."""
    cum = np.cumsum(weights)
    i = int(np.searchsorted(cum, u * cum[-1], side="right"))
    if i >= len(weights):                       # u * total rounded up to total
        i = int(np.flatnonzero(weights > 0)[-1])
    return i


def combine(spec, c: int, xL, xR, lwL, lwR, u1, u2, keep_S: bool = False) -> CombineResult:
    """Algorithm 1 at boundary c on the left block's particles at time c-1 (xL)
    and the right block's particles at time c (xR), with block log-weights
    lwL, lwR.  Returns the N index pairs and the log increment Z_c."""
    N = xL.shape[0]
    S = pair_logweights(spec, c, np.asarray(xL, np.float64), np.asarray(xR, np.float64),
                        np.asarray(lwL, np.float64), np.asarray(lwR, np.float64))
    if np.isnan(S).any():
        raise FloatingPointError(f"NaN pair weight at boundary {c}")
    row_lse = logsumexp(S, axis=1)
    Z = float(logsumexp(row_lse))
    l = np.empty(N, dtype=np.int64)
    r = np.empty(N, dtype=np.int64)
    if not np.isfinite(Z):
        l[:] = np.minimum((u1 * N).astype(np.int64), N - 1)
        r[:] = np.minimum((u2 * N).astype(np.int64), N - 1)
        return CombineResult(l, r, row_lse, Z, True, S if keep_S else None)
    row_w = np.exp(row_lse - np.max(row_lse))
    for n in range(N):
        m = inverse_cdf(row_w, u1[n])
        row = S[m]
        j = inverse_cdf(np.exp(row - np.max(row)), u2[n])
        l[n], r[n] = m, j
    return CombineResult(l, r, row_lse, Z, False, S if keep_S else None)


# --------------------------------------------------------------------------
# Tree: Algorithm 6
# --------------------------------------------------------------------------

def schedule(K: int):
    """Algorithm 6 as a list of levels; each level is a list of
    (a, c, b) = left block [a, c), right block [c, b) to combine at boundary c.
    Blocks are padded to 2^L with null blocks; a block whose right neighbour is
    padding is left unchanged."""
    L = 0
    while (1 << L) < K:
        L += 1
    blocks = [(t, t + 1) for t in range(K)] + [None] * ((1 << L) - K)
    levels = []
    for _ in range(L):
        nodes, nxt = [], []
        for k in range(0, len(blocks), 2):
            left, right = blocks[k], blocks[k + 1]
            if right is None:
                nxt.append(left)
            else:
                nodes.append((left[0], left[1], right[1]))
                nxt.append((left[0], right[1]))
        levels.append(nodes)
        blocks = nxt
    return levels


@dataclass
class Block:
    a: int
    b: int
    x: np.ndarray            # (b - a, N, d_x)
    logw: np.ndarray         # (N,)
    logL: float
    idx: np.ndarray          # (b - a, N) leaf particle index of each trajectory entry


@dataclass
class SmoothResult:
    x: np.ndarray            # (K, N, d_x) output trajectories
    logw: np.ndarray         # (N,) their log-weights (uniform for K >= 2)
    logZ: float              # log L^N_{0:K-1}
    leaves: Leaves
    ancestry: np.ndarray     # (K-1, 2, N): (l_n, r_n) of the combine at boundary c = 1..K-1
    Zc: np.ndarray           # (K-1,) log increments
    row_lse: np.ndarray      # (K-1, N)
    idx: np.ndarray          # (K, N) leaf index of every output entry
    degenerate: bool = False
    levels: list = field(default_factory=list)
    capped: bool = False


def run_tree(spec, leaves: Leaves, seed: int, conditional: bool = False) -> SmoothResult:
    """Algorithm 6 over the leaves; ``conditional`` runs Algorithm 4 at every
    node instead of Algorithm 1."""
    K, N = leaves.x.shape[0], leaves.x.shape[1]
    blocks = {t: Block(t, t + 1, leaves.x[t:t + 1], leaves.logw[t].copy(), float(leaves.logL[t]),
                       np.arange(N)[None, :].copy()) for t in range(K)}
    anc = np.zeros((max(K - 1, 0), 2, N), dtype=np.int64)
    Zc = np.zeros(max(K - 1, 0))
    rows = np.zeros((max(K - 1, 0), N))
    if np.isnan(leaves.raw).any():
        raise FloatingPointError("NaN leaf weight")
    degenerate = leaves.degenerate
    levels = schedule(K)
    for nodes in levels:
        for (a, c, b) in nodes:
            L, R = blocks.pop(a), blocks.pop(c)
            u1, u2 = philox.combine_uniforms(seed, c, N)
            step = conditional_combine if conditional else combine
            res = step(spec, c, L.x[-1], R.x[0], L.logw, R.logw, u1, u2)
            degenerate |= res.degenerate
            anc[c - 1, 0], anc[c - 1, 1] = res.l, res.r
            Zc[c - 1] = res.Z
            rows[c - 1] = res.row_lse
            x = np.concatenate([L.x[:, res.l], R.x[:, res.r]], axis=0)
            idx = np.concatenate([L.idx[:, res.l], R.idx[:, res.r]], axis=0)
            blocks[a] = Block(a, b, x, np.full(N, -np.log(N)), L.logL + R.logL + res.Z, idx)
    top = blocks[0]
    return SmoothResult(x=top.x, logw=top.logw, logZ=top.logL, leaves=leaves, ancestry=anc,
                        Zc=Zc, row_lse=rows, idx=top.idx, degenerate=degenerate, levels=levels)


def smooth(spec, N: int, seed: int) -> SmoothResult:
    """Leaves (Algorithm 2), then the tree of Algorithm 6 with Algorithm 1 at
    every node; log Z = sum_t log L_t + sum_c Z_c."""
    return run_tree(spec, sample_leaves(spec, N, seed), seed)


# --------------------------------------------------------------------------
# Conditional dSMC: Section 3.1 and Algorithm 4
# --------------------------------------------------------------------------

def sample_leaves_conditional(spec, N: int, seed: int, star) -> Leaves:
    """Conditional initialisation (Section 3.2): the star trajectory star[t]
    (K, d_x) is put in front of N - 1 proposal draws, so slot 0 of time t holds
    x*_t and slot n >= 1 the draw an unconditional run puts in slot n; the
    weights of Algorithm 2 are then computed over all N particles."""
    K, d = spec.K, spec.d_x
    star = np.asarray(star, dtype=np.float64).reshape(K, d)
    x = np.empty((K, N, d))
    for t in range(K):
        x[t] = proposal_draw(spec, t, _leaf_variates(spec, seed, t, N, d))
    x[:, 0] = star
    return sample_leaves(spec, N, seed, x=x)


def conditional_combine(spec, c: int, xL, xR, lwL, lwR, u1, u2,
                        keep_S: bool = False) -> CombineResult:
    """Algorithm 4 at boundary c: the pair weights, row sums and increment of
    Algorithm 1 over all N x N pairs, the star's included; N - 1 index pairs
    drawn for slots 1..N-1, while slot 0 keeps (0, 0), so the star trajectory,
    slot 0 of both blocks, is slot 0 of the merged block."""
    res = combine(spec, c, xL, xR, lwL, lwR, u1, u2, keep_S=keep_S)
    res.l[0] = 0
    res.r[0] = 0
    return res


def smooth_conditional(spec, N: int, seed: int, star) -> SmoothResult:
    """Conditional dSMC: conditional leaves, then the tree of Algorithm 6 with
    Algorithm 4 at every node.  Output slot 0 is the star trajectory; log Z is
    computed as in the unconditional run, over all particles."""
    return run_tree(spec, sample_leaves_conditional(spec, N, seed, star), seed, conditional=True)


# --------------------------------------------------------------------------
# Lazy resampling: Section 4.2, Algorithms 7 and 8
# --------------------------------------------------------------------------

def _margin(u, num, den):
    """Distance of the decision u < exp(num - den) from flipping, in units of
    the magnitudes of its log terms (for comparisons with other precisions)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        m = np.abs(np.log(u) - (num - den)) / (np.maximum(1.0, np.abs(num)) + np.maximum(1.0, np.abs(den)))
    return np.where(np.isfinite(m), m, np.inf)


def mh_resampling(S: np.ndarray, seed: int, c: int, B: int, margins: bool = False):
    """Algorithm 7 on the log pair weights S (N x N, target proportional to
    exp S): chain n starts at (n, n) and takes B Metropolis-Hastings steps with
    a proposal uniform over the N^2 pairs, moving when u < W(I*, J*) / W(I, J).
    With ``margins`` also returns each chain's smallest decision margin."""
    N = S.shape[0]
    I, J = np.arange(N), np.arange(N)
    mg = np.full(N, np.inf)
    with np.errstate(invalid="ignore", over="ignore"):
        for b in range(B):
            Ip, Jp, u = philox.lazy_proposals(seed, c, N, philox.PURPOSE_LAZY_MH, b)
            move = u < np.exp(S[Ip, Jp] - S[I, J])
            if margins:
                mg = np.minimum(mg, _margin(u, S[Ip, Jp], S[I, J]))
            I = np.where(move, Ip, I)
            J = np.where(move, Jp, J)
    return (I, J, mg) if margins else (I, J)


def rs_resampling(S: np.ndarray, log_bound: float, seed: int, c: int, cap: int,
                  margins: bool = False):
    """Algorithm 8 on the log pair weights S with log_bound >= max S: chain n
    proposes (I, J) uniformly over the N^2 pairs until u < W(I, J) / W_bar.
    Returns (I, J, capped): after `cap` proposals a chain keeps its last
    proposal and is marked capped.  With ``margins`` also each chain's
    smallest decision margin."""
    N = S.shape[0]
    I = np.zeros(N, dtype=np.int64)
    J = np.zeros(N, dtype=np.int64)
    done = np.zeros(N, dtype=bool)
    mg = np.full(N, np.inf)
    for k in range(cap):
        Ip, Jp, u = philox.lazy_proposals(seed, c, N, philox.PURPOSE_LAZY_RS, k)
        open_ = ~done
        I[open_], J[open_] = Ip[open_], Jp[open_]
        if margins:
            mg[open_] = np.minimum(mg[open_], _margin(u, S[Ip, Jp], log_bound)[open_])
        done |= open_ & (u < np.exp(S[Ip, Jp] - log_bound))
        if done.all():
            break
    return (I, J, ~done, mg) if margins else (I, J, ~done)


def rs_log_bound(spec, c: int, xR, lwL, lwR) -> float:
    """max_m a_m + max_n b_n + max_{x, x'} log p_c(x' | x): every pair weight of
    the combine is at most its exponential (the Gaussian transition density
    peaks at zero residual)."""
    b = lwR - log_proposal(spec, c, xR)
    if spec.weighting == "boundary_obs":
        b = b + log_potential(spec, c, xR)
    d = spec.d_x
    log_pmax = -np.sum(np.log(np.diag(spec.Q_chol))) - 0.5 * d * np.log(2.0 * np.pi)
    return float(np.max(lwL) + np.max(b) + log_pmax)


def lazy_combine(spec, c: int, xL, xR, lwL, lwR, seed: int, scheme: str, param: int,
                 keep_S: bool = False, margins: bool = False) -> CombineResult:
    """Algorithm 1 with its multinomial draw replaced by Algorithm 7 (scheme
    "mh", param = B) or Algorithm 8 (scheme "rs", param = cap).  The pair
    weights are formed here only to evaluate the proposed pairs; row sums and
    Z_c are not estimated (NaN)."""
    N = xL.shape[0]
    xL, xR = np.asarray(xL, np.float64), np.asarray(xR, np.float64)
    lwL, lwR = np.asarray(lwL, np.float64), np.asarray(lwR, np.float64)
    S = pair_logweights(spec, c, xL, xR, lwL, lwR)
    capped = False
    mg = None
    if scheme == "mh":
        out = mh_resampling(S, seed, c, param, margins=margins)
        l, r = out[0], out[1]
        mg = out[2] if margins else None
    elif scheme == "rs":
        out = rs_resampling(S, rs_log_bound(spec, c, xR, lwL, lwR), seed, c, param,
                            margins=margins)
        l, r, capped = out[0], out[1], bool(out[2].any())
        mg = out[3] if margins else None
    else:
        raise ValueError(scheme)
    res = CombineResult(l, r, np.full(N, np.nan), float("nan"), False, S if keep_S else None,
                        capped=capped)
    res.margin = mg
    return res


def smooth_lazy(spec, N: int, seed: int, scheme: str, param: int) -> SmoothResult:
    """Leaves (Algorithm 2), then the tree of Algorithm 6 with lazy combines."""
    leaves = sample_leaves(spec, N, seed)
    K = spec.K
    blocks = {t: Block(t, t + 1, leaves.x[t:t + 1], leaves.logw[t].copy(), float(leaves.logL[t]),
                       np.arange(N)[None, :].copy()) for t in range(K)}
    anc = np.zeros((max(K - 1, 0), 2, N), dtype=np.int64)
    capped = False
    levels = schedule(K)
    for nodes in levels:
        for (a, c, b) in nodes:
            L, R = blocks.pop(a), blocks.pop(c)
            res = lazy_combine(spec, c, L.x[-1], R.x[0], L.logw, R.logw, seed, scheme, param)
            capped |= res.capped
            anc[c - 1, 0], anc[c - 1, 1] = res.l, res.r
            x = np.concatenate([L.x[:, res.l], R.x[:, res.r]], axis=0)
            idx = np.concatenate([L.idx[:, res.l], R.idx[:, res.r]], axis=0)
            blocks[a] = Block(a, b, x, np.full(N, -np.log(N)), float("nan"), idx)
    top = blocks[0]
    return SmoothResult(x=top.x, logw=top.logw, logZ=top.logL if K > 1 else float(leaves.logL[0]),
                        leaves=leaves, ancestry=anc, Zc=np.full(max(K - 1, 0), np.nan),
                        row_lse=np.full((max(K - 1, 0), N), np.nan), idx=top.idx,
                        degenerate=leaves.degenerate, levels=levels, capped=capped)
