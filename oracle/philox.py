"""Philox4x64-10 and the uniform / normal draws of the dSMC oracle.

TEST INFRASTRUCTURE: part of the fp64 CPU oracle; see oracle/__init__.py.

Philox4x64-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 256-bit counter and a
128-bit key go through 10 rounds, each two 64x64->128 multiplications and a
Feistel-like word permutation, with a Weyl key schedule between rounds.

Stream layout (shared contract with the GPU side, each side implementing it
from the generator's published definition):

* key     = (seed, 0x64534D43)
* counter = (w0 = block index (particle or draw), w1 = time t or boundary c,
             w2 = purpose, w3 = sub-block j)
* purpose 2 (LEAF):    four standard normals per block (Box-Muller on its
                       word pairs (w0, w1) and (w2, w3)).  d_x dividing 4
                       (1, 2, 4): the normals of time t form one flat stream,
                       block (q, t, 2, 0) giving normals 4q .. 4q+3, and
                       coordinate i of particle n is normal n d_x + i.  Other
                       d_x: block (n, t, 2, j) gives z[4j .. 4j+3] of particle
                       n.  Uniform proposals take the words themselves, in the
                       same places.
* purpose 3 (COMBINE): block (n, c, 3, 0) gives the two uniforms (u1, u2) of
                       the n-th draw of the combine at boundary c (words w0,
                       w1).

Uniform from a 64-bit word w: (w >> 11) * 2^-53 in [0, 1).
Box-Muller from words (wa, wb): ua = ((wa >> 11) + 1) * 2^-53 in (0, 1],
ub = (wb >> 11) * 2^-53, rad = sqrt(-2 ln ua), z = (rad cos 2 pi ub, rad sin 2 pi ub).
"""
from __future__ import annotations

import numpy as np

KEY1 = 0x64534D43
PURPOSE_LEAF = 2
PURPOSE_COMBINE = 3
PURPOSE_LAZY_MH = 4
PURPOSE_LAZY_RS = 5

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: np.uint64):
    """Full 64x64 -> 128-bit product as (high word, low word), via 32-bit limbs."""
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, a * b


def philox4x64_10(counter, key):
    """Philox4x64-10 block for broadcastable counter words (c0, c1, c2, c3) and a
    key (k0, k1).  Returns the four output words as uint64 arrays."""
    c0, c1, c2, c3 = (np.asarray(w, dtype=np.uint64) for w in counter)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0, k1 = np.uint64(int(key[0]) & 0xFFFFFFFFFFFFFFFF), np.uint64(int(key[1]) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(c0, _M0)
            hi1, lo1 = _mulhilo(c2, _M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def key_of(seed: int):
    return (int(seed) & 0xFFFFFFFFFFFFFFFF, KEY1)


def to_uniform(w: np.ndarray) -> np.ndarray:
    """[0, 1) double with 53 random bits."""
    return (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def to_uniform_open0(w: np.ndarray) -> np.ndarray:
    """(0, 1] double with 53 random bits (never 0, so its log is finite)."""
    return ((w >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53


def _leaf_blocks(seed: int, t: int, N: int, d: int):
    """The leaf Philox words of time t, shape (N, 4 * blocks per particle):
    row n holds the four words of each block particle n draws from, in the
    positions of its coordinates (flat stream for d dividing 4: row n holds
    the words of block floor(n d / 4) rotated so that its coordinates come
    first)."""
    if 4 % d == 0:
        ppb = 4 // d                                   # particles per block
        q = np.arange((N + ppb - 1) // ppb, dtype=np.uint64)
        w = philox4x64_10((q, np.uint64(t), np.uint64(PURPOSE_LEAF), np.uint64(0)), key_of(seed))
        return np.stack(w, axis=1)                     # (blocks, 4): words of block q
    n = np.arange(N, dtype=np.uint64)
    out = []
    for j in range((d + 3) // 4):
        w = philox4x64_10((n, np.uint64(t), np.uint64(PURPOSE_LEAF), np.uint64(j)), key_of(seed))
        out.append(np.stack(w, axis=1))
    return np.concatenate(out, axis=1)                 # (N, 4 * blocks)


def _box_muller(w: np.ndarray) -> np.ndarray:
    """Four normals from each row of four words (pairs (w0, w1), (w2, w3))."""
    z = np.empty(w.shape)
    for p in range(w.shape[1] // 2):
        ua = to_uniform_open0(w[:, 2 * p])
        ub = to_uniform(w[:, 2 * p + 1])
        rad = np.sqrt(-2.0 * np.log(ua))
        z[:, 2 * p] = rad * np.cos(2.0 * np.pi * ub)
        z[:, 2 * p + 1] = rad * np.sin(2.0 * np.pi * ub)
    return z


def leaf_normals(seed: int, t: int, N: int, d: int) -> np.ndarray:
    """Standard normals z[n, 0:d] of the N particles drawn at time t, shape (N, d)."""
    z = _box_muller(_leaf_blocks(seed, t, N, d))
    if 4 % d == 0:
        return z.reshape(-1)[:N * d].reshape(N, d)   # normal n d + i
    return z[:, :d]


def leaf_uniforms(seed: int, t: int, N: int, d: int) -> np.ndarray:
    """Uniforms in [0, 1) of the N particles drawn at time t, shape (N, d):
    the words that give a Gaussian proposal its normals, in the same places."""
    u = to_uniform(_leaf_blocks(seed, t, N, d))
    if 4 % d == 0:
        return u.reshape(-1)[:N * d].reshape(N, d)
    return u[:, :d]


def combine_uniforms(seed: int, c: int, N: int):
    """(u1, u2) of the N draws of the combine at boundary c, each shape (N,)."""
    n = np.arange(N, dtype=np.uint64)
    w = philox4x64_10((n, np.uint64(c), np.uint64(PURPOSE_COMBINE), np.uint64(0)), key_of(seed))
    return to_uniform(w[0]), to_uniform(w[1])


def lazy_proposals(seed: int, c: int, N: int, purpose: int, step: int):
    """Proposal `step` of the N lazy-resampling chains at boundary c.  Block
    (n, c, purpose, step // 2) serves proposals 2j and 2j + 1: proposal
    2j + h takes its indices from word 2h, I* = floor(lo32 * N / 2^32) and
    J* = floor(hi32 * N / 2^32) of its two 32-bit halves (uniform on
    {0..N-1} up to N / 2^32), and u in [0, 1) from word 2h + 1 (53 bits)."""
    n = np.arange(N, dtype=np.uint64)
    w = philox4x64_10((n, np.uint64(c), np.uint64(purpose), np.uint64(step // 2)), key_of(seed))
    h = step % 2
    wi, wu = w[2 * h], w[2 * h + 1]
    I = ((wi & _LO32) * np.uint64(N)) >> _S32
    J = ((wi >> _S32) * np.uint64(N)) >> _S32
    return I.astype(np.int64), J.astype(np.int64), to_uniform(wu)
