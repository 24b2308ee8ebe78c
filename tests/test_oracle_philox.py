"""Pins of the oracle's Philox4x64-10 stream and its uniform / normal draws."""
import os

import numpy as np
import pytest

from oracle import philox as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(v, 16) for v in line.split()]
        rows.append((tuple(w[0:4]), tuple(w[4:6]), tuple(w[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_known_answer_vectors(ctr, key, out):
    got = P.philox4x64_10(ctr, key)
    assert tuple(int(x) for x in got) == out


def test_matches_numpy_philox():
    """numpy.random.Philox is an independent Philox4x64-10; it increments the
    256-bit counter before generating, so its block for counter C is produced
    from state C - 1."""
    g = np.random.default_rng(5)
    for _ in range(50):
        ctr = tuple(int(v) for v in g.integers(0, 2**64, size=4, dtype=np.uint64))
        key = tuple(int(v) for v in g.integers(0, 2**64, size=2, dtype=np.uint64))
        c = sum(v << (64 * i) for i, v in enumerate(ctr))
        bg = np.random.Philox(counter=(c - 1) % (1 << 256), key=key[0] | (key[1] << 64))
        ref = bg.random_raw(4)
        got = P.philox4x64_10(ctr, key)
        assert [int(x) for x in got] == [int(x) for x in ref]


def test_vectorised_counters_match_scalar():
    n = np.arange(100, dtype=np.uint64)
    w = P.philox4x64_10((n, np.uint64(7), np.uint64(2), np.uint64(1)), (3, P.KEY1))
    for i in (0, 17, 99):
        ws = P.philox4x64_10((i, 7, 2, 1), (3, P.KEY1))
        assert [int(a[i]) for a in w] == [int(x) for x in ws]


def test_uniform_ranges():
    w = np.array([0, 2**64 - 1, 2**11, 2**11 - 1], dtype=np.uint64)
    u = P.to_uniform(w)
    assert u[0] == 0.0 and u[1] == 1.0 - 2.0 ** -53 and u[2] == 2.0 ** -53 and u[3] == 0.0
    v = P.to_uniform_open0(w)
    assert v[0] == 2.0 ** -53 and v[1] == 1.0


def test_box_muller_moments():
    z = np.concatenate([P.leaf_normals(11, t, 250_000, 4).reshape(-1) for t in range(4)])
    assert z.size == 4_000_000
    assert abs(z.mean()) < 5e-3 / 2
    assert abs(z.var() - 1.0) < 3e-3
    assert abs(np.mean(z ** 3)) < 6e-3
    assert abs(np.mean(z ** 4) - 3.0) < 3e-2
    # pairs from one Box-Muller transform are uncorrelated
    zz = P.leaf_normals(12, 0, 500_000, 2)
    assert abs(np.mean(zz[:, 0] * zz[:, 1])) < 6e-3


def test_stream_separation():
    """Different purposes / times / seeds give different words."""
    a = P.leaf_normals(1, 0, 64, 1)
    b = P.leaf_normals(1, 1, 64, 1)
    c = P.leaf_normals(2, 0, 64, 1)
    assert not np.allclose(a, b) and not np.allclose(a, c)
    u1, u2 = P.combine_uniforms(1, 1, 64)
    assert not np.allclose(u1, u2)
