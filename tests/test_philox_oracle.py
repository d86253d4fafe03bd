"""Pins of the oracle's Gaussian start-block generator (Section 4: G has independent
N(0, 1) entries), checked against what its published definitions fix: the known-answer
vectors of Philox-4x32-10, closed forms of the uniform and Box-Muller maps, and the
distribution of the draws."""
import json
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def _kat():
    with open(GOLDEN) as f:
        return json.load(f)["vectors"]


def _h(words):
    return np.array([int(w, 16) for w in words], dtype=np.uint64)


@pytest.mark.parametrize("i", [0, 1, 2])
def test_philox_known_answer_vectors(i):
    v = _kat()[i]
    out = P.philox4x32_10(_h(v["counter"]), [int(k, 16) for k in v["key"]])
    assert [int(w) for w in out] == [int(w, 16) for w in v["output"]]


def test_philox_vectorised_equals_one_by_one():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(64, 4), dtype=np.uint64)
    key = (0x01234567, 0x89ABCDEF)
    many = P.philox4x32_10(ctr, key)
    for t in range(0, 64, 9):
        assert np.array_equal(many[t], P.philox4x32_10(ctr[t], key))


def test_uniform52_closed_forms():
    z = np.zeros(1, dtype=np.uint32)
    f = np.full(1, 0xFFFFFFFF, dtype=np.uint32)
    assert P.uniform52(z, z)[0] == 0.5 / 2.0 ** 52
    assert P.uniform52(f, f)[0] == (2.0 ** 52 - 0.5) / 2.0 ** 52
    assert 0.0 < P.uniform52(z, z)[0] and P.uniform52(f, f)[0] < 1.0
    # the top 26 bits of each word; the low 6 bits are dropped
    hi = np.array([1 << 6], dtype=np.uint32)
    lo = np.array([(1 << 6) | 63], dtype=np.uint32)
    assert P.uniform52(hi, z)[0] == (2.0 ** 26 + 0.5) / 2.0 ** 52
    assert P.uniform52(z, lo)[0] == 1.5 / 2.0 ** 52
    assert P.uniform52(np.array([63], dtype=np.uint32), z)[0] == P.uniform52(z, z)[0]


def test_box_muller_closed_forms():
    u1 = np.array([np.exp(-0.5), np.exp(-2.0), 0.3])
    u2 = np.array([0.0, 0.25, 0.5])
    z0, z1 = P.box_muller(u1, u2)
    np.testing.assert_allclose(z0, [1.0, 0.0, -np.sqrt(-2 * np.log(0.3))], atol=1e-15)
    np.testing.assert_allclose(z1, [0.0, 2.0, 0.0], atol=1e-15)
    # radius: z0^2 + z1^2 = -2 ln u1 for any angle
    rng = np.random.default_rng(3)
    a, b = rng.random(100), rng.random(100)
    x, y = P.box_muller(a, b)
    np.testing.assert_allclose(x * x + y * y, -2.0 * np.log(a), rtol=1e-13)


def test_block_entries_depend_on_seed_row_and_column_only():
    G = P.gaussian_block(77, 1001, 6)
    # a shorter block is a prefix; a column drawn alone equals the block's column
    np.testing.assert_array_equal(P.gaussian_block(77, 500, 6), G[:500])
    np.testing.assert_array_equal(P.gaussian_columns(77, 1001, [4, 2]), G[:, [4, 2]])
    # row pairs share one counter: rows 2t and 2t+1 are its cosine and sine normals
    w = P.philox4x32_10(np.array([3, 5, 0, 0]), P.seed_key(77))
    z0, z1 = P.box_muller(P.uniform52(w[:1], w[1:2]), P.uniform52(w[2:3], w[3:4]))
    assert G[6, 5] == z0[0] and G[7, 5] == z1[0]
    # another seed (only its high key word differs) gives another block
    G2 = P.gaussian_block(77 + (1 << 32), 1001, 6)
    assert np.abs(G2 - G).max() > 1.0


def test_block_is_standard_normal():
    G = P.gaussian_block(20210118, 200_003, 5)
    x = G.ravel()
    n = x.size
    assert abs(x.mean()) <= 5.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) <= 5.0 * np.sqrt(2.0 / n)
    assert abs(stats.skew(x)) <= 5.0 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(x)) <= 5.0 * np.sqrt(24.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # each row parity (cosine / sine normals) on its own, and columns uncorrelated
    for half in (G[0::2].ravel(), G[1::2].ravel()):
        assert stats.kstest(half, "norm").pvalue > 1e-4
    C = np.corrcoef(G.T)
    assert np.abs(C - np.eye(5)).max() <= 5.0 / np.sqrt(G.shape[0])
    # the cosine and sine normals of one pair are uncorrelated
    assert abs(np.corrcoef(G[0:-1:2, 0], G[1::2, 0])[0, 1]) <= 5.0 / np.sqrt(G.shape[0] / 2)


def test_uniforms_are_uniform():
    ctr = np.zeros((100_000, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(100_000)
    w = P.philox4x32_10(ctr, P.seed_key(11))
    u = P.uniform52(w[:, 0], w[:, 1])
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # every output word's bits are balanced
    bits = np.unpackbits(w.view(np.uint8)).reshape(-1)
    assert abs(bits.mean() - 0.5) <= 5.0 * 0.5 / np.sqrt(bits.size)
