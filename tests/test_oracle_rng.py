"""Pins for the oracle's random streams: Philox against numpy, samplers against statistics."""
import numpy as np
import pytest
from scipy import stats

from oracle import rng


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((5, 6), (3, 0, 0, 0)),
                                     ((2**64 - 1, 12345), (7, 2**63 + 5, 11, 2**64 - 2))])
def test_philox_scalar_matches_numpy(key, ctr):
    # numpy's Philox increments the counter before each block
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = bg.random_raw(8)
    c1 = ((ctr[0] + 1) & rng.MASK64, ctr[1], ctr[2], ctr[3])
    c2 = ((ctr[0] + 2) & rng.MASK64, ctr[1], ctr[2], ctr[3])
    mine = list(rng.philox4x64_10_scalar(c1, key)) + list(rng.philox4x64_10_scalar(c2, key))
    assert [int(x) for x in raw] == mine


def test_philox_vector_matches_scalar():
    r = np.random.default_rng(0)
    ctr = r.integers(0, 2**63, size=(4, 17), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    key = (0xDEADBEEFCAFEBABE, 0x0123456789ABCDEF)
    vec = rng.philox4x64_10(ctr, key)
    for j in range(ctr.shape[1]):
        assert tuple(int(v) for v in vec[:, j]) == rng.philox4x64_10_scalar(tuple(ctr[:, j]), key)


@pytest.mark.parametrize("seed,purpose,t", [(1, 5, 0), (3, 6, 121), (2**40 + 3, 7, 2**33)])
def test_stream_matches_numpy(seed, purpose, t):
    bg = np.random.Philox(key=np.array([seed, purpose], dtype=np.uint64),
                          counter=np.array([0, t, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(1001)
    assert np.array_equal(rng.stream_words(seed, purpose, t, 1001), raw)
    # an arbitrary window
    assert np.array_equal(rng.stream_words(seed, purpose, t, 50, start=333), raw[333:383])


def test_uniform_ranges():
    w = np.array([0, 1, 2**11 - 1, 2**11, 2**64 - 1], dtype=np.uint64)
    u0 = rng.uniform_closed0(w)
    u1 = rng.uniform_open0(w)
    assert u0[0] == 0.0 and u0[-1] == 1.0 - 2.0**-53
    assert u1[0] == 2.0**-53 and u1[-1] == 1.0
    assert np.all((u1 > 0) & (u1 <= 1)) and np.all((u0 >= 0) & (u0 < 1))


def test_normals_distribution():
    z = rng.normals(9, rng.PURPOSE_OMEGA, 4, 200_000)
    assert np.all(np.isfinite(z))
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01


def test_normals_prefix_property():
    a = rng.normals(1, 6, 0, 1000)
    b = rng.normals(1, 6, 0, 300)
    assert np.array_equal(a[:300], b)


def test_bounded_power_of_two_is_top_bits():
    # for s = 2^j no rejection can happen and the result is the top j bits of the word
    ws = rng.WordStream(11, 5, 3)
    raw = rng.stream_words(11, 5, 3, 64)
    for i in range(64):
        v = rng.bounded(ws, 1 << 13)
        assert v == int(raw[i]) >> (64 - 13)


def test_bounded_uniform_chi2():
    ws = rng.WordStream(12, 5, 0)
    s = 7
    counts = np.bincount([rng.bounded(ws, s) for _ in range(70_000)], minlength=s)
    assert counts.size == s
    assert stats.chisquare(counts).pvalue > 1e-3


def test_floyd_block_properties():
    for t in range(20):
        B = rng.sample_block(1, t, 1000, 97)
        assert B.size == 97 and np.all(np.diff(B) > 0) and B[0] >= 0 and B[-1] < 1000
    assert np.array_equal(rng.sample_block(1, 0, 50, 50), np.arange(50))
    with pytest.raises(ValueError):
        rng.sample_block(1, 0, 10, 11)


def test_floyd_inclusion_uniform():
    n, b, T = 40, 10, 4000
    counts = np.zeros(n)
    for t in range(T):
        counts[rng.sample_block(2, t, n, b)] += 1
    # each index is included with probability b/n
    assert stats.chisquare(counts, np.full(n, T * b / n)).pvalue > 1e-3
    # pairs: P(i and j both in B) = b(b-1)/(n(n-1))
    both = 0
    for t in range(T):
        B = set(rng.sample_block(2, t, n, b).tolist())
        both += (0 in B) and (n - 1 in B)
    p = b * (b - 1) / (n * (n - 1))
    assert abs(both / T - p) < 5 * np.sqrt(p * (1 - p) / T)
