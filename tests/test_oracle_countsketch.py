"""Pins for the oracle's CountSketch (Section 3 lists it among the common
sketches): the hash read off the Philox words exactly as stated, the product
S X against exact integer sums, the distribution of rows and signs, the norm
identity E ||S x||^2 = ||x||^2, and RCLUPP with it on the SVD family."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from gen import make_svd


def _hash(seed, j, s):
    # counter (floor(j/4) lo, hi, 0, 1), word j mod 4: row floor(w s / 2^32), sign by parity
    q = j // 4
    w = oracle.philox4x32_10([q & 0xFFFFFFFF, q >> 32, 0, 1], [seed & 0xFFFFFFFF, seed >> 32])[j % 4]
    return (int(w) * s) >> 32, (-1.0 if int(w) & 1 else 1.0)


@pytest.mark.parametrize("seed,s", [(0, 128), (7, 100), (2**40 + 5, 1024), (2**64 - 1, 3)])
def test_hash_follows_the_stated_definition(seed, s):
    for j in list(range(0, 41)) + [2**32 - 1, 2**32, 2**33 + 6]:
        assert oracle.countsketch_hash(seed, j, s) == _hash(seed, j, s)


def test_product_is_the_exact_signed_bucket_sum():
    rng = np.random.default_rng(3)
    m, n, s, seed = 9001, 3, 17, 11  # three summation blocks and a ragged tail
    x = rng.integers(-1000, 1000, size=(m, n)).astype(np.float64)
    want = [[0] * n for _ in range(s)]
    for j in range(m):
        h, sg = _hash(seed, j, s)
        for k in range(n):
            want[h][k] += int(sg) * int(x[j, k])
    y = oracle.countsketch(np.asfortranarray(x), s, seed)
    assert np.array_equal(y, np.array(want, dtype=np.float64))


def test_rows_uniform_and_signs_balanced():
    s, count = 64, 40000
    hs = np.empty(count, dtype=np.int64)
    sg = np.empty(count)
    for j in range(count):
        hs[j], sg[j] = oracle.countsketch_hash(5, j, s)
    assert hs.min() >= 0 and hs.max() < s
    chi = stats.chisquare(np.bincount(hs, minlength=s))
    assert chi.pvalue > 1e-3, chi
    assert abs(sg.mean()) < 5 / math.sqrt(count)
    # the four rows of one call are not tied to each other
    assert abs(np.corrcoef(hs[0::4], hs[1::4])[0, 1]) < 0.03


def test_norm_identity_in_expectation():
    # E ||S x||^2 = ||x||^2 for any x (one +-1 per column, signs independent)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2000, 1))
    vals = [float(np.sum(oracle.countsketch(np.asfortranarray(x), 50, seed) ** 2)) for seed in range(300)]
    nx = float(np.sum(x ** 2))
    assert abs(np.mean(vals) / nx - 1.0) < 0.02


@pytest.mark.parametrize("method", ["rclupp", "rcluppr", "rcholqr"])
@pytest.mark.parametrize("kappa", [1e4, 1e12])
def test_methods_with_countsketch(method, kappa):
    # the final Q, R do not depend on the sketch in exact arithmetic: the same
    # invariants, and R agrees with the Gaussian-sketch result
    x = make_svd(6000, 24, kappa, seed=9)
    r = oracle.run(method, x, s=48, seed=2, sketch="count")
    g = oracle.run(method, x, s=48, seed=2)
    assert r.ok and g.ok
    m = oracle.metrics(x, r.Q, r.R)
    assert m["orth"] < 1e-13 and m["rel_res"] < 1e-14
    assert np.all(np.diag(r.R) > 0) and np.all(np.tril(r.R, -1) == 0)
    assert np.linalg.norm(r.R - g.R) / np.linalg.norm(g.R) < 1e-15 * kappa
