"""Pins for the oracle's SRHT (Section 3 lists the subsampled randomized
Hadamard transform among the common sketches): S = sqrt(m'/s) R H D with H the
order-m' Walsh-Hadamard matrix. The oracle forms entry (i, j) as
(-1)^popcount(r_i & j) d_j / sqrt(s); the pins rebuild S from scipy's
Sylvester-recursion Hadamard matrix and compute S X a second way, by a fast
Walsh-Hadamard transform of D X, and check the signs and rows against their
stated definitions, the row sample for distinctness, and the exact unit
column norms of S."""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy import stats

import oracle
from gen import make_svd


def _mprime(m):
    k = 0
    while (1 << k) < m:
        k += 1
    return 1 << k, k


def _sign(seed, j):
    # counter (floor(j/4) lo, hi, 0, 2), word j mod 4: -1 for odd words
    q = j // 4
    w = oracle.philox4x32_10([q & 0xFFFFFFFF, q >> 32, 0, 2], [seed & 0xFFFFFFFF, seed >> 32])[j % 4]
    return -1.0 if int(w) & 1 else 1.0


def _row(seed, m, i):
    # pi(i) = f3(f2(f1(i))) mod 2^k with parameters from counter (0, 0, 0, 3)
    mp, k = _mprime(m)
    if k == 0:
        return 0
    a1, b1, a2, b2 = [int(v) for v in oracle.philox4x32_10([0, 0, 0, 3], [seed & 0xFFFFFFFF, seed >> 32])]
    x = ((a1 | 1) * i + b1) % mp
    x ^= x >> ((k + 1) // 2)
    return ((a2 | 1) * x + b2) % mp


@pytest.mark.parametrize("seed", [0, 9, 2**40 + 3, 2**64 - 1])
def test_signs_and_rows_follow_the_stated_definition(seed):
    for j in list(range(0, 37)) + [2**32 - 1, 2**32 + 5]:
        assert oracle.srht_sign(seed, j) == _sign(seed, j)
    for m in (1, 2, 3, 100, 4096, 4097, 4194304):
        for i in (0, 1, 2, 5, min(m, 77) - 1):
            assert oracle.srht_row(seed, m, i) == _row(seed, m, i)


@pytest.mark.parametrize("m", [1, 2, 5, 64, 100, 1000])
def test_row_sample_is_a_permutation(m):
    # every r_i lies in [0, m') and i -> r_i is one-to-one on all of [0, m')
    mp, _ = _mprime(m)
    rows = [oracle.srht_row(7, m, i) for i in range(mp)]
    assert sorted(rows) == list(range(mp))


@pytest.mark.parametrize("m,n,s,seed", [(1, 1, 1, 0), (2, 2, 2, 1), (3, 2, 3, 2), (64, 5, 16, 3), (100, 5, 16, 4),
                                        (1000, 3, 37, 5), (9001, 2, 50, 6)])
def test_matches_the_hadamard_matrix(m, n, s, seed):
    # S rebuilt from scipy's Walsh-Hadamard matrix (Sylvester recursion), the
    # sampled rows and the signs; m not a power of two pads X with zero rows
    mp, _ = _mprime(m)
    x = np.asfortranarray(np.random.default_rng(seed).standard_normal((m, n)))
    H = scipy.linalg.hadamard(mp).astype(np.float64)
    r = [_row(seed, m, i) for i in range(s)]
    d = np.array([_sign(seed, j) for j in range(m)])
    S = H[r][:, :m] * d[None, :] / math.sqrt(s)
    y = oracle.srht(x, s, seed)
    # both sums round: within a few ulps of sum_j |S_ij| |x_jk|
    bound = 4 * m * np.finfo(float).eps * (np.abs(S) @ np.abs(x))
    assert np.all(np.abs(y - S @ x) <= bound + 1e-300)


def _fwht(a):
    # unnormalized fast Walsh-Hadamard transform of the rows of a (length 2^k)
    a = a.copy()
    h = 1
    while h < a.shape[0]:
        for i in range(0, a.shape[0], 2 * h):
            u = a[i:i + h].copy()
            v = a[i + h:i + 2 * h].copy()
            a[i:i + h] = u + v
            a[i + h:i + 2 * h] = u - v
        h *= 2
    return a


def test_matches_a_fast_transform():
    # S X = (1/sqrt(s)) (H_unnormalized (D X_padded))[r]: the transform the
    # SRHT is named for, computed by butterflies instead of entry signs
    m, n, s, seed = 300, 4, 37, 8
    mp, _ = _mprime(m)
    x = np.random.default_rng(1).standard_normal((m, n))
    dx = np.zeros((mp, n))
    dx[:m] = np.array([_sign(seed, j) for j in range(m)])[:, None] * x
    want = _fwht(dx)[[_row(seed, m, i) for i in range(s)]] / math.sqrt(s)
    np.testing.assert_allclose(oracle.srht(np.asfortranarray(x), s, seed), want, rtol=0, atol=1e-12)


def test_columns_of_s_have_unit_norm():
    # every column of S has s entries +-1/sqrt(s): diag(S^T S) = 1 exactly,
    # whatever the sample (a wrong scale, e.g. sqrt(m/s), fails here)
    m, s = 200, 23
    S = oracle.srht(np.asfortranarray(np.eye(m)), s, 4)
    assert np.all(np.abs(np.abs(S) - 1 / math.sqrt(s)) < 1e-15)
    np.testing.assert_allclose(np.sum(S * S, axis=0), np.ones(m), rtol=0, atol=1e-14)


def test_signs_balanced_and_rows_spread():
    count = 40000
    sg = np.array([oracle.srht_sign(5, j) for j in range(count)])
    assert abs(sg.mean()) < 5 / math.sqrt(count)
    m = 1 << 20
    rows = np.array([oracle.srht_row(5, m, i) for i in range(4096)])
    chi = stats.chisquare(np.bincount(rows >> 14, minlength=64))  # 64 equal bins of [0, 2^20)
    assert chi.pvalue > 1e-3, chi


@pytest.mark.parametrize("method", ["rclupp", "rcluppr", "rcholqr"])
@pytest.mark.parametrize("kappa", [1e4, 1e12])
def test_methods_with_srht(method, kappa):
    # the final Q, R do not depend on the sketch in exact arithmetic: the same
    # invariants, and R agrees with the Gaussian-sketch result
    x = make_svd(6000, 24, kappa, seed=9)
    r = oracle.run(method, x, s=48, seed=2, sketch="srht")
    g = oracle.run(method, x, s=48, seed=2)
    assert r.ok and g.ok
    m = oracle.metrics(x, r.Q, r.R)
    assert m["orth"] < 1e-13 and m["rel_res"] < 1e-14
    assert np.all(np.diag(r.R) > 0) and np.all(np.tril(r.R, -1) == 0)
    assert np.linalg.norm(r.R - g.R) / np.linalg.norm(g.R) < 1e-15 * kappa
