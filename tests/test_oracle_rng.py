"""Pins for the oracle's Gaussian sketch (Section 3: S = G / sqrt(s), G i.i.d.
N(0,1)) and for the sketch product Y = S X (Algorithm 2, first step).

Pins: published Philox4x32-10 known-answer vectors, exact-representation of the
uniforms, distributional tests of the Box-Muller normals, the subspace-
embedding property (eq. sketch) against the Marchenko-Pastur edges, and the
sketch product against an exactly rounded sum.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert oracle.philox4x32_10(ctr, key).tolist() == out


def _words_to_normals(w):
    # the documented mapping: u_t = (floor(w_t / 2^9) + 1/2) 2^-23, Box-Muller pairs (u0,u1), (u2,u3)
    u = [((int(x) >> 9) + 0.5) * 2.0 ** -23 for x in w]
    r0 = math.sqrt(-2.0 * math.log(u[0]))
    r1 = math.sqrt(-2.0 * math.log(u[2]))
    return np.array([r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
                     r1 * math.cos(2 * math.pi * u[3]), r1 * math.sin(2 * math.pi * u[3])], dtype=np.float32)


@pytest.mark.parametrize("seed,q,i", [(0, 0, 0), (0, 5, 3), (12345678901234, (1 << 33) + 7, 17), (2**64 - 1, 2**40, 4095)])
def test_counter_and_key_layout(seed, q, i):
    # the counter is (q lo, q hi, i, 0) for sketch row i and tall rows 4q..4q+3,
    # and the key (seed lo, seed hi)
    w = oracle.philox4x32_10([q & 0xFFFFFFFF, q >> 32, i, 0], [seed & 0xFFFFFFFF, seed >> 32])
    z = oracle.normals4(seed, q, i)
    np.testing.assert_allclose(z, _words_to_normals(w), rtol=2e-7, atol=1e-7)


def test_omega_entries_follow_the_counter_layout():
    # Omega[i, j] * sqrt(s) is output j mod 4 of the call for (q = j // 4, i)
    s, cols, j0, seed = 6, 11, 5, 21
    om = oracle.omega(s, cols, seed=seed, j0=j0)
    for c in range(cols):
        j = j0 + c
        for i in range(s):
            z = oracle.normals4(seed, j // 4, i)
            assert om[i, c] * math.sqrt(s) == pytest.approx(float(z[j % 4]), rel=1e-15)


def test_uniforms_exact_and_open_interval():
    # (floor(w/2^9) + 1/2) 2^-23 is an odd multiple of 2^-24 in (0, 1): exact in float32
    for w in (0, 1, 511, 512, 2**31, 2**32 - 1):
        u = ((w >> 9) + 0.5) * 2.0 ** -23
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u


def test_normals_distribution():
    # 4 positions x 50k draws: each marginal N(0,1), positions uncorrelated
    s, cols = 4, 50000
    om = oracle.omega(s, cols, seed=7)
    z = om * math.sqrt(s)
    for t in range(4):
        d = stats.kstest(z[t], "norm")
        assert d.pvalue > 1e-3, (t, d)
        assert abs(z[t].mean()) < 5 / math.sqrt(cols)
        assert abs(z[t].var() - 1.0) < 0.03
    c = np.corrcoef(z)
    assert np.max(np.abs(c - np.eye(4))) < 0.02
    # the four tall rows of one call (the Box-Muller outputs) are uncorrelated too
    w = z.reshape(4, cols // 4, 4).transpose(2, 0, 1).reshape(4, -1)
    cw = np.corrcoef(w)
    assert np.max(np.abs(cw - np.eye(4))) < 0.02


def test_omega_scaling_and_rows():
    s, cols = 64, 4000
    om = oracle.omega(s, cols, seed=3)
    # E ||Omega[:, j]||^2 = 1 (Omega = G / sqrt(s))
    assert abs(np.mean(np.sum(om * om, axis=0)) - 1.0) < 0.02
    # rows are uncorrelated (every sketch row has its own counters)
    c = np.corrcoef(om)
    off = c - np.eye(s)
    assert np.max(np.abs(off)) < 0.08
    # prefix property: Omega for s rows is the first s rows of a larger sketch, up to the 1/sqrt(s) scaling
    om2 = oracle.omega(2 * s, cols, seed=3)
    np.testing.assert_allclose(om * math.sqrt(s), om2[:s] * math.sqrt(2 * s), rtol=1e-15)


def test_omega_window_offset():
    om = oracle.omega(12, 100, seed=11)
    om_w = oracle.omega(12, 30, seed=11, j0=40)
    np.testing.assert_array_equal(om[:, 40:70], om_w)


def test_embedding_marchenko_pastur():
    # eq. (sketch): for an orthonormal basis X, singular values of S X concentrate in
    # [1 - sqrt(n/s), 1 + sqrt(n/s)] (Gaussian sketch, Marchenko-Pastur edges)
    rng = np.random.default_rng(0)
    m, n, s = 20000, 16, 512
    x, _ = np.linalg.qr(rng.standard_normal((m, n)))
    y = oracle.sketch(np.asfortranarray(x), s, seed=5)
    sv = np.linalg.svd(y, compute_uv=False)
    r = math.sqrt(n / s)
    assert sv.max() < 1 + r + 0.1 and sv.min() > 1 - r - 0.1
    # with eps = 0.5 this is an eps-embedding (Section 3, eq. s2-sigman1)
    assert sv.max() ** 2 <= 1.5 and sv.min() ** 2 >= 0.5


def test_sketch_matches_exact_sum():
    rng = np.random.default_rng(1)
    m, n, s = 9000, 3, 10  # spans three summation blocks
    x = np.asfortranarray(rng.standard_normal((m, n)))
    om = oracle.omega(s, m, seed=9)
    y = oracle.sketch(x, s, seed=9)
    for i in range(s):
        for k in range(n):
            exact = math.fsum(float(a) * float(b) for a, b in zip(om[i], x[:, k]))
            bound = 1.02 * (4096 + 3) * oracle.U * float(np.abs(om[i]) @ np.abs(x[:, k]))
            assert abs(y[i, k] - exact) <= bound
            # a typical error is much smaller than the worst-case bound
            assert abs(y[i, k] - exact) <= 1e-12 * float(np.abs(om[i]) @ np.abs(x[:, k]))


def test_sketch_unit_columns_pick_omega_columns():
    m, s = 5000, 8
    idx = [0, 1, 4095, 4096, 4999]
    x = np.zeros((m, len(idx)), order="F")
    for c, j in enumerate(idx):
        x[j, c] = 1.0
    y = oracle.sketch(x, s, seed=21)
    om = oracle.omega(s, m, seed=21)
    np.testing.assert_array_equal(y, om[:, idx])


def test_sketch_seed_changes_sketch():
    x = np.asfortranarray(np.random.default_rng(2).standard_normal((300, 4)))
    assert not np.array_equal(oracle.sketch(x, 8, 1), oracle.sketch(x, 8, 2))
    np.testing.assert_array_equal(oracle.sketch(x, 8, 1), oracle.sketch(x, 8, 1))
