"""Pins for the oracle's small dense steps: LU with partial pivoting (eq. elu),
the R-only Householder QR (eq. eh), Cholesky (eq. C2), the row-wise triangular
solve (eq. ewy), the Gram matrix (eq. C1) and the triangular product (eq. ey).

Pins: LAPACK routines (getrf, geqrf, potrf, trsm via scipy/numpy), exact
rational arithmetic on tiny inputs, componentwise backward-error bounds of the
paper's error model, and special cases.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import oracle

U = oracle.U


def _lapack_perm(piv, r):
    perm = np.arange(r)
    for k, p in enumerate(piv):
        perm[k], perm[p] = perm[p], perm[k]
    return perm


# ------------------------------------------------------------------ LU
@pytest.mark.parametrize("r,n,seed", [(12, 5, 0), (64, 32, 1), (300, 64, 2), (7, 7, 3)])
def test_gepp_matches_lapack_getrf(r, n, seed):
    a = np.random.default_rng(seed).standard_normal((r, n))
    M, N, perm, info = oracle.gepp(a)
    assert info[0] == 0
    lu, piv = sla.lu_factor(a)
    np.testing.assert_array_equal(perm, _lapack_perm(piv, r))
    np.testing.assert_allclose(N, np.triu(lu[:n, :n]), rtol=0, atol=1e-13 * np.abs(N).max())
    Ml = np.tril(lu, -1)[:, :n] + np.eye(r, n)
    np.testing.assert_allclose(M, Ml, rtol=0, atol=1e-13)


def test_gepp_backward_error_and_multipliers():
    # eq. (elu): |P X_s - M N| <= 1.02 n u |M||N|; partial pivoting keeps |M| <= 1
    a = np.random.default_rng(4).standard_normal((200, 40))
    M, N, perm, info = oracle.gepp(a)
    assert np.all(np.abs(M) <= 1.0)
    err = np.abs(a[perm] - M @ N)
    assert np.all(err <= 1.02 * 40 * U * (np.abs(M) @ np.abs(N)) + 1e-300)


def _exact_gepp(rows):
    a = [[Fraction(v) for v in row] for row in rows]
    r, n = len(a), len(a[0])
    perm = list(range(r))
    for k in range(n):
        p = max(range(k, r), key=lambda i: (abs(a[i][k]), -i))
        a[k], a[p] = a[p], a[k]
        perm[k], perm[p] = perm[p], perm[k]
        for i in range(k + 1, r):
            a[i][k] = a[i][k] / a[k][k]
            for j in range(k + 1, n):
                a[i][j] -= a[i][k] * a[k][j]
    return a, perm


@pytest.mark.parametrize("seed", range(6))
def test_gepp_exact_rational_small(seed):
    rng = np.random.default_rng(100 + seed)
    r, n = 6, 4
    a = rng.integers(-9, 10, size=(r, n)).astype(float)
    ex, eperm = _exact_gepp(a.tolist())
    M, N, perm, info = oracle.gepp(a)
    if info[0] != 0:
        pytest.skip("singular draw")
    assert perm.tolist() == eperm
    for i in range(r):
        for j in range(n):
            want = float(ex[i][j])
            got = M[i, j] if i > j else N[i, j] if i <= j and i < n else None
            if got is None:
                continue
            assert abs(got - want) <= 1e-14 * max(1.0, abs(want))


def test_gepp_ties_pick_first_row():
    a = np.array([[1.0, 2.0], [-1.0, 0.0], [1.0, 5.0]])
    M, N, perm, info = oracle.gepp(a)
    assert perm[0] == 0  # |1| = |-1| = |1|: the first one wins (LAPACK idamax rule)
    lu, piv = sla.lu_factor(a)
    np.testing.assert_array_equal(perm, _lapack_perm(piv, 3))


def test_gepp_zero_pivot_and_nonfinite():
    # column 2 is zero: every elimination leaves it exactly zero
    a = np.array([[1.0, 0.0, 3.0], [2.0, 0.0, 1.0], [3.0, 0.0, 2.0], [1.0, 0.0, 5.0]])
    _, _, _, info = oracle.gepp(a)
    assert info.tolist()[:3] == [oracle.LU_ZERO_PIVOT, oracle.ST_LU, 2]
    b = np.random.default_rng(0).standard_normal((5, 3))
    b[3, 1] = np.nan
    _, _, _, info = oracle.gepp(b)
    assert info[0] == oracle.NONFINITE and info[2] == 2


# ------------------------------------------------------------------ Householder R
@pytest.mark.parametrize("r,n,seed", [(10, 4, 0), (128, 64, 1), (65, 64, 2), (1000, 50, 3)])
def test_house_r_matches_lapack_geqrf(r, n, seed):
    a = np.random.default_rng(seed).standard_normal((r, n))
    R = oracle.house_r(a)
    # same reflector convention as LAPACK dgeqrf (dlarfg), so no sign ambiguity
    Rl = np.linalg.qr(a, mode="r")
    np.testing.assert_allclose(R, Rl, rtol=0, atol=50 * n * U * np.abs(Rl).max())
    assert np.all(np.tril(R, -1) == 0)


def test_house_r_gram_identity():
    # R^T R = A^T A in exact arithmetic
    a = np.random.default_rng(5).standard_normal((90, 30))
    R = oracle.house_r(a)
    np.testing.assert_allclose(R.T @ R, a.T @ a, rtol=0, atol=1e-12 * np.abs(a.T @ a).max())


def test_house_r_upper_input():
    # an upper-triangular input needs no reflection: R = A (alpha kept when x = 0)
    a = np.zeros((6, 3))
    a[:3, :3] = np.triu(np.arange(1.0, 10.0).reshape(3, 3))
    np.testing.assert_array_equal(oracle.house_r(a), a[:3, :3])


def test_house_r_sign_convention():
    # dlarfg: beta = -sign(alpha) ||(alpha, x)||
    a = np.array([[3.0], [4.0]])
    assert oracle.house_r(a)[0, 0] == -5.0
    a = np.array([[-3.0], [4.0]])
    assert oracle.house_r(a)[0, 0] == 5.0


# ------------------------------------------------------------------ Cholesky
@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (64, 2), (128, 3)])
def test_chol_matches_lapack_potrf(n, seed):
    b = np.random.default_rng(seed).standard_normal((3 * n + 2, n))
    g = b.T @ b
    R, info = oracle.chol(g)
    assert info[0] == 0
    L = np.linalg.cholesky(g)
    np.testing.assert_allclose(R, L.T, rtol=0, atol=1e-12 * math.sqrt(np.abs(g).max()))
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


def test_chol_reads_upper_triangle_only():
    b = np.random.default_rng(7).standard_normal((20, 6))
    g = b.T @ b
    g2 = np.triu(g) + np.tril(np.full_like(g, 1e9), -1)
    np.testing.assert_array_equal(oracle.chol(g)[0], oracle.chol(g2)[0])


def test_chol_breakdown_column_and_shift():
    g = np.diag([4.0, 1.0, -1.0, 2.0])
    R, info = oracle.chol(g, stage=oracle.ST_CHOL_B)
    assert info.tolist()[:3] == [oracle.CHOL_BREAKDOWN, oracle.ST_CHOL_B, 3]
    R, info = oracle.chol(g, shift=2.0)
    assert info[0] == 0
    np.testing.assert_allclose(np.diag(R), np.sqrt([6.0, 3.0, 1.0, 4.0]), rtol=1e-15)
    g = np.eye(3)
    g[1, 1] = np.inf
    assert oracle.chol(g)[1][0] == oracle.NONFINITE


def test_chol_exact_on_diagonal():
    R, info = oracle.chol(np.diag([4.0, 9.0, 16.0]))
    np.testing.assert_array_equal(R, np.diag([2.0, 3.0, 4.0]))


# ------------------------------------------------------------------ TRSM
def _well_conditioned_upper(n, seed):
    rng = np.random.default_rng(seed)
    return np.triu(rng.standard_normal((n, n))) + n * np.eye(n)


@pytest.mark.parametrize("m,n,seed", [(50, 1, 0), (100, 7, 1), (3000, 64, 2)])
def test_trsm_matches_solve_triangular(m, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((m, n))
    R = _well_conditioned_upper(n, seed)
    w = oracle.trsm(x, R)
    want = sla.solve_triangular(R, x.T, trans="T", lower=False).T  # w R = x  <=>  R^T w^T = x^T
    np.testing.assert_allclose(w, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())


def test_trsm_componentwise_backward_error_ill_conditioned():
    # eq. (ewy): |W R - X| <= 1.02 n u |W||R|, even when R is extremely ill-conditioned
    rng = np.random.default_rng(3)
    n = 40
    R = np.triu(rng.standard_normal((n, n)))
    R[np.arange(n), np.arange(n)] = np.logspace(0, -14, n)
    x = rng.standard_normal((500, n))
    w = oracle.trsm(x, R)
    err = np.abs(w @ R - x)
    bound = 1.02 * n * U * (np.abs(w) @ np.abs(R))
    assert np.all(err <= 4 * bound + 1e-300)


def test_trsm_identity_and_in_place_aliasing():
    x = np.asfortranarray(np.random.default_rng(4).standard_normal((30, 5)))
    np.testing.assert_array_equal(oracle.trsm(x, np.eye(5)), x)
    R = np.diag([2.0, 4.0, 8.0, 0.5, 1.0])
    np.testing.assert_array_equal(oracle.trsm(x, R), x / np.diag(R))


# ------------------------------------------------------------------ Gram
def test_gram_matches_exact_sums():
    rng = np.random.default_rng(8)
    m, n = 9000, 4
    w = rng.standard_normal((m, n))
    G = oracle.gram(w)
    for i in range(n):
        for j in range(n):
            exact = math.fsum(float(a) * float(b) for a, b in zip(w[:, i], w[:, j]))
            assert abs(G[i, j] - exact) <= 1e-13 * float(np.abs(w[:, i]) @ np.abs(w[:, j]))
    assert np.array_equal(G, G.T)


def test_gram_blocks_cover_all_rows():
    # ones in the last (ragged) block must be counted
    m = 4096 * 2 + 17
    w = np.zeros((m, 2), order="F")
    w[-1, 0] = 3.0
    w[0, 1] = 2.0
    w[4096, 1] = 1.0
    G = oracle.gram(w)
    np.testing.assert_array_equal(G, np.array([[9.0, 0.0], [0.0, 5.0]]))


# ------------------------------------------------------------------ triangular product
def test_trmm_matches_matmul():
    rng = np.random.default_rng(9)
    a = np.triu(rng.standard_normal((20, 20)))
    b = np.triu(rng.standard_normal((20, 20)))
    np.testing.assert_allclose(oracle.trmm(a, b), a @ b, rtol=0, atol=1e-14 * 20 * np.abs(a).max() * np.abs(b).max())
    assert np.all(np.tril(oracle.trmm(a, b), -1) == 0)
