"""Pins for the oracle's tournament pivoting (TSLU, Grigori, Demmel and Xiang
2011) of the LU of a tall X, the alternative to partial pivoting in Algorithm 7
step 1 and Algorithm 5 step 1: the tree re-derived with LAPACK's getrf on every
node, partial pivoting when one block holds all rows, the factorization
identities, a singular leaf, and RCLUPPr and LC2 with it against the partial-
pivoting methods."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from gen import make_krylov, make_svd


def _getrf_rows(block_rows, x, n):
    """First n pivot rows of LAPACK getrf on x[block_rows] (in pivot order)."""
    _, piv = sl.lu_factor(x[block_rows])
    order = np.arange(len(block_rows))
    for k, p in enumerate(piv[:n]):
        order[k], order[p] = order[p], order[k]
    return [block_rows[i] for i in order[:n]]


def _tournament(x):
    m, n = x.shape
    L = (m + 255) // 256
    F = 256 // n
    sets = [_getrf_rows(list(range(g * m // L, (g + 1) * m // L)), x, n) for g in range(L)]
    while len(sets) > 1:
        sets = [_getrf_rows(sum(sets[i:i + F], []), x, n) for i in range(0, len(sets), F)]
    return sets[0]


@pytest.mark.parametrize("m,n", [(5000, 16), (9001, 40), (3000, 64), (2600, 100), (70000, 8)])
def test_tree_matches_lapack_per_node(m, n):
    x = make_svd(m, n, 1e6, seed=m + n)
    sel, N, L11, M, info = oracle.tslu(x)
    assert info[0] == 0
    assert [int(v) for v in sel] == _tournament(x)


def test_one_block_is_partial_pivoting():
    x = make_svd(256, 30, 1e5, seed=1)
    sel, N, L11, M, info = oracle.tslu(x)
    Mo, No, po, io = oracle.gepp(x)
    assert [int(v) for v in sel] == [int(v) for v in po[:30]]
    assert np.array_equal(N, No)
    assert np.array_equal(L11, np.tril(Mo[:30], -1) + np.eye(30))


@pytest.mark.parametrize("m,n,kappa", [(20000, 32, 1e10), (4099, 128, 1e4)])
def test_factorization_identities(m, n, kappa):
    x = make_svd(m, n, kappa, seed=5)
    sel, N, L11, M, info = oracle.tslu(x)
    u = oracle.U
    # X[sel] = L_11 N (Gaussian elimination's backward error, gamma_n |L||U|)
    err = np.abs(x[sel] - L11 @ N)
    assert np.all(err <= (n + 1) * u * (np.abs(L11) @ np.abs(N)) + 1e-300)
    # rows sel of M are L_11 exactly; M N = X row-wise (substitution's bound)
    assert np.array_equal(M[sel], L11)
    assert np.all(np.abs(M @ N - x) <= 2 * (n + 2) * u * (np.abs(M) @ np.abs(N)) + 1e-300)
    # upper and unit lower triangular factors; modest growth
    assert np.all(np.tril(N, -1) == 0) and np.all(np.diag(L11) == 1) and np.all(np.triu(L11, 1) == 0)
    assert np.max(np.abs(M)) < 10


def test_singular_leaf_does_not_stop_the_tournament():
    # rows 0..255 all equal (a rank-one leaf): the tournament must still find n
    # independent rows among the other leaves
    m, n = 2048, 12
    x = make_svd(m, n, 1e3, seed=7)
    x[:256] = x[0]
    sel, N, L11, M, info = oracle.tslu(x)
    assert info[0] == 0
    assert np.all(np.abs(np.diag(N)) > 0)
    assert len(set(int(v) for v in sel)) == n
    r = oracle.run("rcluppr", x, s=24, seed=3, lu="tournament")
    assert r.ok and oracle.metrics(x, r.Q, r.R)["orth"] < 1e-13


def test_zero_column_is_a_root_zero_pivot():
    x = make_svd(3000, 10, 1e2, seed=8)
    x[:, 4] = 0.0
    sel, N, L11, M, info = oracle.tslu(x)
    assert info[0] == oracle.LU_ZERO_PIVOT and info[2] == 5


@pytest.mark.parametrize("method", ["rcluppr", "lc2"])
@pytest.mark.parametrize("kappa", [1e4, 1e12, 1e15])
def test_methods_with_tournament_pivoting(method, kappa):
    x = make_svd(12000, 48, kappa, seed=9)
    t = oracle.run(method, x, s=96, seed=2, lu="tournament")
    p = oracle.run(method, x, s=96, seed=2)
    assert t.ok and p.ok
    m = oracle.metrics(x, t.Q, t.R)
    assert m["orth"] < 1e-13 and m["rel_res"] < 1e-14
    assert np.linalg.norm(t.R - p.R) / np.linalg.norm(p.R) < 1e-15 * kappa


def test_krylov_rcluppr_with_tournament_pivoting():
    # numerically rank deficient (kappa beyond 1e15): invariants only
    x = make_krylov(40000, 64, seed=2)
    r = oracle.run("rcluppr", x, s=128, seed=0, lu="tournament")
    assert r.ok
    m = oracle.metrics(x, r.Q, r.R)
    assert m["orth"] < 1e-13 and m["rel_res"] < 1e-14
