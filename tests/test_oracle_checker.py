"""Pins of the oracle's accuracy metrics, the SCholeskyQR3 shift and the
closed-form bounds against values fixed independently of their code.

* chk_orthogonality, chk_residual (Section 5: ||Q^T Q - I||_F and
  ||Q R - X||_F): constructed dyadic inputs whose exact values follow from
  integer arithmetic. Each construction is chosen so that a plausible slip
  fails: a missing factor 2 on the off-diagonal entries, I not subtracted,
  plain instead of compensated summation, R read transposed or through its
  lower triangle, a wrong sign on X.
* orc_scholqr3_shift (Algorithm 4 with the shift of Lemma 3.2,
  s = 11(mnu + n(n+1)u) ||X||_g^2): exact rational evaluation; the reading
  with (n+1)u in place of n(n+1)u must fail. orc_scholqr3 must factor
  G + s I with that s and max_j G_jj as ||X||_g^2.
* oracle/bounds.py (Lemmas 3.1-3.3, the RCLUPP theorem): the tabulated values
  of tests/golden/paper_bounds.txt and the special case epsilon = 0 of h.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import bounds
from gen import make_svd

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_bounds.txt")
U = Fraction(1, 2 ** 53)


def _frac_sqrt(f: Fraction) -> float:
    """sqrt of an exact rational, correctly rounded to within an ulp."""
    return math.sqrt(float(f))


# ------------------------------------------------------------------ orthogonality
def _perturbed_identity(m, n, e_bits, seed, zero_top=False):
    """Q = [I; 0] + 2^-e_bits E with integer E in [-3, 3] and a zero diagonal
    (zero_top: the whole top n x n block zero); returns (Q, E)."""
    rng = np.random.default_rng(seed)
    E = rng.integers(-3, 4, size=(m, n))
    E[np.arange(n), np.arange(n)] = 0
    if zero_top:
        E[:n] = 0
    Q = np.zeros((m, n))
    Q[np.arange(n), np.arange(n)] = 1.0
    Q = np.asfortranarray(Q + np.ldexp(E.astype(np.float64), -e_bits))
    return Q, E


def _exact_orth_sq(E, n, e_bits):
    """||Q^T Q - I||_F^2 for Q = [I; 0] + 2^-e E, exactly (integer arithmetic)."""
    k = 1 << e_bits
    A = E.astype(object)
    A[np.arange(n), np.arange(n)] += k          # A = 2^e Q
    G = A.T.dot(A)                               # 2^(2e) Q^T Q, exact
    tot = 0
    for i in range(n):
        for j in range(n):
            d = G[i, j] - (k * k if i == j else 0)
            tot += d * d
    return Fraction(tot, k ** 4), G


@pytest.mark.parametrize("m,n,e_bits,seed", [(40, 7, 10, 0), (4096, 6, 27, 1), (3000, 1, 20, 2)])
def test_orthogonality_exact_construction(m, n, e_bits, seed):
    Q, E = _perturbed_identity(m, n, e_bits, seed)
    exact_sq, G = _exact_orth_sq(E, n, e_bits)
    want = _frac_sqrt(exact_sq)
    got = oracle.orthogonality(Q)
    assert abs(got - want) <= 4e-16 * want, (got, want)
    # the readings a slip would produce are far from the exact value
    k2 = (1 << e_bits) ** 2
    upper_only = sum((G[i, j] - (k2 if i == j else 0)) ** 2 for j in range(n) for i in range(j + 1))
    if n > 1:
        assert abs(_frac_sqrt(Fraction(upper_only, k2 * k2)) - want) > 1e-3 * want
    no_eye = sum(G[i, j] ** 2 for i in range(n) for j in range(n))
    assert abs(_frac_sqrt(Fraction(no_eye, k2 * k2)) - want) > 0.5 * want


def test_orthogonality_needs_compensated_sums():
    # Q^T Q - I = 2^-54 E^T E: its diagonal entries are sums of multiples of
    # 2^-54 added to 1, which plain summation rounds to multiples of 2^-52
    # (an error of order 1e-5 of the value); the compensated sums keep them
    m, n, e_bits = 4096, 6, 27
    Q, E = _perturbed_identity(m, n, e_bits, 3, zero_top=True)
    assert any(int((E[:, j] ** 2).sum()) % 4 for j in range(n))  # not on the 2^-52 grid
    want = _frac_sqrt(_exact_orth_sq(E, n, e_bits)[0])
    naive = np.linalg.norm(Q.T @ Q - np.eye(n))
    assert abs(naive - want) > 1e-7 * want   # the slip this test guards against
    assert abs(oracle.orthogonality(Q) - want) <= 4e-16 * want


def test_orthogonality_leading_dimension():
    Q, E = _perturbed_identity(50, 5, 12, 4)
    big = np.asfortranarray(np.full((64, 5), 7.0))
    big[:50] = Q
    want = _frac_sqrt(_exact_orth_sq(E, 5, 12)[0])
    view = big[:50]
    assert abs(oracle.orthogonality(np.asfortranarray(view)) - want) <= 4e-16 * want
    # same value through the ld = 64 layout of the C routine
    import ctypes
    lib = oracle._load()
    got = lib.chk_orthogonality(ctypes.c_void_p(big.ctypes.data), 50, 5, 64)
    assert abs(got - want) <= 4e-16 * want


# ------------------------------------------------------------------ residual
def _dyadic_qr_with_perturbation(m, n, seed):
    rng = np.random.default_rng(seed)
    Qi = rng.integers(-8, 9, size=(m, n))                  # Q = Qi / 16
    Ri = np.triu(rng.integers(-8, 9, size=(n, n)))         # upper, not symmetric
    Ri[np.arange(n), np.arange(n)] = rng.integers(1, 9, size=n)
    D = np.zeros((m, n), dtype=np.int64)                   # Delta = D 2^-30
    idx = rng.choice(m * n, size=min(m * n, 11), replace=False)
    D.flat[idx] = rng.integers(-3, 4, size=idx.size)
    Q = np.asfortranarray(Qi / 16.0)
    X = np.asfortranarray(Q @ Ri + np.ldexp(D.astype(np.float64), -30))
    # exact X in units of 2^-30: 2^26 Qi Ri + D
    Xi = (Qi.astype(object).dot(Ri.astype(object))) * (1 << 26) + D.astype(object)
    return Q, Ri, D, X, Xi


@pytest.mark.parametrize("m,n,seed", [(37, 5, 0), (5000, 3, 1), (100, 1, 2)])
def test_residual_exact_construction(m, n, seed):
    Q, Ri, D, X, Xi = _dyadic_qr_with_perturbation(m, n, seed)
    assert np.array_equal(np.ldexp(np.array(Xi, dtype=np.float64), -30), X)  # X held exactly
    R = np.asfortranarray(Ri.astype(np.float64))
    # the strict lower triangle must be ignored: fill it with garbage
    Rg = R.copy(order="F")
    Rg[np.tril_indices(n, -1)] = 1e6
    res, xn = oracle.residual(X, Q, Rg)
    want_res = math.sqrt(float(Fraction(int((D.astype(object) ** 2).sum()), 1 << 60)))
    want_xn = _frac_sqrt(Fraction(int(sum(v * v for v in Xi.flat)), 1 << 60))
    assert abs(res - want_res) <= 4e-16 * max(want_res, 1e-300), (res, want_res)
    assert abs(xn - want_xn) <= 1e-15 * want_xn
    # slips: R transposed, or X added instead of subtracted
    if n > 1:
        rt, _ = oracle.residual(X, Q, np.asfortranarray(R.T))
        assert rt > 1e3 * max(want_res, 2.0 ** -30)
    rn, _ = oracle.residual(np.asfortranarray(-X), Q, R)
    assert rn > 1e3 * max(want_res, 2.0 ** -30)


def test_residual_zero_for_exact_product():
    Q, Ri, D, X, Xi = _dyadic_qr_with_perturbation(200, 4, 5)
    X0 = np.asfortranarray(Q @ Ri.astype(np.float64))
    res, _ = oracle.residual(X0, Q, np.asfortranarray(Ri.astype(np.float64)))
    assert res == 0.0


# ------------------------------------------------------------------ SCholeskyQR3 shift
def _shift_exact(m, n, g: Fraction) -> Fraction:
    return 11 * (m * n * U + n * (n + 1) * U) * g


@pytest.mark.parametrize("m,n,g", [(64, 64, 3.25), (20000, 50, 1.0), (1048576, 64, 0.1875), (7, 1, 5.0)])
def test_scholqr3_shift_closed_form(m, n, g):
    got = oracle.scholqr3_shift(m, n, g)
    want = _shift_exact(m, n, Fraction(g))
    assert abs(Fraction(got) - want) <= 2 * Fraction(2.0 ** -52) * want, (got, float(want))
    if n > 1:  # the (n+1)u reading of Section 5 gives a different shift
        alt = 11 * (m * n * U + (n + 1) * U) * Fraction(g)
        assert abs(Fraction(got) - alt) > Fraction(1, 10 ** 6) * want


def test_scholqr3_factors_shifted_gram():
    # R_1 of Algorithm 4 is the Cholesky factor of G + s I with s from the
    # largest diagonal entry of G (||X||_g^2 = max_j ||X_j||^2): the diagonal of
    # R_1^T R_1 - G is s up to rounding of order n u max_j G_jj (s is about
    # 11 mn u max_j G_jj, 4e5 times larger here), its off-diagonal part is
    # rounding only
    m, n = 3000, 12
    x = make_svd(m, n, 1e6, seed=21)
    x[:, 5] *= 3.0  # a column of larger norm: the max is not column 0
    x = np.asfortranarray(x)
    G = oracle.gram(x)
    gmax = float(np.max(np.diag(G)))
    s = float(_shift_exact(m, n, Fraction(gmax)))
    r = oracle.scholqr3(x)
    assert r.ok
    D = r.R1.T @ r.R1 - G
    noise = 4 * n * 2.0 ** -53 * gmax
    np.testing.assert_allclose(np.diag(D), s, rtol=0, atol=noise)
    assert np.abs(D - np.diag(np.diag(D))).max() <= noise
    # the slips: the shift taken from column 0, or with (n+1)u
    s0 = float(_shift_exact(m, n, Fraction(float(G[0, 0]))))
    alt = float(11 * (m * n * U + (n + 1) * U) * Fraction(gmax))
    assert abs(s0 - s) > 100 * noise and abs(alt - s) > 10 * noise


# ------------------------------------------------------------------ bounds.py
def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, m, n, kappa, val = line.split()
            rows.append((kind, int(m), int(n), float(kappa), float(val)))
    return rows


def _geometric_xf(n, kappa):
    sig = kappa ** (-np.arange(n, dtype=np.float64) / (n - 1))
    return float(np.sqrt(np.sum(sig ** 2)))


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: "%s-%d-%d" % r[:3])
def test_bounds_match_tabulated_values(row):
    kind, m, n, kappa, want = row
    if kind == "h_factor":
        got = bounds.h_factor(0.5)
        tol = 5e-4
    elif kind == "cholqr2_orth":
        got = bounds.cholqr2_bounds(m, n, 1.0)[0]
        tol = 0.05
    elif kind == "cholqr2_kappa_limit":
        got = bounds.cholqr2_kappa_limit(m, n)
        tol = 0.05
    elif kind == "rclupp_delta":
        got = bounds.rclupp_bounds(m, n, _geometric_xf(n, kappa), 1.0)[1]
        tol = 0.05
    elif kind == "rclupp_delta_unitcol":
        got = bounds.rclupp_bounds(m, n, math.sqrt(n), math.sqrt(n))[1]
        tol = 0.05
    else:
        raise AssertionError(kind)
    assert abs(got - want) <= tol * want, (kind, m, n, got, want)


def test_bounds_structure():
    # h at epsilon = 0 reduces to 1/(0.78 - 0.1)
    assert abs(bounds.h_factor(0.0) - 1.0 / 0.68) <= 1e-15
    # the RCLUPP and CholeskyQR2 orthogonality bounds coincide (Theorem vs Lemma 3.1);
    # LC2's constant is 6.5 (Lemma 3.3); SCholeskyQR3's is 6 (Lemma 3.2)
    for m, n in ((2048, 32), (1 << 20, 64)):
        c = bounds.cholqr2_bounds(m, n, 1.0)[0]
        assert bounds.rclupp_bounds(m, n, 1.0, 1.0)[0] == c
        assert abs(bounds.lc2_bounds(m, n, 1.0)[0] / c - 6.5 / 6.0) < 1e-15
        assert bounds.scholqr3_bounds(m, n, 1.0, 1.0)[0] == c
    # residual bounds scale with the norms they multiply
    n = 40
    r1 = bounds.cholqr2_bounds(1000, n, 1.0)[1]
    assert abs(bounds.cholqr2_bounds(1000, n, 3.0)[1] - 3 * r1) <= 1e-15 * r1
    # Lemma 3.2 residual: 6.57 n^2 u ||X||_g + 4.81 n^2 u ||X||_2 -> the two terms separate
    a = bounds.scholqr3_bounds(1000, n, 1.0, 0.0)[1]
    b = bounds.scholqr3_bounds(1000, n, 0.0, 1.0)[1]
    assert abs(a / b - 6.57 / 4.81) < 1e-14
    # Lemma 3.3 residual against Lemma 3.1's: 4.09 n^2 vs 5 n^2 sqrt(n)
    assert abs(bounds.lc2_bounds(1000, n, 1.0)[1] / r1 - 4.09 / (5 * math.sqrt(n))) < 1e-14
    # Delta: the ||X||_F and ||X||_2 terms carry 4.36 n sqrt(n) and 3.02 n^2
    dF = bounds.rclupp_bounds(1000, n, 1.0, 0.0)[1]
    d2 = bounds.rclupp_bounds(1000, n, 0.0, 1.0)[1]
    assert abs(dF / d2 - 4.36 * math.sqrt(n) / (3.02 * n)) < 1e-14
