"""Closed-form rounding-error bounds of the paper (TEST INFRASTRUCTURE ONLY).

Each function returns the upper bound the paper proves for one method; the
tests check measured orthogonality ||Q^T Q - I||_F and residual ||QR - X||_F
against them. u = 2^-53 (Section 1), epsilon = 0.5 (Section 5).
"""
from __future__ import annotations

import math

U = 2.0 ** -53


def _c(m: int, n: int) -> float:
    return m * n * U + n * (n + 1) * U


def cholqr2_bounds(m: int, n: int, x2: float):
    """Lemma 3.1: orthogonality 6(mnu+n(n+1)u), residual 5 n^2 sqrt(n) u ||X||_2."""
    return 6.0 * _c(m, n), 5.0 * n * n * math.sqrt(n) * U * x2


def cholqr2_kappa_limit(m: int, n: int) -> float:
    """Lemma 3.1 / Table 1 sufficient condition: kappa <= 1 / (8 sqrt(mnu+n(n+1)u))."""
    return 1.0 / (8.0 * math.sqrt(_c(m, n)))


def scholqr3_bounds(m: int, n: int, xg: float, x2: float):
    """Lemma 3.2: orthogonality 6(mnu+n(n+1)u), residual 6.57 n^2 u ||X||_g + 4.81 n^2 u ||X||_2."""
    return 6.0 * _c(m, n), 6.57 * n * n * U * xg + 4.81 * n * n * U * x2


def lc2_bounds(m: int, n: int, x2: float):
    """Lemma 3.3: orthogonality 6.5(mnu+n(n+1)u), residual 4.09 n^2 u ||X||_2."""
    return 6.5 * _c(m, n), 4.09 * n * n * U * x2


def h_factor(eps: float = 0.5) -> float:
    """h of the RCLUPP theorem: 1 / (0.78/sqrt(1+eps) - 0.1/sqrt(1-eps))."""
    return 1.0 / (0.78 / math.sqrt(1.0 + eps) - 0.1 / math.sqrt(1.0 - eps))


def rclupp_bounds(m: int, n: int, xf: float, x2: float, eps: float = 0.5):
    """Theorem (RCLUPP): orthogonality 6(mnu+n(n+1)u), residual Delta =
    4.36/sqrt(1-eps) h n sqrt(n) u ||X||_F + 3.02/sqrt(1-eps) h n^2 u ||X||_2."""
    h = h_factor(eps)
    se = math.sqrt(1.0 - eps)
    delta = 4.36 / se * h * n * math.sqrt(n) * U * xf + 3.02 / se * h * n * n * U * x2
    return 6.0 * _c(m, n), delta
