"""Input families of the paper's experiments, regenerated from their definitions.

All matrices are float64 and returned in column-major (Fortran) order, which is
the layout the library and the oracle take (element (i, j) at X[i + j*ld]).

* make_svd      -- Section 5.1.1: X = U diag(sigma) V^T with a geometric spectrum
                   from 1 down to 1/kappa (kappa_2(X) = kappa, ||X||_2 = 1).
* make_lowtri   -- Section 5.1.2: 400 stacked copies of a 50x50 lower-triangular
                   block F (F_ii = 100, F_ij = a below the diagonal).
* make_arrowhead-- Section 5.1.3: X = -5 e_b e_a^T + P_s with E = diag(1,..,1,beta).
* make_krylov   -- columns A^k v / ||A^k v|| with A diagonal, eigenvalues U(0,1)
                   and v Gaussian (a severely ill-conditioned family).
* batch_manifest-- a seeded list of problem shapes for batched runs.
* make_svd_device, make_krylov_device -- the same families drawn on the GPU with
                   torch's generator, for benchmark-sized inputs.
"""
from __future__ import annotations

import functools

import numpy as np


def fortran(a: np.ndarray) -> np.ndarray:
    """Return `a` as a float64 column-major array (copying only if needed)."""
    return np.asfortranarray(a, dtype=np.float64)


def _orthonormal_columns(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """Q factor (m x n, orthonormal columns) of a seeded Gaussian matrix, sign-fixed
    so that the R factor has a positive diagonal (this makes it unique)."""
    g = rng.standard_normal((m, n))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


@functools.lru_cache(maxsize=2)
def _svd_factors(m: int, n: int, seed: int):
    rng = np.random.default_rng(seed)
    u = _orthonormal_columns(rng, m, n)
    v = _orthonormal_columns(rng, n, n)
    u.setflags(write=False)
    v.setflags(write=False)
    return u, v


def make_svd(m: int, n: int, kappa: float, seed: int = 0, norm2: float = 1.0) -> np.ndarray:
    """X = U diag(sigma) V^T, sigma_i = norm2 * kappa^(-(i-1)/(n-1)), i = 1..n.

    U is the Q factor of a seeded m x n Gaussian, V the Q factor of a seeded
    n x n Gaussian (both sign-fixed). kappa_2(X) = kappa, ||X||_2 = norm2.
    The factors depend only on (m, n, seed), so a sweep over kappa reuses them.
    """
    if not (m >= n >= 1):
        raise ValueError("need m >= n >= 1")
    u, v = _svd_factors(m, n, seed)
    if n == 1:
        sig = np.array([1.0])
    else:
        sig = kappa ** (-np.arange(n, dtype=np.float64) / (n - 1))
    sig = sig * norm2
    x = (u * sig) @ v.T
    return fortran(x)


def make_lowtri(a: float, copies: int = 400, nb: int = 50) -> np.ndarray:
    """Stack `copies` copies of F (nb x nb): F_ii = 100, F_ij = a for j < i, 0 above."""
    f = np.tril(np.full((nb, nb), float(a)), k=-1) + 100.0 * np.eye(nb)
    return fortran(np.tile(f, (copies, 1)))


def make_arrowhead(beta: float, m: int = 20000, n: int = 50) -> np.ndarray:
    """X = -5 e_b e_a^T + P_s, e_a = (0,1,...,1) in R^n, e_b = e_1 in R^m,
    P_s = [E; 0] with E = diag(1, ..., 1, beta) (n x n)."""
    x = np.zeros((m, n))
    e = np.ones(n)
    e[-1] = beta
    x[np.arange(n), np.arange(n)] = e
    x[0, 1:] += -5.0
    return fortran(x)


def make_krylov(m: int, n: int, seed: int = 0, block: int = 1 << 20) -> np.ndarray:
    """Krylov-monomial columns x_k = A^k v / ||A^k v||, k = 0..n-1, with
    A = diag(lambda), lambda_i ~ U(0,1) i.i.d., v ~ N(0, I) (seeded).

    Column norms are summed over fixed row blocks in index order, so the result
    does not depend on how the work is split.
    """
    rng = np.random.default_rng(seed)
    lam = rng.random(m)
    v = rng.standard_normal(m)
    x = np.empty((m, n), order="F")

    def _norm(c: np.ndarray) -> float:
        acc = 0.0
        for b0 in range(0, m, block):
            seg = c[b0:b0 + block]
            acc += float(np.dot(seg, seg))
        return float(np.sqrt(acc))

    cur = v / _norm(v)
    x[:, 0] = cur
    for k in range(1, n):
        cur = lam * cur
        cur = cur / _norm(cur)
        x[:, k] = cur
    return x


def batch_manifest(seed: int = 0, count: int = 512, m_lo: int = 10000, m_hi: int = 500000,
                   n_choices=(16, 32, 64, 128), logk_lo: float = 2.0, logk_hi: float = 14.0):
    """Seeded list of batched problems: m ~ U{m_lo..m_hi}, n ~ U(n_choices),
    log10(kappa) ~ U[logk_lo, logk_hi]; input seed 1000+i, sketch seed i, s = 2n."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = rng.choice(np.asarray(n_choices), size=count)
    lk = rng.uniform(logk_lo, logk_hi, size=count)
    out = []
    for i in range(count):
        n = int(ns[i])
        out.append(dict(m=int(ms[i]), n=n, kappa=float(10.0 ** lk[i]), input_seed=1000 + i,
                        seed=i, s=2 * n))
    return out


# ---------------------------------------------------------------------------
# Device-side versions for benchmark-sized inputs (gigabytes): the same
# constructions drawn with torch's generator on the GPU, so the values differ
# from the numpy versions above (which the parity tests use).
# ---------------------------------------------------------------------------
def _torch_colmajor(x):
    import torch
    out = torch.empty((x.shape[1], x.shape[0]), dtype=torch.float64, device=x.device).t()
    out.copy_(x)
    return out


def _orthonormalize_device(u):
    """Orthonormal columns spanning those of a well-conditioned device matrix u
    (a Gaussian, kappa ~ 1 + O(sqrt(n/m))): two Cholesky QR passes whose small
    n x n factors are formed on the host, so the device runs plain matrix
    products only (no device LAPACK)."""
    import torch
    for _ in range(2):
        g = (u.t() @ u).cpu().numpy()
        r = np.linalg.cholesky(g).T                       # upper, g = r^T r
        rinv = np.linalg.inv(r)
        u = u @ torch.from_numpy(np.ascontiguousarray(rinv)).to(u.device)
    return u


def make_svd_device(m: int, n: int, kappa: float, seed: int = 0, device="cuda", orthonormal: bool = True):
    """X = U diag(sigma) V^T on the device, column-major, sigma as in make_svd.

    orthonormal=True: U has orthonormal columns spanning a Gaussian's
    (kappa_2(X) = kappa to rounding).
    orthonormal=False: U is a Gaussian with unit columns, whose condition number
    is 1 + O(sqrt(n/m)), so kappa_2(X) is kappa to within a few percent (cheap
    enough for hundreds of matrices).
    V is the sign-fixed Q factor of a seeded n x n Gaussian, formed on the host."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    u = torch.randn((m, n), generator=g, dtype=torch.float64, device=device)
    if orthonormal:
        u = _orthonormalize_device(u)
    else:
        u /= torch.linalg.vector_norm(u, dim=0, keepdim=True)
    v = _orthonormal_columns(np.random.default_rng(int(seed) + 7919), n, n)
    v = torch.from_numpy(np.ascontiguousarray(v)).to(u.device)
    if n == 1:
        sig = torch.ones(1, dtype=torch.float64, device=device)
    else:
        sig = float(kappa) ** (-torch.arange(n, dtype=torch.float64, device=device) / (n - 1))
    x = (u * sig) @ v.t()
    del u
    return _torch_colmajor(x)


def make_krylov_device(m: int, n: int, seed: int = 0, device="cuda"):
    """make_krylov's family on the device (torch's generator), column-major."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    lam = torch.rand(m, generator=g, dtype=torch.float64, device=device)
    cur = torch.randn(m, generator=g, dtype=torch.float64, device=device)
    out = torch.empty((n, m), dtype=torch.float64, device=device)
    cur = cur / torch.linalg.vector_norm(cur)
    out[0] = cur
    for k in range(1, n):
        cur = lam * cur
        cur = cur / torch.linalg.vector_norm(cur)
        out[k] = cur
    return out.t()
