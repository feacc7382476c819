"""GPU parity of each step of the hot path against the oracle's step, on the
same seeded inputs (inputs of each step come from the oracle, never from the
HIP path). Called through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from gen import make_svd
from gpu_common import gpu, require_gpu, to_dev, to_host

pytestmark = gpu


@pytest.fixture(autouse=True)
def _dev():
    require_gpu()
    import paper_2412_06551_amd  # noqa: F401


def _lib():
    import paper_2412_06551_amd as lib
    return lib


# ---------------------------------------------------------------- generator
def test_philox_words_bit_exact():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(1000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    for k0, k1 in [(0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (0xA4093822, 0x299F31D0), (12345, 678)]:
        t = torch.from_numpy(ctr.view(np.int32)).cuda()
        out = _lib().philox(t, k0, k1).cpu().numpy().view(np.uint32)
        for i in range(0, 1000, 97):
            want = oracle.philox4x32_10(ctr[i], [k0, k1])
            assert out[i].tolist() == want.tolist()


@pytest.mark.parametrize("s,cols,j0,seed", [(64, 3000, 0, 0), (13, 257, 5, 7), (128, 1000, (1 << 32) - 10, 2**40 + 3)])
def test_omega_normals_match(s, cols, j0, seed):
    g = to_host(_lib().omega(s, cols, seed, j0)).astype(np.float64)
    want = oracle.omega(s, cols, seed, j0) * math.sqrt(s)  # unscaled normals
    # both sides compute the same Box-Muller transform of the same Philox words;
    # the oracle in float64, rounded to float32, the device in float32 on the
    # hardware log2, sqrt, sin and cos (in revolutions), measured within 8 float32
    # ulps of max(|z|, 1) of the float32 library transform
    err = np.abs(g - want)
    assert np.all(err <= 8 * 2.0**-24 * np.maximum(np.abs(want), 1.0)), err.max()


# ---------------------------------------------------------------- sketch
@pytest.mark.parametrize("m,n,s,seed", [(2048, 32, 64, 0), (5000 + 37, 64, 128, 3), (700, 16, 40, 1),
                                        (3000, 100, 200, 2), (1025, 5, 5, 4), (3001, 16, 1000, 6),
                                        (40000 + 3, 256, 1024, 8), (50000 + 1, 48, 96, 9)])
def test_sketch_matches_oracle(m, n, s, seed):
    x = make_svd(m, n, 1e6, seed=seed)
    y = to_host(_lib().sketch(to_dev(x), s, seed))
    want = oracle.sketch(x, s, seed)
    om = oracle.omega(s, m, seed)
    # |dY| <= (8 float32 ulps of Omega, as for the normals) |Omega| |X| + summation error
    bound = (8 * 2.0**-24 + 4 * m * oracle.U) * (np.abs(om) @ np.abs(x))
    assert np.all(np.abs(y - want) <= bound)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n,s,seed", [(2048, 32, 64, 0), (5000 + 37, 64, 128, 3), (3000, 100, 200, 2),
                                        (4099, 256, 512, 5), (700, 16, 40, 1), (40000 + 3, 256, 1024, 8)])
def test_sketch_low_precision(prec, m, n, s, seed):
    x = make_svd(m, n, 1e6, seed=seed)
    y = to_host(_lib().sketch(to_dev(x), s, seed, prec=prec))
    want = oracle.sketch(x, s, seed)
    ab = np.abs(oracle.omega(s, m, seed)) @ np.abs(x)
    # inputs rounded to the working precision (FP32: X; BF16: G and X), products
    # exact in FP32, at most m terms added in FP32 per accumulator, then FP64
    uin = 2.0**-24 if prec == "fp32" else 2.0**-8
    assert np.all(np.abs(y - want) <= (2 * uin + (m + 8) * 2.0**-24) * ab)
    # the typical error is at the rounding level: a misplaced row or column would be O(1)
    rel = np.abs(y - want) / ab
    assert np.median(rel) <= 4 * uin + 4 * np.sqrt(m) * 2.0**-24


@pytest.mark.parametrize("grid", ["43", "200"])
def test_sketch_grid_hint(grid, monkeypatch):
    # row chunks not a multiple of 8 (plain workgroup order) and a smaller grid:
    # the same sketch up to summation order
    m, n, s, seed = 30000 + 9, 64, 256, 12
    x = make_svd(m, n, 1e4, seed=seed)
    want = oracle.sketch(x, s, seed)
    monkeypatch.setenv("RCLUPP_SKETCH_GRID", grid)
    y = to_host(_lib().sketch(to_dev(x), s, seed))
    om = oracle.omega(s, m, seed)
    bound = (8 * 2.0**-24 + 4 * m * oracle.U) * (np.abs(om) @ np.abs(x))
    assert np.all(np.abs(y - want) <= bound)


@pytest.mark.parametrize("m,n,s,seed", [(2048, 32, 64, 0), (5000 + 37, 64, 128, 3), (40000 + 3, 256, 1024, 8),
                                        (3001, 5, 40, 1), (7000 + 1, 16, 1792, 2), (20000 + 11, 100, 200, 4)])
def test_countsketch_matches_oracle(m, n, s, seed):
    # every slice width (64, 32, 16, 8 columns), the largest s and a ragged last
    # tile; the sums
    # differ from the oracle's only in their association
    x = make_svd(m, n, 1e6, seed=seed)
    y = to_host(_lib().countsketch(to_dev(x), s, seed))
    want = oracle.countsketch(x, s, seed)
    colsum = np.sum(np.abs(x), axis=0)
    assert np.all(np.abs(y - want) <= 4 * m * oracle.U * colsum[None, :])
    # a misplaced row or sign would be O(|x|): the typical error is at rounding level
    assert np.max(np.abs(y - want)) <= 1e-12 * np.max(colsum)


@pytest.mark.parametrize("m,n,s,seed", [(4096, 32, 64, 0), (5000 + 37, 64, 128, 3), (64, 16, 64, 1),
                                        (3000, 100, 200, 2), (40000 + 3, 256, 1024, 8), (1, 1, 1, 5)])
def test_srht_matches_oracle(m, n, s, seed):
    # a power of two, ragged sizes (X padded to m' rows), all rows of the
    # order-64 Hadamard matrix (s = m = 64) and the 1 x 1 case; the +-1 / sqrt(s)
    # entries are exact on both sides, so only the association of the sums differs
    x = make_svd(m, n, 1e6, seed=seed) if m >= n and m > 1 else np.ones((m, n), order="F")
    y = to_host(_lib().srht(to_dev(x), s, seed))
    want = oracle.srht(x, s, seed)
    colsum = np.sum(np.abs(x), axis=0) / np.sqrt(s)  # = |S| |X| (every |S_ij| = 1 / sqrt(s))
    assert np.all(np.abs(y - want) <= (4 * m + 8) * oracle.U * colsum[None, :])
    # a wrong row sample or sign would be O(|x|): the typical error is at rounding level
    assert np.max(np.abs(y - want)) <= 1e-12 * max(np.max(colsum), 1.0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n,s,seed", [(2048, 32, 64, 0), (5000 + 37, 64, 128, 3), (4099, 256, 512, 5)])
def test_srht_low_precision(prec, m, n, s, seed):
    # X rounded to the working precision (S is exact), products exact in FP32, at
    # most m terms added in FP32 per accumulator, then FP64
    x = make_svd(m, n, 1e6, seed=seed)
    y = to_host(_lib().srht(to_dev(x), s, seed, prec=prec))
    want = oracle.srht(x, s, seed)
    ab = np.broadcast_to(np.sum(np.abs(x), axis=0) / np.sqrt(s), want.shape)
    uin = 2.0**-24 if prec == "fp32" else 2.0**-8
    assert np.all(np.abs(y - want) <= (uin + (m + 8) * 2.0**-24) * ab)
    rel = np.abs(y - want) / ab
    assert np.median(rel) <= 4 * uin + 4 * np.sqrt(m) * 2.0**-24


def test_srht_rejects_more_rows_than_the_hadamard_order():
    x = make_svd(100, 4, 1e2, seed=1)
    with pytest.raises(Exception) as e:
        _lib().srht(to_dev(x), 129, 0)  # m' = 128
    from paper_2412_06551_amd import _native
    assert getattr(e.value, "status", None) == _native.ERR_INVALID_ARG


def test_sketch_leading_dimension():
    x = make_svd(3000, 24, 1e3, seed=5)
    a = to_host(_lib().sketch(to_dev(x, ld=3072), 48, 9))
    b = to_host(_lib().sketch(to_dev(x), 48, 9))
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------- preconditioner
# (300, 64), (512, 200), (300, 6), (1500, 9), (4096, 40): the multi-workgroup
# kernel with 8, 25, 1, 2 and 40 workgroups (the last one also wraps the ring
# of published steps several times)
@pytest.mark.parametrize("s,n,seed", [(64, 32, 0), (128, 64, 1), (100, 50, 2), (16, 16, 3), (256, 128, 4),
                                      (300, 64, 5), (512, 200, 6), (300, 6, 7), (1500, 9, 8), (4096, 40, 9)])
@pytest.mark.parametrize("kappa", [1e2, 1e8])
def test_precond_lu_householder(s, n, seed, kappa):
    x = make_svd(4 * s, n, kappa, seed=seed)
    y = oracle.sketch(x, s, seed)  # oracle input, uploaded
    R1, perm, M, info = _lib().precond(to_dev(y), lu=True, want_m=True)
    assert info.cpu().tolist()[0] == 0
    Mo, No, po, io = oracle.gepp(y)
    assert io[0] == 0
    np.testing.assert_array_equal(perm.cpu().numpy(), po)  # random data: no near-ties
    # M is the oracle's bit for bit: the multipliers are correctly rounded
    # quotients (the register kernel forms them from one reciprocal with
    # Markstein's correction, which gives RN(x / p)) and every entry takes the
    # same fused updates in the same column order as the oracle's elimination
    np.testing.assert_array_equal(to_host(M), Mo)
    R0 = oracle.house_r(Mo)
    r1o = oracle.trmm(R0, No)
    r1o = np.sign(np.diag(r1o))[:, None] * r1o
    r1 = to_host(R1)
    assert np.linalg.norm(r1 - r1o) <= 1e-15 * kappa * n * np.linalg.norm(r1o)
    assert np.all(np.diag(r1) > 0) and np.all(np.tril(r1, -1) == 0)
    # both are (up to row signs) the R factor of Y: R1^T R1 = Y^T Y (eq. elu-ey)
    g = y.T @ y
    assert np.linalg.norm(r1.T @ r1 - g) <= 1e-13 * np.linalg.norm(g)


@pytest.mark.parametrize("s,n", [(64, 32), (128, 64)])
def test_precond_lu_subnormal_pivots(s, n):
    # every entry subnormal: 1 / pivot would overflow, so those steps divide
    # directly; M still equals the oracle's bit for bit (IEEE subnormals)
    y = np.asfortranarray(np.random.default_rng(s).standard_normal((s, n)) * 1e-310)
    assert np.all(np.abs(y) < np.finfo(np.float64).tiny)
    _, perm, M, info = _lib().precond(to_dev(y), lu=True, want_m=True)
    Mo, _, po, io = oracle.gepp(y)
    assert info.cpu().tolist()[0] == 0 and io[0] == 0
    np.testing.assert_array_equal(perm.cpu().numpy(), po)
    np.testing.assert_array_equal(to_host(M), Mo)


def _huge_pivot_sketch(s, n):
    """Three columns with one entry of 1.5 2^1022 (the pivot of that column's
    step) and the rest of order 2^1016; the other columns standard normal.
    No elimination step can overflow (|multipliers| <= 1 and the updated
    entries stay below 2^1019)."""
    rng = np.random.default_rng(s + 3 * n)
    y = rng.standard_normal((s, n))
    for k, j in enumerate((0, n // 3, 2 * n // 3)):
        y[:, j] *= 2.0**1016
        y[5 + 7 * k, j] = (1.5 if k % 2 == 0 else -1.5) * 2.0**1022
    return np.asfortranarray(y)


@pytest.mark.parametrize("s,n", [(64, 32), (128, 64), (256, 128)])
def test_precond_lu_huge_pivots(s, n):
    # entries near the overflow threshold: pivots above 2^1022 have a subnormal
    # reciprocal, so those steps divide directly and M still equals the
    # oracle's bit for bit. R_1 = R_0 N may overflow here, which the kernel
    # reports after M is written.
    y = _huge_pivot_sketch(s, n)
    _, perm, M, info = _lib().precond(to_dev(y), lu=True, want_m=True)
    Mo, No, po, io = oracle.gepp(y)
    assert io[0] == 0
    assert np.sum(np.abs(np.diag(No)) > 2.0**1022) >= 3  # those steps took the direct division
    assert info.cpu().tolist()[0] in (0, oracle.NONFINITE)
    np.testing.assert_array_equal(perm.cpu().numpy(), po)
    np.testing.assert_array_equal(to_host(M), Mo)


@pytest.mark.parametrize("s,n", [(64, 32), (256, 128)])
def test_precond_fp32_huge_pivot(s, n):
    # FP32 LU with a first pivot above 2^126 (its reciprocal is subnormal in
    # FP32): the step divides directly and R_1 keeps FP32 accuracy row by row
    rng = np.random.default_rng(s + n)
    y = rng.standard_normal((s, n))
    y[:, 0] *= 2.0**120
    y[3, 0] = 1.5 * 2.0**126
    y = np.asfortranarray(y)
    R1, _, _, info = _lib().precond(to_dev(y), lu=True, prec="fp32")
    assert info.cpu().tolist()[0] == 0
    Mo, No, _, _ = oracle.gepp(y)
    r1o = oracle.trmm(oracle.house_r(Mo), No)
    r1o = np.sign(np.diag(r1o))[:, None] * r1o
    r1 = to_host(R1)
    assert np.all(np.isfinite(r1)) and np.all(np.diag(r1) > 0)
    kap = np.linalg.cond(Mo) * np.linalg.cond(No[1:, 1:])
    for i in range(n):
        assert np.linalg.norm(r1[i] - r1o[i]) <= 64 * 2.0**-24 * n * kap * np.linalg.norm(r1o[i]), i


@pytest.mark.parametrize("s,n,seed", [(64, 32, 0), (128, 64, 1), (256, 128, 4), (512, 200, 6)])
@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_precond_fp32(s, n, seed, kappa):
    # FP32 LU + Householder on the FP64 sketch, R_1 widened to FP64: an FP32-accurate R factor of Y
    x = make_svd(4 * s, n, kappa, seed=seed)
    y = oracle.sketch(x, s, seed)
    R1, _, _, info = _lib().precond(to_dev(y), lu=True, prec="fp32")
    assert info.cpu().tolist()[0] == 0
    Mo, No, _, _ = oracle.gepp(y)
    r1o = oracle.trmm(oracle.house_r(Mo), No)
    r1o = np.sign(np.diag(r1o))[:, None] * r1o
    r1 = to_host(R1)
    assert np.all(np.diag(r1) > 0) and np.all(np.tril(r1, -1) == 0)
    assert np.linalg.norm(r1 - r1o) <= 64 * 2.0**-24 * kappa * n * np.linalg.norm(r1o)


@pytest.mark.parametrize("s,n", [(64, 32), (40, 40), (300, 64), (520, 150)])
def test_precond_householder_only(s, n):
    x = make_svd(8 * s, n, 1e4, seed=11)
    y = oracle.sketch(x, s, 3)
    R1, _, _, info = _lib().precond(to_dev(y), lu=False)
    r0 = oracle.house_r(y)
    r0 = np.sign(np.diag(r0))[:, None] * r0
    assert np.linalg.norm(to_host(R1) - r0) <= 1e-13 * np.linalg.norm(r0)


@pytest.mark.parametrize("shape", [(32, 8), (300, 40)])
@pytest.mark.parametrize("case", ["zero", "zero_then_nan", "nan_first", "inf"])
def test_precond_info_codes(case, shape):
    # (300, 40): s > 256, the multi-workgroup kernel
    y = np.random.default_rng(0).standard_normal(shape)
    if case in ("zero", "zero_then_nan"):
        y[:, 3] = 0.0
    if case == "zero_then_nan":
        y[7, 6] = np.nan
    if case == "nan_first":
        y[9, 2] = np.nan
        y[:, 5] = 0.0
    if case == "inf":
        y[0, 0] = np.inf
    y = np.asfortranarray(y)
    _, _, _, info = _lib().precond(to_dev(y), lu=True)
    _, _, _, io = oracle.gepp(y)
    assert info.cpu().tolist()[:3] == io.tolist()[:3]


# ---------------------------------------------------------------- tall passes
def _upper(n, seed, cond=None):
    """A well-conditioned upper triangle with mixed-sign diagonal: the R factor of a
    seeded 3n x n Gaussian (kappa ~ 5), rows flipped at random."""
    rng = np.random.default_rng(seed)
    r = np.linalg.qr(rng.standard_normal((3 * n + 2, n)), mode="r")
    r = np.where(rng.random(n) < 0.5, -1.0, 1.0)[:, None] * r
    return np.asfortranarray(np.triu(r))


def _check_trsm(w, wo, x, R):
    """W from the kernel against the oracle's row-wise substitution W_o.
    Row-wise backward error (eq. ewy): |W R - X| <= gamma |W| |R| with
    gamma = 2 (n + 3) u, covering the substitution's gamma_n and the 2u
    perturbation of R_jj from multiplying by its rounded reciprocal.
    Forward: both solutions satisfy such a bound, so
    |W - W_o| <= 2 gamma |W| |R| |R^{-1}| (first order)."""
    n = R.shape[0]
    g = 2 * (n + 3) * oracle.U
    absr = np.abs(R)
    res = np.abs(w @ R - x)
    assert np.all(res <= g * (np.abs(w) @ absr) + 1e-300)
    rinv = np.linalg.solve(R, np.eye(n))
    fwd = np.abs(w - wo)
    bound = 2.2 * g * ((np.abs(w) @ absr) @ np.abs(rinv))
    assert np.all(fwd <= bound + 1e-300), float(np.max(fwd / (bound + 1e-300)))


@pytest.mark.parametrize("m,n", [(1000, 1), (4096 + 77, 16), (3000, 32), (20000 + 5, 50), (9999, 64),
                                 (5000, 100), (3000, 128), (1200, 129), (2500, 200), (1500, 256)])
def test_trsm_gram_matches_oracle(m, n):
    rng = np.random.default_rng(m + n)
    x = np.asfortranarray(rng.standard_normal((m, n)))
    R = _upper(n, n)
    W, G = _lib().trsm_gram(to_dev(x), to_dev(R), gram=True)
    wo = oracle.trsm(x, R)
    w = to_host(W)
    _check_trsm(w, wo, x, R)
    go = oracle.gram(wo)
    g = to_host(G)
    assert np.max(np.abs(g - go)) <= 1e-12 * np.max(np.abs(go))
    np.testing.assert_array_equal(g, g.T)


@pytest.mark.parametrize("m,n", [(5000, 10), (4096, 64), (3000, 200)])
def test_gram_only(m, n):
    x = np.asfortranarray(np.random.default_rng(n).standard_normal((m, n)))
    _, G = _lib().trsm_gram(to_dev(x), None, gram=True)
    go = oracle.gram(x)
    assert np.max(np.abs(to_host(G) - go)) <= 1e-12 * np.max(np.abs(go))


def test_trsm_in_place_and_ld():
    m, n = 7000, 48
    x = np.asfortranarray(np.random.default_rng(1).standard_normal((m, n)))
    R = _upper(n, 2)
    X = to_dev(x, ld=7040)
    W, _ = _lib().trsm_gram(X, to_dev(R), gram=False, out=X)
    wo = oracle.trsm(x, R)
    _check_trsm(to_host(X), wo, x, R)


@pytest.mark.parametrize("n", [16, 100, 256])
def test_trsm_without_gram(n):
    # the solve alone (no Gram asked for) on each kernel family
    m = 3000 + 7
    x = np.asfortranarray(np.random.default_rng(n).standard_normal((m, n)))
    R = _upper(n, 3)
    W, G = _lib().trsm_gram(to_dev(x), to_dev(R), gram=False)
    assert G is None
    _check_trsm(to_host(W), oracle.trsm(x, R), x, R)


@pytest.mark.parametrize("n", [32, 64, 128, 200])
@pytest.mark.parametrize("layout", ["ld16", "ld_odd", "base_off"])
def test_trsm_gram_layouts(n, layout):
    """Both access forms of the tall kernels against the oracle: nontemporal
    when every column run fills whole 128-byte lines (ld a multiple of 16,
    aligned base), ordinary loads and stores otherwise (an odd ld; an aligned
    ld with the matrix starting one row into its buffer, written to an aligned
    W). Also the Gram of X alone."""
    m = 4000 + 3 * n
    rng = np.random.default_rng(7 * n)
    x = np.asfortranarray(rng.standard_normal((m, n)))
    R = _upper(n, 5)
    if layout == "ld16":
        X = to_dev(x, ld=m + 16 - m % 16)
    elif layout == "ld_odd":
        X = to_dev(x, ld=m + 3)
    else:
        X = to_dev(np.vstack([np.zeros((1, n)), x]), ld=m + 1 + 16 - (m + 1) % 16)[1:]
    W, G = _lib().trsm_gram(X, to_dev(R), gram=True)
    wo = oracle.trsm(x, R)
    w = to_host(W)
    _check_trsm(w, wo, x, R)
    go = oracle.gram(wo)
    assert np.max(np.abs(to_host(G) - go)) <= 1e-12 * np.max(np.abs(go))
    _, G0 = _lib().trsm_gram(X, None, gram=True)
    g0 = oracle.gram(x)
    assert np.max(np.abs(to_host(G0) - g0)) <= 1e-12 * np.max(np.abs(g0))
    # in place (W aliases X, same layout)
    _lib().trsm_gram(X, to_dev(R), gram=False, out=X)
    _check_trsm(to_host(X), wo, x, R)


# ---------------------------------------------------------------- Cholesky
@pytest.mark.parametrize("n", [1, 16, 50, 64, 128, 200, 256])
def test_chol_matches_oracle(n):
    b = np.random.default_rng(n).standard_normal((3 * n + 5, n))
    g = np.asfortranarray(b.T @ b)
    Rp = _upper(n, 3 * n)
    R, Rout, info = _lib().chol(to_dev(g), Rprev=to_dev(Rp))
    assert info.cpu().tolist()[0] == 0
    ro, io = oracle.chol(g)
    np.testing.assert_allclose(to_host(R), ro, rtol=0, atol=1e-12 * np.abs(ro).max())
    np.testing.assert_allclose(to_host(Rout), oracle.trmm(ro, Rp), rtol=0,
                               atol=1e-12 * np.abs(ro).max() * np.abs(Rp).max() * n)


def test_chol_shift_and_breakdown():
    m, n = 100000, 20
    b = np.random.default_rng(4).standard_normal((40, n))
    g = np.asfortranarray(b.T @ b)
    R, _, info = _lib().chol(to_dev(g), m=m, shift=True)
    sigma = oracle.scholqr3_shift(m, n, float(np.max(np.diag(g))))
    ro, _ = oracle.chol(g, shift=sigma)
    np.testing.assert_allclose(to_host(R), ro, rtol=0, atol=1e-12 * np.abs(ro).max())
    g2 = np.diag([4.0, 1.0, -1.0, 2.0])
    _, _, info = _lib().chol(to_dev(np.asfortranarray(g2)), stage=5)
    assert info.cpu().tolist()[:3] == [2, 5, 3]


@pytest.mark.parametrize("n", [136, 200, 256])
def test_chol_blocked_shift_breakdown_nonfinite(n):
    # n > 128: the blocked kernel; Algorithm 4's shift, the first failing
    # column of a breakdown (a negative pivot) and of a non-finite entry
    m = 1000000
    b = np.random.default_rng(n + 1).standard_normal((2 * n, n))
    g = np.asfortranarray(b.T @ b)
    R, _, info = _lib().chol(to_dev(g), m=m, shift=True)
    assert info.cpu().tolist()[0] == 0
    sigma = oracle.scholqr3_shift(m, n, float(np.max(np.diag(g))))
    ro, _ = oracle.chol(g, shift=sigma)
    np.testing.assert_allclose(to_host(R), ro, rtol=0, atol=1e-12 * np.abs(ro).max())
    # a column made dependent on the earlier ones after the first blocks: the
    # pivot of column k is exactly zero in exact arithmetic, so it breaks down
    # there (not earlier) in both; the reported index is the oracle's
    k = n - 7
    c = np.random.default_rng(5).standard_normal((2 * n, n))
    c[:, k] = c[:, 3] - 2.0 * c[:, 20]
    gd = np.asfortranarray(c.T @ c)
    gd[k, k] -= 1.0  # now indefinite at column k
    _, _, info = _lib().chol(to_dev(gd), stage=5)
    _, io = oracle.chol(gd, stage=5)
    assert info.cpu().tolist()[:3] == [2, 5, k + 1] == io[:3].tolist()
    gn = g.copy(order="F")
    gn[10, 150 if n > 150 else n - 1] = np.nan
    _, _, info = _lib().chol(to_dev(gn), stage=4)
    assert info.cpu().tolist()[:3] == [3, 4, (150 if n > 150 else n - 1) + 1]


# ---------------------------------------------------------------- tall LU
@pytest.mark.parametrize("m,n", [(1000, 8), (5000 + 13, 32), (20000, 50), (3000, 64), (2000, 100), (700, 17),
                                 (900, 33), (3000 + 1, 128), (1500, 256)])
def test_tall_lu_matches_oracle(m, n):
    # every element takes the steps' fused multiply-adds in step order on both
    # sides (the blocked updates included), so L and N are the oracle's bit
    # for bit; n = 17, 33, 100 end in partial panels and blocks, n = 128 and
    # 256 take the widest updates
    x = np.asfortranarray(np.random.default_rng(m).standard_normal((m, n)))
    M, perm, info = _lib().tall_lu(to_dev(x))
    assert info.cpu().tolist()[0] == 0
    Mo, No, po, io = oracle.gepp(x)
    np.testing.assert_array_equal(perm.cpu().numpy(), po)
    lu = to_host(M)
    np.testing.assert_array_equal(np.tril(lu, -1)[:, :n], np.tril(Mo, -1))
    np.testing.assert_array_equal(np.triu(lu[:n]), No)


# ---------------------------------------------------------------- tournament pivoting
@pytest.mark.parametrize("m,n,kappa", [(5000, 16, 1e6), (9001, 40, 1e10), (3000, 64, 1e4), (2600, 100, 1e8),
                                       (70000 + 3, 8, 1e3), (300, 128, 1e2), (256, 30, 1e5), (40000 + 7, 128, 1e12),
                                       (1000, 1, 1.0), (128, 128, 1e3), (4099, 9, 1e7), (20000, 65, 1e9)])
def test_tournament_lu_matches_oracle(m, n, kappa):
    # the selection is integer work: pivot rows identical; the tree's
    # eliminations use the same operations, so N and L_11 equal the oracle's bit
    # for bit; M = X N^{-1} by the tall substitution meets its row-wise bound
    x = make_svd(m, n, kappa, seed=m % 97)
    M, sel, N, info = _lib().tall_lu_tournament(to_dev(x))
    sel_o, N_o, L_o, M_o, info_o = oracle.tslu(x)
    assert info.cpu().tolist()[0] == 0 and info_o[0] == 0
    sel_h = sel.cpu().numpy()
    np.testing.assert_array_equal(sel_h, sel_o)
    np.testing.assert_array_equal(to_host(N), N_o)
    m_h = to_host(M)
    np.testing.assert_array_equal(m_h[sel_h], L_o)
    bound = 2 * (n + 3) * oracle.U * (np.abs(m_h) @ np.abs(N_o))
    assert np.all(np.abs(m_h @ N_o - x) <= bound + 1e-300)


@pytest.mark.parametrize("kind", ["integers", "shared_high_word"])
def test_tournament_lu_ties(kind):
    # equal magnitudes decide by position: small integers tie exactly; entries
    # 1 + e 2^-40 share the high word of their bit pattern and differ below it
    rng = np.random.default_rng(11)
    m, n = 3000 + 5, 24
    e = rng.integers(-40, 41, size=(m, n)).astype(np.float64)
    x = np.asfortranarray(e if kind == "integers" else 1.0 + e * 2.0**-40)
    M, sel, N, info = _lib().tall_lu_tournament(to_dev(x))
    sel_o, N_o, L_o, _, info_o = oracle.tslu(x)
    assert info.cpu().tolist()[0] == 0 and info_o[0] == 0
    sel_h = sel.cpu().numpy()
    np.testing.assert_array_equal(sel_h, sel_o)
    np.testing.assert_array_equal(to_host(N), N_o)
    np.testing.assert_array_equal(to_host(M)[sel_h], L_o)


def test_tournament_lu_singular_leaf_and_zero_column():
    m, n = 2048, 12
    x = make_svd(m, n, 1e3, seed=7)
    x[:256] = x[0]  # a rank-one leaf
    M, sel, N, info = _lib().tall_lu_tournament(to_dev(x))
    sel_o, N_o, _, _, _ = oracle.tslu(x)
    assert info.cpu().tolist()[0] == 0
    np.testing.assert_array_equal(sel.cpu().numpy(), sel_o)
    y = make_svd(3000, 10, 1e2, seed=8)
    y[:, 4] = 0.0  # a zero column: the root's zero pivot
    _, _, _, info = _lib().tall_lu_tournament(to_dev(y))
    assert info.cpu().tolist()[:3] == [oracle.LU_ZERO_PIVOT, 1, 5]


def test_tall_lu_zero_pivot():
    x = np.asfortranarray(np.random.default_rng(2).standard_normal((3000, 12)))
    x[:, 7] = 0.0
    _, _, info = _lib().tall_lu(to_dev(x))
    assert info.cpu().tolist()[:3] == [1, 1, 8]
