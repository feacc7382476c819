"""GPU parity of the six methods (Algorithms 2-7) against the oracle on the same
seeded inputs, through the C ABI: orthogonality <= 1e-12, relative residual
<= 1e-13, relative R error <= 1e-14 * kappa_2 (kappa_2 as prescribed by the
generator). Sizes span several row tiles with ragged tails; the full-size
1,048,576 x 64 workload is compared in full (the oracle finishes it in
seconds)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import bounds
from gen import make_arrowhead, make_krylov, make_lowtri, make_svd
from gpu_common import TOL_ORTH, TOL_R, TOL_RES, gpu, method_parity, require_gpu, to_dev, to_host

pytestmark = gpu
ALL = ["rclupp", "rcluppr", "cholqr2", "scholqr3", "lc2", "rcholqr"]


@pytest.fixture(autouse=True)
def _dev():
    require_gpu()


def _lib():
    import paper_2412_06551_amd as lib
    return lib


@pytest.mark.parametrize("method", ALL)
def test_small_config_all_methods(method):
    # m = 2048, n = 32, kappa = 1e8, s = 2n = 64, seed 0
    m, n, s, kappa = 2048, 32, 64, 1e8
    x = make_svd(m, n, kappa, seed=0)
    res = _lib().qr(to_dev(x), alg=method, s=s, seed=0)
    if method == "cholqr2":
        # kappa = 1e8 is at CholeskyQR2's limit (Section 2.1): require the oracle's outcome
        orc = oracle.run(method, x)
        if not orc.ok:
            assert res.info_host()[0] == orc.info[0]
            return
    method_parity(x, method, s, 0, kappa, res)


@pytest.mark.parametrize("method", ["rclupp", "rcluppr", "lc2", "rcholqr"])
@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e10, 1e13, 1e15])
def test_kappa_sweep_ragged(method, kappa):
    m, n, s = 30000 + 77, 50, 100
    x = make_svd(m, n, kappa, seed=1)
    res = _lib().qr(to_dev(x), alg=method, s=s, seed=5)
    method_parity(x, method, s, 5, kappa, res)


@pytest.mark.parametrize("method", ["cholqr2", "scholqr3"])
@pytest.mark.parametrize("kappa", [1e2, 1e6])
def test_baselines_in_range(method, kappa):
    m, n = 12345, 64
    x = make_svd(m, n, kappa, seed=2)
    res = _lib().qr(to_dev(x), alg=method)
    method_parity(x, method, 0, 0, kappa, res)


@pytest.mark.parametrize("method,kappa", [("cholqr2", 1e12), ("scholqr3", 1e16)])
def test_baselines_break_down_like_oracle(method, kappa):
    x = make_svd(5000, 40, kappa, seed=3)
    orc = oracle.run(method, x)
    res = _lib().qr(to_dev(x), alg=method)
    info = res.info_host()
    if not orc.ok:
        assert info[0] == orc.info[0] == oracle.CHOL_BREAKDOWN
    else:  # outside the method's range the result is poor on both sides
        assert oracle.orthogonality(to_host(res.Q)) > TOL_ORTH or info[0] != 0


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 33, 64, 65, 100, 128, 200, 256])
def test_column_counts(n):
    m = max(4 * n + 3, 3000)
    kappa = 1e6
    x = make_svd(m, n, kappa, seed=n)
    for method in ("rclupp", "rcluppr"):
        res = _lib().qr(to_dev(x), alg=method, s=2 * n, seed=1)
        method_parity(x, method, 2 * n, 1, kappa, res)


@pytest.mark.parametrize("m,n,s", [(64, 64, 64), (65, 64, 64), (130, 64, 128), (300, 32, 300)])
def test_edge_shapes(m, n, s):
    # m = n (square), s = n, s = m
    x = make_svd(m, n, 1e4, seed=4)
    for method in ("rclupp", "rcluppr", "lc2"):
        res = _lib().qr(to_dev(x), alg=method, s=s, seed=2)
        method_parity(x, method, s, 2, 1e4, res)


def test_leading_dimension_and_simple_entry():
    m, n = 9000, 48
    x = make_svd(m, n, 1e9, seed=6)
    X = to_dev(x, ld=9216)
    a = _lib().qr(X, alg="rclupp", s=96, seed=3)
    method_parity(x, "rclupp", 96, 3, 1e9, a)
    Q, R, info = _lib().qr_simple(X, alg="rclupp", s=96, seed=3)
    assert info[0] == 0
    np.testing.assert_array_equal(to_host(Q), to_host(a.Q))
    np.testing.assert_array_equal(to_host(R), to_host(a.R))
    for method in ALL:
        Q, R, info = _lib().qr_simple(X, alg=method, s=96, seed=3)
        orc = oracle.run(method, x, s=96, seed=3)
        assert info[0] == orc.info[0]


def test_determinism():
    x = make_svd(50000, 64, 1e12, seed=7)
    X = to_dev(x)
    a = _lib().qr(X, alg="rclupp", s=128, seed=9)
    b = _lib().qr(X, alg="rclupp", s=128, seed=9)
    np.testing.assert_array_equal(to_host(a.Q), to_host(b.Q))
    np.testing.assert_array_equal(to_host(a.R), to_host(b.R))


@pytest.mark.parametrize("method", ALL)
def test_info_nonfinite_and_zero_column(method):
    x = make_svd(4000, 16, 1e3, seed=8)
    xn = x.copy(order="F")
    xn[123, 5] = np.nan
    res = _lib().qr(to_dev(xn), alg=method, s=32, seed=0)
    orc = oracle.run(method, xn, s=32, seed=0)
    assert res.info_host()[:3] == orc.info.tolist()[:3], (method, res.info_host(), orc.info)
    xz = x.copy(order="F")
    xz[:, 9] = 0.0
    res = _lib().qr(to_dev(xz), alg=method, s=32, seed=0)
    orc = oracle.run(method, xz, s=32, seed=0)
    assert res.info_host()[0] == orc.info[0], (method, res.info_host(), orc.info)
    if orc.info[0] == oracle.LU_ZERO_PIVOT:
        assert res.info_host()[:3] == orc.info.tolist()[:3]


def test_underflow_scaled_input_is_reported():
    # X scaled to the underflow threshold: R_1's diagonal is subnormal, its
    # reciprocals overflow, and the non-finite solve is reported by the first
    # Cholesky (info, not a silently wrong factor)
    x = make_svd(3000, 16, 1e2, seed=3) * 1e-312
    res = _lib().qr(to_dev(np.asfortranarray(x)), alg="rclupp", s=32, seed=0)
    info = res.info_host()
    assert info[0] == oracle.NONFINITE and info[1] == oracle.ST_CHOL_A, info


def test_invalid_arguments_are_synchronous_errors():
    from paper_2412_06551_amd import _native as nat
    x = to_dev(make_svd(100, 8, 10.0, seed=0))
    with pytest.raises(nat.RclError) as e:
        _lib().qr(x, alg="rclupp", s=4)  # s < n
    assert e.value.status == nat.ERR_INVALID_ARG
    with pytest.raises(nat.RclError):
        _lib().qr(x, alg="rclupp", s=101)  # s > m
    big = torch.zeros((300, 1000), dtype=torch.float64, device="cuda").t()
    with pytest.raises(nat.RclError) as e:
        _lib().qr(big, alg="cholqr2")  # n > 256
    assert e.value.status == nat.ERR_UNSUPPORTED


@pytest.mark.parametrize("beta", [1e-10, 1e-15, 1e-20, 1e-25, 1e-30])
def test_arrowhead_rcluppr(beta):
    # Section 5.1.3's arrowhead family with s = 100
    x = make_arrowhead(beta)
    res = _lib().qr(to_dev(x), alg="rcluppr", s=100, seed=0)
    orc = oracle.rcluppr(x, 100, 0)
    info = res.info_host()
    if orc.ok and info[0] == 0:
        r = to_host(res.R)
        m = oracle.metrics(x, to_host(res.Q), r)
        assert m["orth"] <= TOL_ORTH and m["rel_res"] <= TOL_RES
        # the full parity bar: kappa_2 estimated from the computed singular
        # values (an underestimate when sigma_min is below rounding level,
        # which only tightens the bar)
        sv = np.linalg.svd(x, compute_uv=False)
        rerr = np.linalg.norm(r - orc.R) / np.linalg.norm(orc.R)
        assert rerr <= TOL_R * max(sv[0] / sv[-1], 1.0), (beta, rerr)
        return
    if info[:3] == orc.info.tolist()[:3]:
        return
    # The outcomes differ. That is allowed only where the preconditioned Q_1 lies far
    # outside CholeskyQR2's range (Lemma 3.1): there the first Cholesky's last pivot
    # is at rounding level and its sign is decided by the summation order.
    q1 = oracle.trsm(x, orc.R1)
    sv = np.linalg.svd(q1, compute_uv=False)
    assert sv[0] / sv[-1] > 1e3 * bounds.cholqr2_kappa_limit(*x.shape), (info, orc.info)
    if info[0] != 0:
        assert info[0] == oracle.CHOL_BREAKDOWN and info[1] in (oracle.ST_CHOL_A, oracle.ST_CHOL_B)
    else:
        r = to_host(res.R)
        assert np.all(np.isfinite(r)) and np.all(np.diag(r) > 0) and np.all(np.tril(r, -1) == 0)
        assert oracle.metrics(x, to_host(res.Q), r)["rel_res"] <= TOL_RES


@pytest.mark.parametrize("a", [-0.6, -1.0])
def test_lowtri_family(a):
    x = make_lowtri(a)
    for method in ("rclupp", "rcluppr", "lc2"):
        res = _lib().qr(to_dev(x), alg=method, s=100, seed=0)
        method_parity(x, method, 100, 0, 2.0, res)


def test_krylov_rcluppr_invariants():
    # numerically rank deficient: (Q, R) are not unique, only the invariants are compared
    x = make_krylov(200000, 64, seed=0)
    res = _lib().qr(to_dev(x), alg="rcluppr", s=128, seed=0)
    assert res.info_host()[0] == 0
    m = oracle.metrics(x, to_host(res.Q), to_host(res.R))
    assert m["orth"] <= TOL_ORTH and m["rel_res"] <= TOL_RES
    r = to_host(res.R)
    assert np.all(np.diag(r) > 0) and np.all(np.tril(r, -1) == 0)


def _batch_inputs(shapes, seed0=100):
    rng = np.random.default_rng(0)
    kap = [10 ** rng.uniform(2, 12) for _ in shapes]
    xs = [make_svd(m, n, kap[i], seed=seed0 + i) for i, (m, n) in enumerate(shapes)]
    return xs, kap


def test_batched_grouped_parity_and_isolation():
    # RCLUPP problems of uneven m and n in one call, grouped by (n, s): each result
    # meets the parity bar, and a poisoned problem does not affect the others
    shapes = [(3000, 16), (5000, 32), (2000, 64), (7000, 24), (4000, 128), (9001, 64), (2500, 16), (6100, 128)]
    xs, kap = _batch_inputs(shapes)
    xs[2][5, 5] = np.nan
    Xs = [to_dev(x) for x in xs]
    Qs, Rs, info = _lib().qr_batched(Xs, alg="rclupp", seeds=list(range(len(xs))))
    info = info.cpu().numpy()
    for i, x in enumerate(xs):
        if i == 2:
            assert info[i][0] == oracle.NONFINITE
            continue
        assert info[i][0] == 0, (i, info[i])
        n = x.shape[1]

        class _R:
            pass
        r = _R()
        r.Q, r.R = Qs[i], Rs[i]
        r.info_host = lambda i=i: info[i].tolist()
        method_parity(x, "rclupp", 2 * n, i, kap[i], r)
        # the single-problem call differs only in how rows are split among workgroups
        one = _lib().qr(Xs[i], alg="rclupp", seed=i)
        d = np.linalg.norm(to_host(one.R) - to_host(Rs[i])) / np.linalg.norm(to_host(one.R))
        assert d <= 1e-14 * kap[i]


def test_batched_deterministic_and_graph_replays():
    shapes = [(3000, 16), (5000, 32), (2000, 64), (4000, 128), (6100, 128), (1200, 48)]
    xs, _ = _batch_inputs(shapes, seed0=300)
    Xs = [to_dev(x) for x in xs]
    eager = _lib().Batch(Xs, alg="rclupp")
    q0, r0, i0 = eager.run()
    ref_q = [to_host(q) for q in q0]
    ref_r = [to_host(r) for r in r0]
    ref_i = i0.cpu().numpy().copy()
    q1, r1, _ = eager.run()
    for k in range(len(xs)):
        np.testing.assert_array_equal(to_host(q1[k]), ref_q[k])
        np.testing.assert_array_equal(to_host(r1[k]), ref_r[k])
    g = _lib().Batch(Xs, alg="rclupp", graph=True)
    for rep in range(3):
        # the program's own eager work between the replays
        other = _lib().qr(Xs[1], alg="rclupp", seed=7)
        torch.cuda.synchronize()
        for q in g.Qs:
            q.fill_(-1.0)
        qg, rg, ig = g.run()
        torch.cuda.synchronize()
        assert np.array_equal(ig.cpu().numpy(), ref_i), rep
        for k in range(len(xs)):
            np.testing.assert_array_equal(to_host(qg[k]), ref_q[k])
            np.testing.assert_array_equal(to_host(rg[k]), ref_r[k])
        del other


def test_batched_autotune_parity():
    shapes = [(20000, 16), (15000, 32), (9000, 64), (12000, 128)]
    xs, kap = _batch_inputs(shapes, seed0=500)
    Xs = [to_dev(x) for x in xs]
    b = _lib().Batch(Xs, alg="rclupp", autotune=True)
    for _ in range(2):  # the first call tunes, the second reuses the choice
        Qs, Rs, info = b.run()
        torch.cuda.synchronize()
        for i, x in enumerate(xs):
            assert info[i].cpu().tolist()[0] == 0
            m = oracle.metrics(x, to_host(Qs[i]), to_host(Rs[i]))
            assert m["orth"] <= TOL_ORTH and m["rel_res"] <= TOL_RES


def test_batched_tuning_cache_persists(tmp_path, monkeypatch):
    # the tuned knobs go to the cache file (one line per batch shape) and are
    # read back after the in-memory table is dropped: the second run takes the
    # same plan (equal bits) without tuning again (no second line)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("RCLUPP_TUNE_CACHE", str(cache))
    # an earlier test may have tuned this batch shape: start from an empty table
    _nat().release()
    shapes = [(20000, 16), (15000, 32), (9000, 64), (12000, 128)]
    xs, _ = _batch_inputs(shapes, seed0=550)
    Xs = [to_dev(x) for x in xs]
    b = _lib().Batch(Xs, alg="rclupp", autotune=True)
    q0, r0, i0 = b.run()
    torch.cuda.synchronize()
    lines = cache.read_text().split("\n")
    lines = [ln for ln in lines if ln.strip()]
    assert len(lines) == 1
    key, tall, sk = lines[0].split()
    assert int(tall) in (4, 8, 16, 32, 64) and int(sk) in (16, 32, 64, 128, 256, 512, 1024) and len(key) == 16
    ref_q = [to_host(q) for q in q0]
    _nat().release()  # drops the in-memory table (and the cached graphs)
    q1, r1, i1 = b.run()
    torch.cuda.synchronize()
    for k in range(len(xs)):
        np.testing.assert_array_equal(to_host(q1[k]), ref_q[k])
    assert len([ln for ln in cache.read_text().split("\n") if ln.strip()]) == 1


def test_batched_parity_sample_vs_oracle():
    # problems drawn from the 512-problem manifest (m cut to a tenth), every
    # (n, s) group present, each against the oracle at the parity bar
    from gen import batch_manifest
    man = [p for p in batch_manifest(0, 512)]
    picked = []
    for n in (16, 32, 64, 128):
        picked += [p for p in man if p["n"] == n][:3]
    xs = [make_svd(p["m"] // 10, p["n"], p["kappa"], seed=p["input_seed"]) for p in picked]
    Xs = [to_dev(x) for x in xs]
    Qs, Rs, info = _lib().qr_batched(Xs, alg="rclupp", seeds=[p["seed"] for p in picked], graph=True)
    torch.cuda.synchronize()
    for i, (x, p) in enumerate(zip(xs, picked)):
        class _R:
            pass
        r = _R()
        r.Q, r.R = Qs[i], Rs[i]
        r.info_host = lambda i=i: info[i].cpu().tolist()
        method_parity(x, "rclupp", 2 * p["n"], p["seed"], p["kappa"], r)


def test_batched_sequential_fallback_matches_single():
    # a problem beyond the grouped kernels (n = 200) sends the batch down the
    # single-problem pipeline: identical to separate calls
    shapes = [(3000, 16), (4000, 200), (2000, 64)]
    xs, _ = _batch_inputs(shapes, seed0=700)
    Xs = [to_dev(x) for x in xs]
    Qs, Rs, info = _lib().qr_batched(Xs, alg="rclupp", seeds=[0, 1, 2])
    for i in range(len(xs)):
        one = _lib().qr(Xs[i], alg="rclupp", seed=i)
        assert info[i].cpu().tolist() == one.info_host()
        np.testing.assert_array_equal(to_host(Qs[i]), to_host(one.Q))
        np.testing.assert_array_equal(to_host(Rs[i]), to_host(one.R))


# ------------------------------------------------------------------ mixed precision
# FP32 or BF16 sketch on MFMA and an FP32 preconditioner; the tall passes, the
# Cholesky factors and the last CholeskyQR pass stay FP64, so the final Q and R
# must meet the same bar against the FP64 oracle wherever the rounded
# preconditioner still brings Q_1 into CholeskyQR2's range.
# Beyond that range (a BF16 sketch of X leaves kappa(Q_1) near 2^-9 kappa(X))
# the call escalates to the shifted Cholesky and one more CholeskyQR pass, and
# the same bar applies.
@pytest.mark.parametrize("sk,lu,kappa", [("fp32", "fp32", 1e2), ("fp32", "fp32", 1e8), ("fp32", "fp32", 1e14),
                                         ("fp32", "fp64", 1e14), ("fp32", "fp32", 1e15), ("bf16", "fp32", 1e2),
                                         ("bf16", "fp32", 1e6), ("bf16", "fp64", 1e6), ("bf16", "fp32", 1e10),
                                         ("bf16", "fp32", 1e12), ("bf16", "fp32", 1e14), ("bf16", "fp32", 1e15)])
def test_mixed_rclupp(sk, lu, kappa):
    m, n, s = 40000 + 11, 64, 256
    x = make_svd(m, n, kappa, seed=21)
    res = _lib().qr(to_dev(x), alg="rclupp", s=s, seed=4, sketch_prec=sk, lu_prec=lu)
    method_parity(x, "rclupp", s, 4, kappa, res)
    notes = res.info_host()[3]
    if kappa <= 1e6 or sk == "fp32" and kappa <= 1e8:
        assert notes == 0  # well inside CholeskyQR2's range: no extra pass
    if sk == "bf16" and kappa >= 1e14:
        assert notes == _nat().NOTE_ESCALATED  # kappa(Q_1) near 1e11: the first Cholesky breaks down


def _nat():
    from paper_2412_06551_amd import _native
    return _native


@pytest.mark.parametrize("kappa", [1e4, 1e10, 1e15])
def test_mixed_rcluppr_bf16(kappa):
    # the sketch of the well-conditioned M factor tolerates BF16 at any kappa
    m, n, s = 30000 + 5, 48, 96
    x = make_svd(m, n, kappa, seed=22)
    res = _lib().qr(to_dev(x), alg="rcluppr", s=s, seed=1, sketch_prec="bf16", lu_prec="fp32")
    method_parity(x, "rcluppr", s, 1, kappa, res)


@pytest.mark.parametrize("sk", ["fp32", "bf16"])
@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e14])
def test_mixed_wide(sk, kappa):
    # the n = 256, s = 4n shape of the mixed-precision workload at reduced m
    m, n, s = 20000 + 3, 256, 1024
    x = make_svd(m, n, kappa, seed=23)
    res = _lib().qr(to_dev(x), alg="rclupp", s=s, seed=0, sketch_prec=sk, lu_prec="fp32")
    method_parity(x, "rclupp", s, 0, kappa, res)


_ORACLE_R = {}


@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e14])
@pytest.mark.parametrize("sk,lu", [("fp64", "fp64"), ("fp32", "fp32"), ("bf16", "fp32")])
def test_mixed_workload_shape_vs_oracle(kappa, sk, lu):
    # the mixed-precision workload's n = 256 and s = 4n = 1024 with a quarter of
    # a million rows (m + 5 for a ragged last tile): every form against the
    # FP64 oracle (one oracle run per kappa)
    m, n, s = 262144 + 5, 256, 1024
    x = make_svd(m, n, kappa, seed=24)
    if kappa not in _ORACLE_R:
        _ORACLE_R[kappa] = oracle.run("rclupp", x, s=s, seed=7)
    res = _lib().qr(to_dev(x), alg="rclupp", s=s, seed=7, sketch_prec=sk, lu_prec=lu)
    method_parity(x, "rclupp", s, 7, kappa, res, orc=_ORACLE_R[kappa])
    print("mixed %s/%s kappa=%.0e notes=%d" % (sk, lu, kappa, res.info_host()[3]))


# ------------------------------------------------------------------ CountSketch
# The CountSketch in place of the Gaussian sketch (FP64 sums; FP64 or FP32
# preconditioner): the same bar against the oracle run with the same sketch.
@pytest.mark.parametrize("method", ["rclupp", "rcluppr", "rcholqr"])
@pytest.mark.parametrize("kappa,lu", [(1e4, "fp64"), (1e12, "fp64"), (1e15, "fp64"), (1e8, "fp32"), (1e14, "fp32")])
def test_countsketch_methods(method, kappa, lu):
    if method == "rcholqr" and lu == "fp32" and kappa > 1e8:
        # Algorithm 6 has one CholeskyQR after the preconditioner: an FP32 R_1
        # leaves kappa(Q_1) near 1e-7 kappa(X), beyond one CholeskyQR's reach
        pytest.skip("randomized CholeskyQR with an FP32 preconditioner is limited to kappa(X) near 1e8")
    m, n, s = 30000 + 7, 64, 128
    x = make_svd(m, n, kappa, seed=41)
    orc = oracle.run(method, x, s=s, seed=6, sketch="count")
    res = _lib().qr(to_dev(x), alg=method, s=s, seed=6, sketch="count", lu_prec=lu)
    method_parity(x, method, s, 6, kappa, res, orc=orc)


@pytest.mark.parametrize("kappa", [1e2, 1e14])
def test_countsketch_wide(kappa):
    # the n = 256, s = 4n shape (8-column slices)
    m, n, s = 20000 + 3, 256, 1024
    x = make_svd(m, n, kappa, seed=42)
    res = _lib().qr(to_dev(x), alg="rclupp", s=s, seed=1, sketch="count", lu_prec="fp32")
    method_parity(x, "rclupp", s, 1, kappa, res)


def test_countsketch_rejects_reduced_precision_sums():
    x = make_svd(5000, 16, 1e3, seed=43)
    with pytest.raises(Exception) as e:
        _lib().qr(to_dev(x), alg="rclupp", s=32, sketch="count", sketch_prec="bf16")
    assert getattr(e.value, "status", None) == _nat().ERR_UNSUPPORTED


# ------------------------------------------------------------------ SRHT
# The SRHT in place of the Gaussian sketch, FP64 or BF16 products with an FP64
# or FP32 preconditioner: the same bar against the oracle run with the same
# (FP64) sketch.
@pytest.mark.parametrize("method", ["rclupp", "rcluppr", "rcholqr"])
@pytest.mark.parametrize("kappa,sk,lu", [(1e4, "fp64", "fp64"), (1e12, "fp64", "fp64"), (1e15, "fp64", "fp64"),
                                         (1e8, "bf16", "fp32"), (1e14, "bf16", "fp32")])
def test_srht_methods(method, kappa, sk, lu):
    if method == "rcholqr" and sk == "bf16":
        # Algorithm 6 has one CholeskyQR after the preconditioner: a sketch of X
        # rounded to BF16 (relative error 2^-8) leaves kappa(Q_1) near
        # 4e-3 kappa(X), beyond one CholeskyQR's reach already at kappa(X) = 1e8
        pytest.skip("randomized CholeskyQR with a BF16 sketch is limited to small kappa(X)")
    m, n, s = 30000 + 7, 64, 128
    x = make_svd(m, n, kappa, seed=44)
    orc = oracle.run(method, x, s=s, seed=6, sketch="srht")
    res = _lib().qr(to_dev(x), alg=method, s=s, seed=6, sketch="srht", sketch_prec=sk, lu_prec=lu)
    method_parity(x, method, s, 6, kappa, res, orc=orc)


# ------------------------------------------------------------------ tournament pivoting
@pytest.mark.parametrize("method", ["rcluppr", "lc2"])
@pytest.mark.parametrize("kappa", [1e4, 1e12, 1e15])
def test_tournament_methods(method, kappa):
    m, n, s = 30000 + 9, 64, 128
    x = make_svd(m, n, kappa, seed=44)
    orc = oracle.run(method, x, s=s, seed=5, lu="tournament")
    res = _lib().qr(to_dev(x), alg=method, s=s, seed=5, tall_lu="tournament")
    method_parity(x, method, s, 5, kappa, res, orc=orc)


@pytest.mark.parametrize("n", [16, 100, 128])
def test_tournament_rcluppr_shapes(n):
    m, s = 50000 + 1, 2 * n
    x = make_svd(m, n, 1e10, seed=45)
    res = _lib().qr(to_dev(x), alg="rcluppr", s=s, seed=2, tall_lu="tournament")
    method_parity(x, "rcluppr", s, 2, 1e10, res, orc=oracle.run("rcluppr", x, s=s, seed=2, lu="tournament"))


def test_tournament_rejects_wide():
    x = make_svd(5000, 200, 1e3, seed=46)
    with pytest.raises(Exception) as e:
        _lib().qr(to_dev(x), alg="rcluppr", s=400, tall_lu="tournament")
    assert getattr(e.value, "status", None) == _nat().ERR_UNSUPPORTED


# ------------------------------------------------------------------ full size
@pytest.mark.parametrize("kappa", [1e4, 1e8, 1e12, 1e15])
def test_full_size_rclupp(kappa):
    # 1,048,576 x 64, s = 2n = 128, seed 0: the benchmark workload, compared in full
    m, n, s = 1 << 20, 64, 128
    x = make_svd(m, n, kappa, seed=0)
    X = to_dev(x)
    for method in ("rclupp", "rcluppr"):
        res = _lib().qr(X, alg=method, s=s, seed=0)
        torch.cuda.synchronize()
        method_parity(x, method, s, 0, kappa, res)
        del res


@pytest.mark.parametrize("method,kappa,lu", [("cholqr2", 1e6, "partial"), ("scholqr3", 1e12, "partial"),
                                             ("lc2", 1e15, "partial"), ("rcholqr", 1e15, "partial"),
                                             ("lc2", 1e15, "tournament"), ("rcluppr", 1e15, "tournament")])
def test_full_size_other_methods(method, kappa, lu):
    # the baselines and the tournament-pivoting forms on the 1,048,576 x 64
    # workload (s = 128, seed 0), each inside its range, against the oracle
    m, n, s = 1 << 20, 64, 128
    x = make_svd(m, n, kappa, seed=0)
    sk = s if method in ("rcluppr", "rcholqr") else None
    res = _lib().qr(to_dev(x), alg=method, s=sk, seed=0, tall_lu=lu)
    torch.cuda.synchronize()
    method_parity(x, method, sk, 0, kappa, res, orc=oracle.run(method, x, s=sk, seed=0, lu=lu))


@pytest.mark.parametrize("method", ["cholqr2", "scholqr3"])
def test_full_size_breakdown_like_oracle(method):
    # at kappa = 1e15 both Cholesky-based baselines leave their range; the
    # device reports the breakdown as the oracle does (code and stage)
    m, n = 1 << 20, 64
    x = make_svd(m, n, 1e15, seed=0)
    orc = oracle.run(method, x)
    info = _lib().qr(to_dev(x), alg=method).info_host()
    assert not orc.ok
    assert info[0] == orc.info[0] == oracle.CHOL_BREAKDOWN and info[1] == orc.info[1]

