"""Full-size runs of the mixed-precision and the Krylov workloads, in the launch
configuration the benchmark times, checked by properties that hold at any
size (the CPU oracle would need minutes per run at these sizes; the
1,048,576 x 64 workload is compared with it in full in test_gpu_methods.py):
  * info zero, R upper triangular with a positive diagonal;
  * orthogonality ||Q^T Q - I||_F <= 1e-12 and relative residual
    ||Q R - X||_F / ||X||_F <= 1e-13 (Section 4's targets, as for every
    method test), computed on the device in FP64;
  * the mixed-precision forms give the FP64 form's R to the parity bar
    1e-14 kappa_2 relative (both are the unique R with a positive diagonal of
    the same X); BF16 at kappa = 1e14 takes the escalated tail (shifted
    Cholesky and one more CholeskyQR pass).
Inputs are generated on the device with the recipes of gen.matrices."""
import pytest
import torch

from gen import make_krylov_device, make_svd_device
from gpu_common import TOL_ORTH, TOL_R, TOL_RES, gpu, require_gpu

pytestmark = gpu


@pytest.fixture(autouse=True)
def _dev():
    require_gpu()
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _lib():
    import paper_2412_06551_amd as lib
    return lib


def _props(X, res):
    """Device-side orthogonality and relative residual (row chunks bound the
    temporaries)."""
    assert res.info_host()[0] == 0, res.info_host()
    Q, R = res.Q, res.R
    n = R.shape[0]
    assert bool(torch.all(torch.diagonal(R) > 0)) and bool(torch.all(torch.tril(R, -1) == 0))
    g = torch.zeros((n, n), dtype=torch.float64, device=X.device)
    num = torch.zeros((), dtype=torch.float64, device=X.device)
    den = torch.zeros((), dtype=torch.float64, device=X.device)
    step = 1 << 20
    for r0 in range(0, X.shape[0], step):
        q = Q[r0:r0 + step]
        g += q.t() @ q
        num += torch.sum((q @ R - X[r0:r0 + step]) ** 2)
        den += torch.sum(X[r0:r0 + step] ** 2)
    orth = float(torch.linalg.matrix_norm(g - torch.eye(n, dtype=torch.float64, device=X.device)))
    res_rel = float(torch.sqrt(num / den))
    assert orth <= TOL_ORTH, orth
    assert res_rel <= TOL_RES, res_rel
    return orth, res_rel


@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e14])
def test_full_size_mixed_workload(kappa):
    # 4,194,304 x 256, s = 4n = 1024: FP64, FP32 sketch + FP32 LU, BF16 sketch + FP32 LU,
    # BF16 SRHT + FP32 LU
    m, n, s = 4194304, 256, 1024
    X = make_svd_device(m, n, kappa, seed=0, orthonormal=False)
    ref = _lib().qr(X, alg="rclupp", s=s, seed=0)
    _props(X, ref)
    for sk, lu, kind in (("fp32", "fp32", "gaussian"), ("bf16", "fp32", "gaussian"), ("bf16", "fp32", "srht")):
        res = _lib().qr(X, alg="rclupp", s=s, seed=0, sketch_prec=sk, lu_prec=lu, sketch=kind)
        _props(X, res)
        d = float(torch.linalg.matrix_norm(res.R - ref.R) / torch.linalg.matrix_norm(ref.R))
        assert d <= TOL_R * kappa, (sk, lu, kind, d)
        if sk == "bf16" and kind == "gaussian" and kappa >= 1e14:
            assert res.info_host()[3] == 1  # escalated: kappa(Q_1) near 1e11
        del res
    del ref, X


def test_full_size_krylov_rcluppr():
    # 16,777,216 x 128 Krylov-monomial columns (kappa_2 beyond 1e15), RCLUPPr FP64
    # and with the BF16 sketch of M and the FP32 LU of the sketch
    m, n, s = 16777216, 128, 256
    X = make_krylov_device(m, n, seed=0)
    for sk, lu in (("fp64", "fp64"), ("bf16", "fp32")):
        res = _lib().qr(X, alg="rcluppr", s=s, seed=0, sketch_prec=sk, lu_prec=lu)
        _props(X, res)
        del res
    del X


def test_full_size_krylov_rcluppr_tournament():
    # the same workload with tournament pivoting for the LU of X
    m, n, s = 16777216, 128, 256
    X = make_krylov_device(m, n, seed=0)
    res = _lib().qr(X, alg="rcluppr", s=s, seed=0, tall_lu="tournament")
    _props(X, res)
    del res, X


def test_full_size_batch():
    # the 512-problem batch as the benchmark runs it (grouped by (n, s), graph
    # replay, autotuned rows per workgroup), every problem checked, on the
    # second replay too
    from gen import batch_manifest
    man = batch_manifest(0, 512)
    Xs = [make_svd_device(p["m"], p["n"], p["kappa"], p["input_seed"], orthonormal=False) for p in man]
    batch = _lib().Batch(Xs, alg="rclupp", seeds=[p["seed"] for p in man], graph=True, autotune=True)
    for _ in range(2):
        _, _, info = batch.run()
        torch.cuda.synchronize()
        assert int(torch.count_nonzero(info[:, 0])) == 0
        for X, Q, R in zip(Xs, batch.Qs, batch.Rs):
            n = R.shape[0]
            assert bool(torch.all(torch.diagonal(R) > 0)) and bool(torch.all(torch.tril(R, -1) == 0))
            orth = float(torch.linalg.matrix_norm(Q.t() @ Q - torch.eye(n, dtype=torch.float64, device=X.device)))
            res = float(torch.linalg.matrix_norm(Q @ R - X) / torch.linalg.matrix_norm(X))
            assert orth <= TOL_ORTH and res <= TOL_RES, (X.shape, orth, res)
    del batch, Xs
