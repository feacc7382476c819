"""Helpers shared by the GPU parity tests (tests call the HIP library through
the C ABI binding and compare with the CPU oracle on the same seeded inputs)."""
import numpy as np
import pytest
import torch

import oracle

gpu = pytest.mark.gpu

# Parity bar for whole methods (orthogonality, relative residual, relative R
# error divided by the prescribed condition number).
TOL_ORTH = 1e-12
TOL_RES = 1e-13
TOL_R = 1e-14


def have_gpu() -> bool:
    return torch.cuda.is_available()


def require_gpu():
    if not have_gpu():
        pytest.skip("no HIP device")


def to_dev(a: np.ndarray, ld: int = None) -> torch.Tensor:
    """Column-major float64 device copy (optionally with a larger leading dimension)."""
    a = np.asfortranarray(a, dtype=np.float64)
    m, n = a.shape
    ld = m if ld is None else ld
    base = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    t = base.t()[:m]
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return t


def to_host(t: torch.Tensor) -> np.ndarray:
    return np.asfortranarray(t.detach().cpu().numpy())


def method_parity(x: np.ndarray, method: str, s: int, seed: int, kappa: float, gpu_res, orc=None,
                  tol_r=TOL_R):
    """Assert the HIP result meets the parity bar against the oracle."""
    q = to_host(gpu_res.Q)
    r = to_host(gpu_res.R)
    info = gpu_res.info_host()
    if orc is None:
        orc = oracle.run(method, x, s=s, seed=seed)
    assert orc.ok, ("oracle failed", orc.info)
    assert info[0] == 0, ("gpu info", info, method)
    assert np.all(np.tril(r, -1) == 0), "R not upper triangular"
    assert np.all(np.diag(r) > 0), "diag(R) not positive"
    m = oracle.metrics(x, q, r)
    assert m["orth"] <= TOL_ORTH, (method, m)
    assert m["rel_res"] <= TOL_RES, (method, m)
    rerr = np.linalg.norm(r - orc.R) / np.linalg.norm(orc.R)
    assert rerr <= tol_r * max(kappa, 1.0), (method, rerr, kappa)
    return m, rerr
