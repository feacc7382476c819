"""CPU FP64 oracle for RCLUPP / RCLUPPr and the CholeskyQR-type baselines.

TEST INFRASTRUCTURE ONLY: the plain, step-by-step reference implementation
written from the paper (arXiv 2412.06551) that the GPU library is checked
against. Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it. It shares no code with the GPU library; the only module both
sides use is the seeded input generator package ``gen``.

The arithmetic lives in ``oracle.c`` (algorithms and their steps) and
``checker.c`` (accuracy metrics), compiled with gcc into ``liboracle.so``.
This module only marshals numpy arrays (float64, column-major).

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
(``tests/test_oracle_*.py``) against library routines, closed forms,
invariants, exact rational arithmetic or the paper's bounds.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ("oracle.c", "checker.c")
# the oracle's reading (fused multiply-add in the LU elimination and the
# substitution) and the other one (product and sum rounded separately), which
# only serves to document outcomes outside the paper's conditions
VARIANTS = {"": [], "separate_muladd": ["-DORC_SEPARATE_MULADD"]}


def _lib_path(variant: str = "") -> str:
    return os.path.join(_HERE, "liboracle%s.so" % ("_" + variant if variant else ""))


_LIB_PATH = _lib_path()

# info codes / stages (the oracle's own definition of the documented convention)
OK, LU_ZERO_PIVOT, CHOL_BREAKDOWN, NONFINITE, SINGULAR = 0, 1, 2, 3, 4
ST_LU, ST_QR, ST_PRECOND, ST_CHOL_A, ST_CHOL_B = 1, 2, 3, 4, 5

U = 2.0 ** -53  # unit roundoff of float64 (Section 1)


def build(force: bool = True) -> str:
    """Compile liboracle.so (and its separate-multiply-add variant) with gcc
    (plain C11, OpenMP, no FP contraction)."""
    for variant, defs in VARIANTS.items():
        path = _lib_path(variant)
        if not force and os.path.exists(path):
            continue
        srcs = [os.path.join(_HERE, s) for s in _SOURCES]
        tmp = path + ".tmp%d" % os.getpid()
        # no implicit contraction; the explicit fma() calls use the FMA instruction
        cmd = ["gcc", "-std=c11", "-O2", "-mfma", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off"] + defs + \
            ["-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return _LIB_PATH


_libs = {}


def _load(variant: str = ""):
    if variant in _libs:
        return _libs[variant]
    if variant not in VARIANTS:
        raise ValueError("unknown oracle variant %r" % variant)
    path = _lib_path(variant)
    stale = not os.path.exists(path) or any(
        os.path.getmtime(os.path.join(_HERE, s)) > os.path.getmtime(path) for s in _SOURCES)
    if stale:
        build(force=True)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    U64 = ctypes.c_uint64
    I32 = ctypes.c_int32
    D = ctypes.c_double
    sig = {
        "orc_max_threads": ([], ctypes.c_int),
        "orc_set_threads": ([ctypes.c_int], None),
        "orc_philox4x32_10": ([P, P, P], None),
        "orc_normals4": ([U64, U64, ctypes.c_uint32, P], None),
        "orc_omega": ([U64, I64, I64, I64, P], None),
        "orc_sketch": ([P, I64, I64, I64, I64, U64, P], None),
        "orc_gram": ([P, I64, I64, I64, P], None),
        "orc_gepp": ([P, I64, I64, I64, P, P, I32], ctypes.c_int),
        "orc_house_r": ([P, I64, I64, I64, P], None),
        "orc_chol": ([P, I64, D, P, P, I32], ctypes.c_int),
        "orc_trsm": ([P, I64, I64, I64, P, P, I64], None),
        "orc_trmm": ([P, P, I64, P], None),
        "orc_rclupp": ([P, I64, I64, I64, I64, U64, P, I64, P, P, P, P, P], ctypes.c_int),
        "orc_rcluppr": ([P, I64, I64, I64, I64, U64, P, I64, P, P, P, P, P], ctypes.c_int),
        "orc_cholqr2": ([P, I64, I64, I64, P, I64, P, P, P, P], ctypes.c_int),
        "orc_scholqr3": ([P, I64, I64, I64, P, I64, P, P, P, P, P], ctypes.c_int),
        "orc_scholqr3_shift": ([I64, I64, D], D),
        "orc_lc2": ([P, I64, I64, I64, P, I64, P, P, P, P], ctypes.c_int),
        "orc_rcholqr": ([P, I64, I64, I64, I64, U64, P, I64, P, P, P, P], ctypes.c_int),
        "orc_rclupp_f": ([P, I64, I64, I64, I64, U64, P, I64, P, P, P, P, P, ctypes.c_int], ctypes.c_int),
        "orc_rcluppr_f": ([P, I64, I64, I64, I64, U64, P, I64, P, P, P, P, P, ctypes.c_int], ctypes.c_int),
        "orc_rcholqr_f": ([P, I64, I64, I64, I64, U64, P, I64, P, P, P, P, ctypes.c_int], ctypes.c_int),
        "orc_countsketch_hash": ([U64, U64, I64, P, P], None),
        "orc_countsketch": ([P, I64, I64, I64, I64, U64, P], None),
        "orc_srht_sign": ([U64, U64], ctypes.c_double),
        "orc_srht_row": ([U64, I64, I64], I64),
        "orc_srht": ([P, I64, I64, I64, I64, U64, P], None),
        "orc_tslu": ([P, I64, I64, I64, P, P, P, P, I64, P], ctypes.c_int),
        "orc_lc2_f": ([P, I64, I64, I64, P, I64, P, P, P, P, ctypes.c_int], ctypes.c_int),
        "chk_orthogonality": ([P, I64, I64, I64], D),
        "chk_residual": ([P, I64, P, I64, P, I64, I64, P, P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _libs[variant] = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _f64(a) -> np.ndarray:
    return np.asfortranarray(a, dtype=np.float64)


def _ld(a: np.ndarray) -> int:
    """Leading dimension of a column-major 2-D array (or 1 for vectors)."""
    if a.ndim == 1:
        return max(1, a.shape[0])
    if not a.flags.f_contiguous and a.shape[1] > 1:
        raise ValueError("expected a column-major array")
    return max(1, a.shape[0])


def max_threads() -> int:
    return int(_load().orc_max_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


# --------------------------------------------------------------------------
# Sketch generator
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    """Raw Philox4x32-10 output words for counter ctr[4] and key key[2]."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals4(seed: int, q: int, i: int) -> np.ndarray:
    """The four float32 normals of sketch row i for tall rows 4q..4q+3."""
    z = np.zeros(4, dtype=np.float32)
    _load().orc_normals4(ctypes.c_uint64(seed), ctypes.c_uint64(q), ctypes.c_uint32(i), _ptr(z))
    return z


def omega(s: int, cols: int, seed: int, j0: int = 0) -> np.ndarray:
    """Omega[:, j0:j0+cols] (s x cols), Omega = G / sqrt(s)."""
    om = np.zeros((s, cols), order="F")
    _load().orc_omega(ctypes.c_uint64(seed), s, j0, cols, _ptr(om))
    return om


def tslu(x):
    """Tournament pivoting of a tall x (n <= 128): (sel, N, L11, M, info) with
    x[sel] = L11 N and M = x N^{-1} in x's row order, rows sel equal to L11."""
    x = _f64(x)
    m, n = x.shape
    sel = np.zeros(n, dtype=np.int64)
    N = np.zeros((n, n), order="F")
    L11 = np.zeros((n, n), order="F")
    M = np.zeros((m, n), order="F")
    info = np.zeros(4, dtype=np.int32)
    _load().orc_tslu(_ptr(x), m, n, _ld(x), _ptr(sel), _ptr(N), _ptr(L11), _ptr(M), m, _ptr(info))
    return sel, N, L11, M, info


def countsketch_hash(seed: int, j: int, s: int):
    """(h_j, sigma_j): the row and sign of column j of the CountSketch."""
    h = np.zeros(1, dtype=np.int64)
    sg = np.zeros(1)
    _load().orc_countsketch_hash(ctypes.c_uint64(seed), ctypes.c_uint64(j), s, _ptr(h), _ptr(sg))
    return int(h[0]), float(sg[0])


def countsketch(x, s: int, seed: int) -> np.ndarray:
    """Y = S X for the CountSketch S (s x m, one +-1 per column)."""
    x = _f64(x)
    m, n = x.shape
    y = np.zeros((s, n), order="F")
    _load().orc_countsketch(_ptr(x), m, n, _ld(x), s, ctypes.c_uint64(seed), _ptr(y))
    return y


def srht_sign(seed: int, j: int) -> float:
    """d_j, the random sign of tall row j in the SRHT's D."""
    return float(_load().orc_srht_sign(ctypes.c_uint64(seed), ctypes.c_uint64(j)))


def srht_row(seed: int, m: int, i: int) -> int:
    """r_i, the row of the order-2^ceil(log2 m) Walsh-Hadamard matrix that row i
    of the SRHT samples."""
    return int(_load().orc_srht_row(ctypes.c_uint64(seed), m, i))


def srht(x, s: int, seed: int) -> np.ndarray:
    """Y = S X for the SRHT S = sqrt(m'/s) R H D (s x m)."""
    x = _f64(x)
    m, n = x.shape
    y = np.zeros((s, n), order="F")
    _load().orc_srht(_ptr(x), m, n, _ld(x), s, ctypes.c_uint64(seed), _ptr(y))
    return y


def sketch(x, s: int, seed: int) -> np.ndarray:
    """Y = Omega X (s x n)."""
    x = _f64(x)
    m, n = x.shape
    y = np.zeros((s, n), order="F")
    _load().orc_sketch(_ptr(x), m, n, _ld(x), s, ctypes.c_uint64(seed), _ptr(y))
    return y


# --------------------------------------------------------------------------
# Small dense steps
# --------------------------------------------------------------------------
def gepp(a, stage: int = ST_LU):
    """LU with partial pivoting of a (r x n, r >= n).

    Returns (M, N, perm, info): M r x n unit lower-trapezoidal, N n x n upper,
    perm[p] = original row now at position p, so a[perm] = M @ N.
    """
    a = np.array(_f64(a), order="F", copy=True)
    r, n = a.shape
    perm = np.zeros(r, dtype=np.int64)
    info = np.zeros(4, dtype=np.int32)
    _load().orc_gepp(_ptr(a), r, n, _ld(a), _ptr(perm), _ptr(info), stage)
    M = np.tril(a, -1)[:, :n].copy(order="F")
    M[np.arange(n), np.arange(n)] = 1.0
    N = np.triu(a[:n, :n]).copy(order="F")
    return M, N, perm, info


def house_r(a) -> np.ndarray:
    """R factor (n x n) of the thin Householder QR of a (r x n, r >= n)."""
    a = np.array(_f64(a), order="F", copy=True)
    r, n = a.shape
    R = np.zeros((n, n), order="F")
    _load().orc_house_r(_ptr(a), r, n, _ld(a), _ptr(R))
    return R


def chol(g, shift: float = 0.0, stage: int = ST_CHOL_A):
    """Upper Cholesky factor R of g + shift*I (reads the upper triangle)."""
    g = _f64(g)
    n = g.shape[0]
    R = np.zeros((n, n), order="F")
    info = np.zeros(4, dtype=np.int32)
    _load().orc_chol(_ptr(g), n, float(shift), _ptr(R), _ptr(info), stage)
    return R, info


def trsm(x, R) -> np.ndarray:
    """W = X R^{-1} by row-wise substitution."""
    x = _f64(x)
    R = _f64(R)
    m, n = x.shape
    w = np.zeros((m, n), order="F")
    _load().orc_trsm(_ptr(x), m, n, _ld(x), _ptr(R), _ptr(w), _ld(w))
    return w


def gram(w) -> np.ndarray:
    """G = W^T W (blocked sums)."""
    w = _f64(w)
    m, n = w.shape
    G = np.zeros((n, n), order="F")
    _load().orc_gram(_ptr(w), m, n, _ld(w), _ptr(G))
    return G


def trmm(a, b) -> np.ndarray:
    """C = A B for upper-triangular n x n A, B."""
    a = _f64(a)
    b = _f64(b)
    n = a.shape[0]
    c = np.zeros((n, n), order="F")
    _load().orc_trmm(_ptr(a), _ptr(b), n, _ptr(c))
    return c


def scholqr3_shift(m: int, n: int, g_max_diag: float) -> float:
    return float(_load().orc_scholqr3_shift(m, n, float(g_max_diag)))


# --------------------------------------------------------------------------
# Whole methods
# --------------------------------------------------------------------------
@dataclass
class Result:
    Q: np.ndarray
    R: np.ndarray
    info: np.ndarray
    R1: np.ndarray
    R2: np.ndarray
    R4: np.ndarray

    @property
    def ok(self) -> bool:
        return int(self.info[0]) == OK


# method flags: the sketch (Gaussian by default) and the pivoting of the LU of X
SKETCH_FLAGS = {"gaussian": 0, "count": 1, "srht": 4}
LU_FLAGS = {"partial": 0, "tournament": 2}


def _run(name: str, x, s=None, seed=None, variant: str = "", sketch: str = "gaussian", lu: str = "partial") -> Result:
    x = _f64(x)
    m, n = x.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    R1 = np.zeros((n, n), order="F")
    R2 = np.zeros((n, n), order="F")
    R4 = np.zeros((n, n), order="F")
    info = np.zeros(4, dtype=np.int32)
    lib = _load(variant)
    f = getattr(lib, "orc_" + name)
    flags = SKETCH_FLAGS[sketch] | LU_FLAGS[lu]
    if name in ("rclupp", "rcluppr"):
        if not (n <= s <= m):
            raise ValueError("need n <= s <= m")
        f = getattr(lib, "orc_" + name + "_f")
        f(_ptr(x), m, n, _ld(x), s, ctypes.c_uint64(seed), _ptr(Q), m, _ptr(R), _ptr(info), _ptr(R1), _ptr(R2),
          _ptr(R4), flags)
    elif name == "rcholqr":
        if not (n <= s <= m):
            raise ValueError("need n <= s <= m")
        f = getattr(lib, "orc_rcholqr_f")
        f(_ptr(x), m, n, _ld(x), s, ctypes.c_uint64(seed), _ptr(Q), m, _ptr(R), _ptr(info), _ptr(R1), _ptr(R2), flags)
    elif name == "scholqr3":
        f(_ptr(x), m, n, _ld(x), _ptr(Q), m, _ptr(R), _ptr(info), _ptr(R1), _ptr(R2), _ptr(R4))
    elif name == "lc2":
        lib.orc_lc2_f(_ptr(x), m, n, _ld(x), _ptr(Q), m, _ptr(R), _ptr(info), _ptr(R1), _ptr(R2), flags)
    else:  # cholqr2
        f(_ptr(x), m, n, _ld(x), _ptr(Q), m, _ptr(R), _ptr(info), _ptr(R1), _ptr(R2))
    return Result(Q, R, info, R1, R2, R4)


def rclupp(x, s: int, seed: int = 0) -> Result:
    """Algorithm 2 (RCLUPP)."""
    return _run("rclupp", x, s, seed)


def rcluppr(x, s: int, seed: int = 0) -> Result:
    """Algorithm 7 (RCLUPPr)."""
    return _run("rcluppr", x, s, seed)


def cholqr2(x) -> Result:
    """Algorithm 3 (CholeskyQR2)."""
    return _run("cholqr2", x)


def scholqr3(x) -> Result:
    """Algorithm 4 (Shifted CholeskyQR3)."""
    return _run("scholqr3", x)


def lc2(x) -> Result:
    """Algorithm 5 (LU-CholeskyQR2)."""
    return _run("lc2", x)


def rcholqr(x, s: int, seed: int = 0) -> Result:
    """Algorithm 6 (randomized CholeskyQR, single sketch)."""
    return _run("rcholqr", x, s, seed)


METHODS = {"rclupp": rclupp, "rcluppr": rcluppr, "cholqr2": cholqr2, "scholqr3": scholqr3, "lc2": lc2,
           "rcholqr": rcholqr}


def run(method: str, x, s=None, seed: int = 0, variant: str = "", sketch: str = "gaussian",
        lu: str = "partial") -> Result:
    """Run one method; variant "separate_muladd" takes the other rounding
    reading of the LU elimination and the substitution (see VARIANTS); sketch
    "count" takes the CountSketch for the sketched methods; lu "tournament"
    takes tournament pivoting for the LU of X (RCLUPPr, LC2)."""
    if lu != "partial" and method not in ("rcluppr", "lc2"):
        raise ValueError("only RCLUPPr and LC2 factor X")
    if sketch != "gaussian" or lu != "partial":
        if sketch != "gaussian" and method not in ("rclupp", "rcluppr", "rcholqr"):
            raise ValueError("only the sketched methods take a sketch")
        return _run(method, x, s, seed, variant, sketch, lu)
    if variant:
        if method in ("rclupp", "rcluppr", "rcholqr"):
            return _run(method, x, s, seed, variant)
        return _run(method, x, variant=variant)
    f = METHODS[method]
    if method in ("rclupp", "rcluppr", "rcholqr"):
        return f(x, s, seed)
    return f(x)


# --------------------------------------------------------------------------
# Metrics (Section 5: orthogonality and residual)
# --------------------------------------------------------------------------
def orthogonality(q) -> float:
    q = _f64(q)
    m, n = q.shape
    return float(_load().chk_orthogonality(_ptr(q), m, n, _ld(q)))


def residual(x, q, R):
    """(||QR - X||_F, ||X||_F), R taken as upper triangular."""
    x = _f64(x)
    q = _f64(q)
    R = _f64(R)
    m, n = x.shape
    res = ctypes.c_double()
    xn = ctypes.c_double()
    _load().chk_residual(_ptr(x), _ld(x), _ptr(q), _ld(q), _ptr(R), m, n, ctypes.byref(res), ctypes.byref(xn))
    return float(res.value), float(xn.value)


def metrics(x, q, R) -> dict:
    orth = orthogonality(q)
    res, xn = residual(x, q, R)
    return dict(orth=orth, res=res, rel_res=res / xn if xn > 0 else float("nan"), xnorm=xn)
