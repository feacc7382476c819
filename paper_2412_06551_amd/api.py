"""PyTorch-facing wrappers of the C ABI: device memory and streams come from
torch, every computation runs in librclupp.so on the current HIP device.

Matrices are float64 and column-major: an m x n matrix is a tensor of shape
(m, n) with stride (1, ld), ld >= m, e.g. ``torch.empty((n, m)).t()``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _native as nat


def _require_device() -> None:
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the tall-skinny QR library runs on the GPU only")
    nat.load()


def colmajor(a: torch.Tensor) -> torch.Tensor:
    """Column-major float64 device copy of a 2-D tensor (shape kept)."""
    if a.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    m, n = a.shape
    out = torch.empty((n, m), dtype=torch.float64, device=a.device if a.is_cuda else "cuda").t()
    out.copy_(a)
    return out


def new_colmajor(m: int, n: int, device="cuda", ld: Optional[int] = None) -> torch.Tensor:
    ld = m if ld is None else ld
    base = torch.empty((n, ld), dtype=torch.float64, device=device)
    return base.t()[:m]


def _ld(a: torch.Tensor) -> int:
    if a.dtype != torch.float64 or not a.is_cuda or a.dim() != 2:
        raise ValueError("expected a float64 CUDA (HIP) matrix")
    m, n = a.shape
    if a.stride(0) != 1 and n > 1 and m > 1:
        raise ValueError("expected a column-major matrix (stride(0) == 1)")
    return max(a.stride(1), m) if n > 1 else max(m, 1)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _opts(sketch_prec="fp64", lu_prec="fp64", sketch="gaussian", tall_lu="partial") -> nat.Opts:
    o = nat.Opts()
    o.sketch_prec = nat.PREC[sketch_prec]
    o.lu_prec = nat.PREC[lu_prec]
    o.sketch_kind = nat.SKETCH[sketch]
    o.tall_lu = nat.TALL_LU[tall_lu]
    return o


@dataclass
class QRResult:
    Q: torch.Tensor
    R: torch.Tensor
    info: torch.Tensor  # int32[4] on the device: code, stage, index, reserved

    def info_host(self):
        return [int(v) for v in self.info.cpu().tolist()]

    @property
    def ok(self) -> bool:
        return self.info_host()[0] == nat.INFO_OK


def workspace_size(alg: str, m: int, n: int, s: Optional[int] = None, sketch_prec="fp64", lu_prec="fp64",
                   sketch="gaussian", tall_lu="partial") -> int:
    nat.load()
    s = _default_s(alg, n, m, s)
    o = _opts(sketch_prec, lu_prec, sketch, tall_lu)
    b = ctypes.c_size_t()
    nat.check(nat.load().rclupp_workspace_size(nat.ALG[alg], m, n, s, ctypes.byref(o), ctypes.byref(b)),
              "rclupp_workspace_size")
    return int(b.value)


def _default_s(alg, n, m, s):
    """s = 2n by default (Section 5), capped at m; an explicit s is passed through
    unchanged so the library validates it (n <= s <= m)."""
    if s is None:
        s = min(2 * n, m) if alg in nat.SKETCHED else 0
    return int(s)


def qr(X: torch.Tensor, alg: str = "rclupp", s: Optional[int] = None, seed: int = 0, sketch_prec: str = "fp64",
       lu_prec: str = "fp64", Q: Optional[torch.Tensor] = None, R: Optional[torch.Tensor] = None,
       workspace: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None, stream=None,
       sketch: str = "gaussian", tall_lu: str = "partial") -> QRResult:
    """X = Q R by one of the six methods (rclupp_qr_ex). Q shares X's leading
    dimension; sketch is "gaussian" or "count" (CountSketch); tall_lu (RCLUPPr,
    LC2) is "partial" or "tournament" pivoting."""
    _require_device()
    m, n = X.shape
    ld = _ld(X)
    s = _default_s(alg, n, m, s)
    if Q is None:
        Q = new_colmajor(m, n, device=X.device, ld=ld)
    if _ld(Q) != ld:
        raise ValueError("Q must have the leading dimension of X")
    if R is None:
        R = torch.empty((n, n), dtype=torch.float64, device=X.device).t()
    if info is None:
        info = torch.zeros(4, dtype=torch.int32, device=X.device)
    nbytes = workspace_size(alg, m, n, s, sketch_prec, lu_prec, sketch, tall_lu)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=X.device)
    o = _opts(sketch_prec, lu_prec, sketch, tall_lu)
    st = nat.load().rclupp_qr_ex(nat.ALG[alg], _ptr(X), m, n, ld, s, ctypes.c_uint64(seed), _ptr(Q), _ptr(R),
                                 ctypes.byref(o), _ptr(workspace), workspace.numel(), _ptr(info), _stream(stream))
    nat.check(st, "rclupp_qr_ex(%s)" % alg)
    return QRResult(Q, R, info)


def qr_noalloc(X: torch.Tensor, Q: torch.Tensor, R: torch.Tensor, alg: str = "rclupp", s: Optional[int] = None,
               seed: int = 0, sketch_prec: str = "fp64", lu_prec: str = "fp64", info: Optional[torch.Tensor] = None,
               stream=None) -> QRResult:
    """X = Q R through rclupp_qr_noalloc: the library takes its workspace from its
    fixed device scratch and allocates nothing; the caller provides Q (X's
    leading dimension), R (n x n) and optionally info (int32[4] on the device)."""
    _require_device()
    m, n = X.shape
    ld = _ld(X)
    s = _default_s(alg, n, m, s)
    if _ld(Q) != ld or tuple(Q.shape) != (m, n):
        raise ValueError("Q must be m x n with the leading dimension of X")
    if tuple(R.shape) != (n, n) or _ld(R) != n:
        raise ValueError("R must be a column-major n x n matrix")
    o = _opts(sketch_prec, lu_prec)
    st = nat.load().rclupp_qr_noalloc(nat.ALG[alg], _ptr(X), m, n, ld, s, ctypes.c_uint64(seed), _ptr(Q), _ptr(R),
                                      ctypes.byref(o), _ptr(info), _stream(stream))
    nat.check(st, "rclupp_qr_noalloc(%s)" % alg)
    return QRResult(Q, R, info)


_SIMPLE = {"rclupp": "rclupp_qr", "rcluppr": "rcluppr_qr", "cholqr2": "cholqr2_qr", "scholqr3": "scholqr3_qr",
           "lc2": "lc2_qr", "rcholqr": "rcholqr_qr"}


def qr_simple(X: torch.Tensor, alg: str = "rclupp", s: Optional[int] = None, seed: int = 0, stream=None):
    """The 9-argument entry point; returns (Q, R, info list) after synchronizing the stream."""
    _require_device()
    m, n = X.shape
    ld = _ld(X)
    s = _default_s(alg, n, m, s)
    Q = new_colmajor(m, n, device=X.device, ld=ld)
    R = torch.empty((n, n), dtype=torch.float64, device=X.device).t()
    lib = nat.load()
    st = getattr(lib, _SIMPLE[alg])(_ptr(X), m, n, ld, s, ctypes.c_uint64(seed), _ptr(Q), _ptr(R), _stream(stream))
    nat.check(st, _SIMPLE[alg])
    inf = nat.Info()
    nat.check(lib.rclupp_last_info(_stream(stream), ctypes.byref(inf)), "rclupp_last_info")
    return Q, R, [inf.code, inf.stage, inf.index, inf.reserved]


class Batch:
    """A reusable batched QR (rclupp_qr_batched) over fixed input matrices: Q, R,
    the workspace and the outcome records are allocated once, so repeated run()
    calls hit the library's captured graph when graph=True."""

    def __init__(self, Xs: Sequence[torch.Tensor], alg: str = "rclupp", s: Optional[Sequence[int]] = None,
                 seeds: Optional[Sequence[int]] = None, sketch_prec="fp64", lu_prec="fp64", graph: bool = False,
                 autotune: bool = False):
        _require_device()
        b = len(Xs)
        self.alg = alg
        self.count = b
        self.Xs = list(Xs)
        self.probs = (nat.Problem * max(b, 1))()
        self.Qs, self.Rs = [], []
        for i, X in enumerate(Xs):
            m, n = X.shape
            ld = _ld(X)
            si = _default_s(alg, n, m, None if s is None else s[i])
            Q = new_colmajor(m, n, device=X.device, ld=ld)
            R = torch.empty((n, n), dtype=torch.float64, device=X.device).t()
            self.Qs.append(Q)
            self.Rs.append(R)
            p = self.probs[i]
            p.X, p.Q, p.R = X.data_ptr(), Q.data_ptr(), R.data_ptr()
            p.m, p.n, p.ld, p.s = m, n, ld, si
            p.seed = i if seeds is None else seeds[i]
        self.opts = _opts(sketch_prec, lu_prec)
        self.opts.batch_flags = (nat.BATCH_GRAPH if graph else 0) | (nat.BATCH_AUTOTUNE if autotune else 0)
        lib = nat.load()
        nb = ctypes.c_size_t()
        nat.check(lib.rclupp_batched_workspace_size(nat.ALG[alg], self.probs, b, ctypes.byref(self.opts),
                                                    ctypes.byref(nb)), "rclupp_batched_workspace_size")
        self.ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device="cuda")
        self.info = torch.zeros((max(b, 1), 4), dtype=torch.int32, device="cuda")

    def run(self, stream=None):
        lib = nat.load()
        nat.check(lib.rclupp_qr_batched(nat.ALG[self.alg], self.probs, self.count, ctypes.byref(self.opts),
                                        _ptr(self.ws), self.ws.numel(), _ptr(self.info), _stream(stream)),
                  "rclupp_qr_batched")
        return self.Qs, self.Rs, self.info[:self.count]


def qr_batched(Xs: Sequence[torch.Tensor], alg: str = "rclupp", s: Optional[Sequence[int]] = None,
               seeds: Optional[Sequence[int]] = None, sketch_prec="fp64", lu_prec="fp64", graph: bool = False,
               autotune: bool = False, stream=None):
    """Many independent QRs in one call (rclupp_qr_batched). Returns (Qs, Rs, info[batch, 4])."""
    return Batch(Xs, alg, s, seeds, sketch_prec, lu_prec, graph, autotune).run(stream)


# ---------------------------------------------------------------------- steps
def omega(s: int, cols: int, seed: int, j0: int = 0) -> torch.Tensor:
    """Raw normals G (float32, s x cols, column-major) of the sketch S = G / sqrt(s)."""
    _require_device()
    g = torch.empty((cols, s), dtype=torch.float32, device="cuda").t()
    nat.check(nat.load().rclupp_omega(ctypes.c_uint64(seed), s, j0, cols, _ptr(g), _stream()), "rclupp_omega")
    return g


def philox(ctr: torch.Tensor, k0: int, k1: int) -> torch.Tensor:
    """Raw Philox4x32-10 words for counters ctr (int32 tensor [count, 4] on the device)."""
    _require_device()
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    nat.check(nat.load().rclupp_philox(_ptr(ctr), ctr.shape[0], ctypes.c_uint32(k0), ctypes.c_uint32(k1),
                                       _ptr(out), _stream()), "rclupp_philox")
    return out


def sketch(X: torch.Tensor, s: int, seed: int = 0, prec: str = "fp64") -> torch.Tensor:
    _require_device()
    m, n = X.shape
    Y = new_colmajor(s, n)
    nat.check(nat.load().rclupp_sketch(_ptr(X), m, n, _ld(X), s, ctypes.c_uint64(seed), nat.PREC[prec], _ptr(Y),
                                       _stream()), "rclupp_sketch")
    return Y


def countsketch(X: torch.Tensor, s: int, seed: int = 0) -> torch.Tensor:
    """Y = S X for the CountSketch S (s x n, column-major)."""
    _require_device()
    m, n = X.shape
    Y = new_colmajor(s, n)
    nat.check(nat.load().rclupp_countsketch(_ptr(X), m, n, _ld(X), s, ctypes.c_uint64(seed), _ptr(Y), _stream()),
              "rclupp_countsketch")
    return Y


def srht(X: torch.Tensor, s: int, seed: int = 0, prec: str = "fp64") -> torch.Tensor:
    """Y = S X for the SRHT S = sqrt(m'/s) R H D (s x n, column-major)."""
    _require_device()
    m, n = X.shape
    Y = new_colmajor(s, n)
    nat.check(nat.load().rclupp_srht(_ptr(X), m, n, _ld(X), s, ctypes.c_uint64(seed), nat.PREC[prec], _ptr(Y),
                                     _stream()), "rclupp_srht")
    return Y


def precond(Y: torch.Tensor, lu: bool = True, prec: str = "fp64", want_m: bool = False):
    """R_1 = D R_0 N from the s x n sketch; returns (R1, perm, M, info)."""
    _require_device()
    s, n = Y.shape
    if _ld(Y) != s:
        Y = colmajor(Y)
    R1 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    perm = torch.empty(s, dtype=torch.int32, device="cuda")
    M = new_colmajor(s, n) if want_m else None
    info = torch.zeros(4, dtype=torch.int32, device="cuda")
    nat.check(nat.load().rclupp_precond(_ptr(Y), s, n, 1 if lu else 0, nat.PREC[prec], _ptr(R1),
                                        _ptr(perm) if lu else None, _ptr(M), _ptr(info), _stream()),
              "rclupp_precond")
    return R1, perm, M, info


def trsm_gram(X: torch.Tensor, R: Optional[torch.Tensor] = None, gram: bool = True, out: Optional[torch.Tensor] = None):
    """(W, G): W = X R^{-1} (if R given), G = W^T W (if gram)."""
    _require_device()
    m, n = X.shape
    W = None
    if R is not None:
        W = out if out is not None else new_colmajor(m, n)
        if _ld(R) != n:
            R = colmajor(R)
    G = torch.empty((n, n), dtype=torch.float64, device="cuda").t() if gram else None
    nat.check(nat.load().rclupp_trsm_gram(_ptr(X), m, n, _ld(X), _ptr(R), _ptr(W), _ld(W) if W is not None else m,
                                          _ptr(G), _stream()), "rclupp_trsm_gram")
    return W, G


def chol(G: torch.Tensor, m: int = 0, shift: bool = False, Rprev: Optional[torch.Tensor] = None,
         stage: int = nat.STAGE_CHOL_A):
    """(R, Rout, info): R^T R = G (+ shift), Rout = R Rprev if Rprev is given."""
    _require_device()
    n = G.shape[0]
    if _ld(G) != n:
        G = colmajor(G)
    R = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    Rout = torch.empty((n, n), dtype=torch.float64, device="cuda").t() if Rprev is not None else None
    if Rprev is not None and _ld(Rprev) != n:
        Rprev = colmajor(Rprev)
    info = torch.zeros(4, dtype=torch.int32, device="cuda")
    nat.check(nat.load().rclupp_chol(_ptr(G), n, m, 1 if shift else 0, _ptr(R), _ptr(Rprev), _ptr(Rout), stage,
                                     _ptr(info), _stream()), "rclupp_chol")
    return R, Rout, info


def tall_lu(X: torch.Tensor):
    """(LU packed m x n with rows in pivoted order, perm int32[m], info)."""
    _require_device()
    m, n = X.shape
    M = new_colmajor(m, n)
    perm = torch.empty(m, dtype=torch.int32, device="cuda")
    info = torch.zeros(4, dtype=torch.int32, device="cuda")
    nat.check(nat.load().rclupp_tall_lu(_ptr(X), m, n, _ld(X), _ptr(M), m, _ptr(perm), _ptr(info), _stream()),
              "rclupp_tall_lu")
    return M, perm, info


def tall_lu_tournament(X: torch.Tensor):
    """(M in X's row order, sel int32[n], N (n x n), info) of tournament pivoting."""
    _require_device()
    m, n = X.shape
    M = new_colmajor(m, n)
    sel = torch.empty(n, dtype=torch.int32, device="cuda")
    N = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    info = torch.zeros(4, dtype=torch.int32, device="cuda")
    nat.check(nat.load().rclupp_tall_lu_tournament(_ptr(X), m, n, _ld(X), _ptr(M), m, _ptr(sel), _ptr(N), _ptr(info),
                                                   _stream()), "rclupp_tall_lu_tournament")
    return M, sel, N, info
