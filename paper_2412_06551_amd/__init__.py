"""MI355X (gfx950) tall-skinny QR: RCLUPP / RCLUPPr (arXiv 2412.06551) and the
CholeskyQR-type baselines, as hand-written HIP kernels behind a C ABI
(include/rclupp.h). This package is the thin Python binding; importing it does
not touch the GPU, the first call does (and fails loudly without a device or
without the built librclupp.so).
"""
from . import _native  # noqa: F401
from .api import (  # noqa: F401
    QRResult,
    chol,
    colmajor,
    countsketch,
    srht,
    new_colmajor,
    omega,
    philox,
    precond,
    qr,
    qr_batched,
    qr_noalloc,
    Batch,
    qr_simple,
    sketch,
    tall_lu,
    tall_lu_tournament,
    trsm_gram,
    workspace_size,
)

__all__ = ["qr", "qr_simple", "qr_noalloc", "qr_batched", "Batch", "workspace_size", "sketch", "countsketch", "srht", "omega",
           "philox", "precond", "trsm_gram", "chol", "tall_lu", "tall_lu_tournament", "colmajor", "new_colmajor",
           "QRResult"]
