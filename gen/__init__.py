"""Seeded synthetic test matrices for the tall-skinny QR methods.

This package only builds inputs; it contains none of the QR methods'
arithmetic, and it is shared by the CPU oracle, the tests and the benchmark.
"""
from .matrices import (  # noqa: F401
    make_svd,
    make_lowtri,
    make_arrowhead,
    make_krylov,
    make_svd_device,
    make_krylov_device,
    batch_manifest,
    fortran,
)
