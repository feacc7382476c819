"""The C ABI library loads on a host without a GPU and exports every function
include/rclupp.h declares; host-side argument checks that return before any
device work (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2412_06551_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rclupp.h")


def declared_functions():
    """Names of the functions declared in the public header."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|char\s*\*|const\s+char\s*\*)\s*\**\s*(rclupp_\w+|\w+_qr)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return nat.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for need in ("rclupp_qr", "rcluppr_qr", "cholqr2_qr", "scholqr3_qr", "lc2_qr", "rcholqr_qr", "rclupp_qr_ex",
                 "rclupp_qr_batched", "rclupp_qr_noalloc", "rclupp_status_string"):
        assert need in names, need


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert sorted(nat.EXPORTS) == declared_functions()


def test_status_strings(lib):
    for st in range(0, 7):
        s = nat.status_string(st)
        assert s and s != "unknown status", st
    assert "rclupp_qr_noalloc" in nat.status_string(nat.ERR_SCRATCH_LIMIT)


def test_noalloc_rejects_sizes_beyond_its_scratch(lib):
    # RCLUPPr keeps an m-long pivot vector for its tall LU: at m = 2^26 that
    # alone is 256 MiB, beyond the fixed scratch; the call returns before it
    # touches the device (the pointers are never dereferenced)
    m, n, s = 1 << 26, 8, 16
    assert 4 * m > nat.NOALLOC_MAX_BYTES
    fake = ctypes.c_void_p(1 << 20)
    o = nat.Opts()
    st = lib.rclupp_qr_noalloc(nat.ALG["rcluppr"], fake, m, n, m, s, 0, fake, fake, ctypes.byref(o), None, None)
    assert st == nat.ERR_SCRATCH_LIMIT
    # argument errors come first, as for rclupp_qr_ex
    st = lib.rclupp_qr_noalloc(nat.ALG["rclupp"], fake, 100, 200, 100, 400, 0, fake, fake, None, None, None)
    assert st == nat.ERR_INVALID_ARG
    st = lib.rclupp_qr_noalloc(nat.ALG["rclupp"], None, 100, 10, 100, 20, 0, fake, fake, None, None, None)
    assert st == nat.ERR_INVALID_ARG


def test_tall_lu_rejects_overlapping_output(lib):
    # M must not overlap X (the LU reads X until its last column has entered
    # M); the check comes before any device work
    m, n = 1000, 8
    x = ctypes.c_void_p(1 << 24)
    perm = ctypes.c_void_p(1 << 30)
    for off in (0, 8 * m, 8 * (7 * m + 999)):
        st = lib.rclupp_tall_lu(x, m, n, m, ctypes.c_void_p((1 << 24) + off), m, perm, None, None)
        assert st == nat.ERR_INVALID_ARG, off
