"""ctypes binding of the C ABI in include/rclupp.h (argument marshalling only).

Every computation runs in librclupp.so (HIP kernels for gfx950). Loading fails
loudly when the library is missing or no HIP device is present: there is no
CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librclupp.so")

# status codes (rclupp_status)
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_ALLOC, ERR_HIP, ERR_WORKSPACE, ERR_SCRATCH_LIMIT = 0, 1, 2, 3, 4, 5, 6
# fixed scratch of the allocation-free form (RCLUPP_NOALLOC_MAX_BYTES)
NOALLOC_MAX_BYTES = 128 << 20
# info codes and stages (rclupp_info_code, rclupp_stage)
INFO_OK, INFO_LU_ZERO_PIVOT, INFO_CHOL_BREAKDOWN, INFO_NONFINITE, INFO_SINGULAR, INFO_SYNC_TIMEOUT = 0, 1, 2, 3, 4, 5
STAGE_NONE, STAGE_LU, STAGE_QR, STAGE_PRECOND, STAGE_CHOL_A, STAGE_CHOL_B, STAGE_CHOL_X = 0, 1, 2, 3, 4, 5, 6
# outcome notes (rclupp_info.reserved bits)
NOTE_ESCALATED = 1
# precisions and algorithms (rclupp_prec, rclupp_alg)
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
ALG = {"rclupp": 0, "rcluppr": 1, "cholqr2": 2, "scholqr3": 3, "lc2": 4, "rcholqr": 5}
SKETCHED = ("rclupp", "rcluppr", "rcholqr")
MAX_N = 256

EXPORTS = [
    "rclupp_qr", "rcluppr_qr", "cholqr2_qr", "scholqr3_qr", "lc2_qr", "rcholqr_qr",
    "rclupp_last_info", "rclupp_status_string", "rclupp_workspace_size", "rclupp_qr_ex",
    "rclupp_batched_workspace_size", "rclupp_qr_batched", "rclupp_omega", "rclupp_philox",
    "rclupp_sketch", "rclupp_precond", "rclupp_trsm_gram", "rclupp_chol", "rclupp_tall_lu",
    "rclupp_trace_enable", "rclupp_trace_read", "rclupp_release", "rclupp_qr_noalloc", "rclupp_countsketch",
    "rclupp_tall_lu_tournament", "rclupp_srht",
]


class Info(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("stage", ctypes.c_int32), ("index", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


BATCH_GRAPH = 1
BATCH_AUTOTUNE = 2


# sketch kinds (rclupp_opts.sketch_kind)
SKETCH = {"gaussian": 0, "count": 1, "srht": 2}


# pivoting of the LU of X (rclupp_opts.tall_lu)
TALL_LU = {"partial": 0, "tournament": 1}


class Opts(ctypes.Structure):
    _fields_ = [("sketch_prec", ctypes.c_int32), ("lu_prec", ctypes.c_int32), ("batch_flags", ctypes.c_int32),
                ("sketch_kind", ctypes.c_int32), ("tall_lu", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class Problem(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("R", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("s", ctypes.c_int64), ("seed", ctypes.c_uint64)]


class RclError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s failed: %s (status %d)" % (what, status_string(status), status))
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load librclupp.so and declare the signatures (no device work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("librclupp.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I64, U64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t
    qr_sig = [P, I64, I64, I64, I64, U64, P, P, P]
    sigs = {
        "rclupp_qr": qr_sig, "rcluppr_qr": qr_sig, "cholqr2_qr": qr_sig, "scholqr3_qr": qr_sig,
        "lc2_qr": qr_sig, "rcholqr_qr": qr_sig,
        "rclupp_last_info": [P, ctypes.POINTER(Info)],
        "rclupp_workspace_size": [ctypes.c_int, I64, I64, I64, ctypes.POINTER(Opts), ctypes.POINTER(SZ)],
        "rclupp_qr_ex": [ctypes.c_int, P, I64, I64, I64, I64, U64, P, P, ctypes.POINTER(Opts), P, SZ, P, P],
        "rclupp_qr_noalloc": [ctypes.c_int, P, I64, I64, I64, I64, U64, P, P, ctypes.POINTER(Opts), P, P],
        "rclupp_batched_workspace_size": [ctypes.c_int, ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(Opts),
                                          ctypes.POINTER(SZ)],
        "rclupp_qr_batched": [ctypes.c_int, ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(Opts), P, SZ, P, P],
        "rclupp_omega": [U64, I64, I64, I64, P, P],
        "rclupp_philox": [P, I64, ctypes.c_uint32, ctypes.c_uint32, P, P],
        "rclupp_sketch": [P, I64, I64, I64, I64, U64, ctypes.c_int, P, P],
        "rclupp_countsketch": [P, I64, I64, I64, I64, U64, P, P],
        "rclupp_srht": [P, I64, I64, I64, I64, U64, ctypes.c_int, P, P],
        "rclupp_precond": [P, I64, I64, ctypes.c_int, ctypes.c_int, P, P, P, P, P],
        "rclupp_trsm_gram": [P, I64, I64, I64, P, P, I64, P, P],
        "rclupp_chol": [P, I64, I64, ctypes.c_int, P, P, P, I32, P, P],
        "rclupp_tall_lu": [P, I64, I64, I64, P, I64, P, P, P],
        "rclupp_tall_lu_tournament": [P, I64, I64, I64, P, I64, P, P, P, P],
        "rclupp_trace_enable": [ctypes.c_int],
        "rclupp_trace_read": [ctypes.c_int, ctypes.c_char_p, ctypes.c_int, P, P, P],
        "rclupp_release": [],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.rclupp_status_string.argtypes = [ctypes.c_int]
    lib.rclupp_status_string.restype = ctypes.c_char_p
    _lib = lib
    # free the library's process-lifetime HIP objects (pinned tables, cached
    # graphs, events, streams) before the HIP runtime is torn down at exit
    atexit.register(release)
    return lib


def release() -> None:
    """rclupp_release: free the library's process-lifetime objects (no-op if
    the library was never loaded)."""
    if _lib is not None:
        check(_lib.rclupp_release(), "rclupp_release")


def status_string(status: int) -> str:
    try:
        return load().rclupp_status_string(int(status)).decode()
    except Exception:  # pragma: no cover - only used in error paths
        return "status %d" % status


def trace_enable(max_marks: int) -> None:
    check(load().rclupp_trace_enable(int(max_marks)), "rclupp_trace_enable")


def trace_read(max_stages: int = 32, name_len: int = 32):
    """{stage name: (total ms, launches)} for the traced calls since trace_enable."""
    names = ctypes.create_string_buffer(max_stages * name_len)
    ms = (ctypes.c_float * max_stages)()
    cnt = (ctypes.c_int * max_stages)()
    count = ctypes.c_int()
    check(load().rclupp_trace_read(max_stages, names, name_len, ms, cnt, ctypes.byref(count)), "rclupp_trace_read")
    out = {}
    raw = names.raw
    for k in range(min(count.value, max_stages)):
        nm = raw[k * name_len:(k + 1) * name_len].split(b"\0", 1)[0].decode()
        out[nm] = (float(ms[k]), int(cnt[k]))
    return out


def check(status: int, what: str) -> None:
    if status != OK:
        raise RclError(status, what)
