"""Host logic of bench.py (no device): the algorithmic byte and flop counts,
the dominant-kernel roofline entry, the per-kernel rates, the traffic lookup
keyed to the kernel source, and the one-GPU guard."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_counts(bench):
    m, n, s = 1 << 20, 64, 128
    by = bench.tall_bytes(m, n)
    assert by["total"] == 56 * m * n == by["sketch"] + 3 * by["trsm_gram"]
    fl = bench.tall_flops(m, n, s)
    assert fl["sketch"] == 2 * s * m * n
    assert fl["trsm_gram"] == m * n * n + m * n * (n + 1)
    assert fl["total"] == fl["sketch"] + 2 * fl["trsm_gram"] + fl["trsm_final"]


def test_roofline_picks_dominant_kernel_and_bound(bench):
    m, n, s = 1 << 20, 64, 128
    # stage -> (total ms, launches): the substitution+Gram pass dominates
    st = {"sketch": (4.0, 10), "trsm_gram": (6.0, 20), "trsm_final": (2.2, 10)}
    e = bench.roofline_entry(st, m, n, s)
    assert e["kernel"] == "trsm_gram" and e["bound"] == "hbm" and e["unit"] == "GB/s"
    achieved = 16 * m * n / (0.3e-3) / 1e9
    assert abs(e["achieved"] - round(achieved, 1)) < 0.11
    assert abs(e["frac"] - achieved / bench.HBM_PEAK_GBS) < 1e-4
    # n = 256: arithmetic intensity n/8 = 32 flop/B is past the FP64 ridge (9.8)
    e2 = bench.roofline_entry({"trsm_gram": (1.0, 1)}, m, 256, 1024)
    assert e2["bound"] == "mfma" and e2["unit"] == "TFLOP/s"


def test_stage_rates_both_ceilings(bench):
    m, n, s = 1 << 20, 64, 128
    r = bench.stage_rates({"sketch": (0.4, 1), "trsm_final": (0.2, 1)}, m, n, s)
    assert set(r) == {"sketch", "trsm_final"}
    sk = r["sketch"]
    assert abs(sk["GB_s"] - 8 * m * n / 0.4e-3 / 1e9) < 0.1
    assert abs(sk["TFLOP_s"] - 2 * s * m * n / 0.4e-3 / 1e12) < 0.01
    assert abs(sk["frac_matrix"] - sk["TFLOP_s"] / bench.FP64_PEAK_TFLOPS) < 1e-3
    # a BF16 sketch is priced against the BF16 matrix peak
    r2 = bench.stage_rates({"sketch": (0.4, 1)}, m, n, s, sketch_prec="bf16")
    assert r2["sketch"]["prec"] == "bf16"
    assert abs(r2["sketch"]["frac_matrix"] - r2["sketch"]["TFLOP_s"] / 2500.0) < 1e-4


def test_sketch_bound_follows_its_precision(bench):
    # s = 1024: arithmetic intensity s/4 = 256 flop/B, past the FP64 (9.8) and
    # FP32 (19.7) ridges, below the BF16 ridge (312.5)
    m, n, s = 4194304, 256, 1024
    st = {"sketch": (10.0, 1)}
    e64 = bench.rate_entry("sketch", 10.0, 1, m, n, s, "fp64")
    e32 = bench.rate_entry("sketch", 10.0, 1, m, n, s, "fp32")
    e16 = bench.rate_entry("sketch", 10.0, 1, m, n, s, "bf16")
    assert (e64["bound"], e64["peak"]) == ("mfma", 78.6)
    assert (e32["bound"], e32["peak"]) == ("mfma", 157.3)
    assert (e16["bound"], e16["unit"]) == ("hbm", "GB/s")
    assert abs(e16["achieved"] - 8 * m * n / 10e-3 / 1e9) < 0.1
    assert bench.roofline_entry(st, m, n, s)["kernel"] == "sketch"


def test_attainable_time_matches_the_closed_form(bench):
    # max(bytes / 8 TB/s, flops / 78.6 TFLOP/s) per tall pass
    assert abs(bench.attainable_ms(1 << 20, 64, 128) - 0.62) < 0.01
    assert abs(bench.attainable_ms(4194304, 256, 1024) - 45.5) < 0.1


def test_traffic_lookup_is_keyed_to_the_source(bench):
    # a kernel with no source mapping, or an entry not in the file: no traffic figure
    assert bench.measured_traffic("precond") is None
    assert bench.measured_traffic("sketch", workload="no such workload") is None
    assert bench.kernel_source_hash("precond") is None
    h = bench.kernel_source_hash("trsm_gram")
    assert isinstance(h, str) and len(h) == 16


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_tall_lu_moved_bytes(bench):
    """The blocked LU's byte count: closed forms for one level of panels and
    for the three levels at n = 128, and the widths the library launches."""
    import re
    m = 1000
    # one level of w-column panels: column steps n (w + 1) / 2, and after
    # each panel but the last its L (w / 2) and the later columns
    n, w = 64, 8
    later = sum(n - c1 for c1 in range(w, n, w))
    one = n * (w + 1) / 2 + (n // w - 1) * w / 2 + later
    assert bench.tall_lu_moved_bytes(m, n, widths=(w, w, n)) == int(one * 16 * m)
    # three levels at n = 128: 320 + 240 + 96 + 240 passes
    assert bench.tall_lu_moved_bytes(m, 128) == 896 * 16 * m
    # a single column: its step
    assert bench.tall_lu_moved_bytes(m, 1) == 16 * m
    # the default widths are the ones the library uses
    src = open(os.path.join(ROOT, "paper_2412_06551_amd", "csrc", "k_tall_lu.hip")).read()
    got = re.search(r"LU_W0 = (\d+), LU_W1 = (\d+), LU_W2 = (\d+);", src)
    assert got and tuple(int(x) for x in got.groups()) == (4, 16, 32)
