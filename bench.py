#!/usr/bin/env python3
"""Throughput benchmark of the MI355X tall-skinny QR library.

Headline workload (one step = one full RCLUPP factorization, Algorithm 2, every
stage on the GPU): X = U diag(sigma) V^T with m = 4,194,304, n = 256 (8 GiB),
a geometric spectrum with kappa_2 = 1e14, U the orthonormalized Q factor of a
seeded Gaussian and V a seeded orthogonal matrix (generated on the device,
seed 0); Gaussian sketch with s = 4n = 1024 rows, sketch seed 0; FP64
throughout. Inputs are resident in HBM before the timed region.

Reported (one JSON line):
  value       = algorithmic bytes of the tall passes / time per step (GB/s):
                sketch 8mn + three substitution passes 16mn each = 56mn bytes;
  tflops      = algorithmic FP64 flops / time: 2smn (sketch) + 2(mn^2 + mn(n+1))
                (two substitution+Gram passes) + mn^2 (final substitution);
  roofline    = the dominant kernel's algorithmic rate (per launch, from HIP
                events recorded between the launches on the library's stream)
                against MI355X's published peak for its binding resource;
  stage_rates = each tall stage against both ceilings (HBM and the matrix peak
                of its precision);
  mixed       = the same shape at kappa in {1e2, 1e8, 1e14}: plain FP64 against
                the FP32 (sketch and LU) and BF16 (sketch; FP32 LU) forms and the
                CountSketch (FP64 sums; FP32 LU), each with its time, accuracy,
                sketch roofline and whether the call escalated to the extra
                shifted-Cholesky pass;
  c2          = m = 1,048,576, n = 64, s = 2n, kappa = 1e15 (FP64 RCLUPP, with
                its roofline, the other five methods and the oracle comparison);
  batched     = 512 problems (m in [1e4, 5e5], n in {16, 32, 64, 128}, kappa
                log-uniform in [1e2, 1e14], s = 2n) in one call: QRs/s and the
                fraction of the batch's attainable roofline time;
  krylov      = RCLUPPr on m = 16,777,216, n = 128 Krylov-monomial columns;
  cpu_baseline= the CPU oracle (oracle/) timed on the host cores on a bounded
                sample of the headline matrix (its first 2^20 rows), and the GPU
                result on the same sample compared with it (accuracy).
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
       python bench.py --only {mixed,c2,batched,krylov}   (one extra leg alone, for a
                                                           kernel trace of that workload)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tall QR GB/s + FP64 TFLOP/s (plain vs mixed, orth≤1e-12); batched QRs/s"
M, N, S, KAPPA, SEED = 4194304, 256, 1024, 1e14, 0
C2_M, C2_N, C2_S, C2_KAPPA = 1 << 20, 64, 128, 1e15
CPU_SAMPLE_ROWS = 1 << 20
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 (vector and matrix), TFLOP/s
MATRIX_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # dense MFMA peaks
TALL_STAGES = ("sketch", "trsm_gram", "trsm_final")


def tall_bytes(m, n):
    """Algorithmic HBM bytes per RCLUPP step and per kernel launch."""
    return {"sketch": 8 * m * n, "trsm_gram": 16 * m * n, "trsm_final": 16 * m * n,
            "total": 8 * m * n + 3 * 16 * m * n}


def tall_lu_moved_bytes(m, n, widths=(4, 16, 32)):
    """HBM bytes the blocked partial-pivoting LU moves (rows taken as m): every
    column step's read and write of the rest of its panel, and every block
    update's read of its L columns and read and write of the columns it
    updates (a column's first update reads it from X), with panels of
    widths[0] columns inside blocks of widths[1] inside blocks of widths[2]
    (the launch order of the library)."""
    w0, w1, w2 = widths
    passes = 0.0

    def update(c0, c1, ce):
        return 0.5 * (c1 - c0) + (ce - c1)

    for b0 in range(0, n, w2):
        b1 = min(b0 + w2, n)
        for s0 in range(b0, b1, w1):
            s1 = min(s0 + w1, b1)
            for c0 in range(s0, s1, w0):
                c1 = min(c0 + w0, s1)
                passes += sum(c1 - k for k in range(c0, c1))
                if c1 < s1:
                    passes += update(c0, c1, s1)
            if s1 < b1:
                passes += update(s0, s1, b1)
        if b1 < n:
            passes += update(b0, b1, n)
    return int(passes * 16 * m)


def tall_flops(m, n, s):
    return {"sketch": 2 * s * m * n, "trsm_gram": m * n * n + m * n * (n + 1), "trsm_final": m * n * n,
            "total": 2 * s * m * n + 2 * (m * n * n + m * n * (n + 1)) + m * n * n}


def stage_prec(name, sketch_prec):
    """Arithmetic of a tall stage: the sketch follows the option, the rest is FP64."""
    return sketch_prec if name == "sketch" else "fp64"


def kernel_source_hash(name):
    src = {"sketch": "k_sketch.hip", "trsm_gram": "k_tall.hip", "trsm_final": "k_tall.hip"}.get(name)
    if src is None:
        return None
    with open(os.path.join(ROOT, "paper_2412_06551_amd", "csrc", src), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(name, workload="c3"):
    """HBM bytes per launch from the committed rocprofv3 counter runs of this
    workload, if they were taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(name)
    if not e or e.get("source_sha256_16") != kernel_source_hash(name):
        return None
    return e.get("bytes_per_launch")


def rate_entry(name, ms, cnt, m, n, s, sketch_prec="fp64"):
    """Per-launch algorithmic rate of one tall stage against the ceiling that
    binds it: HBM when its arithmetic intensity is below the ridge of its
    precision's matrix peak, that peak otherwise."""
    by = tall_bytes(m, n)[name]
    fl = tall_flops(m, n, s)[name]
    prec = stage_prec(name, sketch_prec)
    peak = MATRIX_PEAK_TFLOPS[prec]
    t = ms / cnt / 1e3
    if fl / by > peak * 1e12 / (HBM_PEAK_GBS * 1e9):
        achieved = fl / t / 1e12
        ent = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
               "frac": round(achieved / peak, 4), "prec": prec}
    else:
        achieved = by / t / 1e9
        ent = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4), "prec": prec}
    ent["kernel"] = name
    ent["avg_launch_ms"] = round(ms / cnt, 5)
    ent["launches"] = cnt
    return ent


def stage_rates(stages, m, n, s, sketch_prec="fp64"):
    """Every tall stage against both ceilings (HBM and the matrix peak of its
    precision), from the same per-launch event timings as the roofline entry."""
    by = tall_bytes(m, n)
    fl = tall_flops(m, n, s)
    out = {}
    for name in TALL_STAGES:
        if name not in stages:
            continue
        ms, cnt = stages[name]
        t = ms / cnt / 1e3
        prec = stage_prec(name, sketch_prec)
        gbs = by[name] / t / 1e9
        tfs = fl[name] / t / 1e12
        out[name] = {"avg_launch_ms": round(ms / cnt, 5), "GB_s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                     "TFLOP_s": round(tfs, 2), "prec": prec, "frac_matrix": round(tfs / MATRIX_PEAK_TFLOPS[prec], 4)}
    return out


def roofline_entry(stages, m, n, s, sketch_prec="fp64", workload="c3"):
    """Dominant tall kernel (largest total time) and its rate against its roof."""
    best = None
    for name in TALL_STAGES:
        if name not in stages:
            continue
        ms, cnt = stages[name]
        if best is None or ms > best[1]:
            best = (name, ms, cnt)
    if best is None:
        return None
    name, ms, cnt = best
    ent = rate_entry(name, ms, cnt, m, n, s, sketch_prec)
    ent["traffic"] = measured_traffic(name, workload) if sketch_prec == "fp64" else None
    return ent


def attainable_ms(m, n, s):
    """Attainable-roofline time of one FP64 RCLUPP: every tall pass at
    max(bytes / HBM peak, flops / FP64 peak)."""
    by, fl = tall_bytes(m, n), tall_flops(m, n, s)
    t = 0.0
    for name, k in (("sketch", 1), ("trsm_gram", 2), ("trsm_final", 1)):
        t += k * max(by[name] / (HBM_PEAK_GBS * 1e9), fl[name] / (FP64_PEAK_TFLOPS * 1e12))
    return t * 1e3


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def copy_rate(X, Q, reps=5):
    """The streaming rate a plain copy reaches on this GPU: torch's elementwise
    multiply by 1.0 of X into Q (8mn bytes read, 8mn written), timed with
    events; the ceiling the HBM-bound kernels are compared against besides the
    published peak."""
    import torch
    torch.mul(X, 1.0, out=Q)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        torch.mul(X, 1.0, out=Q)
    e1.record(st)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps / 1e3
    gbs = 2 * X.numel() * 8 / t / 1e9
    return {"GB_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "kernel": "torch elementwise copy of X (8mn bytes read, 8mn written)"}


def gpu_accuracy(X, Q, R):
    """||Q^T Q - I||_F and ||QR - X||_F / ||X||_F in FP64 with plain torch
    products over row chunks (bounded temporaries)."""
    import torch
    n = Q.shape[1]
    g = torch.zeros((n, n), dtype=torch.float64, device=Q.device)
    num = torch.zeros((), dtype=torch.float64, device=Q.device)
    den = torch.zeros((), dtype=torch.float64, device=Q.device)
    step = 1 << 20
    for r0 in range(0, X.shape[0], step):
        q = Q[r0:r0 + step]
        g += q.t() @ q
        num += torch.sum((q @ R - X[r0:r0 + step]) ** 2)
        den += torch.sum(X[r0:r0 + step] ** 2)
    g -= torch.eye(n, dtype=torch.float64, device=Q.device)
    return float(torch.linalg.matrix_norm(g)), float(torch.sqrt(num / den))


class Runner:
    """Q, R, outcome record and workspace for repeated calls on one input."""

    def __init__(self, lib, X, alg, s, seed, sketch_prec="fp64", lu_prec="fp64", sketch="gaussian",
                 tall_lu="partial"):
        import torch
        m, n = X.shape
        self.lib, self.X, self.alg, self.s, self.seed = lib, X, alg, s, seed
        self.sp, self.lp, self.kind, self.tl = sketch_prec, lu_prec, sketch, tall_lu
        self.stream = torch.cuda.current_stream()
        self.Q = torch.empty((n, m), dtype=torch.float64, device=X.device).t()
        self.R = torch.empty((n, n), dtype=torch.float64, device=X.device).t()
        self.info = torch.zeros(4, dtype=torch.int32, device=X.device)
        self.ws = torch.empty(max(lib.workspace_size(alg, m, n, s, sketch_prec, lu_prec, sketch, tall_lu=tall_lu), 256),
                              dtype=torch.uint8, device=X.device)

    def __call__(self):
        self.lib.qr(self.X, alg=self.alg, s=self.s, seed=self.seed, sketch_prec=self.sp, lu_prec=self.lp, Q=self.Q,
                    R=self.R, workspace=self.ws, info=self.info, stream=self.stream, sketch=self.kind,
                    tall_lu=self.tl)

    def time(self, reps, warmup=1):
        import torch
        for _ in range(warmup):
            self()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(reps):
            self()
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def trace(self, reps):
        """Per-stage totals over `reps` traced calls: {stage: (ms, launches)}."""
        import torch
        from paper_2412_06551_amd import _native as nat
        nat.trace_enable(64 * reps)
        for _ in range(reps):
            self()
        stages = nat.trace_read()
        nat.trace_enable(0)
        torch.cuda.synchronize()
        return stages

    def info_host(self):
        return [int(v) for v in self.info.cpu().tolist()]


def bench_mixed(lib, reps=3, x_headline=None):
    """The headline shape at kappa 1e2, 1e8 and 1e14: FP64 against the FP32
    and BF16 forms."""
    import torch
    from gen import make_svd_device
    m, n, s = M, N, S
    by = tall_bytes(m, n)["total"]
    fl = tall_flops(m, n, s)["total"]
    out = {"workload": "rclupp m=%d n=%d s=%d (SVD-based, device-generated seed 0)" % (m, n, s), "kappa": {}}
    for kappa in (1e2, 1e8, 1e14):
        if kappa == KAPPA and x_headline is not None:
            X = x_headline
        else:
            print("bench: mixed leg, generating %dx%d kappa=%.0e" % (m, n, kappa), file=sys.stderr, flush=True)
            X = make_svd_device(m, n, kappa, seed=SEED)
        row = {}
        r64 = None
        for tag, sk, lu, kind in (("fp64", "fp64", "fp64", "gaussian"), ("fp32", "fp32", "fp32", "gaussian"),
                                  ("bf16", "bf16", "fp32", "gaussian"), ("count", "fp64", "fp32", "count"),
                                  ("srht", "bf16", "fp32", "srht")):
            run = Runner(lib, X, "rclupp", s, SEED, sk, lu, kind)
            ms = run.time(reps)
            stages = run.trace(1)
            info = run.info_host()
            orth, res = gpu_accuracy(X, run.Q, run.R)
            ent = {"sketch": kind, "sketch_prec": sk, "lu_prec": lu, "ms": round(ms, 3),
                   "GB_s": round(by / (ms / 1e3) / 1e9, 1),
                   "fp64_tflops": round(fl / (ms / 1e3) / 1e12, 3), "info": info,
                   "escalated": bool(info[3] & 1), "orth": orth, "rel_res": res}
            if "sketch" in stages and kind == "gaussian":
                ent["sketch_roofline"] = rate_entry("sketch", *stages["sketch"], m, n, s, sk)
            elif "sketch" in stages:
                # CountSketch, BF16 SRHT: one read of X (8mn bytes) against HBM
                t = stages["sketch"][0] / stages["sketch"][1] / 1e3
                gbs = 8 * m * n / t / 1e9
                ent["sketch_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                          "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                          "avg_launch_ms": round(t * 1e3, 5)}
            if tag == "fp64":
                r64 = run.R.clone()
            else:
                ent["r_rel_diff_vs_fp64"] = float(torch.linalg.matrix_norm(run.R - r64) / torch.linalg.matrix_norm(r64))
                ent["speedup_vs_fp64"] = round(row["fp64"]["ms"] / ms, 3)
            row[tag] = ent
            print("bench: mixed kappa=%.0e %s %.3f ms info=%s orth=%.2e" % (kappa, tag, ms, info, orth),
                  file=sys.stderr, flush=True)
            del run
            torch.cuda.empty_cache()
        out["kappa"]["%.0e" % kappa] = row
        if X is not x_headline:
            del X
        torch.cuda.empty_cache()
    return out


def bench_c2(lib, steps=10, with_cpu=True, copy_calibration=False):
    """1,048,576 x 64, s = 2n, kappa = 1e15: FP64 RCLUPP, its roofline, the other
    methods, and the whole result against the oracle."""
    import numpy as np
    import torch

    import oracle
    from gen import make_svd
    m, n, s = C2_M, C2_N, C2_S
    print("bench: c2 leg, generating %dx%d" % (m, n), file=sys.stderr, flush=True)
    x = make_svd(m, n, C2_KAPPA, seed=SEED)
    X = torch.empty((n, m), dtype=torch.float64, device="cuda").t()
    X.copy_(torch.from_numpy(x))
    run = Runner(lib, X, "rclupp", s, SEED)
    if copy_calibration:
        torch.mul(X, 1.0, out=run.Q)
        torch.cuda.synchronize()
    ms = run.time(steps, warmup=2)
    stages = run.trace(steps)
    by, fl = tall_bytes(m, n), tall_flops(m, n, s)
    out = {"workload": "rclupp m=%d n=%d s=%d kappa=%.0e (SVD-based, host-generated seed 0)" % (m, n, s, C2_KAPPA),
           "ms": round(ms, 5), "GB_s": round(by["total"] / (ms / 1e3) / 1e9, 1),
           "fp64_tflops": round(fl["total"] / (ms / 1e3) / 1e12, 3), "info": run.info_host(),
           "attainable_ms": round(attainable_ms(m, n, s), 4),
           "stages_ms_per_step": {k: round(v[0] / steps, 5) for k, v in stages.items()},
           "roofline": roofline_entry(stages, m, n, s, workload="c2"), "stage_rates": stage_rates(stages, m, n, s)}
    other = {}
    for alg, tl in (("rcluppr", "partial"), ("cholqr2", "partial"), ("scholqr3", "partial"), ("lc2", "partial"),
                    ("rcholqr", "partial"), ("rcluppr", "tournament"), ("lc2", "tournament")):
        o = Runner(lib, X, alg, s, SEED, tall_lu=tl)
        t = o.time(max(2, steps // 4))
        other[alg if tl == "partial" else alg + "_tournament"] = {"ms": round(t, 4), "info": o.info_host()}
        del o
    out["other_methods_ms"] = other
    if with_cpu:
        q = np.asfortranarray(run.Q.cpu().numpy())
        r = np.asfortranarray(run.R.cpu().numpy())
        t0 = time.perf_counter()
        orc = oracle.rclupp(x, s, SEED)
        t = time.perf_counter() - t0
        met = oracle.metrics(x, q, r)
        out["vs_oracle"] = {"orth": met["orth"], "rel_res": met["rel_res"],
                            "r_rel_err": float(np.linalg.norm(r - orc.R) / np.linalg.norm(orc.R)),
                            "oracle_seconds": round(t, 3), "oracle_GB_s": round(by["total"] / t / 1e9, 3)}
    return out


def bench_batched(lib, reps=3):
    import torch
    from gen import batch_manifest, make_svd_device
    man = batch_manifest(0, 512)
    print("bench: batched leg, generating %d problems" % len(man), file=sys.stderr, flush=True)
    Xs = [make_svd_device(p["m"], p["n"], p["kappa"], p["input_seed"], orthonormal=False) for p in man]
    seeds = [p["seed"] for p in man]
    by = sum(tall_bytes(p["m"], p["n"])["total"] for p in man)
    t_roof = sum(attainable_ms(p["m"], p["n"], 2 * p["n"]) for p in man)
    # grouped launches captured in a hipGraph, rows per workgroup autotuned on the first call
    batch = lib.Batch(Xs, alg="rclupp", seeds=seeds, graph=True, autotune=True)
    batch.run()
    batch.run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        Qs, Rs, info = batch.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    info = info.cpu()
    worst_orth, worst_res = 0.0, 0.0
    for i in range(0, len(man), 64):  # a sample of the results
        o, r = gpu_accuracy(Xs[i], Qs[i], Rs[i])
        worst_orth, worst_res = max(worst_orth, o), max(worst_res, r)
    # the same problems as one plain FP64 RCLUPP call each, on the same stream
    for X, p in zip(Xs[:4], man[:4]):
        lib.qr(X, alg="rclupp", s=2 * p["n"], seed=p["seed"])
    torch.cuda.synchronize()
    e0.record(stream)
    for X, p in zip(Xs, man):
        lib.qr(X, alg="rclupp", s=2 * p["n"], seed=p["seed"])
    e1.record(stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    return {"problems": len(man), "ms": round(ms, 3), "qrs_per_s": round(len(man) / (ms / 1e3), 1),
            "sequential_ms": round(seq_ms, 3), "speedup_vs_sequential": round(seq_ms / ms, 2),
            "GB_s": round(by / (ms / 1e3) / 1e9, 1), "failed": int((info[:, 0] != 0).sum()),
            "roofline": {"bound": "attainable", "attainable_ms": round(t_roof, 3),
                         "frac": round(t_roof / ms, 4),
                         "note": "sum over problems and tall passes of max(bytes / HBM peak, flops / FP64 peak)"},
            "sample_worst_orth": worst_orth, "sample_worst_rel_res": worst_res,
            "workload": "512 x RCLUPP, batch_manifest(seed 0), U = normalised Gaussian columns",
            "launch": "grouped by (n, s), hipGraph replay, autotuned rows per workgroup"}


def bench_krylov(lib):
    import torch
    from gen import make_krylov_device
    m, n, s = 16777216, 128, 256
    print("bench: krylov leg, generating %dx%d" % (m, n), file=sys.stderr, flush=True)
    X = make_krylov_device(m, n, 0)
    run = Runner(lib, X, "rcluppr", s, SEED)
    ms = run.time(1)
    stages = run.trace(1)
    orth, res = gpu_accuracy(X, run.Q, run.R)
    out = {"workload": "rcluppr m=%d n=%d s=%d Krylov-monomial (device-generated)" % (m, n, s), "ms": round(ms, 3),
           "GB_s": round(tall_bytes(m, n)["total"] / (ms / 1e3) / 1e9, 1), "info": run.info_host(), "orth": orth,
           "rel_res": res, "stages_ms": {k: round(v[0], 4) for k, v in stages.items()}}
    if "tall_lu" in stages:
        # one read and one write of X is the tall LU's algorithmic traffic;
        # "moved" counts what its blocked form streams (the column steps of
        # partial pivoting cannot avoid most of it)
        t = stages["tall_lu"][0] / 1e3
        gbs = 16 * m * n / t / 1e9
        moved = tall_lu_moved_bytes(m, n)
        out["tall_lu_roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(gbs / HBM_PEAK_GBS, 4), "ms": round(stages["tall_lu"][0], 3),
                                   "moved_bytes": moved, "moved_GB_s": round(moved / t / 1e9, 1),
                                   "moved_frac": round(moved / t / 1e9 / HBM_PEAK_GBS, 4)}
    del run
    torch.cuda.empty_cache()
    # the mixed-precision form: BF16 sketch of M, FP32 LU/Householder of the sketch
    run = Runner(lib, X, "rcluppr", s, SEED, "bf16", "fp32")
    ms2 = run.time(1)
    orth2, res2 = gpu_accuracy(X, run.Q, run.R)
    out["mixed_bf16_sketch_fp32_lu"] = {"ms": round(ms2, 3), "info": run.info_host(), "orth": orth2, "rel_res": res2}
    del run
    torch.cuda.empty_cache()
    # tournament pivoting for the LU of X (TSLU tree, then M = X N^{-1})
    run = Runner(lib, X, "rcluppr", s, SEED, tall_lu="tournament")
    ms3 = run.time(1)
    st3 = run.trace(1)
    orth3, res3 = gpu_accuracy(X, run.Q, run.R)
    out["tournament_lu"] = {"ms": round(ms3, 3), "info": run.info_host(), "orth": orth3, "rel_res": res3,
                            "tall_lu_ms": round(st3["tall_lu"][0], 3) if "tall_lu" in st3 else None}
    return out


def cpu_baseline(lib, X, s, seed, rows=CPU_SAMPLE_ROWS):
    """The oracle's RCLUPP on the first `rows` rows of the headline matrix (a
    bounded sample), and the GPU's RCLUPP on the same rows compared with it."""
    import numpy as np
    import torch

    import oracle
    n = X.shape[1]
    xs = torch.empty((n, rows), dtype=torch.float64, device=X.device).t()
    xs.copy_(X[:rows])
    x = np.asfortranarray(xs.cpu().numpy())
    run = Runner(lib, xs, "rclupp", s, seed)
    run()
    torch.cuda.synchronize()
    q = np.asfortranarray(run.Q.cpu().numpy())
    r = np.asfortranarray(run.R.cpu().numpy())
    t0 = time.perf_counter()
    res = oracle.rclupp(x, s, seed)
    t = time.perf_counter() - t0
    met = oracle.metrics(x, q, r)
    base = {"value": round(tall_bytes(rows, n)["total"] / t / 1e9, 3), "unit": "GB/s", "cores": oracle.max_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "seconds": round(t, 3),
            "sample": "oracle RCLUPP (FP64, s=%d, seed %d) on rows 0..%d of the headline matrix (%d x %d, "
                      "1/%d of its rows), one run; value = 56 * rows * n bytes / time"
                      % (s, seed, rows - 1, rows, n, X.shape[0] // rows)}
    acc = {"sample_rows": rows, "orth": met["orth"], "rel_res": met["rel_res"],
           "r_rel_err_vs_oracle": float(np.linalg.norm(r - res.R) / np.linalg.norm(res.R)),
           "gpu_info": run.info_host(), "oracle_info": int(res.info[0])}
    return base, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-extras", action="store_true", help="skip the extra legs")
    ap.add_argument("--kappa", type=float, default=KAPPA)
    ap.add_argument("--only", choices=("mixed", "c2", "batched", "krylov"),
                    help="run just that extra leg and print its JSON object (for kernel traces of that workload; "
                         "not the benchmark line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain elementwise copy of X (8mn bytes read, 8mn written) before timing, "
                         "as the reference kernel for the HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_06551_amd as lib
    from gen import make_svd_device

    torch.cuda.set_device(0)
    if args.only:
        legs = {"mixed": bench_mixed,
                "c2": lambda l: bench_c2(l, with_cpu=not args.no_cpu, copy_calibration=args.copy_calibration),
                "batched": bench_batched, "krylov": bench_krylov}
        print(json.dumps({args.only: legs[args.only](lib)}), flush=True)
        return
    m, n, s = M, N, S
    print("bench: generating %dx%d kappa=%.0e input on the device" % (m, n, args.kappa), file=sys.stderr, flush=True)
    X = make_svd_device(m, n, args.kappa, seed=SEED)
    run = Runner(lib, X, "rclupp", s, SEED)
    if args.copy_calibration:
        torch.mul(X, 1.0, out=run.Q)
        torch.cuda.synchronize()
    ms = run.time(args.steps, warmup=args.warmup)
    gpu_info = run.info_host()
    print("bench: rclupp %.4f ms/step info=%s" % (ms, gpu_info), file=sys.stderr, flush=True)
    # stage timing over a second timed region (events between the library's launches)
    stages = run.trace(args.steps)
    orth, res = gpu_accuracy(X, run.Q, run.R)
    hbm_copy = copy_rate(X, run.Q)

    by, fl = tall_bytes(m, n), tall_flops(m, n, s)
    out = {
        "metric": METRIC,
        "value": round(by["total"] / (ms / 1e3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rclupp m=%d n=%d s=%d kappa=%.0e (SVD-based geometric spectrum, device-generated "
                               "seed %d)" % (m, n, s, args.kappa, SEED),
                   "method": "RCLUPP (Algorithm 2), FP64", "m": m, "n": n, "s": s, "kappa": args.kappa},
        "tflops": round(fl["total"] / (ms / 1e3) / 1e12, 3),
        "attainable_ms": round(attainable_ms(m, n, s), 3),
        "gpu_info": gpu_info,
        "orth": orth,
        "rel_res": res,
        "stages_ms_per_step": {k: round(v[0] / args.steps, 5) for k, v in stages.items()},
        "roofline": roofline_entry(stages, m, n, s),
        "hbm_copy": hbm_copy,
        "stage_rates": stage_rates(stages, m, n, s),
    }
    del run
    torch.cuda.empty_cache()

    if not args.no_extras:
        t_extra = time.time()
        legs = (("mixed", lambda: bench_mixed(lib, x_headline=X)),
                ("c2", lambda: bench_c2(lib, with_cpu=not args.no_cpu)),
                ("batched", lambda: bench_batched(lib)), ("krylov", lambda: bench_krylov(lib)))
        for key, fn in legs:
            if time.time() - t_extra > 200:
                out[key] = {"skipped": "time budget of the extra legs spent"}
                continue
            try:
                out[key] = fn()
            except Exception as e:  # a leg that cannot run is reported, not fatal
                out[key] = {"error": repr(e)[:300]}
            torch.cuda.empty_cache()

    if not args.no_cpu:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        base, acc = cpu_baseline(lib, X, s, SEED)
        out["cpu_baseline"] = base
        out["accuracy"] = acc
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
