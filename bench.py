#!/usr/bin/env python3
"""Throughput benchmark of the MI355X tall-skinny QR library.

Workload (one step = one full RCLUPP factorization, Algorithm 2, every stage on
the GPU): X = U diag(sigma) V^T, m = 1,048,576, n = 64, geometric spectrum with
kappa_2 = 1e15, seed 0; Gaussian sketch with s = 2n = 128 rows, sketch seed 0;
FP64 throughout. Inputs are resident in HBM before the timed region.

Reported (one JSON line):
  value       = algorithmic bytes of the tall passes / time per step (GB/s):
                sketch 8mn + three substitution passes 16mn each = 56mn bytes;
  tflops      = algorithmic FP64 flops / time: 2smn (sketch) + 2(mn^2 + mn(n+1))
                (two substitution+Gram passes) + mn^2 (final substitution);
  roofline    = the dominant kernel's algorithmic rate (per launch, from HIP
                events recorded between the launches on the library's stream)
                against MI355X's published peak for its binding resource;
  stage_rates = each tall kernel (sketch, substitution+Gram, final substitution)
                against both ceilings: algorithmic GB/s over the HBM peak and
                algorithmic FP64 TFLOP/s over the FP64 MFMA peak;
  cpu_baseline= the CPU oracle (oracle/) timed on the host cores on the same
                input; the same leg also checks the GPU result against it.
Further legs (skipped with --no-extras), each with its own time and accuracy:
  other_methods_ms = the other five methods on the same input;
  mixed        = m = 4,194,304, n = 256, s = 4n = 1024, kappa = 1e8: plain FP64
                 RCLUPP against the FP32 (sketch and LU) and BF16 (sketch) forms;
  batched      = 512 problems (m in [1e4, 5e5], n in {16, 32, 64, 128}, kappa
                 log-uniform in [1e2, 1e14], s = 2n) in one call: QRs/s;
  krylov       = RCLUPPr on m = 16,777,216, n = 128 Krylov-monomial columns.
Large inputs are generated on the GPU (gen.make_*_device).
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
       python bench.py --only {mixed,batched,krylov}   (one extra leg alone, for a
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
M, N, S, KAPPA, SEED = 1 << 20, 64, 128, 1e15, 0
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 (vector and matrix), TFLOP/s


def tall_bytes(m, n):
    """Algorithmic HBM bytes per RCLUPP step and per kernel launch."""
    return {"sketch": 8 * m * n, "trsm_gram": 16 * m * n, "trsm_final": 16 * m * n,
            "total": 8 * m * n + 3 * 16 * m * n}


def tall_flops(m, n, s):
    return {"sketch": 2 * s * m * n, "trsm_gram": m * n * n + m * n * (n + 1), "trsm_final": m * n * n,
            "total": 2 * s * m * n + 2 * (m * n * n + m * n * (n + 1)) + m * n * n}


def kernel_source_hash(name):
    src = {"sketch": "k_sketch.hip", "trsm_gram": "k_tall.hip", "trsm_final": "k_tall.hip"}.get(name)
    if src is None:
        return None
    with open(os.path.join(ROOT, "paper_2412_06551_amd", "csrc", src), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(name)
    if not e or e.get("source_sha256_16") != kernel_source_hash(name):
        return None
    return e.get("bytes_per_launch")


def stage_rates(stages, m, n, s):
    """Every tall kernel's rate against both of its ceilings (HBM and FP64 MFMA),
    from the same per-launch event timings as the roofline entry."""
    by = tall_bytes(m, n)
    fl = tall_flops(m, n, s)
    out = {}
    for name in ("sketch", "trsm_gram", "trsm_final"):
        if name not in stages:
            continue
        ms, cnt = stages[name]
        t = ms / cnt / 1e3
        gbs = by[name] / t / 1e9
        tfs = fl[name] / t / 1e12
        out[name] = {"avg_launch_ms": round(ms / cnt, 5), "GB_s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                     "fp64_TFLOP_s": round(tfs, 2), "frac_fp64": round(tfs / FP64_PEAK_TFLOPS, 4)}
    return out


def roofline_entry(stages, m, n, s):
    """Dominant kernel (largest total time among the tall kernels) and its rate."""
    by = tall_bytes(m, n)
    fl = tall_flops(m, n, s)
    best = None
    for name in ("sketch", "trsm_gram", "trsm_final"):
        if name not in stages:
            continue
        ms, cnt = stages[name]
        if best is None or ms > best[1]:
            best = (name, ms, cnt)
    if best is None:
        return None
    name, ms, cnt = best
    avg_s = ms / cnt / 1e3
    # binding resource from arithmetic intensity vs the FP64 ridge (78.6 TF / 8 TB/s)
    ai = fl[name] / by[name]
    if ai > FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
        achieved = fl[name] / avg_s / 1e12
        ent = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": round(achieved / FP64_PEAK_TFLOPS, 4)}
    else:
        achieved = by[name] / avg_s / 1e9
        ent = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4)}
    ent["kernel"] = name
    ent["avg_launch_ms"] = round(ms / cnt, 5)
    ent["launches"] = cnt
    ent["traffic"] = measured_traffic(name)
    return ent


def cpu_baseline(x, s, seed, q_gpu, r_gpu, budget_s=12.0):
    """Oracle RCLUPP on the host cores (same input), plus the GPU result's accuracy."""
    import numpy as np

    import oracle
    m, n = x.shape
    times = []
    res = None
    t_end = time.time() + budget_s
    while not times or (time.time() < t_end and len(times) < 5):
        t0 = time.perf_counter()
        res = oracle.rclupp(x, s, seed)
        times.append(time.perf_counter() - t0)
    t = min(times)
    met = oracle.metrics(x, q_gpu, r_gpu)
    rerr = float(np.linalg.norm(r_gpu - res.R) / np.linalg.norm(res.R))
    base = {"value": round(tall_bytes(m, n)["total"] / t / 1e9, 3), "unit": "GB/s", "cores": oracle.max_threads(),
            "kind": "oracle", "seconds_per_qr": round(t, 3),
            "sample": "full workload, %d run(s) of oracle RCLUPP (best taken)" % len(times)}
    acc = {"orth": met["orth"], "rel_res": met["rel_res"], "r_rel_err_vs_oracle": rerr,
           "oracle_info": int(res.info[0])}
    return base, acc


def gpu_accuracy(X, Q, R):
    """||Q^T Q - I||_F and ||QR - X||_F / ||X||_F in FP64 with plain torch products."""
    import torch
    n = Q.shape[1]
    qtq = Q.t() @ Q
    qtq -= torch.eye(n, dtype=torch.float64, device=Q.device)
    orth = float(torch.linalg.matrix_norm(qtq))
    res = float(torch.linalg.matrix_norm(Q @ R - X) / torch.linalg.matrix_norm(X))
    return orth, res


def time_qr(lib, X, alg, s, seed, reps, sketch_prec="fp64", lu_prec="fp64"):
    """Median-free simple timing: one warm-up call, then `reps` calls between events."""
    import torch
    m, n = X.shape
    stream = torch.cuda.current_stream()
    Q = torch.empty((n, m), dtype=torch.float64, device=X.device).t()
    R = torch.empty((n, n), dtype=torch.float64, device=X.device).t()
    info = torch.zeros(4, dtype=torch.int32, device=X.device)
    ws = torch.empty(lib.workspace_size(alg, m, n, s, sketch_prec, lu_prec), dtype=torch.uint8, device=X.device)

    def call():
        lib.qr(X, alg=alg, s=s, seed=seed, sketch_prec=sketch_prec, lu_prec=lu_prec, Q=Q, R=R, workspace=ws,
               info=info, stream=stream)

    call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, info.cpu().tolist(), Q, R


def bench_mixed(lib, reps=3, kappa=1e8):
    import torch
    from gen import make_svd_device
    m, n, s = 4194304, 256, 1024
    print("bench: mixed leg, generating %dx%d" % (m, n), file=sys.stderr, flush=True)
    X = make_svd_device(m, n, kappa, seed=0)
    by = tall_bytes(m, n)["total"]
    fl = tall_flops(m, n, s)["total"]
    out = {"workload": "rclupp m=%d n=%d s=%d kappa=%.0e (SVD-based, device-generated)" % (m, n, s, kappa)}
    r64 = None
    for tag, sk, lu in (("fp64", "fp64", "fp64"), ("fp32", "fp32", "fp32"), ("bf16", "bf16", "fp32")):
        ms, info, Q, R = time_qr(lib, X, "rclupp", s, 0, reps, sk, lu)
        orth, res = gpu_accuracy(X, Q, R)
        ent = {"sketch_prec": sk, "lu_prec": lu, "ms": round(ms, 3), "GB_s": round(by / (ms / 1e3) / 1e9, 1),
               "fp64_tflops": round(fl / (ms / 1e3) / 1e12, 3), "info": info, "orth": orth, "rel_res": res}
        if tag == "fp64":
            r64 = R.clone()
        else:
            ent["r_rel_diff_vs_fp64"] = float(torch.linalg.matrix_norm(R - r64) / torch.linalg.matrix_norm(r64))
        out[tag] = ent
        print("bench: mixed %s %.3f ms info=%s orth=%.2e" % (tag, ms, info, orth), file=sys.stderr, flush=True)
        del Q, R
        torch.cuda.empty_cache()
    return out


def bench_batched(lib, reps=3):
    import torch
    from gen import batch_manifest, make_svd_device
    man = batch_manifest(0, 512)
    print("bench: batched leg, generating %d problems" % len(man), file=sys.stderr, flush=True)
    Xs = [make_svd_device(p["m"], p["n"], p["kappa"], p["input_seed"], orthonormal=False) for p in man]
    seeds = [p["seed"] for p in man]
    by = sum(tall_bytes(p["m"], p["n"])["total"] for p in man)
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
            "sample_worst_orth": worst_orth, "sample_worst_rel_res": worst_res,
            "workload": "512 x RCLUPP, batch_manifest(seed 0), U = normalised Gaussian columns",
            "launch": "grouped by (n, s), hipGraph replay, autotuned rows per workgroup"}


def bench_krylov(lib):
    import torch
    from gen import make_krylov_device
    m, n, s = 16777216, 128, 256
    print("bench: krylov leg, generating %dx%d" % (m, n), file=sys.stderr, flush=True)
    X = make_krylov_device(m, n, 0)
    ms, info, Q, R = time_qr(lib, X, "rcluppr", s, 0, 1)
    orth, res = gpu_accuracy(X, Q, R)
    out = {"workload": "rcluppr m=%d n=%d s=%d Krylov-monomial (device-generated)" % (m, n, s), "ms": round(ms, 3),
           "GB_s": round(tall_bytes(m, n)["total"] / (ms / 1e3) / 1e9, 1), "info": info, "orth": orth,
           "rel_res": res}
    # the mixed-precision form: BF16 sketch of M, FP32 LU/Householder of the sketch
    del Q, R
    torch.cuda.empty_cache()
    ms2, info2, Q, R = time_qr(lib, X, "rcluppr", s, 0, 1, sketch_prec="bf16", lu_prec="fp32")
    orth2, res2 = gpu_accuracy(X, Q, R)
    out["mixed_bf16_sketch_fp32_lu"] = {"ms": round(ms2, 3), "info": info2, "orth": orth2, "rel_res": res2}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extras", action="store_true", help="skip the other methods")
    ap.add_argument("--kappa", type=float, default=KAPPA)
    ap.add_argument("--only", choices=("mixed", "batched", "krylov"),
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

    import numpy as np
    import torch

    import paper_2412_06551_amd as lib
    from paper_2412_06551_amd import _native as nat
    from gen import make_svd

    torch.cuda.set_device(0)
    if args.only:
        leg = {"mixed": bench_mixed, "batched": bench_batched, "krylov": bench_krylov}[args.only]
        print(json.dumps({args.only: leg(lib)}), flush=True)
        return
    dev = torch.device("cuda:0")
    m, n, s = M, N, S
    print("bench: generating %dx%d kappa=%.0e input" % (m, n, args.kappa), file=sys.stderr, flush=True)
    x = make_svd(m, n, args.kappa, seed=SEED)
    X = torch.empty((n, m), dtype=torch.float64, device=dev).t()
    X.copy_(torch.from_numpy(x))
    Q = torch.empty((n, m), dtype=torch.float64, device=dev).t()
    R = torch.empty((n, n), dtype=torch.float64, device=dev).t()
    info = torch.zeros(4, dtype=torch.int32, device=dev)
    ws = torch.empty(lib.workspace_size("rclupp", m, n, s), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        torch.mul(X, 1.0, out=Q)
        torch.cuda.synchronize()

    def step(alg="rclupp"):
        lib.qr(X, alg=alg, s=s, seed=SEED, Q=Q, R=R, workspace=ws if alg == "rclupp" else None, info=info,
               stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gpu_info = info.cpu().tolist()
    print("bench: rclupp %.4f ms/step info=%s" % (ms, gpu_info), file=sys.stderr, flush=True)

    # stage timing over a second timed region (events between the library's launches)
    nat.trace_enable(64 * args.steps)
    for _ in range(args.steps):
        step()
    stages = nat.trace_read()
    nat.trace_enable(0)
    torch.cuda.synchronize()

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
        "config": {"workload": "rclupp m=%d n=%d s=%d kappa=%.0e (SVD-based geometric spectrum, seed %d)"
                               % (m, n, s, args.kappa, SEED),
                   "method": "RCLUPP (Algorithm 2)", "m": m, "n": n, "s": s, "kappa": args.kappa},
        "tflops": round(fl["total"] / (ms / 1e3) / 1e12, 3),
        "gpu_info": gpu_info,
        "stages_ms_per_step": {k: round(v[0] / args.steps, 5) for k, v in stages.items()},
        "roofline": roofline_entry(stages, m, n, s),
        "stage_rates": stage_rates(stages, m, n, s),
    }

    if not args.no_extras:
        extra = {}
        for alg in ("rcluppr", "cholqr2", "scholqr3", "lc2", "rcholqr"):
            lib.qr(X, alg=alg, s=s, seed=SEED)
            torch.cuda.synchronize()
            k = max(2, args.steps // 4)
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            last = None
            for _ in range(k):
                last = lib.qr(X, alg=alg, s=s, seed=SEED)
            a1.record(stream)
            torch.cuda.synchronize()
            t = a0.elapsed_time(a1) / k
            extra[alg] = {"ms": round(t, 4), "info": last.info_host()}
        out["other_methods_ms"] = extra
        step()
        torch.cuda.synchronize()
        t_extra = time.time()
        for key, fn in (("mixed", bench_mixed), ("batched", bench_batched), ("krylov", bench_krylov)):
            if time.time() - t_extra > 150:
                out[key] = {"skipped": "time budget of the extra legs spent"}
                continue
            try:
                out[key] = fn(lib)
            except Exception as e:  # a leg that cannot run is reported, not fatal
                out[key] = {"error": repr(e)[:300]}
            torch.cuda.empty_cache()

    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        q = np.asfortranarray(Q.cpu().numpy())
        r = np.asfortranarray(R.cpu().numpy())
        base, acc = cpu_baseline(x, s, SEED, q, r)
        out["cpu_baseline"] = base
        out["accuracy"] = acc
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
