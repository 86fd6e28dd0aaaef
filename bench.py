#!/usr/bin/env python3
"""Benchmark of the SparseStack sketch on MI355X (one GPU).

Workload (the coherent least-squares configuration): A is 4,194,304 x 200
float64 with Pareto(1.5) row factors, 1% of rows spiked x1e3 and column
scaling with condition number 1e8; S is a SparseStack with d = 800 rows in
zeta = 8 blocks. A step is one SA = S A (bucket-plan pass, sketch kernel and
partial reduction) with A resident in HBM. The reported value is the whole
step's algorithmic throughput: (n*m*8 + d*m*8) bytes / step time.

The JSON line also carries
  roofline      the sketch kernel's own average duration (HIP events on its
                stream), as a fraction of the 8 TB/s HBM peak;
  lsqr          sketch-and-precondition solves of the same system to
                tol = 1e-10 (LSQR's least-squares test), with the sketch read
                from the float64 A, a float32 copy and a bfloat16 copy: wall
                time per solve (median), iterations, the sketch / QR / LSQR
                split, and the LSQR iteration's HBM roofline;
  cpu_baseline  the plain CPU oracle timed on a bounded row sample of the
                same matrix on this host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "SA apply GB/s (% HBM peak); sketch-precond LSQR solve time to 1e-10 vs FP64"
HBM_PEAK_GBS = 8000.0
N, M, D, ZETA = 1 << 22, 200, 800, 8
DATA_SEED, SKETCH_SEED = 200, 2000


def kernel_source_digest():
    p = os.path.join(HERE, "paper_2508_21189_amd", "csrc", "ss_rows.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    p = os.path.join(HERE, "profiles", "ss_rows_coherent_f64_traffic.json")
    try:
        with open(p) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_digest():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(A_dev, rows):
    """Oracle SA on the first `rows` rows (the pattern of those rows is the
    pattern of the full sketch); single-threaded scipy sparse product."""
    import numpy as np

    from oracle import sketches as sk
    A = A_dev[:rows].cpu().numpy()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        sk.sparsestack_apply(A, D, ZETA, SKETCH_SEED)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    gbs = (rows * M * 8 + D * M * 8) / t / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d rows, SA via scipy.sparse (single-threaded) incl. Philox pattern; "
                      "median of 3 runs, %.2f s each" % (rows, N, t)}


def lsqr_variants(libsketch, torch, A, b, reps, tol=1e-10):
    """Median wall time of lstsq_sketch_precond per sketch input precision."""
    import statistics
    S = libsketch.Sketch("sparsestack", D, N, ZETA, SKETCH_SEED)
    out = {}
    for name, dt in (("f64", None), ("f32", torch.float32), ("bf16", torch.bfloat16)):
        As = A.to(dt) if dt is not None else None
        S.lstsq_precond(A, b, tol=tol, maxit=300, A_sketch=As)  # warm-up (workspace, code objects)
        walls, infos = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, rc, info = S.lstsq_precond(A, b, tol=tol, maxit=300, A_sketch=As)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
        res = S.residual(A, b, x)
        med = statistics.median(walls)
        it = infos[-1]
        per_iter = statistics.median(i["t_lsqr_ms"] / max(1, i["iters"]) for i in infos)
        out[name] = {"solve_ms": round(med, 3), "status": rc, "iters": it["iters"], "converged": it["converged"],
                     "t_sketch_ms": round(statistics.median(i["t_sketch_ms"] for i in infos), 3),
                     "t_qr_ms": round(statistics.median(i["t_qr_ms"] for i in infos), 3),
                     "t_lsqr_ms": round(statistics.median(i["t_lsqr_ms"] for i in infos), 3),
                     "lsqr_ms_per_iter": round(per_iter, 4),
                     "resnorm": res, "rnorm_est": it["rnorm_est"]}
        print("bench: lsqr %s %.2f ms, %d iterations" % (name, med, it["iters"]), file=sys.stderr, flush=True)
        del As
    f64 = out["f64"]
    per_iter = f64["lsqr_ms_per_iter"]
    it_bytes = N * M * 8
    out["tol"] = tol
    out["speedup_vs_f64"] = {k: round(f64["solve_ms"] / out[k]["solve_ms"], 3) for k in ("f32", "bf16")}
    out["roofline_iteration"] = {"bound": "hbm", "achieved": round(it_bytes / (per_iter * 1e-3) / 1e9, 2),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(it_bytes / (per_iter * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "alg_bytes_per_iteration": it_bytes,
                                 "note": "one fused pass over A per iteration plus the small step kernels"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of A (a kernel of known traffic, for counter calibration)")
    ap.add_argument("--lsqr-reps", type=int, default=3, help="timed solves per sketch precision (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the row-sharded design is described in DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2508_21189_amd import inputs, libsketch
    torch.cuda.set_device(0)
    print("bench: generating %d x %d float64 input" % (N, M), file=sys.stderr, flush=True)
    A, b, _, nspk = inputs.coherent(N, M, exponent=8.0, seed=DATA_SEED)
    S = libsketch.Sketch("sparsestack", D, N, ZETA, SKETCH_SEED)
    out = torch.empty((D, M), dtype=torch.float64, device="cuda")
    ws = torch.empty(S.workspace_size(0, torch.float64, M), dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        S.apply(A, out=out, ws=ws)
    torch.cuda.synchronize()
    S.timing(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.apply(A, out=out, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = S.timing(2)
    S.timing(0)
    print("bench: timed %d steps" % args.steps, file=sys.stderr, flush=True)

    ms_step = (t1 - t0) * 1e3 / args.steps
    alg_bytes = N * M * 8 + D * M * 8
    value = alg_bytes / (ms_step * 1e-3) / 1e9
    kern_avg_ms = kern_ms / max(1, launches)
    achieved = alg_bytes / (kern_avg_ms * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "coherent least squares: A 4194304x200 f64 (Pareto 1.5 rows, 1%% spikes x1e3, "
                               "kappa(D)=1e8), SparseStack d=800 zeta=8",
                   "n": N, "m": M, "d": D, "zeta": ZETA, "spiked_rows": nspk},
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "ss_rows_kernel<double>", "kernel_avg_ms": round(kern_avg_ms, 4),
                     "alg_bytes_per_launch": alg_bytes},
    }
    if args.copy_probe:
        Acopy = A.clone()  # reads and writes n*m*8 bytes
        torch.cuda.synchronize()
        del Acopy
    if args.lsqr_reps > 0:
        rec["lsqr"] = lsqr_variants(libsketch, torch, A, b, args.lsqr_reps)
    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(A, args.cpu_rows)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
