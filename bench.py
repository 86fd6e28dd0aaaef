#!/usr/bin/env python3
"""Benchmark of the SparseStack sketch on MI355X (one GPU).

Workload (the coherent least-squares configuration): A is 4,194,304 x 200
float64 with Pareto(1.5) row factors, 1% of rows spiked x1e3 and column
scaling with condition number 1e8; S is a SparseStack with d = 800 rows in
zeta = 8 blocks. A step is one SA = S A (sketch kernel + partial reduction)
with A resident in HBM. The reported value is the whole step's algorithmic
throughput: (n*m*8 + d*m*8) bytes / step time.

The JSON line also carries
  roofline      the sketch kernel's own average duration (HIP events on its
                stream), as a fraction of the 8 TB/s HBM peak;
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
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
    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(A, args.cpu_rows)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
