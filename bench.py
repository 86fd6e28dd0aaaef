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
                tol = 1e-10 (LSQR's least-squares test): SparseStack with the
                sketch read from the float64 A, a float32 copy and a bfloat16
                copy, and the Gaussian and SRTT sketches: wall time per solve
                (median), iterations, the sketch / QR / LSQR split, and the
                LSQR iteration's HBM roofline;
  lsqr_mixed    the same on the 8388608 x 500, kappa = 1e10 system, where the
                float32 / bfloat16 sketch copies pay off, with the Gaussian
                sketch beside them, each sketch kernel's HBM roofline, and
                every solution's errors against the oracle's exact solution
                (Householder TSQR of [A b] on the host);
  rsvd          Alg. 1 on a 65536 x 16384 float32 matrix with known spectrum
                (k = 512) for the four sketch kinds, with the spectral error;
  gen_nystrom,  generalized Nystrom (outer and SVD forms) and psd Nystrom,
  nystrom       SparseStack against Gaussian;
  batched       512 independent float32 least-squares problems solved by
                lstsq_sketch_solve_batched: problems per second and the
                p50 / p99 per-problem device time;
  injectivity   the injectivity / dilation sweep of Fig. 2;
  stream_read_ref  a plain streaming read of A in the same run;
  cpu_baseline  the plain CPU oracle timed per step (sketch, QR, LSQR,
                exact TSQR) on a bounded row sample of the same system on this
                host, with the host's core count and BLAS thread count.
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


APPLY_KERNEL = "ss_idx_kernel<double,200,16>"


def kernel_source_digest():
    p = os.path.join(HERE, "paper_2508_21189_amd", "csrc", "ss_idx.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    p = os.path.join(HERE, "profiles", "ss_idx_coherent_f64_traffic.json")
    try:
        with open(p) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_digest():
        return None
    return t.get("hbm_bytes_per_launch")


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([int(i.get("num_threads", 1)) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        return None


def cpu_baseline(A_cpu, b_cpu, rows):
    """The oracle, as it stands, timed per step on the first `rows` rows of the
    coherent system (the pattern of those rows is the full sketch's): the
    sketch S A (scipy.sparse product, single-threaded, Philox pattern
    included), the Householder QR of S A, sketch-and-precondition LSQR to
    tol 1e-10 on the sample system, and the exact least-squares solve by TSQR
    (LAPACK, all BLAS threads). The reported value is the sketch's rate."""
    import numpy as np

    from oracle import lstsq as ol
    from oracle import sketches as sk
    A = A_cpu[:rows].numpy()
    b = b_cpu[:rows].numpy()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        SA = sk.sparsestack_apply(A, D, ZETA, SKETCH_SEED)
        times.append(time.perf_counter() - t0)
    t_sa = float(np.median(times))
    Sb = sk.sparsestack_apply(b[:, None], D, ZETA, SKETCH_SEED)[:, 0]
    t0 = time.perf_counter()
    ol.householder_qr(np.column_stack([SA, Sb]))
    t_qr = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, info = ol.sketch_and_precondition(A, b, SA, Sb, tol=1e-10, maxit=300)
    t_lsqr = time.perf_counter() - t0
    t0 = time.perf_counter()
    xs, rs, _ = ol.exact_lstsq_tsqr(A, b)
    t_tsqr = time.perf_counter() - t0
    gbs = (rows * M * 8 + D * M * 8) / t_sa / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": len(os.sched_getaffinity(0)),
            "blas_threads": _blas_threads(), "kind": "oracle",
            "sample": "first %d of %d rows of the coherent system; SA via scipy.sparse (single-threaded, Philox "
                      "pattern included), median of 3 runs" % (rows, N),
            "steps_s": {"sketch_SA": round(t_sa, 3), "qr_of_SA": round(t_qr, 4),
                        "sketch_precond_lsqr_tol1e-10": round(t_lsqr, 3), "lsqr_iters": int(info["iters"]),
                        "exact_tsqr": round(t_tsqr, 3)},
            "sample_lsqr_vs_tsqr": {"A_x_minus_xstar_rel_b": float(np.linalg.norm(A @ (x - xs)) /
                                                                    np.linalg.norm(b))}}


def apply_roofline(S, A, torch, transpose=False, reps=5, kernel=None):
    """Average device time of the dominant kernel of S A (or A S^T) over reps
    calls (HIP events on the call's stream) and its rate against the 8 TB/s
    HBM peak, counting A read once and the result written once."""
    dt_out = torch.float64 if A.dtype == torch.float64 else torch.float32
    fn = (lambda: S.apply_T(A, out_dtype=dt_out)) if transpose else (lambda: S.apply(A, out_dtype=dt_out))
    fn()
    torch.cuda.synchronize()
    S.timing(1)
    for _ in range(reps):
        y = fn()
    torch.cuda.synchronize()
    ms, cnt = S.timing(2)
    S.timing(0)
    kms = ms / max(1, cnt)
    alg = A.numel() * A.element_size() + y.numel() * y.element_size()
    gbs = alg / (kms * 1e-3) / 1e9
    return {"kernel_ms": round(kms, 4), "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "alg_bytes": int(alg), "kernel": kernel}


def _solve_stats(libsketch, torch, S, A, b, reps, tol, As=None, keep_x=None):
    """Median wall time (and its split) of reps sketch-and-precondition solves
    (the last solution goes to keep_x[0] when a list is given)."""
    import statistics
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
    it = infos[-1]
    med = lambda key: round(statistics.median(i[key] for i in infos), 3)
    if keep_x is not None:
        keep_x.append(x)
    return {"solve_ms": round(statistics.median(walls), 3), "status": rc, "iters": it["iters"],
            "converged": it["converged"], "t_sketch_ms": med("t_sketch_ms"), "t_qr_ms": med("t_qr_ms"),
            "t_lsqr_ms": med("t_lsqr_ms"),
            "lsqr_ms_per_iter": round(statistics.median(i["t_lsqr_ms"] / max(1, i["iters"]) for i in infos), 4),
            "resnorm": res, "rnorm_est": it["rnorm_est"]}


def lsqr_variants(libsketch, torch, A, b, reps, tol=1e-10):
    """Sketch-and-precondition solves of the coherent system: SparseStack with
    the sketch reading float64 / float32 / bfloat16 copies of A, and the
    Gaussian (matrix-core GEMM), SRTT and SparseRTT (Walsh-Hadamard; SparseRTT
    with the default column sparsity ceil(1.5 ln d)) sketches."""
    out = {}
    variants = (("sparsestack_f64", "sparsestack", ZETA, None), ("sparsestack_f32", "sparsestack", ZETA, torch.float32),
                ("sparsestack_bf16", "sparsestack", ZETA, torch.bfloat16), ("gaussian_f64", "gaussian", 1, None),
                ("srtt_f64", "srtt", 1, None), ("sparsertt_f64", "sparsertt", 0, None))
    for name, kind, zeta, dt in variants:
        S = libsketch.Sketch(kind, D, N, zeta, SKETCH_SEED)
        As = A.to(dt) if dt is not None else None
        out[name] = _solve_stats(libsketch, torch, S, A, b, reps, tol, As)
        print("bench: lsqr %s %.2f ms, %d iterations" % (name, out[name]["solve_ms"], out[name]["iters"]),
              file=sys.stderr, flush=True)
        del As, S
        torch.cuda.empty_cache()
    f64 = out["sparsestack_f64"]
    per_iter = f64["lsqr_ms_per_iter"]
    it_bytes = N * M * 8
    out["tol"] = tol
    out["speedup_vs_sparsestack_f64"] = {k: round(f64["solve_ms"] / out[k]["solve_ms"], 3) for k in out
                                         if isinstance(out[k], dict) and k != "sparsestack_f64"}
    out["roofline_iteration"] = {"bound": "hbm", "achieved": round(it_bytes / (per_iter * 1e-3) / 1e9, 2),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(it_bytes / (per_iter * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "alg_bytes_per_iteration": it_bytes,
                                 "note": "one fused pass over A per iteration plus the small step kernels"}
    return out


def lsqr_mixed(libsketch, inputs, torch, reps, tol=1e-10, exact=True):
    """The mixed-precision system: A 8388608 x 500 iid N(0,1) with column
    scaling kappa(D) = 1e10, SparseStack d = 2000, zeta = 8, the sketch reading
    A itself (float64) or its float32 / bfloat16 copy; QR and LSQR in float64.
    Also: the Gaussian (matrix-core) sketch of the same system, each sketch
    kernel's HBM roofline, and (exact=True) every solution's error against
    the oracle's exact least-squares solution computed on the host."""
    n3, m3, d3 = 1 << 23, 500, 2000
    print("bench: generating %d x %d float64 input" % (n3, m3), file=sys.stderr, flush=True)
    A, b, _ = inputs.scaled_gaussian(n3, m3, exponent=10.0, seed=DATA_SEED + 1)
    out = {"workload": "A %dx%d f64 iid N(0,1), kappa(D)=1e10; SparseStack d=%d zeta=8" % (n3, m3, d3)}
    S = libsketch.Sketch("sparsestack", d3, n3, 8, SKETCH_SEED + 1)
    SA64 = S.apply(A)
    nb = float(b.norm())
    x64 = None
    sols = {}
    out["apply_roofline"] = {}
    # the apply kernel each precision takes at d/zeta = 250 buckets a block:
    # FP64 the bucket-indexed kernel in three bucket parts, FP32 / BF16 the
    # sorted kernel (BF16 rows of 1000 B: 4-byte loads)
    kern = {"f64": "ss_idx_kernel<double,200,16,parts>", "f32": "ss_rows_kernel<float,64,16>",
            "bf16": "ss_rows_kernel<bf16,64,4>"}
    for name, dt in (("f64", None), ("f32", torch.float32), ("bf16", torch.bfloat16)):
        As = A.to(dt) if dt is not None else None
        out["apply_roofline"][name] = apply_roofline(S, As if As is not None else A, torch, kernel=kern[name])
        xs = []
        out[name] = _solve_stats(libsketch, torch, S, A, b, reps, tol, As, keep_x=xs)
        sols[name] = xs[0]
        if dt is None:
            x64 = xs[0]
        else:
            # reported, not gated: how far the low-precision sketch (rounded
            # input and float32 accumulation) is from the float64 sketch, and
            # how far the solution lands from the float64-sketch solution
            SAlo = S.apply(As, out_dtype=torch.float64)
            out[name]["sketch_rel_diff_vs_f64"] = float((SAlo - SA64).norm() / SA64.norm())
            out[name]["A_x_diff_vs_f64_sketch_rel_b"] = float((A @ (xs[0] - x64)).norm()) / nb
            out[name]["x_diff_vs_f64_sketch_rel"] = float((xs[0] - x64).norm() / x64.norm())
            del SAlo
        print("bench: mixed %s %.2f ms, %d iterations" % (name, out[name]["solve_ms"], out[name]["iters"]),
              file=sys.stderr, flush=True)
        del As
        torch.cuda.empty_cache()
    # the Gaussian sketch (matrix-core GEMM, d = 2000) of the same system
    Sg = libsketch.Sketch("gaussian", d3, n3, 1, SKETCH_SEED + 1)
    xs = []
    out["gaussian_f64"] = _solve_stats(libsketch, torch, Sg, A, b, 1, tol, None, keep_x=xs)
    sols["gaussian_f64"] = xs[0]
    print("bench: mixed gaussian %.2f ms, %d iterations" % (out["gaussian_f64"]["solve_ms"],
                                                           out["gaussian_f64"]["iters"]), file=sys.stderr, flush=True)
    del Sg
    out["speedup_vs_f64"] = {k: round(out["f64"]["solve_ms"] / out[k]["solve_ms"], 3)
                             for k in ("f32", "bf16", "gaussian_f64")}
    if exact:
        # the oracle's exact solution x* (Householder TSQR of [A b] on the
        # host, from the same bytes) and each solution's errors against it
        import numpy as np

        from oracle import lstsq as ol
        t0 = time.perf_counter()
        Ah, bh = A.cpu(), b.cpu()
        xstar, rstar, _ = ol.exact_lstsq_tsqr(Ah.numpy(), bh.numpy())
        t_tsqr = time.perf_counter() - t0
        del Ah, bh
        xs_d = torch.from_numpy(np.ascontiguousarray(xstar)).cuda()
        cn = torch.sqrt(torch.stack([torch.sum(A[:, j] ** 2) for j in range(m3)]))  # column norms
        out["vs_oracle_exact"] = {"how": "oracle exact_lstsq_tsqr of [A b] on %d host cores, %.1f s"
                                         % (len(os.sched_getaffinity(0)), t_tsqr)}
        for name, x in sols.items():
            r = float((A @ x - b).norm())
            out["vs_oracle_exact"][name] = {
                "A_x_minus_xstar_rel_b": float((A @ (x - xs_d)).norm()) / nb,
                "resnorm_rel_diff": abs(r - rstar) / rstar,
                "col_scaled_forward_err": float((cn * (x - xs_d)).norm() / (cn * xs_d).norm())}
        print("bench: mixed errors against the oracle's exact solution done (TSQR %.1f s)" % t_tsqr,
              file=sys.stderr, flush=True)
    del A, b, S, SA64, x64, sols
    torch.cuda.empty_cache()
    return out


def rsvd_variants(libsketch, inputs, torch, reps):
    """Alg. 1 on A = U diag(i^-2) V^T (65536 x 16384, float32), k = 512, with
    SparseStack (zeta = 8), SRTT, SparseRTT (default xi) and Gaussian sketches; the spectral error
    ||A - U S V^T||_2 is estimated on the device by 30 power iterations."""
    import statistics
    rows, cols, k = 65536, 16384, 512
    print("bench: generating the %d x %d low-rank matrix" % (rows, cols), file=sys.stderr, flush=True)
    A, sig = inputs.lowrank_decay(rows, cols, seed=DATA_SEED + 2, dtype=torch.float32)
    A64 = A.double()
    out = {"workload": "A %dx%d f32 = U diag(i^-2) V^T, k=%d" % (rows, cols, k), "floor_sigma_k+1": float(sig[k])}
    for kind, zeta in (("sparsestack", 8), ("srtt", 1), ("sparsertt", 0), ("gaussian", 1)):
        S = libsketch.Sketch(kind, k, cols, zeta, SKETCH_SEED + 2)
        if kind == "sparsestack":
            # the column-mode apply Y = A S^T that the RSVD's sketch step runs
            out["apply_roofline_colmode"] = apply_roofline(S, A, torch, transpose=True,
                                                           kernel="ss_cols_idx_kernel<float,64,2>")
        S.rsvd(A)
        walls, infos = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, s, Vt, rc, info = S.rsvd(A)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        x = torch.randn(cols, dtype=torch.float64, device="cuda", generator=g)
        x /= x.norm()
        est = 0.0
        for _ in range(30):
            y = A64 @ x - U @ (s * (Vt @ x))
            z = A64.T @ y - Vt.T @ (s * (U.T @ y))
            nz = z.norm()
            est = float(nz.sqrt())
            x = z / nz
        it = infos[-1]
        out[kind] = {"total_ms": round(statistics.median(walls), 3), "status": rc,
                     "t_sketch_ms": round(it["t_sketch_ms"], 3), "t_orth_ms": round(it["t_orth_ms"], 3),
                     "t_project_ms": round(it["t_project_ms"], 3), "t_svd_ms": round(it["t_svd_ms"], 3),
                     "jacobi_sweeps": it["jacobi_sweeps"], "spectral_error": est}
        print("bench: rsvd %s %.2f ms, error %.3e" % (kind, out[kind]["total_ms"], est), file=sys.stderr, flush=True)
        del U, Vt, S
        torch.cuda.empty_cache()
    del A, A64
    torch.cuda.empty_cache()
    return out


def gn_variants(libsketch, inputs, torch, reps):
    """Generalized Nystrom (Alg. 4 outer form, Alg. 5 SVD form) on the
    131072 x 40000 float32 snapshot stand-in, k = 200, p = ceil(1.5 k) = 300,
    with SparseStack (zeta = 4) and Gaussian test matrices; the relative error
    ||A - A_hat||_F / ||A||_F is computed on the device afterwards."""
    import statistics
    rows, cols, k, p = 131072, 40000, 200, 300
    print("bench: generating the %d x %d snapshot stand-in" % (rows, cols), file=sys.stderr, flush=True)
    A = inputs.snapshots_stand_in(rows, cols, seed=DATA_SEED + 3)
    nA = sum(float(torch.sum(A[r0:r0 + 8192].double() ** 2)) for r0 in range(0, rows, 8192)) ** 0.5

    def rel_err(L, R, s=None):
        # ||A - L diag(s) R^T||_F / ||A||_F in row blocks
        acc = 0.0
        Rs = (R * s[None, :]) if s is not None else R
        for r0 in range(0, rows, 8192):
            E = A[r0:r0 + 8192].double() - L[r0:r0 + 8192] @ Rs.T
            acc += float(torch.sum(E * E))
        return (acc ** 0.5) / nA

    out = {"workload": "snapshot stand-in A %dx%d f32 (rank-300 i^-2 spectrum + noise 1e-6, centred), k=%d p=%d"
                       % (rows, cols, k, p)}
    for kind, zeta in (("sparsestack", 4), ("gaussian", 1)):
        So = libsketch.Sketch(kind, k, cols, zeta, SKETCH_SEED + 3)
        Sp = libsketch.Sketch(kind, p, rows, zeta, SKETCH_SEED + 4)
        res = {}
        for form in ("outer", "svd"):
            r = libsketch.gen_nystrom(So, Sp, A, form=form)
            walls = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = libsketch.gen_nystrom(So, Sp, A, form=form)
                torch.cuda.synchronize()
                walls.append((time.perf_counter() - t0) * 1e3)
            info = r[-1]
            err = rel_err(r[0], r[1]) if form == "outer" else rel_err(r[0], r[2], r[1])
            res[form] = {"total_ms": round(statistics.median(walls), 3), "status": r[-2], "rank": info["rank"],
                         "t_sketch_ms": round(info["t_sketch_ms"], 3), "t_core_ms": round(info["t_core_ms"], 3),
                         "t_factors_ms": round(info["t_factors_ms"], 3), "rel_error_fro": err}
            print("bench: gen_nystrom %s %s %.2f ms, error %.3e" % (kind, form, res[form]["total_ms"], err),
                  file=sys.stderr, flush=True)
            del r
            torch.cuda.empty_cache()
        out[kind] = res
        del So, Sp
    out["speedup_vs_gaussian"] = {f: round(out["gaussian"][f]["total_ms"] / out["sparsestack"][f]["total_ms"], 3)
                                  for f in ("outer", "svd")}
    del A
    torch.cuda.empty_cache()
    return out


def nystrom_variants(libsketch, inputs, torch, reps):
    """Nystrom (Alg. 2) on a 32768 x 32768 float32 psd stand-in (rank 1000,
    i^-2 spectrum, + 1e-6 I), k = 512, SparseStack (zeta = 4) and Gaussian
    Omega; relative error ||A - U diag(lam) U^T||_F / ||A||_F on the device."""
    import statistics
    n, k = 32768, 512
    print("bench: generating the %d x %d psd stand-in" % (n, n), file=sys.stderr, flush=True)
    A = inputs.psd_stand_in(n, seed=DATA_SEED + 4)
    nA = sum(float(torch.sum(A[r0:r0 + 4096].double() ** 2)) for r0 in range(0, n, 4096)) ** 0.5
    out = {"workload": "psd stand-in A %dx%d f32 (rank 1000, i^-2 spectrum, + 1e-6 I), k=%d" % (n, n, k)}
    for kind, zeta in (("sparsestack", 4), ("gaussian", 1)):
        S = libsketch.Sketch(kind, k, n, zeta, SKETCH_SEED + 5)
        r = libsketch.nystrom_psd(S, A)
        walls = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = libsketch.nystrom_psd(S, A)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
        U, lam, rc, info = r
        acc = 0.0
        Ul = U * lam[None, :]
        for r0 in range(0, n, 4096):
            E = A[r0:r0 + 4096].double() - Ul[r0:r0 + 4096] @ U.T
            acc += float(torch.sum(E * E))
        out[kind] = {"total_ms": round(statistics.median(walls), 3), "status": rc,
                     "t_sketch_ms": round(info["t_sketch_ms"], 3), "t_core_ms": round(info["t_core_ms"], 3),
                     "jacobi_sweeps": info["jacobi_sweeps"], "rel_error_fro": acc ** 0.5 / nA}
        print("bench: nystrom %s %.2f ms, error %.3e" % (kind, out[kind]["total_ms"], out[kind]["rel_error_fro"]),
              file=sys.stderr, flush=True)
        del U, lam, Ul, r, S
        torch.cuda.empty_cache()
    out["speedup_vs_gaussian"] = round(out["gaussian"]["total_ms"] / out["sparsestack"]["total_ms"], 3)
    del A
    torch.cuda.empty_cache()
    return out


def batched_solves(libsketch, torch, reps, nprob=512):
    """Many independent least-squares problems (lstsq_sketch_solve_batched):
    n log-uniform in [1e4, 1e6], k uniform in [16, 256], float32 N(0,1)
    entries, b = A x_planted + 1e-4 noise, each problem with its own
    SparseStack (d = 4k, zeta = 4, its own seed). Reports problems per second
    over the whole batch (wall clock, one call, caller workspace) and the
    p50 / p99 of the per-problem device times (from the start of a problem's
    sketch to the end of the batched solve that finishes it)."""
    import numpy as np
    import statistics
    rng = np.random.default_rng(DATA_SEED + 5)
    ns = np.exp(rng.uniform(np.log(1e4), np.log(1e6), nprob)).astype(np.int64)
    ks = rng.integers(16, 257, nprob)
    print("bench: generating %d least-squares problems (%.1f GB float32)" % (nprob, float((ns * ks).sum()) * 4e-9),
          file=sys.stderr, flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(DATA_SEED + 5)
    problems, planted = [], []
    for i in range(nprob):
        n, k = int(ns[i]), int(ks[i])
        A = torch.randn((n, k), generator=g, dtype=torch.float32, device="cuda")
        x = torch.randn(k, generator=g, dtype=torch.float32, device="cuda")
        b = A @ x + 1e-4 * torch.randn(n, generator=g, dtype=torch.float32, device="cuda")
        problems.append((A, b, SKETCH_SEED + 1000 + i))
        planted.append(x.double())
    ws = torch.empty(libsketch.batched_workspace_size(problems), dtype=torch.uint8, device="cuda")
    libsketch.solve_batched(problems[:8], ws=ws)  # warm-up (code objects)
    walls, lat = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, status, ranks, t_ms, rc = libsketch.solve_batched(problems, ws=ws)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        lat = t_ms
    err = [float((x - xp).norm() / xp.norm()) for x, xp in zip(xs, planted)]
    # the same batch through a batch plan: one graph launch per batch (default chunk lengths, then tuned ones
    # from a fresh cache); the plan's workspace and graph are made outside the timed region
    plans = {}
    import tempfile
    with tempfile.TemporaryDirectory() as tdir:
        old_cache = os.environ.get("SKETCH_TUNE_CACHE")
        os.environ["SKETCH_TUNE_CACHE"] = os.path.join(tdir, "tune.json")
        try:
            for name, flags in (("default", libsketch.SK_BATCH_NOTUNE), ("tuned", libsketch.SK_BATCH_AUTOTUNE)):
                plan = libsketch.BatchPlan(problems, 4, 4, flags)
                plan.bind()
                plan.launch()
                plan.results()
                pw = []
                for _ in range(max(1, reps)):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    plan.launch()
                    _, rk, pt, prc = plan.results()
                    pw.append(time.perf_counter() - t0)
                same = all(torch.equal(a, b) for a, b in zip(plan.xs, xs)) if name == "default" else None
                inf = plan.info()
                plans[name] = {"wall_s": round(statistics.median(pw), 4),
                               "problems_per_s": round(nprob / statistics.median(pw), 1),
                               "device_ms": round(pt[0], 3), "status": prc, "kernel_nodes": inf.kernel_nodes,
                               "tuned_problems": inf.tuned}
                if same is not None:
                    plans[name]["bitwise_equal_to_one_call"] = same
                print("bench: batch plan (%s) %.3f s (%.0f problems/s)" % (name, plans[name]["wall_s"],
                                                                          plans[name]["problems_per_s"]),
                      file=sys.stderr, flush=True)
                plan.close()
                del plan
        finally:
            if old_cache is None:
                os.environ.pop("SKETCH_TUNE_CACHE", None)
            else:
                os.environ["SKETCH_TUNE_CACHE"] = old_cache
    lat_sorted = sorted(lat)
    wall = statistics.median(walls)
    out = {"workload": "%d problems, n log-uniform [1e4, 1e6], k uniform [16, 256], f32 N(0,1), d=4k, zeta=4"
           % nprob, "total_gb": round(float((ns * ks).sum()) * 4e-9, 2), "wall_s": round(wall, 4),
           "problems_per_s": round(nprob / wall, 1),
           "p50_ms": round(lat_sorted[len(lat) // 2], 4), "p99_ms": round(lat_sorted[min(len(lat) - 1,
                                                                                          int(0.99 * len(lat)))], 4),
           "latency": "per problem, from the start of its sketch to the end of the batch's factorization and solve",
           "status": rc, "all_full_rank": all(r == int(k) for r, k in zip(ranks, ks)),
           "median_rel_err_vs_planted": statistics.median(err), "plan": plans}
    print("bench: batched %d problems %.3f s (%.0f problems/s), p50 %.3f ms, p99 %.3f ms" %
          (nprob, wall, out["problems_per_s"], out["p50_ms"], out["p99_ms"]), file=sys.stderr, flush=True)
    del problems, planted, ws, xs
    torch.cuda.empty_cache()
    return out


def injectivity_sweep(libsketch, torch, trials, trials_1e7, steps):
    """Fig. 2: injectivity alpha and dilation beta of SparseStack on the
    coordinate basis Q = [e_1 ... e_r], k = 2r, r = 10^2 .. 10^7, zeta in
    {1, 2, 4, 8}; median and 10% / 90% quantiles over trials (sketch seeds),
    each estimate from `steps` Lanczos steps on S^T S (sketch_sv_extremes)."""
    import numpy as np
    out = {"workload": "SparseStack on Q = [e_1..e_r], k = 2r, Lanczos %d steps" % steps,
           "gaussian_limit": {"alpha": (1 - 2 ** -0.5) ** 2, "beta": (1 + 2 ** -0.5) ** 2}, "points": []}
    t_all = time.perf_counter()
    for e in range(2, 8):
        r = 10 ** e
        nt = trials if e < 7 else trials_1e7
        for zeta in (1, 2, 4, 8):
            al, be, t_ms = [], [], []
            for t in range(nt):
                S = libsketch.Sketch("sparsestack", 2 * r, r, zeta, SKETCH_SEED + 100 * e + t)
                a, b, rc, info = libsketch.sv_extremes(S, steps=steps, start_seed=t)
                al.append(a)
                be.append(b)
                t_ms.append(info["t_build_ms"] + info["t_iter_ms"])
                del S
            q = lambda x: [float(v) for v in np.quantile(x, [0.1, 0.5, 0.9])]
            out["points"].append({"r": r, "zeta": zeta, "trials": nt, "alpha_q10_med_q90": q(al),
                                  "beta_q10_med_q90": q(be), "ms_per_estimate": round(float(np.median(t_ms)), 2)})
        print("bench: injectivity r=1e%d done" % e, file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    out["total_s"] = round(time.perf_counter() - t_all, 2)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed-exact", action="store_true",
                    help="skip the host TSQR of the mixed-precision system (errors against the oracle's x*)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of A (a kernel of known traffic, for counter calibration)")
    ap.add_argument("--lsqr-reps", type=int, default=3, help="timed solves per sketch variant (0 = skip)")
    ap.add_argument("--mixed-reps", type=int, default=2,
                    help="timed solves per precision of the 8388608 x 500 mixed-precision system (0 = skip)")
    ap.add_argument("--rsvd-reps", type=int, default=1, help="timed randomized SVDs per sketch kind (0 = skip)")
    ap.add_argument("--gn-reps", type=int, default=1,
                    help="timed generalized Nystrom calls per sketch kind and form (0 = skip)")
    ap.add_argument("--nystrom-reps", type=int, default=1, help="timed Nystrom calls per sketch kind (0 = skip)")
    ap.add_argument("--batched-reps", type=int, default=2,
                    help="timed runs of the 512-problem batched least-squares leg (0 = skip)")
    ap.add_argument("--inj-trials", type=int, default=10,
                    help="trials per point of the injectivity sweep for r <= 1e6 (0 = skip the sweep)")
    ap.add_argument("--inj-trials-1e7", type=int, default=3, help="trials per point at r = 1e7")
    ap.add_argument("--inj-steps", type=int, default=400, help="Lanczos steps per estimate")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (it would shard A by rows, "
              "each GPU sketching its block and one all-reduce summing the d x m partials). Run with --gpus 1.",
              file=sys.stderr)
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
        "config": {"workload": "coherent least squares: A 4194304x200 f64 (Pareto 1.5 rows, 1% spikes x1e3, "
                               "kappa(D)=1e8), SparseStack d=800 zeta=8",
                   "n": N, "m": M, "d": D, "zeta": ZETA, "spiked_rows": nspk},
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": APPLY_KERNEL, "kernel_avg_ms": round(kern_avg_ms, 4),
                     "alg_bytes_per_launch": alg_bytes},
    }
    # context: a plain streaming read of the same bytes in the same run (a
    # column sum of A by torch, i.e. not this library; reported, not used)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cs = torch.empty(M, dtype=torch.float64, device="cuda")
    torch.sum(A, dim=0, out=cs)
    reads = []
    for _ in range(5):
        ev0.record()
        torch.sum(A, dim=0, out=cs)
        ev1.record()
        ev1.synchronize()
        reads.append(ev0.elapsed_time(ev1))
    read_ms = sorted(reads)[len(reads) // 2]
    read_gbs = N * M * 8 / (read_ms * 1e-3) / 1e9
    rec["stream_read_ref"] = {"GBs": round(read_gbs, 1), "frac_of_peak": round(read_gbs / HBM_PEAK_GBS, 4),
                              "apply_frac_of_ref": round(achieved / read_gbs, 4),
                              "how": "torch.sum(A, dim=0) over the same 6.71 GB, median of 5 (HIP events)"}
    del cs
    if args.copy_probe:
        Acopy = A.clone()  # reads and writes n*m*8 bytes
        torch.cuda.synchronize()
        del Acopy
    # the Gaussian comparison sketch (Def. 1.4) of the same A: G generated in
    # the kernel, FP64 matrix cores; its roofline is the FP64 MFMA peak
    Sg = libsketch.Sketch("gaussian", D, N, 1, SKETCH_SEED)
    rg = apply_roofline(Sg, A, torch, reps=3)
    flops = 2.0 * D * N * M
    tfs = flops / (rg["kernel_ms"] * 1e-3) / 1e12
    rec["gaussian_roofline"] = {"bound": "mfma", "achieved": round(tfs, 2), "peak": 78.6, "unit": "TFLOP/s",
                                "frac": round(tfs / 78.6, 4), "kernel": "gauss_rows_kernel (FP64 MFMA, G generated "
                                "in-kernel)", "kernel_avg_ms": rg["kernel_ms"], "flops_per_launch": flops}
    del Sg
    if args.lsqr_reps > 0:
        rec["lsqr"] = lsqr_variants(libsketch, torch, A, b, args.lsqr_reps)
    cpu_sample = (A[:args.cpu_rows].cpu(), b[:args.cpu_rows].cpu()) if not args.no_cpu else None
    del A, b, out, ws, S
    torch.cuda.empty_cache()
    if args.mixed_reps > 0:
        rec["lsqr_mixed"] = lsqr_mixed(libsketch, inputs, torch, args.mixed_reps, exact=not args.no_mixed_exact)
    if args.rsvd_reps > 0:
        rec["rsvd"] = rsvd_variants(libsketch, inputs, torch, args.rsvd_reps)
    if args.gn_reps > 0:
        rec["gen_nystrom"] = gn_variants(libsketch, inputs, torch, args.gn_reps)
    if args.nystrom_reps > 0:
        rec["nystrom"] = nystrom_variants(libsketch, inputs, torch, args.nystrom_reps)
    if args.batched_reps > 0:
        rec["batched"] = batched_solves(libsketch, torch, args.batched_reps)
    if args.inj_trials > 0:
        rec["injectivity"] = injectivity_sweep(libsketch, torch, args.inj_trials, max(1, args.inj_trials_1e7),
                                               args.inj_steps)
    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(cpu_sample[0], cpu_sample[1], args.cpu_rows)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
