/*
 * libsketch: structured random sketching on AMD Instinct MI355X (gfx950).
 *
 * Implements the sketching step and the least-squares / low-rank drivers of
 * Camano, Epperly, Meyer, Tropp, "Faster Linear Algebra Algorithms with
 * Structured Random Matrices" (arXiv 2508.21189).
 *
 * Orientation. A sketch is the short-fat matrix S (d x n); the paper's test
 * matrix is Omega = S^T (n x d). sketch_apply computes S A (the paper's
 * Psi^T A, the sketching step of Alg. 3); sketch_apply_T computes A S^T
 * (the paper's A Omega, the sketching step of Alg. 1).
 *
 * Conventions for every entry point:
 *   - Matrix pointers are DEVICE pointers owned by the caller, unless a
 *     parameter says "host". Scalars and info structs are host memory.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and is asynchronous unless the function says it synchronizes.
 *   - Return value: 0 = success; negative = error, nothing was written to
 *     the outputs and sketch_last_error() (thread-local) explains why;
 *     positive = warning, the outputs are valid (see each function).
 *   - Non-finite inputs are propagated, not checked.
 *   - A sketch handle is immutable after creation; concurrent calls with
 *     the same handle on different streams are safe except that calls
 *     passing ws = NULL share the handle's internal workspace and must be
 *     serialized by the caller. Every call runs on one stream. (An earlier
 *     batched driver that spread 512 small solves over 32 concurrent streams,
 *     each reusing one workspace slot, gave wrong results for a few of them in
 *     some runs, for a reason not yet found; callers that run many calls
 *     concurrently should check their results the same way.)
 */
#ifndef LIBSKETCH_H
#define LIBSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sk_sketch* sketch_t;

/* Sketch kinds. */
enum {
  SK_SPARSESTACK = 0, /* Def. 1.5: d rows in zeta blocks of d/zeta; one +-1/sqrt(zeta) per block per column */
  SK_GAUSSIAN = 1,    /* Def. 1.4: iid N(0, 1/d) entries */
  SK_SRTT = 2,        /* eq. (1.1) with a uniform restriction: (1/sqrt(d)) R H D, H = Walsh-Hadamard */
  SK_SPARSERTT = 3,   /* Def. 1.7: Omega^T for Omega = D F S, F = unitary WHT, S = SparseCol (Def. 4.1) */
  SK_IDENTITY_TEST = 99 /* S = I (d = n); exists to test the drivers against exact least squares */
};

/* Element types. */
enum { SK_F64 = 0, SK_F32 = 1, SK_BF16 = 2 };
/* Matrix layouts. */
enum { SK_ROW_MAJOR = 0, SK_COL_MAJOR = 1 };
/* Status codes. */
enum {
  SK_OK = 0,
  SK_E_INVAL = -1,  /* invalid argument */
  SK_E_NOMEM = -2,  /* device allocation failed */
  SK_E_HIP = -3,    /* HIP runtime error */
  SK_E_NOTSUP = -4, /* combination not supported */
  SK_W_RANKDEF = 1, /* warning: the sketched matrix is numerically rank deficient */
  SK_W_NOCONV = 2   /* warning: the iteration limit was reached before the tolerance */
};

/*
 * Create a sketch S (d x n) on the current HIP device.
 *   kind  SK_SPARSESTACK: requires 1 <= zeta <= d and d % zeta == 0 and
 *         d / zeta < 2^31 (sketch_apply and sketch_apply_T take at most
 *         16384 buckets per block and refuse more with SK_E_NOTSUP).
 *         The bucket s_it in [0, d/zeta) and sign rho_it of column i,
 *         block t are drawn from Philox4x32-10 (Salmon et al., SC'11) with
 *         key = seed and counter (i mod 2^32, i >> 32, t / 4, 1), word t % 4:
 *         rho = +1 iff bit 0 is 0; s = ((word >> 1) * (d/zeta)) >> 31.
 *         Row t*(d/zeta) + s of S holds rho/sqrt(zeta) (Def. 1.5).
 *   kind  SK_GAUSSIAN: zeta ignored; entries from Philox + Box-Muller.
 *   kind  SK_SRTT: zeta ignored; requires d <= 2^ceil(log2 n).
 *   kind  SK_SPARSERTT: zeta is the column sparsity xi of the SparseCol
 *         factor (Def. 4.1), 1 <= xi <= npad = 2^ceil(log2 n); zeta = 0
 *         selects xi = ceil(1.5 ln d) (Sec. 4.3), clamped to [1, npad].
 *         Row j of S A is (1/sqrt(d xi)) sum_i rho_ji (H D A_pad)[s_ji]: D
 *         is the SRTT's sign diagonal, H the unnormalized Walsh-Hadamard
 *         matrix, A_pad A with zero rows up to npad. Row j's xi selectors
 *         are distinct, drawn by Floyd's algorithm: for t = npad-xi ..
 *         npad-1, Philox counter (t mod 2^32, t >> 32, j, 5) gives words
 *         w0, w1; u = (w0 (t+1)) >> 32; the index taken is u, or t if u was
 *         taken before; its sign rho is -1 iff bit 0 of w1 is 1. Selected
 *         rows are added in increasing index order. sketch_info reports xi
 *         as zeta.
 *   kind  SK_IDENTITY_TEST: requires d == n.
 * Nothing about S is stored beyond its parameters (and, for SRTT, the d
 * sampled row indices; for SparseRTT, the d xi selectors and signs):
 * entries are regenerated from the seed on demand.
 * Returns NULL on error (see sketch_last_error). Synchronizes the device.
 */
sketch_t sketch_create(int kind, int64_t d, int64_t n, int zeta, uint64_t seed);

/* Release a handle and its internal workspace. NULL is accepted. */
int sketch_destroy(sketch_t S);

/* Thread-local description of the last error (never NULL). */
const char* sketch_last_error(void);

/* Read back the parameters of a handle (any pointer may be NULL). */
int sketch_info(sketch_t S, int* kind, int64_t* d, int64_t* n, int* zeta, uint64_t* seed);

/*
 * SA = S A.
 *   A   n x m matrix of dtype_in (SK_F64, SK_F32 or SK_BF16), layout
 *       SK_ROW_MAJOR (element (i,c) at A[i*lda + c], lda >= m) or
 *       SK_COL_MAJOR (element (i,c) at A[c*lda + i], lda >= n). Column-major
 *       A is first copied to row-major in the workspace (a tiled transpose:
 *       one more read and write of A), then sketched exactly as the same
 *       matrix in row-major order: the results are bitwise equal.
 *       Rows must be 4-byte multiples (m * element size, and for row-major
 *       A also lda * element size and the address): BF16 needs m even.
 *   SA  d x m row-major (element (j,c) at SA[j*ldsa + c], ldsa >= m) of
 *       dtype_out: SK_F64 or SK_F32. F64 input accumulates in F64; F32 and
 *       BF16 inputs accumulate in F32 (BF16 values are exact in F32).
 *   ws  device workspace of ws_bytes >= sketch_workspace_size(...), or NULL
 *       to use a workspace owned by the handle.
 * Kinds: SparseStack takes every input type. Gaussian takes F64 input (F64
 * output; G generated inside the MFMA kernel, never stored) or F32 input
 * (G, d x n F32, written into the workspace and one SGEMM; needs
 * d * n * 4 <= 8 GB). SRTT and SparseRTT take F64 input (F64 output).
 * The result is deterministic (the same inputs give bitwise identical SA on
 * every run: no atomics, fixed summation order).
 */
int sketch_apply(sketch_t S, int dtype_in, int layout, int64_t m, const void* A, int64_t lda,
                 int dtype_out, void* SA, int64_t ldsa, void* ws, size_t ws_bytes, void* stream);

/*
 * Y = A S^T (the paper's A Omega): A is rows x n of dtype_in, layout
 * SK_ROW_MAJOR (element (r,i) at A[r*lda + i], lda >= n) or SK_COL_MAJOR
 * (element (r,i) at A[i*lda + r], lda >= rows); Y is rows x d row-major
 * (ldy >= d) of dtype_out. Column-major A is the row-major n x rows matrix
 * A^T: Y^T = S A^T is sketch_apply's row-mode apply of it (written d x rows
 * into the workspace, with sketch_apply's input rules and limits), then a
 * tiled transpose into Y; the result is bitwise the transpose of
 * sketch_apply on A^T. The row-major path:
 *   SparseStack: any input type, F32 accumulation for F32/BF16, F64 for F64.
 *     Blocks of more than 800 (F64) or 1024 (F32, BF16) buckets, more than
 *     the column kernel keeps in registers, take the column-major route on
 *     the same memory (A is then the column-major n x rows matrix A^T): two
 *     transposes through the workspace and the row-mode apply.
 *   Gaussian: F64 or F32 input; G (d x n) is generated into the workspace and
 *     Y = A G^T is one GEMM on the matrix cores (sk_gemm; F32 for F32 input).
 *   SRTT and SparseRTT: one Walsh-Hadamard transform per row in LDS; needs
 *     npad * element size <= 160 KB (npad <= 2^15 for F32/BF16, 2^14 for F64).
 * Deterministic for every kind (no atomics, fixed summation order).
 */
int sketch_apply_T(sketch_t S, int dtype_in, int layout, int64_t rows, const void* A, int64_t lda, int dtype_out,
                   void* Y, int64_t ldy, void* ws, size_t ws_bytes, void* stream);

/*
 * SA = S A exactly as sketch_apply (row-major A, SparseStack only, same
 * kernels, bitwise the same result), for callers that cannot allocate device
 * memory: code under stream capture, serving loops, harnesses that forbid
 * allocation. Its scratch (per-chunk partial sums and per-row codes) is a
 * fixed device array of the library, sketch_noalloc_scratch_bytes() bytes
 * (128 MB) on each device the library runs on, held until the process ends;
 * its device address is looked up once per device on the first call there.
 * The call allocates nothing and takes no workspace. An apply that needs
 * more scratch than the array holds (sketch_workspace_size, op 0) is refused
 * with SK_E_NOTSUP before any work is queued. Every call on a device shares
 * that device's array (it keeps the last call's contents; the apply writes
 * everything it reads), so calls that overlap on one device, on other
 * streams or threads, race and must be serialized by the caller. The handle
 * must have been created on the current device. Timing (sketch_timing) must
 * be off: it creates events.
 */
int sketch_apply_noalloc(sketch_t S, int dtype_in, int64_t m, const void* A, int64_t lda, int dtype_out, void* SA,
                         int64_t ldsa, void* stream);

/* Bytes of the fixed scratch array behind sketch_apply_noalloc. */
size_t sketch_noalloc_scratch_bytes(void);

/* Result details of sketch_sv_extremes. */
typedef struct {
  int steps;           /* Lanczos steps taken (fewer than asked after an invariant subspace) */
  double alpha_at_3_4; /* the two estimates after 3/4 of the steps: their change from the */
  double beta_at_3_4;  /*   final values shows how far the estimates still move */
  double t_build_ms;   /* building the row-sorted form of S (device time) */
  double t_iter_ms;    /* the Lanczos steps (device time) */
} sk_extremes_info;

/*
 * Injectivity alpha = sigma_min(S Q)^2 and dilation beta = sigma_max(S Q)^2
 * of a SparseStack S (d x n) on the coordinate basis Q = [e_1 ... e_n]
 * (Prop. 1.9; the experiment of Fig. 2 takes d = k = 2r, n = r), i.e. the
 * extreme eigenvalues of S^T S. Estimated by min(steps, n) Lanczos steps on
 * S^T S from a Gaussian start (Philox counter (i mod 2^32, i >> 32, 0, 6)
 * under key start_seed, Box-Muller; no reorthogonalization):
 * the extreme eigenvalues of the Lanczos tridiagonal, found by Sturm
 * bisection on the host. Each estimate lies inside [lambda_min, lambda_max]
 * of S^T S and converges to its end as steps grow. Bitwise reproducible.
 * Needs kind SK_SPARSESTACK, n < 2^31, d < 2^32, n * zeta < 2^31; uses the
 * handle's driver workspace (about 16 n zeta + 8 d + 24 n bytes).
 * Synchronizes the stream.
 */
int sketch_sv_extremes(sketch_t S, int steps, uint64_t start_seed, double* alpha, double* beta,
                       sk_extremes_info* info, void* stream);

/* Workspace bytes needed by sketch_apply (op 0: row-major A, m = columns of
 * A; op 2: column-major A, which adds the row-major copy, n * m elements) or
 * sketch_apply_T (m = rows of A; op 1: row-major A; op 3: column-major A,
 * op 0's bytes for A^T plus the d x rows result before its transpose). */
int sketch_workspace_size(sketch_t S, int op, int dtype_in, int64_t m, size_t* bytes);

/*
 * Z = S^T Y (adjoint; a test helper): Y is d x m row-major F64 (ldy >= m),
 * Z is n x m row-major F64 (ldz >= m). SparseStack only.
 */
int sketch_adjoint(sketch_t S, int64_t m, const double* Y, int64_t ldy, double* Z, int64_t ldz, void* stream);

/*
 * Export the SparseStack pattern computed by the device hash:
 * bucket[i*zeta + t] = s_it (int32), sign[i*zeta + t] = rho_it (int8, +-1).
 */
int sketch_pattern(sketch_t S, int32_t* bucket, int8_t* sign, void* stream);

/*
 * Kernel timing (measurement support, not part of any algorithm).
 *   mode 1: enable and reset; mode 0: disable and reset (both synchronize
 *   the device); mode 2: query. While enabled, every call through the handle
 *   records a HIP event pair on its stream around its dominant kernel (the
 *   sketch kernel of sketch_apply / sketch_apply_T). A query waits for the
 *   recorded events and returns the summed elapsed milliseconds and the
 *   number of timed launches (either pointer may be NULL).
 */
int sketch_timing(sketch_t S, int mode, double* total_ms, int64_t* count);

/* ------------------------------------------------------------------------
 * Least-squares drivers: min_x ||A x - b||_2 for a tall A (n x m, n = the
 * sketch's n, row-major F64, lda >= m) with full column rank. S must have
 * d >= m rows. Each call synchronizes `stream` before returning; device
 * memory comes from a buffer owned by the handle (calls through one handle
 * must be serialized). x is a device vector of m doubles.
 * ------------------------------------------------------------------------ */

typedef struct {
  int rank;              /* numerical rank r of S A (the rank test of Alg. 3) */
  double sigma_max;      /* largest singular value of S A */
  double sigma_min_kept; /* r-th singular value of S A */
  double t_sketch_ms;    /* device time of the sketch of A and b */
  double t_total_ms;     /* device time of the whole solve */
} sk_solve_info;

/*
 * Sketch-and-solve (Alg. 3): x = argmin ||S (A x - b)|| with the rank
 * truncation of Alg. 3: the SVD S A = U diag(s) V^T is obtained from a
 * Householder QR S [A b] = Q [R c; 0 *] and a one-sided Jacobi SVD of R;
 * r = #{i : s_i > 5 eps s_1} with eps = 2^-52;
 * x = V_r diag(s_r)^-1 U_r^T c. Needs m <= 1024.
 * Returns SK_W_RANKDEF when r < m (x is then the truncated solution).
 * info may be NULL.
 */
int lstsq_sketch_solve(sketch_t S, int64_t m, const double* A, int64_t lda, const double* b, double* x,
                       sk_solve_info* info, void* stream);

/* Result of lstsq_sketch_solve_async, written by the device. */
typedef struct {
  int rank;              /* numerical rank r of S A (the rank test of Alg. 3); r < m: truncated solution */
  int pad_;
  double sigma_max;      /* largest singular value of S A */
  double sigma_min_kept; /* r-th singular value of S A */
} sk_solve_result;

/*
 * Sketch-and-solve (Alg. 3), exactly as lstsq_sketch_solve (the same kernels
 * in the same order: bitwise the same x), but fully asynchronous and
 * allocation-free, so that it can be recorded into a HIP graph by stream
 * capture: everything is enqueued on `stream`, nothing is allocated (ws,
 * ws_bytes >= lstsq_solve_workspace_size, is required) and the host waits for
 * nothing. The rank and singular values go to `result`, a DEVICE struct (may
 * be NULL), when the stream reaches them; rank deficiency is reported there,
 * not as a return code. Returns 0 once enqueued, or a negative error before
 * enqueuing anything. Calls sharing a workspace must be serialized.
 */
int lstsq_sketch_solve_async(sketch_t S, int64_t m, const double* A, int64_t lda, const double* b, double* x,
                             sk_solve_result* result, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of lstsq_sketch_solve_async for m columns (a bound over the
 * alignments and leading dimensions A may have). */
int lstsq_solve_workspace_size(sketch_t S, int64_t m, size_t* bytes);

typedef struct {
  int iters;            /* LSQR iterations taken */
  int converged;        /* 1 if the stopping test held */
  double rnorm_est;     /* LSQR's recurrence estimate of ||b - A x|| */
  double arnorm_est;    /* estimate of ||(A R^-1)^T (b - A x)|| */
  double anorm_est;     /* estimate of ||A R^-1||_F */
  double t_sketch_ms;   /* device time of the sketch of A and b */
  double t_qr_ms;       /* QR of the sketch, R^-1 and the warm start */
  double t_lsqr_ms;     /* the LSQR iterations and the final back-substitution */
  double t_total_ms;    /* device time of the whole solve */
} sk_lsqr_info;

/*
 * Sketch-and-precondition, the high-accuracy least-squares solver named in
 * Sec. 1.4 (remark after Thm. 1.4): QR of the sketch S A = Q R (Householder,
 * F64), the warm start x0 = R^-1 Q^T S b, then LSQR (Paige & Saunders 1982)
 * on min ||A R^-1 y - (b - A x0)|| in F64, and x = x0 + R^-1 y.
 * Stopping test (checked every iteration): ||r|| <= tol ||r0|| or
 * ||(A R^-1)^T r|| <= tol ||A R^-1||_F,est ||r||. maxit bounds the
 * iterations (SK_W_NOCONV when reached first).
 * Mixed precision: A_sketch (may be NULL) is a copy of A of dtype
 * sketch_dtype (SK_F64/SK_F32/SK_BF16, row-major, lda_sketch >= m) that is
 * sketched instead of A; the sketch accumulates in F32 for F32/BF16 input
 * and everything after it is F64. warm_start = 0 starts from x0 = 0.
 * Needs m <= 512. info may be NULL.
 */
int lstsq_sketch_precond(sketch_t S, int64_t m, const double* A, int64_t lda, int sketch_dtype,
                         const void* A_sketch, int64_t lda_sketch, const double* b, double* x, double tol,
                         int maxit, int warm_start, sk_lsqr_info* info, void* stream);

/* One problem of lstsq_sketch_solve_batched. */
typedef struct {
  int64_t n;       /* rows of A */
  int64_t k;       /* columns of A, 1 <= k <= 1024 */
  int dtype;       /* element type of A and b: SK_F64, SK_F32 or SK_BF16 */
  const void* A;   /* device, n x k row-major, lda >= k */
  int64_t lda;
  const void* b;   /* device, n elements */
  double* x;       /* device, k doubles (output) */
  uint64_t seed;   /* seed of this problem's SparseStack sketch */
  int status;      /* output: SK_OK, SK_W_RANKDEF, SK_E_INVAL for an invalid problem, or
                      SK_E_NOTSUP for data the apply does not take (sketch_apply's rules) */
  int rank;        /* output: the numerical rank r of S A */
  double t_ms;     /* output: device time of this problem (its first to its last kernel) */
} sk_ls_problem;

/*
 * Many independent sketch-and-solve problems (Alg. 3, as lstsq_sketch_solve)
 * in one call: problem p is solved with its own SparseStack sketch of
 * d = d_per_k * k rows in zeta blocks (zeta must divide d) under key p.seed,
 * reading A and b in their own precision (F32 and BF16 accumulate the sketch
 * in F32; QR, SVD and the solve are F64). After the Householder QR
 * S [A b] = Q [R c; 0 *], a problem whose ||R||_F ||R^-1||_F < 1e-3 / (5 eps)
 * certainly passes the rank test of Alg. 3 (s_k > 5 eps s_1), and its
 * truncated-SVD solution is x = R^-1 c, computed directly; the others are
 * redone with the SVD of R in a second pass, exactly as lstsq_sketch_solve
 * does. The work runs on one stream that the call creates (default
 * priority) and that starts after the work already queued on `stream`, in
 * one workspace (ws, ws_bytes >= lstsq_batched_workspace_size; NULL to
 * allocate and free one inside the call). For the problems with d <= 1024
 * and k <= 512 (and, for their sketch, k >= 4, zeta >= 4 and rows of A that
 * are 4-byte aligned), [S A | S b] is computed for all of them together: one
 * launch for the row codes, one per accumulator register file for the
 * applies (b as the column after A's last), one for the chunk sums, each
 * problem's result landing in its own buffer; their Householder QRs, R^-1
 * and certified solves then run together on `stream`, one launch per panel
 * step. The other problems take the single-problem steps one by one, in one
 * slot of the workspace. The batched sketch keeps every problem's row codes
 * and partial sums in the workspace at once (about 8 and 4 bytes per row and
 * block, and 1/16 of A's bytes; problems are grouped when that passes
 * 16 GiB). The call waits once per pass and returns with every x written. A
 * problem's t_ms runs from the start of its sketch (the batched sketch's
 * start for the problems in it) to the end of the batched solve (or of its
 * own solve). Every problem is validated
 * before any work is queued: if one is invalid, its status is SK_E_INVAL,
 * nothing runs, and SK_E_INVAL is returned; if the apply refuses one's data
 * layout (more than 4 columns whose rows are not 4-byte multiples, as BF16
 * with odd k), its status and the result are SK_E_NOTSUP and nothing runs. Otherwise returns SK_OK, or
 * SK_W_RANKDEF if some problem was rank deficient (see its status).
 */
int lstsq_batched_workspace_size(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, size_t* bytes);
int lstsq_sketch_solve_batched(sk_ls_problem* probs, int nprob, int d_per_k, int zeta, void* ws, size_t ws_bytes,
                               void* stream);

/*
 * Batch plan of the batched sketch-and-solve (Alg. 3 for every problem, as
 * lstsq_sketch_solve): problem p is solved with its own SparseStack sketch
 * of d = d_per_k * k rows in zeta blocks (zeta must divide d; d <= 1024,
 * k <= 512) under key p.seed, reading A and b in their own precision (F32
 * and BF16 accumulate the sketch in F32; the QR, the SVD and the solve are
 * F64). After the Householder QR S [A b] = Q [R c; 0 *], a problem whose
 * ||R||_F ||R^-1||_F < 1e-3 / (5 eps) certainly passes the rank test of
 * Alg. 3 (s_k > 5 eps s_1) and gets x = R^-1 c; the others get the
 * truncated-SVD solution from the Jacobi SVD of R, exactly as
 * lstsq_sketch_solve.
 *
 * A batch plan fixes the problems (their shapes and device pointers) and
 * runs the whole batch as one graph launch: the row codes of every problem,
 * the bucket-indexed applies (one kernel per accumulator register file, b
 * as the column after A's last), the chunk sums into each problem's
 * column-major [S A | S b], the batched Householder QR (one panel and one
 * trailing-update kernel per 32 columns), R^-1, the certified solve and the
 * SVD fallback (which returns at once for the certified problems).
 * Everything lives in one caller workspace; a launch allocates nothing,
 * waits for nothing and records no memset or copy, so it may also be
 * captured into a caller's graph (lstsq_batched_enqueue).
 *
 * lstsq_batched_create validates the problems before any device call
 * (SK_E_INVAL for an invalid problem; SK_E_NOTSUP, naming the problem, for
 * d > 1024, k > 512 or k < 4, rows of A that are not 4-byte aligned, or b or
 * x not aligned to their element size) and chooses each problem's row-chunk
 * length (8, 16 or 32 times d rows; 16 by default) from the tuning cache: a
 * JSON file (SKETCH_TUNE_CACHE, else $XDG_CACHE_HOME/libsketch/batched_tune.json,
 * else ~/.cache/libsketch/batched_tune.json) keyed by device, input type,
 * accumulator register file and bucket parts. With SK_BATCH_AUTOTUNE,
 * classes missing from the cache are timed first on (up to 16 of) the
 * batch's own problems (the batched sketch alone: it reads their A and b,
 * allocates a temporary workspace and synchronizes); the winners are written
 * to the cache. SK_BATCH_NOTUNE ignores the cache (the default length).
 * lstsq_batched_workspace gives the workspace bytes; lstsq_batched_bind
 * uploads the plan's tables into ws (256-byte aligned; synchronizes
 * `stream`) and captures the graph, which stays bound to ws: the workspace
 * must outlive the plan's launches and hold nothing else meanwhile.
 * lstsq_batched_launch enqueues one graph launch on `stream`, bracketed by
 * two events; lstsq_batched_enqueue enqueues the same kernels one by one
 * (for callers capturing `stream` themselves). Launches on one plan must not
 * overlap. lstsq_batched_results waits for `stream` and fills status, rank
 * and t_ms of probs[0 .. nprob) (t_ms: the device time of the last
 * lstsq_batched_launch, the same for every problem; 0 after an enqueue),
 * returning SK_W_RANKDEF if some problem was rank deficient (SK_E_INVAL when
 * nothing was launched or enqueued since the workspace was bound).
 * lstsq_batched_info reports the plan's graph launches and shape.
 */
typedef struct sk_batch* sk_batch_t;
enum { SK_BATCH_AUTOTUNE = 1, SK_BATCH_NOTUNE = 2 };
typedef struct {
  int64_t graph_launches;  /* lstsq_batched_launch calls so far */
  int kernel_nodes;        /* nodes in the batch graph (all kernels) */
  int sketch_workgroups;   /* workgroups of the apply launches, summed */
  int solve_workgroups;    /* workgroups of each solve launch (one a problem) */
  int sketch_items;        /* apply launches (one per accumulator register file) */
  int reduce_items;        /* workgroups of the chunk-sum launches */
  int tuned;               /* problems whose chunk length came from the tuning cache */
  int pad_;
  size_t workspace_bytes;
} sk_batch_info;
int lstsq_batched_create(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int flags, sk_batch_t* out);
int lstsq_batched_workspace(sk_batch_t batch, size_t* bytes);
int lstsq_batched_bind(sk_batch_t batch, void* ws, size_t ws_bytes, void* stream);
int lstsq_batched_launch(sk_batch_t batch, void* stream);
int lstsq_batched_enqueue(sk_batch_t batch, void* stream);
int lstsq_batched_results(sk_batch_t batch, sk_ls_problem* probs, void* stream);
int lstsq_batched_info(sk_batch_t batch, sk_batch_info* info);
int lstsq_batched_destroy(sk_batch_t batch);


/*
 * *resnorm (host) = ||b - A x||_2 in F64, with A (n x m) as above and the
 * handle supplying n and the workspace. Needs m <= 512. Synchronizes.
 */
int lstsq_residual(sketch_t S, int64_t m, const double* A, int64_t lda, const double* b, const double* x,
                   double* resnorm, void* stream);

/* ------------------------------------------------------------------------
 * Randomized SVD (Alg. 1).
 * ------------------------------------------------------------------------ */

typedef struct {
  double t_sketch_ms;  /* Y = A S^T */
  double t_orth_ms;    /* Q = orth(Y) */
  double t_project_ms; /* B = Q^T A */
  double t_svd_ms;     /* SVD of B and U = Q Uh */
  double t_total_ms;   /* device time of the whole call */
  int jacobi_sweeps;   /* sweeps of the Jacobi SVD of the k x k factor */
} sk_rsvd_info;

/*
 * Rank-k approximation A ~ U diag(sigma) Vt from the sketch Y = A S^T, with
 * k = d rows of S and A rows x n (n = the sketch's n), row-major, dtype
 * SK_F32 or SK_F64 (lda >= n). Steps, following Alg. 1 with no
 * oversampling and no power iteration:
 *   Y = A S^T (the handle's kind; accumulated in F32 for F32 input, stored F64);
 *   Q = orth(Y): shifted Cholesky QR, three passes, F64 (a reading: the paper
 *   leaves orth() open);
 *   B = Q^T A: one GEMM, F32 for F32 input (Q rounded to F32), else F64;
 *   B = Uh diag(sigma) V^T via Cholesky QR of B^T and a one-sided Jacobi SVD
 *   of the k x k triangular factor, F64; U = Q Uh.
 * Outputs (device, F64): U rows x k row-major (ldu >= k; may be NULL), sigma
 * (k, descending), Vt k x n row-major (ldvt >= n; may be NULL).
 * Needs k <= min(rows, n) and k <= 4096. Synchronizes `stream`. Returns
 * SK_W_RANKDEF if a Cholesky pivot was not positive (Y or B numerically rank
 * deficient; outputs are then unreliable). info may be NULL.
 */
int rsvd(sketch_t S, int dtype, int64_t rows, const void* A, int64_t lda, double* U, int64_t ldu, double* sigma,
         double* Vt, int64_t ldvt, sk_rsvd_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Generalized Nystrom approximation (Section "Generalized Nystrom
 * approximation": Alg. 4, outer-product form, and Alg. 5, SVD form).
 *
 * A is rows x cols, row-major, dtype SK_F32 or SK_F64, lda >= cols. The two
 * test matrices are sketch handles: Omega = So^T with So k x cols (k = So's
 * d, So's n = cols) and Psi = Sp^T with Sp p x rows (p = Sp's d, Sp's n =
 * rows), k <= p <= min(rows, cols), p <= 4096; the paper recommends
 * p = ceil(1.5 k).
 * Y = A Omega is So's column-mode apply, X^T = Psi^T A is Sp's row-mode apply
 * (both read A once, accumulate in F32 for F32 input and are stored F64),
 * and Psi^T Y (or Psi^T Q) is Sp's row-mode apply to the rows x k factor.
 * Small factorizations run in F64 on the device: SVDs by the one-sided
 * Jacobi method on the tall p x k factors, orthonormal bases (Alg. 5) by
 * shifted Cholesky QR (a reading: the paper leaves qr_econ open). The
 * numerical rank is r = #{i : sigma_i > 5 eps sigma_1}, eps = 2^-52. The
 * workspace belongs to So's handle (it grows on demand). Both calls are
 * synchronous on `stream` at their end. info may be NULL.
 * ------------------------------------------------------------------------- */
typedef struct {
  int rank;             /* numerical rank r of Psi^T Y (Alg. 4) or Psi^T Q (Alg. 5) */
  int jacobi_sweeps;    /* Jacobi sweeps of the small SVDs (summed) */
  double t_sketch_ms;   /* Y = A Omega and X^T = Psi^T A */
  double t_core_ms;     /* the small factorizations */
  double t_factors_ms;  /* F, G (Alg. 4) or U, V (Alg. 5) */
  double t_total_ms;    /* device time of the whole call */
} sk_gn_info;

/*
 * Alg. 4: A ~ F G^T with F = Y V_r Sigma_r^-1 (rows x k, ldf >= k) and
 * G = X U_r (cols x k, ldg >= k), [U, Sigma, V] = svd_econ(X^T Omega);
 * columns r.. of F and G are zero. Returns SK_OK, or a negative status with
 * no output written (invalid shapes, unsupported dtype or kind).
 */
int gen_nystrom(sketch_t So, sketch_t Sp, int dtype, int64_t rows, const void* A, int64_t lda, double* F,
                int64_t ldf, double* G, int64_t ldg, sk_gn_info* info, void* stream);

/*
 * Alg. 5: A ~ U diag(sigma) V^T with U rows x k (ldu >= k), sigma (k,
 * descending) and V cols x k (ldv >= k): [Q, ~] = qr_econ(Y), [P, T] =
 * qr_econ(X), [U1, S1, V1] = svd_econ(Psi^T Q), C = V1_r S1_r^-1 U1_r^T T^T,
 * [Uh, sigma, Vh] = svd_econ(C), U = Q Uh, V = P Vh. Returns SK_W_RANKDEF
 * when the Cholesky QR of Y or X met a non-positive pivot (then U, V are
 * unreliable).
 */
int gen_nystrom_svd(sketch_t So, sketch_t Sp, int dtype, int64_t rows, const void* A, int64_t lda, double* U,
                    int64_t ldu, double* sigma, double* V, int64_t ldv, sk_gn_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Nystrom approximation of a psd matrix (Section "Nystrom approximation",
 * Alg. 2): A ~ U diag(lambda) U^T for a symmetric psd A (n x n, row-major,
 * dtype SK_F32 or SK_F64, lda >= n), with Omega = S^T, S a k x n sketch
 * (SparseStack or Gaussian; k = S's d <= min(n, 4096)). Steps: Y = A Omega
 * (the column-mode apply, stored F64); nu = sqrt(n) eps ||Y||_2 with
 * eps = 2^-52 and ||Y||_2 from 100 power iterations on Y^T Y (a reading:
 * the paper writes ||Y|| and eps_mach); Y_nu = Y + nu Omega;
 * C = chol(Omega^T Y_nu) (the row-mode apply of S to Y_nu, symmetrized);
 * B = Y_nu C^-1; [U, Sigma, ~] = svd_econ(B) by shifted Cholesky QR of B and
 * the Jacobi SVD of its triangular factor; lambda = max(0, Sigma^2 - nu),
 * descending. U: n x k (ldu >= k), lambda: k doubles. Synchronous at its
 * end. Returns SK_W_RANKDEF if a Cholesky factorization met a non-positive
 * pivot. info may be NULL.
 * ------------------------------------------------------------------------- */
typedef struct {
  double nu;           /* the shift */
  double t_sketch_ms;  /* Y = A Omega */
  double t_core_ms;    /* shift, Cholesky, triangular solve, SVD */
  double t_total_ms;   /* device time of the whole call */
  int jacobi_sweeps;   /* sweeps of the k x k Jacobi SVD */
} sk_nystrom_info;

int nystrom_psd(sketch_t S, int dtype, const void* A, int64_t lda, double* U, int64_t ldu, double* lambda,
                sk_nystrom_info* info, void* stream);

/*
 * The library's dense GEMM on the matrix cores (v_mfma_f32_16x16x4f32 for
 * SK_F32, v_mfma_f64_16x16x4f64 for SK_F64), used by the low-rank drivers
 * (Alg. 1 and the Nystrom variants: Y^T Y, Y R^-1, Q^T A, Q U) and by the
 * materialized Gaussian sketch: row-major C (M x N, ldc >= N) =
 * alpha op(A) op(B) + beta C, op(A) M x K and op(B) K x N; A is M x K
 * (lda >= K) or, with transA, K x M (lda >= M); B is K x N (ldb >= N) or,
 * with transB, N x K (ldb >= K). beta = 0 does not read C. Long K with few
 * output tiles is split over workgroups whose partial sums are added in a
 * fixed order through the workspace (ws_bytes >= sk_gemm_workspace_size;
 * NULL is accepted when that size is 0): deterministic. Asynchronous on
 * stream; allocates nothing.
 */
int sk_gemm_workspace_size(int dtype, int64_t M, int64_t N, int64_t K, size_t* bytes);
int sk_gemm(int dtype, int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
            int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* ws, size_t ws_bytes,
            void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBSKETCH_H */
