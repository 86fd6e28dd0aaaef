// Least-squares drivers on top of the sketch apply:
//   * lstsq_sketch_solve      sketch-and-solve (Alg. 3): QR of [S A | S b],
//                             SVD of the triangular factor, truncated solve;
//   * lstsq_sketch_precond    sketch-and-precondition: QR of the sketch,
//                             warm start R^-1 Q^T S b, LSQR on A R^-1 in FP64;
//   * lstsq_residual          ||b - A x|| in FP64 (one fused pass).
// All device memory comes from one handle-owned buffer carved per call.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "sk_dense.hpp"
#include "sk_drivers.hpp"
#include "sk_gauss.hpp"
#include "sk_launch.hpp"
#include "sk_lowrank.hpp"
#include "sk_lsqr.hpp"
#include "sk_srtt.hpp"

namespace sk {

namespace {

// Bump allocator over a device buffer (sizes only when base is null).
struct Carver {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + std::max<size_t>(1, count) * sizeof(T);
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

int driver_workspace(sk_sketch* S, size_t bytes, char** out, hipStream_t st) {
  const int rc = grow_buffer(&S->dws, &S->dws_bytes, bytes, st);
  if (rc != SK_OK) return rc;
  if (!S->h_pinned) SK_HIP(hipHostMalloc(&S->h_pinned, 4096, hipHostMallocDefault));
  *out = static_cast<char*>(S->dws);
  return SK_OK;
}

// Event pairs marking the phases of one driver call.
struct Phases {
  hipEvent_t ev[6] = {};
  int n = 0;
  hipStream_t st;
  explicit Phases(hipStream_t s, bool enabled = true) : st(s) {
    if (!enabled) n = 6;  // no events (stream capture, no host involvement)
  }
  int mark() {
    if (n >= 6) return SK_OK;
    SK_HIP(hipEventCreate(&ev[n]));
    SK_HIP(hipEventRecord(ev[n], st));
    ++n;
    return SK_OK;
  }
  double ms(int a, int b) const {
    float t = 0;
    if (a < n && b < n && hipEventElapsedTime(&t, ev[a], ev[b]) == hipSuccess) return t;
    return 0.0;
  }
  ~Phases() {
    for (int i = 0; i < n; ++i)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
  }
};

// Two events without timing, for the queued stopping tests of LSQR.
struct EventPair {
  hipEvent_t e[2] = {};
  int create() {
    for (auto& x : e) SK_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    return SK_OK;
  }
  ~EventPair() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

#define SK_TRY(expr)            \
  do {                          \
    int _rc = (expr);           \
    if (_rc < 0) return _rc;    \
  } while (0)

struct SketchBufs {
  double* SA;
  double* Sb;
  void* aws;
  size_t aws_bytes;
  double* W;
  double* tau;
  double* Tbuf;
  double* R;
  double* c;
};

// b is of type dtb (F64 unless a batched problem brings F32 or BF16).
int sketch_bufs(Carver& cv, const sk_sketch* S, int k, int dts, const void* As, int64_t ldas, const void* b,
                SketchBufs* B, int dtb = SK_F64) {
  size_t wa = 0, wb = 0;
  if (S->kind == SK_GAUSSIAN || trig_kind(S->kind)) {
    if (dts != SK_F64 || dtb != SK_F64) {
      set_error("the Gaussian, SRTT and SparseRTT sketches read F64 only");
      return SK_E_NOTSUP;
    }
    // one pass over [A | b]
    wa = S->kind == SK_GAUSSIAN ? gauss_workspace(S, k + 1) : srtt_workspace(S, k + 1);
  } else {
    SK_TRY(apply_workspace_for(S, dts, k, As, ldas, &wa));
    SK_TRY(apply_workspace_for(S, dtb, 1, b, 1, &wb));
  }
  const int64_t d = S->d;
  B->SA = cv.take<double>((size_t)d * k);
  B->Sb = cv.take<double>((size_t)d);
  B->aws_bytes = std::max(wa, wb);
  B->aws = cv.take<char>(B->aws_bytes);
  B->W = cv.take<double>((size_t)d * (k + 1));
  B->tau = cv.take<double>((size_t)k);
  B->Tbuf = cv.take<double>(qr_tbuf_doubles(k));
  B->R = cv.take<double>((size_t)k * k);
  B->c = cv.take<double>((size_t)k);
  return SK_OK;
}

// S A (any input precision, F64 result), S b, and the Householder QR of
// [S A | S b]: R (k x k) and c = (Q^T S b)[0:k].
int sketch_and_factor(sk_sketch* S, int k, int dts, const void* As, int64_t ldas, const void* b, const SketchBufs& B,
                      Phases& ph, hipStream_t st, int dtb = SK_F64) {
  const int64_t d = S->d;
  if (S->kind == SK_GAUSSIAN) {
    SK_TRY(launch_gauss_rows(S, k, (const double*)As, ldas, (const double*)b, B.SA, k, B.Sb, B.aws, B.aws_bytes, st));
  } else if (trig_kind(S->kind)) {
    SK_TRY(launch_srtt_rows(S, k, (const double*)As, ldas, (const double*)b, B.SA, k, B.Sb, B.aws, B.aws_bytes, st));
  } else {
    SK_TRY(apply_dispatch(S, dts, k, As, ldas, SK_F64, B.SA, k, B.aws, B.aws_bytes, st));
    SK_TRY(apply_dispatch(S, dtb, 1, b, 1, SK_F64, B.Sb, 1, B.aws, B.aws_bytes, st));
  }
  SK_TRY(ph.mark());
  SK_TRY(launch_to_columns(B.SA, k, B.Sb, d, k, B.W, d, st));
  SK_TRY(qr_columns(B.W, d, d, k, 1, B.tau, B.Tbuf, st));
  SK_TRY(launch_extract_r(B.W, d, k, 1, B.R, B.c, st));
  return SK_OK;
}

bool dtype_ok(int dt) { return dt == SK_F64 || dt == SK_F32 || dt == SK_BF16; }

// ---- batched sketch-and-solve
bool batched_problem_valid(const sk_ls_problem& p, int d_per_k, int zeta) {
  if (p.n < 1 || p.k < 1 || p.k > 1024 || p.lda < p.k || !p.A || !p.b || !p.x || !dtype_ok(p.dtype)) return false;
  const int64_t d = (int64_t)d_per_k * p.k;
  return d >= p.k && d % zeta == 0;
}

// Problem p's SparseStack as a description that owns no memory: every buffer
// its kernels use is carved from the batch workspace.
void batched_sketch(const sk_ls_problem& p, int d_per_k, int zeta, int device, sk_sketch* W) {
  W->kind = SK_SPARSESTACK;
  W->d = (int64_t)d_per_k * p.k;
  W->n = p.n;
  W->zeta = zeta;
  W->nb = W->d / zeta;
  W->seed = p.seed;
  W->k0 = (uint32_t)p.seed;
  W->k1 = (uint32_t)(p.seed >> 32);
  W->device = device;
}

struct SolveBufs {
  SketchBufs B;
  double *U, *V, *sv, *work, *z;
};

int batched_bufs(Carver& cv, const sk_sketch* W, const sk_ls_problem& p, SolveBufs* X) {
  const int k = (int)p.k;
  SK_TRY(sketch_bufs(cv, W, k, p.dtype, p.A, p.lda, p.b, &X->B, p.dtype));
  X->U = cv.take<double>((size_t)k * k);
  X->V = cv.take<double>((size_t)k * k);
  X->sv = cv.take<double>((size_t)k);
  X->work = cv.take<double>((size_t)2 * k * k);
  X->z = cv.take<double>((size_t)k);
  return SK_OK;
}

// The problems' sketches run back to back on one stream (each apply fills
// the chip by itself), with one workspace slot. Spreading them over several
// concurrent streams, each with a slot reused by its problems in turn, gave
// wrong solutions for one to five problems of a 512-problem batch (k = 16..256)
// in some runs with 32 streams, and a GPU memory fault with 4; the cause has
// not been found, and that arrangement is not used.
int batch_streams(int nprob) { return std::min(nprob, 1); }

// Problems whose factorization runs in the batched launches (all problems
// of a batch at once: d <= 1024, the 32-column register panel; k <= 512,
// the blocked inverse); the others take the per-problem steps on their
// stream.
bool batch_factored(const sk_ls_problem& p, int d_per_k) {
  return (int64_t)d_per_k * p.k <= 1024 && p.k <= 512;
}

// Buffers of a batch-factored problem, live from its sketch to the batched
// solve: W = [S A | S b] (d x (k + 1), column-major), tau, T, R, c, X = R^-1
// and X^T.
struct FactorBufs {
  double *W, *tau, *T, *R, *c, *X, *XT;
};
void factor_bufs(Carver& cv, int64_t d, int k, FactorBufs* F) {
  F->W = cv.take<double>((size_t)d * (k + 1));
  F->tau = cv.take<double>((size_t)k);
  F->T = cv.take<double>(qr_tbuf_doubles(k));
  F->R = cv.take<double>((size_t)k * k);
  F->c = cv.take<double>((size_t)k);
  F->X = cv.take<double>((size_t)k * k);
  F->XT = cv.take<double>((size_t)k * k);
}

// Batch-factored problems whose sketch [S A | S b] also runs in the batched
// launches (the bucket-indexed kernels with b as an extra column: k >= 4,
// zeta >= 4, 4-byte aligned rows); the others are sketched one by one.
bool batch_sketched(const sk_ls_problem& p, const sk_sketch* W, int d_per_k) {
  return batch_factored(p, d_per_k) && idx_batch_fits(W, p.dtype, p.k, p.A, p.lda);
}

// Workspace layout: the rank of every problem (nprob ints); the table of the
// batch-factored problems (QrBatch entries) and their factor buffers; the
// area of the batched sketches (tables, row codes, partial sums); then one
// slot per stream holding the buffers of one problem's sketch (and of a
// whole problem for the per-problem path), reused by the problems of that
// stream in turn (they run in stream order).
struct BatchLayout {
  size_t ranks_bytes, table_off, factors_off, bsk_off, bsk_bytes, slots_off, slot_bytes, total;
  std::vector<size_t> factor_at;  // offset of each problem's factor buffers (batch-factored ones)
  std::vector<char> sketched;     // problems in the batched sketch
  std::vector<sk_sketch> sks;     // every problem's sketch description
  int n_factored = 0;
};
// On failure *bad is the problem the apply refused (its data layout).
int batched_layout(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int device, BatchLayout* L,
                   int* bad = nullptr) {
  size_t mx = 0;
  L->sks.assign((size_t)nprob, sk_sketch{});
  L->sketched.assign((size_t)nprob, 0);
  for (int i = 0; i < nprob; ++i) {
    sk_sketch& W = L->sks[i];
    batched_sketch(probs[i], d_per_k, zeta, device, &W);
    L->sketched[i] = batch_sketched(probs[i], &W, d_per_k) ? 1 : 0;
    // (every problem may need the slot: one that the full-rank certificate
    // rejects is redone on the per-problem path)
    Carver cv;
    SolveBufs X;
    const int rc = batched_bufs(cv, &W, probs[i], &X);
    if (rc < 0) {
      if (bad) *bad = i;
      return rc;
    }
    mx = std::max(mx, cv.off);
  }
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  L->ranks_bytes = al((size_t)nprob * sizeof(int));
  L->n_factored = 0;
  for (int i = 0; i < nprob; ++i) L->n_factored += batch_factored(probs[i], d_per_k) ? 1 : 0;
  L->table_off = L->ranks_bytes;
  L->factors_off = al(L->table_off + sizeof(QrBatch) * (size_t)std::max(1, L->n_factored));
  Carver fc;
  L->factor_at.assign((size_t)nprob, 0);
  std::vector<IdxBatchJob> jobs;
  for (int i = 0; i < nprob; ++i) {
    if (!batch_factored(probs[i], d_per_k)) continue;
    L->factor_at[i] = al(fc.off);
    FactorBufs F;
    factor_bufs(fc, (int64_t)d_per_k * probs[i].k, (int)probs[i].k, &F);
    if (L->sketched[i])
      jobs.push_back(
          IdxBatchJob{&L->sks[i], probs[i].dtype, probs[i].k, probs[i].A, probs[i].lda, probs[i].b, nullptr, 0});
  }
  L->bsk_off = al(L->factors_off + fc.off);
  L->bsk_bytes = 0;
  if (!jobs.empty()) {
    const int rc = idx_batch_workspace(jobs.data(), (int)jobs.size(), &L->bsk_bytes);
    if (rc < 0) return rc;
  }
  L->slots_off = al(L->bsk_off + L->bsk_bytes);
  L->slot_bytes = al(mx);
  L->total = L->slots_off + (size_t)batch_streams(nprob) * L->slot_bytes;
  return SK_OK;
}

int batched_check(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, const char* who) {
  if (!probs || nprob < 1 || d_per_k < 1 || zeta < 1) {
    set_error(std::string(who) + ": need problems, nprob >= 1, d_per_k >= 1 and zeta >= 1");
    return SK_E_INVAL;
  }
  for (int i = 0; i < nprob; ++i) {
    if (!batched_problem_valid(probs[i], d_per_k, zeta)) {
      set_error(std::string(who) + ": problem " + std::to_string(i) +
                " is invalid (need n >= 1, 1 <= k <= 1024, lda >= k, pointers, a dtype, zeta | d_per_k * k)");
      return SK_E_INVAL;
    }
  }
  return SK_OK;
}

}  // namespace

void drivers_release(sk_sketch* S) {
  blas_release(S);
  if (S->dws) (void)hipFreeAsync(S->dws, nullptr);
  if (S->h_pinned) (void)hipHostFree(S->h_pinned);
  S->dws = nullptr;
  S->h_pinned = nullptr;
  S->dws_bytes = 0;
}

}  // namespace sk

using namespace sk;

extern "C" {

int lstsq_sketch_solve(sketch_t S, int64_t m, const double* A, int64_t lda, const double* b, double* x,
                       sk_solve_info* info, void* stream) {
  if (!S || !A || !b || !x || m < 1 || lda < m) {
    set_error("lstsq_sketch_solve: invalid argument");
    return SK_E_INVAL;
  }
  if (S->d < m || m > 1024) {
    set_error("lstsq_sketch_solve: need m <= d and m <= 1024");
    return SK_E_INVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int k = (int)m;
  Carver cv;
  SketchBufs B;
  SK_TRY(sketch_bufs(cv, S, k, SK_F64, A, lda, b, &B));
  double* U = cv.take<double>((size_t)k * k);
  double* V = cv.take<double>((size_t)k * k);
  double* sv = cv.take<double>((size_t)k);
  double* work = cv.take<double>((size_t)2 * k * k);
  double* z = cv.take<double>((size_t)k);
  int* rank = cv.take<int>(1);
  char* base = nullptr;
  SK_TRY(driver_workspace(S, cv.off, &base, st));
  Carver cv2{base, 0};
  SK_TRY(sketch_bufs(cv2, S, k, SK_F64, A, lda, b, &B));
  U = cv2.take<double>((size_t)k * k);
  V = cv2.take<double>((size_t)k * k);
  sv = cv2.take<double>((size_t)k);
  work = cv2.take<double>((size_t)2 * k * k);
  z = cv2.take<double>((size_t)k);
  rank = cv2.take<int>(1);

  Phases ph(st);
  SK_TRY(ph.mark());
  SK_TRY(sketch_and_factor(S, k, SK_F64, A, lda, b, B, ph, st));
  SK_TRY(launch_jacobi_svd(B.R, k, U, sv, V, work, st));
  SK_TRY(launch_svd_solve(U, sv, V, B.c, k, std::ldexp(1.0, -52), x, z, rank, st));
  SK_TRY(ph.mark());
  char* hp = static_cast<char*>(S->h_pinned);
  SK_HIP(hipMemcpyAsync(hp, rank, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(hp + 8, sv, sizeof(double), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  const int r = *reinterpret_cast<int*>(hp);
  if (r > 0) {
    SK_HIP(hipMemcpyAsync(hp + 16, sv + (r - 1), sizeof(double), hipMemcpyDeviceToHost, st));
    SK_HIP(hipStreamSynchronize(st));
  }
  if (info) {
    info->rank = r;
    info->sigma_max = *reinterpret_cast<double*>(hp + 8);
    info->sigma_min_kept = r > 0 ? *reinterpret_cast<double*>(hp + 16) : 0.0;
    info->t_sketch_ms = ph.ms(0, 1);
    info->t_total_ms = ph.ms(0, 2);
  }
  return r < k ? SK_W_RANKDEF : SK_OK;
}

// rank, sigma_1 and sigma_r of a solve into the caller's device struct
__global__ void solve_result_kernel(const int* rank, const double* sv, sk_solve_result* out) {
  const int r = *rank;
  out->rank = r;
  out->sigma_max = sv[0];
  out->sigma_min_kept = r > 0 ? sv[r - 1] : 0.0;
}

// Workspace of one sketch-and-solve (Alg. 3) for an A at this address and
// leading dimension (the apply's plan depends on the alignment).
static size_t solve_ws_bytes(sk_sketch* S, int k, const void* A, int64_t lda, const void* b, int* rc) {
  Carver cv;
  SketchBufs B;
  *rc = sketch_bufs(cv, S, k, SK_F64, A, lda, b, &B);
  cv.take<double>((size_t)k * k);
  cv.take<double>((size_t)k * k);
  cv.take<double>((size_t)k);
  cv.take<double>((size_t)2 * k * k);
  cv.take<double>((size_t)k);
  cv.take<int>(1);
  return cv.off + 256;  // (+256: the caller's buffer is carved from a 256-byte aligned start)
}

int lstsq_solve_workspace_size(sketch_t S, int64_t m, size_t* bytes) {
  if (!S || !bytes || m < 1 || S->d < m || m > 1024) {
    set_error("lstsq_solve_workspace_size: invalid argument (need m <= d, m <= 1024)");
    return SK_E_INVAL;
  }
  // the bound over the alignments and leading dimensions an A may have
  size_t best = 0;
  const uintptr_t addrs[2] = {256, 8};
  for (uintptr_t ad : addrs)
    for (int64_t ld : {m, m + 1}) {
      int rc = SK_OK;
      const size_t need = solve_ws_bytes(S, (int)m, (const void*)ad, ld, (const void*)ad, &rc);
      if (rc < 0) return rc;
      best = std::max(best, need);
    }
  *bytes = best;
  return SK_OK;
}

int lstsq_sketch_solve_async(sketch_t S, int64_t m, const double* A, int64_t lda, const double* b, double* x,
                             sk_solve_result* result, void* ws, size_t ws_bytes, void* stream) {
  if (!S || !A || !b || !x || !ws || m < 1 || lda < m) {
    set_error("lstsq_sketch_solve_async: invalid argument (a workspace is required)");
    return SK_E_INVAL;
  }
  if (S->d < m || m > 1024) {
    set_error("lstsq_sketch_solve_async: need m <= d and m <= 1024");
    return SK_E_INVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int k = (int)m;
  int rc = SK_OK;
  const size_t need = solve_ws_bytes(S, k, A, lda, b, &rc);
  if (rc < 0) return rc;
  if (ws_bytes < need) {
    set_error("lstsq_sketch_solve_async: workspace too small (see lstsq_solve_workspace_size)");
    return SK_E_INVAL;
  }
  Carver cv{(char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255), 0};
  SketchBufs B;
  SK_TRY(sketch_bufs(cv, S, k, SK_F64, A, lda, b, &B));
  double* U = cv.take<double>((size_t)k * k);
  double* V = cv.take<double>((size_t)k * k);
  double* sv = cv.take<double>((size_t)k);
  double* work = cv.take<double>((size_t)2 * k * k);
  double* z = cv.take<double>((size_t)k);
  int* rank = cv.take<int>(1);
  Phases ph(st, false);
  SK_TRY(sketch_and_factor(S, k, SK_F64, A, lda, b, B, ph, st));
  SK_TRY(launch_jacobi_svd(B.R, k, U, sv, V, work, st));
  SK_TRY(launch_svd_solve(U, sv, V, B.c, k, std::ldexp(1.0, -52), x, z, rank, st));
  if (result) {
    hipLaunchKernelGGL(solve_result_kernel, dim3(1), dim3(1), 0, st, rank, sv, result);
    SK_HIP(hipGetLastError());
  }
  return SK_OK;
}

int lstsq_batched_workspace_size(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, size_t* bytes) {
  if (!bytes) {
    set_error("lstsq_batched_workspace_size: null output");
    return SK_E_INVAL;
  }
  SK_TRY(batched_check(probs, nprob, d_per_k, zeta, "lstsq_batched_workspace_size"));
  int device = 0;
  SK_HIP(hipGetDevice(&device));
  BatchLayout L;
  SK_TRY(batched_layout(probs, nprob, d_per_k, zeta, device, &L));
  *bytes = L.total;
  return SK_OK;
}

int lstsq_sketch_solve_batched(sk_ls_problem* probs, int nprob, int d_per_k, int zeta, void* ws, size_t ws_bytes,
                               void* stream) {
  if (probs && nprob > 0) {
    for (int i = 0; i < nprob; ++i) {
      probs[i].status = batched_problem_valid(probs[i], d_per_k, zeta) ? SK_OK : SK_E_INVAL;
      probs[i].rank = 0;
      probs[i].t_ms = 0.0;
    }
  }
  SK_TRY(batched_check(probs, nprob, d_per_k, zeta, "lstsq_sketch_solve_batched"));
  int device = 0;
  SK_HIP(hipGetDevice(&device));
  BatchLayout L;
  int bad = -1;
  const int lrc = batched_layout(probs, nprob, d_per_k, zeta, device, &L, &bad);
  if (lrc < 0) {
    if (bad >= 0) probs[bad].status = lrc;
    return lrc;
  }
  const size_t need = L.total;
  if (ws && ws_bytes < need) {
    set_error("lstsq_sketch_solve_batched: workspace too small (see lstsq_batched_workspace_size)");
    return SK_E_INVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  void* own = nullptr;
  if (!ws) SK_HIP(hipMalloc(&own, need));
  char* base = static_cast<char*>(ws ? ws : own);
  std::vector<hipEvent_t> ev((size_t)2 * nprob, nullptr);
  const int NS = batch_streams(nprob);
  std::vector<hipStream_t> ss((size_t)NS, nullptr);
  hipEvent_t ready = nullptr;
  int rc = SK_OK;
  // start and end events of the problems sketched one by one (made when
  // first needed: the problems of the batched sketch share one start)
  auto event = [&](int j) -> hipEvent_t {
    if (!ev[j] && hipEventCreate(&ev[j]) != hipSuccess) {
      set_error("lstsq_sketch_solve_batched: hipEventCreate failed");
      ev[j] = nullptr;
    }
    return ev[j];
  };
  // the problems' streams start after the work already queued on `stream`
  if (rc == SK_OK && (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
                      hipEventRecord(ready, st) != hipSuccess)) {
    set_error("lstsq_sketch_solve_batched: event on the caller's stream failed");
    rc = SK_E_HIP;
  }
  for (int j = 0; j < NS && rc == SK_OK; ++j) {
    if (hipStreamCreateWithFlags(&ss[j], hipStreamNonBlocking) != hipSuccess ||
        hipStreamWaitEvent(ss[j], ready, 0) != hipSuccess) {
      set_error("lstsq_sketch_solve_batched: stream creation failed");
      rc = SK_E_HIP;
    }
  }
  int* ranks = reinterpret_cast<int*>(base);
  QrBatch* table = reinterpret_cast<QrBatch*>(base + L.table_off);
  std::vector<QrBatch> host_table;
  int kmax = 0;
  hipEvent_t batch_done = nullptr;
  std::vector<hipEvent_t> joined((size_t)NS, nullptr);
  const double eps = std::ldexp(1.0, -52);
  // Pass 1: the sketches on the streams; the Householder QR, R^-1 and, where
  // the rank test of Alg. 3 is certain to pass, x = R^-1 c, for all the
  // batch-factored problems at once on the caller's stream (the others take
  // these steps on their own stream). Pass 2 redoes the problems it could
  // not certify with the SVD of R (the same steps as lstsq_sketch_solve).
  std::vector<int> h((size_t)nprob, 0);
  std::vector<char> redo((size_t)nprob, 0);
  std::vector<double> t_ms((size_t)nprob, 0.0);
  // the batched sketches' host tables, alive until the stream has run them
  IdxBatchProgram stage;
  hipEvent_t bsk_start = nullptr;
  for (int pass = 0; pass < 2 && rc == SK_OK; ++pass) {
    bool queued = false;
    if (pass == 0) {
      // the batched sketches first: [S A | S b] of every such problem
      // straight into its factor buffer W
      std::vector<IdxBatchJob> jobs;
      for (int i = 0; i < nprob; ++i) {
        if (!L.sketched[i]) continue;
        const sk_ls_problem& p = probs[i];
        Carver fc{base, L.factors_off + L.factor_at[i]};
        FactorBufs F;
        factor_bufs(fc, L.sks[i].d, (int)p.k, &F);
        jobs.push_back(IdxBatchJob{&L.sks[i], p.dtype, p.k, p.A, p.lda, p.b, F.W, 0});
        host_table.push_back(
            QrBatch{F.W, L.sks[i].d, L.sks[i].d, (int)p.k, 0, F.tau, F.T, F.R, F.c, F.X, F.XT, p.x, ranks + i});
        kmax = std::max(kmax, (int)p.k);
      }
      if (!jobs.empty()) {
        if (hipEventCreate(&bsk_start) != hipSuccess || hipEventRecord(bsk_start, ss[0]) != hipSuccess) {
          set_error("lstsq_sketch_solve_batched: event on the caller's stream failed");
          rc = SK_E_HIP;
        }
        if (rc == SK_OK)
          rc = launch_idx_batch(jobs.data(), (int)jobs.size(), base + L.bsk_off, L.bsk_bytes, &stage, ss[0]);
        queued = rc == SK_OK;
      }
    }
    for (int i = 0; i < nprob && rc == SK_OK; ++i) {
      if (pass == 1 && !redo[i]) continue;
      if (pass == 0 && L.sketched[i]) continue;
      const sk_ls_problem& p = probs[i];
      const int k = (int)p.k;
      const int slot = i % NS;
      hipStream_t ps = ss[slot];
      sk_sketch W;
      batched_sketch(p, d_per_k, zeta, device, &W);
      Carver cv{base, L.slots_off + (size_t)slot * L.slot_bytes};
      SolveBufs X;
      Phases ph(ps);
      if ((rc = batched_bufs(cv, &W, p, &X)) < 0) break;
      if (!event(2 * i) || hipEventRecord(ev[2 * i], ps) != hipSuccess) {
        rc = SK_E_HIP;
        break;
      }
      if (pass == 0 && batch_factored(p, d_per_k)) {
        // the sketch into this stream's slot, [S A | S b] into the problem's own buffers
        Carver fc{base, L.factors_off + L.factor_at[i]};
        FactorBufs F;
        factor_bufs(fc, W.d, k, &F);
        if ((rc = apply_dispatch(&W, p.dtype, k, p.A, p.lda, SK_F64, X.B.SA, k, X.B.aws, X.B.aws_bytes, ps)) < 0) break;
        if ((rc = apply_dispatch(&W, p.dtype, 1, p.b, 1, SK_F64, X.B.Sb, 1, X.B.aws, X.B.aws_bytes, ps)) < 0) break;
        if ((rc = launch_to_columns(X.B.SA, k, X.B.Sb, W.d, k, F.W, W.d, ps)) < 0) break;
        host_table.push_back(QrBatch{F.W, W.d, W.d, k, 0, F.tau, F.T, F.R, F.c, F.X, F.XT, p.x, ranks + i});
        kmax = std::max(kmax, k);
        queued = true;
        continue;
      }
      if ((rc = sketch_and_factor(&W, k, p.dtype, p.A, p.lda, p.b, X.B, ph, ps, p.dtype)) < 0) break;
      if (pass == 0) {
        // U and V hold R^-1 and its transpose here
        if ((rc = launch_trinv(X.B.R, k, X.U, X.V, ps)) < 0) break;
        if ((rc = launch_certified_tri_solve(X.B.R, X.U, X.B.c, k, eps, p.x, ranks + i, ps)) < 0) break;
      } else {
        if ((rc = launch_jacobi_svd(X.B.R, k, X.U, X.sv, X.V, X.work, ps)) < 0) break;
        if ((rc = launch_svd_solve(X.U, X.sv, X.V, X.B.c, k, eps, p.x, X.z, ranks + i, ps)) < 0) break;
      }
      if (!event(2 * i + 1) || hipEventRecord(ev[2 * i + 1], ps) != hipSuccess) {
        rc = SK_E_HIP;
        break;
      }
      queued = true;
    }
    if (pass == 0 && rc == SK_OK && !host_table.empty()) {
      // the caller's stream waits for every sketch, then factors and solves
      // the batch-factored problems together
      for (int j = 0; j < NS && rc == SK_OK; ++j) {
        if (hipEventCreateWithFlags(&joined[j], hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(joined[j], ss[j]) != hipSuccess || hipStreamWaitEvent(st, joined[j], 0) != hipSuccess) {
          set_error("lstsq_sketch_solve_batched: joining the streams failed");
          rc = SK_E_HIP;
        }
      }
      const int nf = (int)host_table.size();
      if (rc == SK_OK && hipMemcpyAsync(table, host_table.data(), sizeof(QrBatch) * (size_t)nf,
                                        hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("lstsq_sketch_solve_batched: uploading the batch table failed");
        rc = SK_E_HIP;
      }
      if (rc == SK_OK) rc = qr_trinv_batched(table, nf, kmax, st);
      if (rc == SK_OK) rc = certified_tri_solve_batched(table, nf, eps, st);
      if (rc == SK_OK && (hipEventCreate(&batch_done) != hipSuccess || hipEventRecord(batch_done, st) != hipSuccess)) {
        set_error("lstsq_sketch_solve_batched: event on the caller's stream failed");
        rc = SK_E_HIP;
      }
      if (rc == SK_OK && hipStreamSynchronize(st) != hipSuccess) {
        set_error("lstsq_sketch_solve_batched: synchronization failed");
        rc = SK_E_HIP;
      }
    }
    // everything queued has finished before the ranks are read and before the
    // events, the streams and the workspace go
    for (int j = 0; j < NS; ++j) {
      if (ss[j] && hipStreamSynchronize(ss[j]) != hipSuccess && rc == SK_OK) {
        set_error("lstsq_sketch_solve_batched: stream synchronization failed");
        rc = SK_E_HIP;
      }
    }
    if (rc != SK_OK || !queued) break;
    if (hipMemcpy(h.data(), ranks, sizeof(int) * nprob, hipMemcpyDeviceToHost) != hipSuccess) {
      set_error("lstsq_sketch_solve_batched: reading the ranks failed");
      rc = SK_E_HIP;
      break;
    }
    for (int i = 0; i < nprob; ++i) {
      if (pass == 0 || redo[i]) {
        // a batch-factored problem ends with the batch's solve
        float t = 0.f;
        const bool batch = pass == 0 && batch_factored(probs[i], d_per_k);
        const bool bsk = pass == 0 && L.sketched[i];
        (void)hipEventElapsedTime(&t, bsk ? bsk_start : ev[2 * i], batch ? batch_done : ev[2 * i + 1]);
        t_ms[i] += t;
      }
      redo[i] = h[i] < 0;
      probs[i].rank = h[i];
    }
  }
  bool rankdef = false;
  if (rc == SK_OK) {
    for (int i = 0; i < nprob; ++i) {
      probs[i].t_ms = t_ms[i];
      probs[i].status = h[i] < probs[i].k ? SK_W_RANKDEF : SK_OK;
      rankdef = rankdef || h[i] < probs[i].k;
    }
  }
  for (int j = 0; j < NS; ++j)
    if (ss[j]) (void)hipStreamSynchronize(ss[j]);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : joined)
    if (e) (void)hipEventDestroy(e);
  if (batch_done) (void)hipEventDestroy(batch_done);
  if (bsk_start) (void)hipEventDestroy(bsk_start);
  if (ready) (void)hipEventDestroy(ready);
  for (auto& s2 : ss)
    if (s2) (void)hipStreamDestroy(s2);
  if (own) (void)hipFree(own);
  if (rc < 0) return rc;
  return rankdef ? SK_W_RANKDEF : SK_OK;
}

int lstsq_sketch_precond(sketch_t S, int64_t m, const double* A, int64_t lda, int sketch_dtype, const void* A_sketch,
                         int64_t lda_sketch, const double* b, double* x, double tol, int maxit, int warm_start,
                         sk_lsqr_info* info, void* stream) {
  if (!S || !A || !b || !x || m < 1 || lda < m || !(tol >= 0.0) || maxit < 0) {
    set_error("lstsq_sketch_precond: invalid argument");
    return SK_E_INVAL;
  }
  if (S->d < m || m > 512) {
    set_error("lstsq_sketch_precond: need m <= d and m <= 512");
    return SK_E_INVAL;
  }
  if (A_sketch && (!dtype_ok(sketch_dtype) || lda_sketch < m)) {
    set_error("lstsq_sketch_precond: A_sketch needs dtype F64/F32/BF16 and lda_sketch >= m");
    return SK_E_INVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int k = (int)m;
  const int64_t n = S->n;
  const void* As = A_sketch ? A_sketch : (const void*)A;
  const int dts = A_sketch ? sketch_dtype : SK_F64;
  const int64_t ldas = A_sketch ? lda_sketch : lda;
  const int groups = lsqr_pass_groups(n);

  double *Rinv, *RinvT, *x0, *v, *wd, *y, *wv, *u, *part;
  LsqrDev* sd;
  SketchBufs B;
  auto carve = [&](Carver& cv) -> int {
    SK_TRY(sketch_bufs(cv, S, k, dts, As, ldas, b, &B));
    Rinv = cv.take<double>((size_t)k * k);
    RinvT = cv.take<double>((size_t)k * k);
    x0 = cv.take<double>((size_t)k);
    v = cv.take<double>((size_t)k);
    wd = cv.take<double>((size_t)k);
    y = cv.take<double>((size_t)k);
    wv = cv.take<double>((size_t)k);
    u = cv.take<double>((size_t)n);
    part = cv.take<double>((size_t)(groups + 1) * (k + 1));
    sd = cv.take<LsqrDev>(1);
    return SK_OK;
  };
  Carver cv;
  SK_TRY(carve(cv));
  char* base = nullptr;
  SK_TRY(driver_workspace(S, cv.off, &base, st));
  Carver cv2{base, 0};
  SK_TRY(carve(cv2));
  double* qv = part + (size_t)groups * (k + 1);

  Phases ph(st);
  SK_TRY(ph.mark());                                                // 0
  SK_TRY(sketch_and_factor(S, k, dts, As, ldas, b, B, ph, st));     // 1: after the sketch
  SK_TRY(launch_trinv(B.R, k, Rinv, RinvT, st));
  if (warm_start)
    SK_TRY(launch_rinv_vec(Rinv, k, B.c, x0, st));
  else
    SK_TRY(launch_fill(x0, k, 0.0, st));
  SK_TRY(ph.mark());                                                // 2: after QR
  SK_HIP(hipMemcpyAsync(u, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  SK_TRY(launch_lsqr_setup(sd, tol, maxit, st));
  SK_TRY(launch_lsqr_pass(A, lda, n, k, x0, &sd->coef, nullptr, u, part, st));
  SK_TRY(launch_lsqr_init(sd, qv, Rinv, RinvT, k, v, wd, y, wv, st));
  // Iterations go out in batches, each followed by a snapshot of the device
  // state into one of two pinned slots. The host keeps two batches queued:
  // while it waits for one snapshot the GPU already runs the next batch, so
  // the stopping test costs no idle time. Launches after the device has set
  // done (converged or maxit reached) return at once.
  static_assert(2 * sizeof(LsqrDev) <= 4096, "two state slots in the pinned page");
  LsqrDev* hs = static_cast<LsqrDev*>(S->h_pinned);
  EventPair ev;
  SK_TRY(ev.create());
  auto snapshot = [&](int slot) -> int {
    SK_HIP(hipMemcpyAsync(&hs[slot], sd, sizeof(LsqrDev), hipMemcpyDeviceToHost, st));
    SK_HIP(hipEventRecord(ev.e[slot], st));
    return SK_OK;
  };
  const int batch = 4;
  int issued = 0;
  auto issue = [&](int slot) -> int {
    const int nb = std::min(batch, maxit - issued);
    for (int j = 0; j < nb; ++j) {
      SK_TRY(launch_lsqr_pass(A, lda, n, k, wv, &sd->coef, &sd->done, u, part, st));
      SK_TRY(launch_lsqr_step(sd, qv, Rinv, RinvT, k, v, wd, y, wv, st));
    }
    issued += nb;
    return snapshot(slot);
  };
  SK_TRY(snapshot(0));  // state after the initialization
  int inflight = 1, pending = 0;
  if (issued < maxit) {
    SK_TRY(issue(1));
    ++inflight;
  }
  for (;;) {
    SK_HIP(hipEventSynchronize(ev.e[pending]));
    --inflight;
    if (hs[pending].done) break;
    if (issued < maxit) {
      SK_TRY(issue(pending));
      ++inflight;
    } else if (inflight == 0) {
      break;
    }
    pending ^= 1;
  }
  SK_TRY(launch_lsqr_finish(Rinv, k, x0, y, x, st));
  SK_TRY(ph.mark());                                                // 3: solution written
  SK_HIP(hipMemcpyAsync(&hs[0], sd, sizeof(LsqrDev), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  if (info) {
    info->iters = hs->iters;
    info->converged = hs->converged;
    info->rnorm_est = hs->rnorm;
    info->arnorm_est = hs->arnorm;
    info->anorm_est = hs->anorm;
    info->t_sketch_ms = ph.ms(0, 1);
    info->t_qr_ms = ph.ms(1, 2);
    info->t_lsqr_ms = ph.ms(2, 3);
    info->t_total_ms = ph.ms(0, 3);
  }
  return hs->converged ? SK_OK : SK_W_NOCONV;
}

int lstsq_residual(sketch_t S, int64_t m, const double* A, int64_t lda, const double* b, const double* x,
                   double* resnorm, void* stream) {
  if (!S || !A || !b || !x || !resnorm || m < 1 || lda < m) {
    set_error("lstsq_residual: invalid argument");
    return SK_E_INVAL;
  }
  if (m > 512) {
    set_error("lstsq_residual: need m <= 512");
    return SK_E_INVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = S->n;
  const int k = (int)m;
  const int groups = lsqr_pass_groups(n);
  double *u, *part, *coef;
  auto carve = [&](Carver& cv) {
    u = cv.take<double>((size_t)n);
    part = cv.take<double>((size_t)(groups + 1) * (k + 1));
    coef = cv.take<double>(1);
  };
  Carver cv;
  carve(cv);
  char* base = nullptr;
  SK_TRY(driver_workspace(S, cv.off, &base, st));
  Carver cv2{base, 0};
  carve(cv2);
  SK_HIP(hipMemcpyAsync(u, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  SK_TRY(launch_fill(coef, 1, -1.0, st));
  {
    KernelTimer timer(S, st);
    SK_TRY(launch_lsqr_pass(A, lda, n, k, x, coef, nullptr, u, part, st));
  }
  double* hp = static_cast<double*>(S->h_pinned);
  SK_HIP(hipMemcpyAsync(hp, part + (size_t)groups * (k + 1) + k, sizeof(double), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  *resnorm = std::sqrt(*hp);
  return SK_OK;
}

}  // extern "C"
