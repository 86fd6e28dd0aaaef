// Randomized SVD driver (Alg. 1): Y = A Omega, Q = orth(Y), B = Q^T A,
// B = Uh diag(s) V^T, U = Q Uh.
//
// orth() is left open by the paper; here it is shifted Cholesky QR in three
// passes (Fukaya, Kannan, Nakatsukasa, Zhang, Yamamoto, SIAM J. Sci. Comput.
// 2020): the first pass factors Y^T Y + s I with s = 11 (rows k + k (k+1)) u
// trace(Y^T Y), which keeps the Cholesky factorization defined up to
// kappa(Y) ~ 1/u, and two plain passes restore orthogonality to working
// precision. All products are GEMMs; the k x k factorizations are the
// blocked Cholesky and triangular inverse kernels. The SVD of the short-fat
// B (k x cols) goes through the same QR of B^T = Q_b R_b and a one-sided
// Jacobi SVD of R_b^T = Uh diag(s) W^T, so V = Q_b W.
#include <algorithm>
#include <cmath>
#include <string>

#include "sk_dense.hpp"
#include "sk_drivers.hpp"
#include "sk_lowrank.hpp"

namespace sk {

namespace {

struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + std::max<size_t>(1, count) * sizeof(T);
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

#define SK_TRY2(expr)         \
  do {                        \
    int _rc = (expr);         \
    if (_rc < 0) return _rc;  \
  } while (0)

int lowrank_workspace(sk_sketch* S, size_t bytes, char** out, hipStream_t st) {
  SK_TRY2(grow_buffer(&S->dws, &S->dws_bytes, bytes, st));
  if (!S->h_pinned) SK_HIP(hipHostMalloc(&S->h_pinned, 4096, hipHostMallocDefault));
  *out = static_cast<char*>(S->dws);
  return SK_OK;
}

constexpr int kGramChunks = 16;

struct OrthBufs {
  double *G, *Rinv, *RinvT, *Rtmp, *Dinv;
  double* Gpart;  // kGramChunks partial Gram matrices
  int* fail;
};

// Q = orth(X) for X (r x k, row-major, F64) by shifted Cholesky QR in three
// passes, ping-ponging between X and alt. Returns the buffer holding Q. When
// Racc is non-null it receives R with X = Q R (upper, k x k).
int orth_cholqr3(sk_sketch* S, double* X, double* alt, int64_t r, int k, const OrthBufs& b, double* Racc,
                 double** Qout, hipStream_t st) {
  const double u = std::ldexp(1.0, -53);
  double* cur = X;
  double* nxt = alt;
  for (int pass = 0; pass < 3; ++pass) {
    SK_TRY2(gram_rm(S, cur, k, r, k, b.G, b.Gpart, kGramChunks, st));
    const double coef = pass == 0 ? 11.0 * ((double)r * k + (double)k * (k + 1)) * u : 0.0;
    SK_TRY2(launch_cholesky_upper(b.G, k, coef, b.Dinv, b.fail, st));
    SK_TRY2(launch_trinv(b.G, k, b.Rinv, b.RinvT, st));
    SK_TRY2(gemm_rm(S, SK_F64, false, false, r, k, k, 1.0, cur, k, b.Rinv, k, 0.0, nxt, k, st));
    std::swap(cur, nxt);
    if (Racc) {
      if (pass == 0) {
        SK_HIP(hipMemcpyAsync(Racc, b.G, sizeof(double) * k * k, hipMemcpyDeviceToDevice, st));
      } else {
        SK_TRY2(gemm_rm(S, SK_F64, false, false, k, k, k, 1.0, b.G, k, Racc, k, 0.0, b.Rtmp, k, st));
        SK_HIP(hipMemcpyAsync(Racc, b.Rtmp, sizeof(double) * k * k, hipMemcpyDeviceToDevice, st));
      }
    }
  }
  *Qout = cur;
  return SK_OK;
}

struct Marks {
  hipEvent_t ev[8] = {};
  int n = 0;
  hipStream_t st;
  explicit Marks(hipStream_t s) : st(s) {}
  int mark() {
    if (n >= 8) return SK_OK;
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
  ~Marks() {
    for (int i = 0; i < n; ++i) (void)hipEventDestroy(ev[i]);
  }
};

// Applies a sketch (row mode) into a caller-carved workspace.
int apply_into(sk_sketch* S, int dtype, int64_t m, const void* A, int64_t lda, double* out, int64_t ldo, void* ws,
               size_t ws_bytes, hipStream_t st) {
  return apply_dispatch(S, dtype, m, A, lda, SK_F64, out, ldo, ws, ws_bytes, st);
}

}  // namespace

}  // namespace sk

using namespace sk;

extern "C" int rsvd(sketch_t S, int dtype, int64_t rows, const void* A, int64_t lda, double* U, int64_t ldu,
                    double* sigma, double* Vt, int64_t ldvt, sk_rsvd_info* info, void* stream) {
  if (!S || !A || !sigma || rows < 1 || (dtype != SK_F64 && dtype != SK_F32) || lda < S->n ||
      (U && ldu < S->d) || (Vt && ldvt < S->n)) {
    set_error("rsvd: invalid argument");
    return SK_E_INVAL;
  }
  const int k = (int)S->d;
  const int64_t cols = S->n;
  if (k > rows || k > cols || k > 4096) {
    set_error("rsvd: need k = d <= min(rows, cols) and k <= 4096");
    return SK_E_INVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  size_t aws_bytes = 0;
  {
    int rc = apply_workspace(S, 1, dtype, rows, &aws_bytes);
    if (rc != SK_OK) return rc;
  }
  double *Y, *Y2, *Bd, *Qb, *Qb2, *Ut, *Wt, *sv, *jw, *Racc;
  float *Qf, *Bf;
  void* aws;
  OrthBufs ob;
  int* jflag;
  auto carve = [&](Carve& c) {
    aws = c.take<char>(aws_bytes);
    Y = c.take<double>((size_t)rows * k);
    Y2 = c.take<double>((size_t)rows * k);
    Qf = dtype == SK_F32 ? c.take<float>((size_t)rows * k) : nullptr;
    Bf = dtype == SK_F32 ? c.take<float>((size_t)k * cols) : nullptr;
    Bd = c.take<double>((size_t)k * cols);
    Qb = c.take<double>((size_t)cols * k);
    Qb2 = c.take<double>((size_t)cols * k);
    ob.G = c.take<double>((size_t)k * k);
    ob.Rinv = c.take<double>((size_t)k * k);
    ob.RinvT = c.take<double>((size_t)k * k);
    ob.Rtmp = c.take<double>((size_t)k * k);
    ob.Dinv = c.take<double>(32 * 32);
    ob.Gpart = c.take<double>((size_t)kGramChunks * k * k);
    ob.fail = c.take<int>(1);
    jflag = c.take<int>(1);
    Racc = c.take<double>((size_t)k * k);
    Ut = c.take<double>((size_t)k * k);
    Wt = c.take<double>((size_t)k * k);
    sv = c.take<double>((size_t)k);
    jw = c.take<double>(jacobi_work_doubles(k, k));
  };
  Carve c0;
  carve(c0);
  char* base = nullptr;
  SK_TRY2(lowrank_workspace(S, c0.off, &base, st));
  Carve c1{base, 0};
  carve(c1);
  int* h = static_cast<int*>(S->h_pinned);

  Marks mk(st);
  SK_TRY2(mk.mark());  // 0
  SK_TRY2(launch_set_int(ob.fail, 0, st));
  SK_TRY2(apply_T_dispatch(S, dtype, rows, A, lda, SK_F64, Y, k, aws, aws_bytes, st));
  SK_TRY2(mk.mark());  // 1: sketch
  double* Q = nullptr;
  SK_TRY2(orth_cholqr3(S, Y, Y2, rows, k, ob, nullptr, &Q, st));
  SK_TRY2(mk.mark());  // 2: orth
  if (dtype == SK_F64) {
    SK_TRY2(gemm_rm(S, SK_F64, true, false, k, cols, rows, 1.0, Q, k, A, lda, 0.0, Bd, cols, st));
  } else {
    SK_TRY2(launch_convert(SK_F64, Q, k, SK_F32, Qf, k, rows, k, st));
    SK_TRY2(gemm_rm(S, SK_F32, true, false, k, cols, rows, 1.0, Qf, k, A, lda, 0.0, Bf, cols, st));
    SK_TRY2(launch_convert(SK_F32, Bf, cols, SK_F64, Bd, cols, k, cols, st));
  }
  SK_TRY2(mk.mark());  // 3: projection
  SK_TRY2(launch_transpose(Bd, k, cols, Qb, st));
  double* Qbf = nullptr;
  SK_TRY2(orth_cholqr3(S, Qb, Qb2, cols, k, ob, Racc, &Qbf, st));
  int sweeps = 0;
  // R_b^T = Uh diag(s) W^T: the column-major view of R_b's memory is R_b^T
  SK_TRY2(jacobi_svd_rounds(Racc, k, k, 1, Ut, sv, Wt, jw, jflag, h + 1, 40, &sweeps, st));
  SK_HIP(hipMemcpyAsync(sigma, sv, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  if (U) SK_TRY2(gemm_rm(S, SK_F64, false, false, rows, k, k, 1.0, Q, k, Ut, k, 0.0, U, ldu, st));
  if (Vt) SK_TRY2(gemm_rm(S, SK_F64, true, true, k, cols, k, 1.0, Wt, k, Qbf, k, 0.0, Vt, ldvt, st));
  SK_TRY2(mk.mark());  // 4: svd
  SK_HIP(hipMemcpyAsync(h, ob.fail, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  if (info) {
    info->t_sketch_ms = mk.ms(0, 1);
    info->t_orth_ms = mk.ms(1, 2);
    info->t_project_ms = mk.ms(2, 3);
    info->t_svd_ms = mk.ms(3, 4);
    info->t_total_ms = mk.ms(0, 4);
    info->jacobi_sweeps = sweeps;
  }
  if (*h) {
    set_error("rsvd: Cholesky QR met a non-positive pivot (the sketch is numerically rank deficient)");
    return SK_W_RANKDEF;
  }
  return SK_OK;
}

// ---------------------------------------------------------------------------
// Generalized Nystrom (Alg. 4 and Alg. 5). Omega = So^T (cols x k), Psi =
// Sp^T (rows x p): Y = A Omega is the column-mode apply of So, X^T = Psi^T A
// the row-mode apply of Sp, and Psi^T Y (or Psi^T Q) the row-mode apply of Sp
// to the n x k factor.
// ---------------------------------------------------------------------------
namespace {

struct GnCheck {
  int64_t cols;
  int k, p;
};

int gn_check(const char* who, sketch_t So, sketch_t Sp, int dtype, int64_t rows, const void* A, int64_t lda,
             GnCheck* c) {
  if (!So || !Sp || !A || rows < 1 || (dtype != SK_F64 && dtype != SK_F32)) {
    set_error(std::string(who) + ": invalid argument");
    return SK_E_INVAL;
  }
  c->cols = So->n;
  c->k = (int)So->d;
  c->p = (int)Sp->d;
  if (Sp->n != rows || lda < c->cols || c->k > c->p || (int64_t)c->p > rows || (int64_t)c->p > c->cols ||
      c->k > 4096 || c->p > 4096) {
    set_error(std::string(who) +
              ": need Omega^T = So (k x cols), Psi^T = Sp (p x rows), k <= p <= min(rows, cols), p <= 4096, "
              "lda >= cols");
    return SK_E_INVAL;
  }
  return SK_OK;
}

}  // namespace

extern "C" int gen_nystrom(sketch_t So, sketch_t Sp, int dtype, int64_t rows, const void* A, int64_t lda, double* F,
                           int64_t ldf, double* G, int64_t ldg, sk_gn_info* info, void* stream) {
  GnCheck c;
  SK_TRY2(gn_check("gen_nystrom", So, Sp, dtype, rows, A, lda, &c));
  if (!F || !G || ldf < c.k || ldg < c.k) {
    set_error("gen_nystrom: F (rows x k, ldf >= k) and G (cols x k, ldg >= k) are required");
    return SK_E_INVAL;
  }
  const int k = c.k, p = c.p;
  const int64_t cols = c.cols;
  hipStream_t st = (hipStream_t)stream;
  size_t wT = 0, wA = 0, wY = 0;
  SK_TRY2(apply_workspace(So, 1, dtype, rows, &wT));
  SK_TRY2(apply_workspace(Sp, 0, dtype, cols, &wA));
  SK_TRY2(apply_workspace(Sp, 0, SK_F64, k, &wY));
  void *awT, *awA, *awY;
  double *Y, *Xt, *M, *Um, *sv, *Vm, *jw, *Vs, *Ur;
  int *jflag, *rk;
  auto carve = [&](Carve& cv) {
    awT = cv.take<char>(wT);
    awA = cv.take<char>(wA);
    awY = cv.take<char>(wY);
    Y = cv.take<double>((size_t)rows * k);
    Xt = cv.take<double>((size_t)p * cols);
    M = cv.take<double>((size_t)p * k);
    Um = cv.take<double>((size_t)p * k);
    sv = cv.take<double>(k);
    Vm = cv.take<double>((size_t)k * k);
    jw = cv.take<double>(jacobi_work_doubles(p, k));
    Vs = cv.take<double>((size_t)k * k);
    Ur = cv.take<double>((size_t)p * k);
    jflag = cv.take<int>(1);
    rk = cv.take<int>(1);
  };
  Carve c0;
  carve(c0);
  char* base = nullptr;
  SK_TRY2(lowrank_workspace(So, c0.off, &base, st));
  Carve c1{base, 0};
  carve(c1);
  int* h = static_cast<int*>(So->h_pinned);

  Marks mk(st);
  SK_TRY2(mk.mark());  // 0
  SK_TRY2(apply_T_dispatch(So, dtype, rows, A, lda, SK_F64, Y, k, awT, wT, st));
  SK_TRY2(apply_into(Sp, dtype, cols, A, lda, Xt, cols, awA, wA, st));
  SK_TRY2(mk.mark());  // 1: both sketches of A
  SK_TRY2(apply_into(Sp, SK_F64, k, Y, k, M, k, awY, wY, st));  // Psi^T Y = X^T Omega
  int sweeps = 0;
  SK_TRY2(jacobi_svd_rounds(M, p, k, 0, Um, sv, Vm, jw, jflag, h + 1, 60, &sweeps, st));
  SK_TRY2(launch_gn_truncate(sv, k, Vm, Vs, Um, p, Ur, rk, st));
  SK_TRY2(mk.mark());  // 2: core
  SK_TRY2(gemm_rm(So, SK_F64, false, false, rows, k, k, 1.0, Y, k, Vs, k, 0.0, F, ldf, st));     // F = Y V_r S_r^-1
  SK_TRY2(gemm_rm(So, SK_F64, true, false, cols, k, p, 1.0, Xt, cols, Ur, k, 0.0, G, ldg, st));  // G = X U_r
  SK_TRY2(mk.mark());  // 3: factors
  SK_HIP(hipMemcpyAsync(h, rk, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  if (info) {
    info->rank = *h;
    info->t_sketch_ms = mk.ms(0, 1);
    info->t_core_ms = mk.ms(1, 2);
    info->t_factors_ms = mk.ms(2, 3);
    info->t_total_ms = mk.ms(0, 3);
    info->jacobi_sweeps = sweeps;
  }
  return SK_OK;
}

extern "C" int gen_nystrom_svd(sketch_t So, sketch_t Sp, int dtype, int64_t rows, const void* A, int64_t lda,
                               double* U, int64_t ldu, double* sigma, double* V, int64_t ldv, sk_gn_info* info,
                               void* stream) {
  GnCheck c;
  SK_TRY2(gn_check("gen_nystrom_svd", So, Sp, dtype, rows, A, lda, &c));
  if (!U || !sigma || !V || ldu < c.k || ldv < c.k) {
    set_error("gen_nystrom_svd: U (rows x k, ldu >= k), sigma (k) and V (cols x k, ldv >= k) are required");
    return SK_E_INVAL;
  }
  const int k = c.k, p = c.p;
  const int64_t cols = c.cols;
  hipStream_t st = (hipStream_t)stream;
  size_t wT = 0, wA = 0, wY = 0;
  SK_TRY2(apply_workspace(So, 1, dtype, rows, &wT));
  SK_TRY2(apply_workspace(Sp, 0, dtype, cols, &wA));
  SK_TRY2(apply_workspace(Sp, 0, SK_F64, k, &wY));
  void *awT, *awA, *awY;
  double *Y, *Y2, *Xt, *Xb, *Xb2, *T, *M1, *U1, *s1, *V1, *jw, *Vs, *U1r, *W1, *C, *Uc, *sc, *Vc;
  OrthBufs ok_, op_;
  int *jflag, *rk;
  auto orth_bufs = [&](Carve& cv, OrthBufs& o, int n) {
    o.G = cv.take<double>((size_t)n * n);
    o.Rinv = cv.take<double>((size_t)n * n);
    o.RinvT = cv.take<double>((size_t)n * n);
    o.Rtmp = cv.take<double>((size_t)n * n);
    o.Dinv = cv.take<double>(32 * 32);
    o.Gpart = cv.take<double>((size_t)kGramChunks * n * n);
    o.fail = cv.take<int>(1);
  };
  auto carve = [&](Carve& cv) {
    awT = cv.take<char>(wT);
    awA = cv.take<char>(wA);
    awY = cv.take<char>(wY);
    Y = cv.take<double>((size_t)rows * k);
    Y2 = cv.take<double>((size_t)rows * k);
    Xt = cv.take<double>((size_t)p * cols);
    Xb = cv.take<double>((size_t)cols * p);
    Xb2 = cv.take<double>((size_t)cols * p);
    T = cv.take<double>((size_t)p * p);
    M1 = cv.take<double>((size_t)p * k);
    U1 = cv.take<double>((size_t)p * k);
    s1 = cv.take<double>(k);
    V1 = cv.take<double>((size_t)k * k);
    jw = cv.take<double>(jacobi_work_doubles(p, k));
    Vs = cv.take<double>((size_t)k * k);
    U1r = cv.take<double>((size_t)p * k);
    W1 = cv.take<double>((size_t)k * p);
    C = cv.take<double>((size_t)k * p);
    Uc = cv.take<double>((size_t)p * k);
    sc = cv.take<double>(k);
    Vc = cv.take<double>((size_t)k * k);
    orth_bufs(cv, ok_, k);
    orth_bufs(cv, op_, p);
    jflag = cv.take<int>(1);
    rk = cv.take<int>(1);
  };
  Carve c0;
  carve(c0);
  char* base = nullptr;
  SK_TRY2(lowrank_workspace(So, c0.off, &base, st));
  Carve c1{base, 0};
  carve(c1);
  int* h = static_cast<int*>(So->h_pinned);

  Marks mk(st);
  SK_TRY2(mk.mark());  // 0
  SK_TRY2(launch_set_int(ok_.fail, 0, st));
  SK_TRY2(launch_set_int(op_.fail, 0, st));
  SK_TRY2(apply_T_dispatch(So, dtype, rows, A, lda, SK_F64, Y, k, awT, wT, st));
  SK_TRY2(apply_into(Sp, dtype, cols, A, lda, Xt, cols, awA, wA, st));
  SK_TRY2(mk.mark());  // 1: both sketches of A
  double* Q = nullptr;
  SK_TRY2(orth_cholqr3(So, Y, Y2, rows, k, ok_, nullptr, &Q, st));  // [Q, ~] = qr_econ(Y)
  SK_TRY2(launch_transpose(Xt, p, cols, Xb, st));                   // X = A^T Psi (cols x p)
  double* P = nullptr;
  SK_TRY2(orth_cholqr3(So, Xb, Xb2, cols, p, op_, T, &P, st));     // [P, T] = qr_econ(X)
  SK_TRY2(apply_into(Sp, SK_F64, k, Q, k, M1, k, awY, wY, st));    // Psi^T Q
  int sw1 = 0, sw2 = 0;
  SK_TRY2(jacobi_svd_rounds(M1, p, k, 0, U1, s1, V1, jw, jflag, h + 1, 60, &sw1, st));
  SK_TRY2(launch_gn_truncate(s1, k, V1, Vs, U1, p, U1r, rk, st));
  // C = V1_r S1_r^-1 U1_r^T T^T = Vs (T U1r)^T
  SK_TRY2(gemm_rm(So, SK_F64, true, true, k, p, p, 1.0, U1r, k, T, p, 0.0, W1, p, st));
  SK_TRY2(gemm_rm(So, SK_F64, false, false, k, p, k, 1.0, Vs, k, W1, p, 0.0, C, p, st));
  // svd_econ(C), C k x p: the Jacobi SVD of C^T (the column-major view of C)
  // gives C^T = Uc diag(sc) Vc^T, i.e. C = Vc diag(sc) Uc^T
  SK_TRY2(jacobi_svd_rounds(C, p, k, 1, Uc, sc, Vc, jw, jflag, h + 1, 60, &sw2, st));
  SK_TRY2(mk.mark());  // 2: core
  SK_HIP(hipMemcpyAsync(sigma, sc, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  SK_TRY2(gemm_rm(So, SK_F64, false, false, rows, k, k, 1.0, Q, k, Vc, k, 0.0, U, ldu, st));  // U = Q Uhat
  SK_TRY2(gemm_rm(So, SK_F64, false, false, cols, k, p, 1.0, P, p, Uc, k, 0.0, V, ldv, st));  // V = P Vhat
  SK_TRY2(mk.mark());  // 3: factors
  SK_HIP(hipMemcpyAsync(h, rk, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(h + 2, ok_.fail, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(h + 3, op_.fail, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  if (info) {
    info->rank = h[0];
    info->t_sketch_ms = mk.ms(0, 1);
    info->t_core_ms = mk.ms(1, 2);
    info->t_factors_ms = mk.ms(2, 3);
    info->t_total_ms = mk.ms(0, 3);
    info->jacobi_sweeps = sw1 + sw2;
  }
  if (h[2] || h[3]) {
    set_error("gen_nystrom_svd: Cholesky QR of Y or X met a non-positive pivot (numerically rank deficient)");
    return SK_W_RANKDEF;
  }
  return SK_OK;
}

// ---------------------------------------------------------------------------
// Nystrom approximation of a psd matrix (Alg. 2), Omega = S^T (n x k).
// ---------------------------------------------------------------------------
extern "C" int nystrom_psd(sketch_t S, int dtype, const void* A, int64_t lda, double* U, int64_t ldu, double* lambda,
                           sk_nystrom_info* info, void* stream) {
  if (!S || !A || !U || !lambda || (dtype != SK_F64 && dtype != SK_F32)) {
    set_error("nystrom_psd: invalid argument");
    return SK_E_INVAL;
  }
  const int64_t n = S->n;
  const int k = (int)S->d;
  if (lda < n || ldu < k || k > n || k > 4096) {
    set_error("nystrom_psd: need A n x n (lda >= n), U n x k (ldu >= k), k = d <= min(n, 4096)");
    return SK_E_INVAL;
  }
  if (S->kind != SK_SPARSESTACK && S->kind != SK_GAUSSIAN) {
    set_error("nystrom_psd: Omega must be a SparseStack or Gaussian sketch");
    return SK_E_NOTSUP;
  }
  hipStream_t st = (hipStream_t)stream;
  size_t wT = 0, wY = 0;
  SK_TRY2(apply_workspace(S, 1, dtype, n, &wT));
  SK_TRY2(apply_workspace(S, 0, SK_F64, k, &wY));
  void *awT, *awY;
  double *Y, *B, *B2, *Om, *C, *Cinv, *CinvT, *R, *Ur, *sv, *jw, *nu;
  OrthBufs ob;
  int* jflag;
  auto carve = [&](Carve& cv) {
    awT = cv.take<char>(wT);
    awY = cv.take<char>(wY);
    Y = cv.take<double>((size_t)n * k);
    B = cv.take<double>((size_t)n * k);
    B2 = cv.take<double>((size_t)n * k);
    Om = S->kind == SK_GAUSSIAN ? cv.take<double>((size_t)n * k) : nullptr;
    C = cv.take<double>((size_t)k * k);
    Cinv = cv.take<double>((size_t)k * k);
    CinvT = cv.take<double>((size_t)k * k);
    R = cv.take<double>((size_t)k * k);
    Ur = cv.take<double>((size_t)k * k);
    sv = cv.take<double>(k);
    jw = cv.take<double>(jacobi_work_doubles(k, k));
    nu = cv.take<double>(1);
    ob.G = cv.take<double>((size_t)k * k);
    ob.Rinv = cv.take<double>((size_t)k * k);
    ob.RinvT = cv.take<double>((size_t)k * k);
    ob.Rtmp = cv.take<double>((size_t)k * k);
    ob.Dinv = cv.take<double>(32 * 32);
    ob.Gpart = cv.take<double>((size_t)kGramChunks * k * k);
    ob.fail = cv.take<int>(1);
    jflag = cv.take<int>(1);
  };
  Carve c0;
  carve(c0);
  char* base = nullptr;
  SK_TRY2(lowrank_workspace(S, c0.off, &base, st));
  Carve c1{base, 0};
  carve(c1);
  int* h = static_cast<int*>(S->h_pinned);

  Marks mk(st);
  SK_TRY2(mk.mark());  // 0
  SK_TRY2(launch_set_int(ob.fail, 0, st));
  SK_TRY2(apply_T_dispatch(S, dtype, n, A, lda, SK_F64, Y, k, awT, wT, st));  // Y = A Omega
  SK_TRY2(mk.mark());                                                         // 1: sketch
  // nu = sqrt(n) eps ||Y||_2
  SK_TRY2(gram_rm(S, Y, k, n, k, ob.G, ob.Gpart, kGramChunks, st));
  SK_TRY2(launch_nystrom_shift(ob.G, k, n, nu, st));
  // Y_nu = Y + nu Omega
  if (S->kind == SK_SPARSESTACK) {
    SK_TRY2(launch_add_omega_ss(Y, n, k, S->zeta, (int)S->nb, S->k0, S->k1, inv_sqrt_host((double)S->zeta), nu, st));
  } else {
    SK_TRY2(launch_gauss_fill_f64(S, Om, st));
    SK_TRY2(launch_add_omega_dense(Y, n, k, Om, nu, st));
  }
  // C = chol(Omega^T Y_nu): Omega^T Y_nu = S Y_nu, symmetrized, upper factor
  SK_TRY2(apply_into(S, SK_F64, k, Y, k, C, k, awY, wY, st));
  SK_TRY2(launch_symmetrize(C, k, st));
  SK_TRY2(launch_cholesky_upper(C, k, 0.0, ob.Dinv, ob.fail, st));
  // B = Y_nu C^-1; [U, Sigma, ~] = svd_econ(B) by Cholesky QR of B and the
  // Jacobi SVD of its triangular factor
  SK_TRY2(launch_trinv(C, k, Cinv, CinvT, st));
  SK_TRY2(gemm_rm(S, SK_F64, false, false, n, k, k, 1.0, Y, k, Cinv, k, 0.0, B, k, st));
  double* Q = nullptr;
  SK_TRY2(orth_cholqr3(S, B, B2, n, k, ob, R, &Q, st));
  int sweeps = 0;
  // only the left singular vectors of B are needed: no V accumulation
  SK_TRY2(jacobi_svd_rounds(R, k, k, 0, Ur, sv, nullptr, jw, jflag, h + 1, 60, &sweeps, st));
  SK_TRY2(gemm_rm(S, SK_F64, false, false, n, k, k, 1.0, Q, k, Ur, k, 0.0, U, ldu, st));
  SK_TRY2(launch_remove_shift(sv, k, nu, lambda, st));  // Lambda = max(0, Sigma^2 - nu)
  SK_TRY2(mk.mark());                                     // 2: core
  double hnu = 0.0;
  SK_HIP(hipMemcpyAsync(h + 2, ob.fail, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(&hnu, nu, sizeof(double), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  if (info) {
    info->nu = hnu;
    info->t_sketch_ms = mk.ms(0, 1);
    info->t_core_ms = mk.ms(1, 2);
    info->t_total_ms = mk.ms(0, 2);
    info->jacobi_sweeps = sweeps;
  }
  if (h[2]) {
    set_error("nystrom_psd: a Cholesky factorization met a non-positive pivot (A not psd to working precision?)");
    return SK_W_RANKDEF;
  }
  return SK_OK;
}
