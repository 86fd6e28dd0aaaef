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

int lowrank_workspace(sk_sketch* S, size_t bytes, char** out) {
  if (S->dws_bytes < bytes) {
    if (S->dws) {
      SK_HIP(hipDeviceSynchronize());
      SK_HIP(hipFree(S->dws));
      S->dws = nullptr;
      S->dws_bytes = 0;
    }
    void* p = nullptr;
    SK_HIP(hipMalloc(&p, bytes));
    S->dws = p;
    S->dws_bytes = bytes;
  }
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
    jw = c.take<double>(jacobi_work_doubles(k));
  };
  Carve c0;
  carve(c0);
  char* base = nullptr;
  SK_TRY2(lowrank_workspace(S, c0.off, &base));
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
  SK_TRY2(jacobi_svd_rounds(Racc, k, 1, Ut, sv, Wt, jw, jflag, h + 1, 40, &sweeps, st));
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
