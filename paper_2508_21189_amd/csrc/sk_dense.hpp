// Dense FP64 building blocks of the least-squares and low-rank drivers.
#pragma once
#include "sk_common.hpp"

namespace sk {

// W (column-major, ldw) := columns of the row-major d x k0 matrix M, then r (if non-null).
int launch_to_columns(const double* M, int64_t ldm, const double* r, int64_t d, int k0, double* W, int64_t ldw,
                      hipStream_t st);
// Blocked Householder QR of the first k columns of W (d x (k + extra_cols),
// column-major), applying Q^T to the extra columns as well. tau: k entries;
// Tbuf: qr_tbuf_doubles(k) doubles.
int qr_columns(double* W, int64_t ldw, int64_t d, int k, int extra_cols, double* tau, double* Tbuf, hipStream_t st);
size_t qr_tbuf_doubles(int k);
// R (k x k row-major, upper) and c = first k entries of the (transformed) column k.
int launch_extract_r(const double* W, int64_t ldw, int k, int has_rhs, double* R, double* c, hipStream_t st);
// X = R^{-1} (k x k row-major, upper) and XT = X^T. k <= 8192.
int launch_trinv(const double* R, int k, double* X, double* XT, hipStream_t st);
// One-sided Jacobi SVD of a k x k row-major matrix R: R = U diag(s) V^T with
// s descending. U, V: k x k row-major. work: 2 k^2 doubles.
int launch_jacobi_svd(const double* R, int k, double* U, double* s, double* V, double* work, hipStream_t st);
// x = V_r diag(s_r)^{-1} U_r^T c with r = #{s_i > 5 eps s_1} (written to
// *rank_out, device). z: k doubles of scratch.
// Alg. 3's solve when its rank test certainly passes: *rank_out = k and
// x = X c if ||R||_F ||X||_F < 1e-3 / (5 eps) (R upper triangular, X = R^-1,
// both k x k row-major), else *rank_out = -1 and x untouched.
int launch_certified_tri_solve(const double* R, const double* X, const double* c, int k, double eps, double* x,
                               int* rank_out, hipStream_t st);
int launch_svd_solve(const double* U, const double* s, const double* V, const double* c, int k, double eps, double* x,
                     double* z, int* rank_out, hipStream_t st);
// x[0:n) = value
int launch_fill(double* x, int64_t n, double value, hipStream_t st);

// One small problem of a batch (device memory): W (d x (k + 1), column-major,
// ldw) = [S A | S b] on entry; tau (k), T (qr_tbuf_doubles(k)), R (k x k),
// c (k), X and XT (k x k) are its outputs; x (k) and *rank its solution.
// k = 0 marks an entry that the batched launches skip. Uc, Vc (k x k) and
// sv, z (k) are the SVD fallback's buffers (null: no fallback for it).
struct QrBatch {
  double* W;
  int64_t ldw, d;
  int k, pad;
  double *tau, *T, *R, *c, *X, *XT, *x;
  int* rank;
  double *Uc, *Vc, *sv, *z;
};
// For every problem of the table B (nprob entries, d <= 1024, k <= kmax <=
// 512): the blocked Householder QR of W (32-column panels), R and c, and X =
// R^-1, XT = X^T: one launch per panel and per trailing update for the whole
// batch, then one each for R, the diagonal blocks and the columns of X.
int qr_trinv_batched(const QrBatch* B, int nprob, int kmax, hipStream_t st);
// Alg. 3's certified solve (launch_certified_tri_solve) for every problem of B.
int certified_tri_solve_batched(const QrBatch* B, int nprob, double eps, hipStream_t st);
// For every problem of B whose certificate failed (*rank < 0): the Jacobi SVD
// of R and the truncated solve (Alg. 3), one workgroup a problem, with X and
// XT as U and V (R^-1 is not needed any more) and Uc, Vc, sv, z as the rest.
int svd_fallback_batched(const QrBatch* B, int nprob, double eps, hipStream_t st);

}  // namespace sk
