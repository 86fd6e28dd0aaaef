// Dense FP64 building blocks of the randomized SVD (lowrank.hip, blas.cpp).
#pragma once
#include "sk_common.hpp"

namespace sk {

// G (k x k row-major, symmetric; the upper triangle is read) := R, upper,
// with G + shift I = R^T R and shift = shift_coef * trace(G) (no shift when
// shift_coef <= 0). Dinv: 32 x 32 doubles of scratch. *fail (device) is set
// to 1 on a non-positive pivot.
int launch_cholesky_upper(double* G, int k, double shift_coef, double* Dinv, int* fail, hipStream_t st);
int launch_set_int(int* p, int v, hipStream_t st);
// Y (c x r) = X^T for X r x c row-major.
int launch_transpose(const double* X, int64_t r, int64_t c, double* Y, hipStream_t st);
// One-sided Jacobi SVD M = U diag(s) V^T of a rows x k matrix (rows >= k; M
// row-major, or column-major when input_colmajor), by block visits (one
// launch for the diagonal blocks and one per round of block pairs in every
// sweep); U (rows x k) and V (k x k) row-major, s descending. Columns of U
// whose singular value is 0 are 0. V = null skips the right vectors (no
// rotation accumulation). work: jacobi_work_doubles(rows, k); flag: one
// device int; h_flag: pinned host int. Synchronizes the stream once per sweep.
size_t jacobi_work_doubles(int64_t rows, int k);
int jacobi_svd_rounds(const double* M, int64_t rows, int k, int input_colmajor, double* U, double* s, double* V,
                      double* work, int* flag, int* h_flag, int max_sweeps, int* sweeps, hipStream_t st);

// Numerical rank r = #{i : s_i > 5 eps s_0} of a descending s (k), written to
// *rank (device), and the truncated factors Vs = V[:, :r] diag(1/s[:r]) and
// Ur = U[:, :r] (zero past r; V k x k, U p x k, row-major).
int launch_gn_truncate(const double* s, int k, const double* V, double* Vs, const double* U, int p, double* Ur,
                       int* rank, hipStream_t st);

// Nystrom (Alg. 2) helpers: *nu = sqrt(n) 2^-52 sqrt(lambda_max(G)) (G = Y^T Y,
// power iteration); Y += nu Omega for Omega = S^T of a SparseStack sketch, or
// of a dense G (k x n) written out; B <- (B + B^T)/2; lambda = max(0, s^2 - nu).
int launch_nystrom_shift(const double* G, int k, int64_t n, double* nu, hipStream_t st);
int launch_add_omega_ss(double* Y, int64_t n, int k, int zeta, int nb, uint32_t k0, uint32_t k1, double scale,
                        const double* nu, hipStream_t st);
int launch_add_omega_dense(double* Y, int64_t n, int k, const double* G, const double* nu, hipStream_t st);
int launch_symmetrize(double* B, int k, hipStream_t st);
int launch_remove_shift(const double* s, int k, const double* nu, double* lambda, hipStream_t st);
// G (d x n, F64 row-major) = the entries of a Gaussian sketch.
int launch_gauss_fill_f64(const sk_sketch* S, double* G, hipStream_t st);

// Row-major GEMM on the handle's rocBLAS handle and stream:
// C (M x N) = alpha op(A) op(B) + beta C; dtype SK_F64 or SK_F32.
int gemm_rm(sk_sketch* S, int dtype, bool transA, bool transB, int64_t M, int64_t N, int64_t K, double alpha,
            const void* A, int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, hipStream_t st);
void blas_release(sk_sketch* S);
// G (k x k row-major) = X^T X for X r x k row-major (ld ldx), over at most
// max_chunks row chunks; part: max_chunks * k * k doubles of scratch.
int gram_rm(sk_sketch* S, const double* X, int64_t ldx, int64_t r, int k, double* G, double* part, int max_chunks,
            hipStream_t st);
// out[e] = sum_c P[c * count + e], c = 0 .. np-1 in order.
int launch_sum_partials(const double* P, int np, int64_t count, double* out, hipStream_t st);

}  // namespace sk
