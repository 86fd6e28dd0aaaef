// Plain library GEMMs (rocBLAS) used by the randomized SVD for its dense
// products: Y^T Y, Y R^-1, Q^T A, Q U, W^T Q_b^T. The Gram matrices of the
// tall factors are split over row chunks (one strided-batched GEMM; the
// partial Grams are then added in chunk order), since a k x k result alone
// gives the GPU only (k/128)^2 output tiles to work on. Row-major operands are
// passed as their column-major transposes (C^T = op(B)^T op(A)^T).
#include <rocblas/rocblas.h>

#include <algorithm>
#include <climits>

#include "sk_lowrank.hpp"

namespace sk {

static int blas_handle(sk_sketch* S, rocblas_handle* h) {
  if (!S->blas) {
    rocblas_handle nh = nullptr;
    if (rocblas_create_handle(&nh) != rocblas_status_success) {
      set_error("rocblas_create_handle failed");
      return SK_E_HIP;
    }
    S->blas = nh;
  }
  *h = (rocblas_handle)S->blas;
  return SK_OK;
}

void blas_release(sk_sketch* S) {
  if (S->blas) rocblas_destroy_handle((rocblas_handle)S->blas);
  S->blas = nullptr;
}

int gemm_rm(sk_sketch* S, int dtype, bool transA, bool transB, int64_t M, int64_t N, int64_t K, double alpha,
            const void* A, int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, hipStream_t st) {
  if (M > INT_MAX || N > INT_MAX || K > INT_MAX || lda > INT_MAX || ldb > INT_MAX || ldc > INT_MAX) {
    set_error("gemm: dimension beyond 32-bit range");
    return SK_E_NOTSUP;
  }
  rocblas_handle h;
  int rc = blas_handle(S, &h);
  if (rc != SK_OK) return rc;
  if (rocblas_set_stream(h, st) != rocblas_status_success) {
    set_error("rocblas_set_stream failed");
    return SK_E_HIP;
  }
  const rocblas_operation oa = transA ? rocblas_operation_transpose : rocblas_operation_none;
  const rocblas_operation ob = transB ? rocblas_operation_transpose : rocblas_operation_none;
  rocblas_status s;
  if (dtype == SK_F64) {
    s = rocblas_dgemm(h, ob, oa, (rocblas_int)N, (rocblas_int)M, (rocblas_int)K, &alpha, (const double*)B,
                      (rocblas_int)ldb, (const double*)A, (rocblas_int)lda, &beta, (double*)C, (rocblas_int)ldc);
  } else {
    const float af = (float)alpha, bf = (float)beta;
    s = rocblas_sgemm(h, ob, oa, (rocblas_int)N, (rocblas_int)M, (rocblas_int)K, &af, (const float*)B,
                      (rocblas_int)ldb, (const float*)A, (rocblas_int)lda, &bf, (float*)C, (rocblas_int)ldc);
  }
  if (s != rocblas_status_success) {
    set_error("rocBLAS gemm failed");
    return SK_E_HIP;
  }
  return SK_OK;
}

int gram_rm(sk_sketch* S, const double* X, int64_t ldx, int64_t r, int k, double* G, double* part, int max_chunks,
            hipStream_t st) {
  int chunks = (int)std::min<int64_t>(max_chunks, std::max<int64_t>(1, r / 512));
  if (chunks <= 1) return gemm_rm(S, SK_F64, true, false, k, k, r, 1.0, X, ldx, X, ldx, 0.0, G, k, st);
  const int64_t rc = (r + chunks - 1) / chunks;
  const int64_t full = r / rc, rem = r - full * rc;
  if (rc > INT_MAX || ldx > INT_MAX) {
    set_error("gram: dimension beyond 32-bit range");
    return SK_E_NOTSUP;
  }
  rocblas_handle h;
  int rc2 = blas_handle(S, &h);
  if (rc2 != SK_OK) return rc2;
  if (rocblas_set_stream(h, st) != rocblas_status_success) {
    set_error("rocblas_set_stream failed");
    return SK_E_HIP;
  }
  const double one = 1.0, zero = 0.0;
  const rocblas_stride sx = (rocblas_stride)(rc * ldx), sp = (rocblas_stride)k * k;
  // column-major view: part_c (k x k) = X_c^T X_c with X_c^T = (k x rc, ld ldx)
  rocblas_status s = rocblas_dgemm_strided_batched(
      h, rocblas_operation_none, rocblas_operation_transpose, k, k, (rocblas_int)rc, &one, X, (rocblas_int)ldx, sx, X,
      (rocblas_int)ldx, sx, &zero, part, k, sp, (rocblas_int)full);
  if (s == rocblas_status_success && rem > 0)
    s = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, k, k, (rocblas_int)rem, &one,
                      X + full * rc * ldx, (rocblas_int)ldx, X + full * rc * ldx, (rocblas_int)ldx, &zero,
                      part + full * sp, k);
  if (s != rocblas_status_success) {
    set_error("rocBLAS gemm failed");
    return SK_E_HIP;
  }
  return launch_sum_partials(part, (int)(full + (rem > 0 ? 1 : 0)), (int64_t)k * k, G, st);
}

}  // namespace sk
