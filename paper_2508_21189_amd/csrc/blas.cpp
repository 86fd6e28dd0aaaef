// Plain library GEMMs (rocBLAS) used by the randomized SVD for its dense
// products: Y^T Y, Y R^-1, Q^T A, Q U, W^T Q_b^T. Row-major operands are
// passed as their column-major transposes (C^T = op(B)^T op(A)^T).
#include <rocblas/rocblas.h>

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

}  // namespace sk
