// The low-rank drivers' dense products (Y^T Y, Y R^-1, Q^T A, Q U, W^T Q_b^T)
// on the project's matrix-core GEMM (gemm.hip). Split-K partial sums live in
// a handle-owned buffer that grows on the call's stream.
#include "sk_drivers.hpp"
#include "sk_gemm.hpp"
#include "sk_lowrank.hpp"

namespace sk {

void blas_release(sk_sketch* S) {
  if (S->gws) (void)hipFreeAsync(S->gws, nullptr);
  S->gws = nullptr;
  S->gws_bytes = 0;
}

int gemm_rm(sk_sketch* S, int dtype, bool transA, bool transB, int64_t M, int64_t N, int64_t K, double alpha,
            const void* A, int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, hipStream_t st) {
  const size_t need = gemm_workspace(dtype, M, N, K);
  if (need > 0) {
    const int rc = grow_buffer(&S->gws, &S->gws_bytes, need, st);
    if (rc != SK_OK) return rc;
  }
  return gemm_launch(dtype, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, S->gws, S->gws_bytes, st);
}

int gram_rm(sk_sketch* S, const double* X, int64_t ldx, int64_t r, int k, double* G, double* part, int max_chunks,
            hipStream_t st) {
  // G = X^T X: the GEMM splits the long dimension r itself (in a fixed order)
  (void)part;
  (void)max_chunks;
  return gemm_rm(S, SK_F64, true, false, k, k, r, 1.0, X, ldx, X, ldx, 0.0, G, k, st);
}

}  // namespace sk
