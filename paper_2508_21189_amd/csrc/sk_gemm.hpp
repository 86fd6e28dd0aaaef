// Dense GEMM on the matrix cores (gemm.hip).
#pragma once
#include "sk_common.hpp"

namespace sk {

struct GemmArgs {
  int64_t M, N, K;
  const void* A;
  const void* B;
  void* C;
  void* P;  // split-K partial sums ([split][M][N]), or null
  int64_t lda, ldb, ldc;
  int64_t k_per_split;
  double alpha, beta;
};

// Workspace bytes gemm_launch needs for this shape (split-K partials; 0 when
// the output tiles alone fill the chip).
size_t gemm_workspace(int dtype, int64_t M, int64_t N, int64_t K);
// Row-major C (M x N, ldc) = alpha op(A) op(B) + beta C with op(A) M x K and
// op(B) K x N; A is M x K (lda) or, transposed, K x M; B is K x N (ldb) or,
// transposed, N x K. dtype SK_F32 or SK_F64. beta = 0 does not read C.
int gemm_launch(int dtype, bool transA, bool transB, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
                int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* ws,
                size_t ws_bytes, hipStream_t st);

}  // namespace sk
