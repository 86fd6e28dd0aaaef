// Gaussian sketch (Def. 1.4) launchers (gauss.hip).
#pragma once
#include "sk_common.hpp"

namespace sk {

// Workspace bytes of launch_gauss_rows for m_eff output columns.
size_t gauss_workspace(const sk_sketch* S, int m_eff);
// SA = G A (d x m, row-major, ldsa) and, when rhs is non-null, Srhs = G rhs
// (d doubles) in the same pass over the rows. A: n x m row-major F64.
int launch_gauss_rows(const sk_sketch* S, int64_t m, const double* A, int64_t lda, const double* rhs, double* SA,
                      int64_t ldsa, double* Srhs, void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace sk
