// SRTT sketch (eq. 1.1, Walsh-Hadamard) launchers (srtt.hip).
#pragma once
#include "sk_common.hpp"

namespace sk {

// Workspace bytes of launch_srtt_rows for m_eff output columns (the padded
// work matrix npad x m_eff, or 0 when npad <= 256).
size_t srtt_workspace(const sk_sketch* S, int m_eff);
// SA = (1/sqrt(d)) R H D A_pad (d x m row-major, ldsa) and, when rhs is
// non-null, Srhs for the extra column in the same passes. A: n x m row-major F64.
int launch_srtt_rows(const sk_sketch* S, int64_t m, const double* A, int64_t lda, const double* rhs, double* SA,
                     int64_t ldsa, double* Srhs, void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace sk
