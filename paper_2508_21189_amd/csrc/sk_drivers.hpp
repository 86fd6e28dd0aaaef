// Dispatch layer between the C-ABI and the kernel launchers.
#pragma once
#include "sk_launch.hpp"

namespace sk {

int handle_workspace(sk_sketch* S, size_t bytes, void** out, hipStream_t st);
// Stream-ordered growth of a handle-owned buffer (no device-wide sync).
int grow_buffer(void** buf, size_t* cur, size_t bytes, hipStream_t st);

// Bytes of workspace needed by sketch_apply (op 0) or sketch_apply_T (op 1).
int apply_workspace(const sk_sketch* S, int op, int dtype_in, int64_t m, size_t* bytes);

// Exact workspace bytes of sketch_apply for this A (alignment-dependent plan).
int apply_workspace_for(const sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, size_t* bytes);

// SA = S A for a column-major A (n x m, lda >= n): a row-major copy in the
// workspace (op 2 of apply_workspace), then the row-mode apply.
int apply_T_colmajor(sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                     int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st);
int apply_colmajor(sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, int dtype_out, void* SA,
                   int64_t ldsa, void* ws, size_t ws_bytes, hipStream_t st);
int apply_dispatch(sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, int dtype_out, void* SA,
                   int64_t ldsa, void* ws, size_t ws_bytes, hipStream_t st);
int apply_T_dispatch(sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                     int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st);

// out (rows x cols, ldo) = (Tout) in (rows x cols, ldi); any dtype pair.
int launch_convert(int dtype_in, const void* in, int64_t ldi, int dtype_out, void* out, int64_t ldo, int64_t rows,
                   int64_t cols, hipStream_t st);

// Row mode of the Gaussian sketch for F32 input (cols_dense.hip): G written
// out (d x n F32) and one SGEMM; F32 or F64 output.
size_t gauss_rows_f32_workspace(const sk_sketch* S, int64_t m, int dtype_out);
int launch_gauss_rows_f32(sk_sketch* S, int64_t m, const float* A, int64_t lda, int dtype_out, void* SA, int64_t ldsa,
                          void* ws, size_t ws_bytes, hipStream_t st);

// Column mode of the Gaussian and SRTT sketches (cols_dense.hip).
int cols_dense_workspace(const sk_sketch* S, int dtype_in, int dtype_out, int64_t rows, size_t* bytes);
int launch_cols_dense(sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                      int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st);

// Frees driver-owned device memory attached to a handle.
void drivers_release(sk_sketch* S);

}  // namespace sk
