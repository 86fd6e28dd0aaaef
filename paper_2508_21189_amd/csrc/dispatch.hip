// Sketch-kind dispatch for sketch_apply / sketch_apply_T, plus small helpers.
#include "sk_drivers.hpp"
#include "sk_gauss.hpp"
#include "sk_srtt.hpp"

#include <algorithm>

namespace sk {

template <typename Ti, typename To>
__global__ void convert_kernel(const Ti* __restrict__ in, int64_t ldi, To* __restrict__ out, int64_t ldo,
                               int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / cols, c = idx - r * cols;
    out[r * ldo + c] = (To)in[r * ldi + c];
  }
}

template <typename To>
__global__ void convert_bf16_kernel(const uint16_t* __restrict__ in, int64_t ldi, To* __restrict__ out, int64_t ldo,
                                    int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / cols, c = idx - r * cols;
    out[r * ldo + c] = (To)bf16_to_f32(in[r * ldi + c]);
  }
}

int launch_convert(int dtype_in, const void* in, int64_t ldi, int dtype_out, void* out, int64_t ldo, int64_t rows,
                   int64_t cols, hipStream_t st) {
  const int64_t total = rows * cols;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192));
  if (dtype_out != SK_F64 && dtype_out != SK_F32) {
    set_error("convert: output must be F64 or F32");
    return SK_E_NOTSUP;
  }
#define SK_CONV(TI, TO) \
  hipLaunchKernelGGL((convert_kernel<TI, TO>), dim3(blocks), dim3(256), 0, st, (const TI*)in, ldi, (TO*)out, ldo, rows, cols)
  if (dtype_in == SK_F64 && dtype_out == SK_F64) SK_CONV(double, double);
  else if (dtype_in == SK_F64 && dtype_out == SK_F32) SK_CONV(double, float);
  else if (dtype_in == SK_F32 && dtype_out == SK_F64) SK_CONV(float, double);
  else if (dtype_in == SK_F32 && dtype_out == SK_F32) SK_CONV(float, float);
  else if (dtype_out == SK_F64)
    hipLaunchKernelGGL((convert_bf16_kernel<double>), dim3(blocks), dim3(256), 0, st, (const uint16_t*)in, ldi,
                       (double*)out, ldo, rows, cols);
  else
    hipLaunchKernelGGL((convert_bf16_kernel<float>), dim3(blocks), dim3(256), 0, st, (const uint16_t*)in, ldi,
                       (float*)out, ldo, rows, cols);
#undef SK_CONV
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// Column-major A (n x m, column c at A + c*lda) to row-major At (n x m,
// ld ldt >= m), through 64 x 64 tiles in LDS so that both the reads (along a column)
// and the writes (along a row) are coalesced. Elements are moved as raw
// bytes of their type.
template <typename T>
__global__ void __launch_bounds__(256) colmajor_to_rowmajor_kernel(const T* __restrict__ A, int64_t lda, int64_t n,
                                                                    int64_t m, T* __restrict__ At, int64_t ldt) {
  __shared__ T tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4 threads
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t i = i0 + tx, c = c0 + cc;
    if (i < n && c < m) tile[cc][tx] = A[c * lda + i];
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii, c = c0 + tx;
    if (i < n && c < m) At[i * ldt + c] = tile[tx][ii];
  }
}

static int launch_colmajor_to_rowmajor(int dtype, const void* A, int64_t lda, int64_t n, int64_t m, void* At,
                                       int64_t ldt, hipStream_t st) {
  const int64_t gx = (n + 63) / 64, gy = (m + 63) / 64;
  if (gx > 0x7fffffff || gy > 65535) {
    set_error("sketch_apply: column-major A too large for the transpose grid");
    return SK_E_NOTSUP;
  }
  const dim3 grid((unsigned)gx, (unsigned)gy);
  if (dtype == SK_F64)
    hipLaunchKernelGGL(colmajor_to_rowmajor_kernel<double>, grid, dim3(256), 0, st, (const double*)A, lda, n, m,
                       (double*)At, ldt);
  else if (dtype == SK_F32)
    hipLaunchKernelGGL(colmajor_to_rowmajor_kernel<float>, grid, dim3(256), 0, st, (const float*)A, lda, n, m,
                       (float*)At, ldt);
  else
    hipLaunchKernelGGL(colmajor_to_rowmajor_kernel<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)A, lda, n,
                       m, (uint16_t*)At, ldt);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// The row-major copy of a column-major A: rows padded to a multiple of 8
// elements, so that every row starts 16-byte aligned and the apply takes its
// 16-byte loads whatever m is (the summation order does not depend on the
// padding); its bytes, 256-aligned.
static int64_t colmajor_copy_ld(int64_t m) { return (m + 7) & ~(int64_t)7; }
static size_t colmajor_copy_bytes(const sk_sketch* S, int dtype_in, int64_t m) {
  return ((size_t)S->n * colmajor_copy_ld(m) * dtype_size(dtype_in) + 255) & ~(size_t)255;
}

// The d x rows result S A^T of sketch_apply_T with column-major A, before
// its transpose (F64 output is the worst case), 256-aligned.
static size_t colmajor_T_result_bytes(const sk_sketch* S, int64_t rows) {
  return ((size_t)S->d * rows * 8 + 255) & ~(size_t)255;
}

int apply_workspace(const sk_sketch* S, int op, int dtype_in, int64_t m, size_t* bytes) {
  if (op == 3) {  // sketch_apply_T with column-major A: op 0 on A^T (m = rows), then the result
    size_t rest = 0;
    int rc = apply_workspace(S, 0, dtype_in, m, &rest);
    if (rc != SK_OK) return rc;
    *bytes = colmajor_T_result_bytes(S, m) + rest;
    return SK_OK;
  }
  if (op == 2) {  // sketch_apply with column-major A: the row-major copy, then op 0 on it
    size_t rest = 0;
    int rc = apply_workspace(S, 0, dtype_in, m, &rest);
    if (rc != SK_OK) return rc;
    *bytes = colmajor_copy_bytes(S, dtype_in, m) + rest;
    return SK_OK;
  }
  *bytes = 0;
  if (op == 0 && S->kind == SK_SPARSESTACK) {
    RowsPlan p;
    // alignment is unknown here: plan for the 16-byte path (same partial size)
    int rc = plan_rows(S, dtype_in, m, nullptr, m, &p);
    if (rc != SK_OK) {
      // fall back to a size estimate independent of alignment
      p.n_chunks = 256;
      p.partial_bytes = (size_t)p.n_chunks * S->d * m * (dtype_in == SK_F64 ? 8 : 4);
      p.plan_bytes = (size_t)((S->n + 15) / 16 + 1) * S->zeta * (2 * (S->nb + 1) + 64);
    }
    *bytes = p.partial_bytes + p.plan_bytes;
  } else if (op == 0 && S->kind == SK_GAUSSIAN) {
    // F64 input: split-K partials; F32 input: G written out (+ F32 staging
    // of an F64 result)
    *bytes = dtype_in == SK_F32 ? gauss_rows_f32_workspace(S, m, SK_F64) : gauss_workspace(S, (int)m);
  } else if (op == 0 && trig_kind(S->kind)) {
    *bytes = srtt_workspace(S, (int)m);
  } else if (op == 1 && S->kind == SK_SPARSESTACK) {
    if (!cols_kernel_fits(S, dtype_in)) {  // through the row-mode apply of A^T
      size_t rest = 0;
      int rc = apply_workspace(S, 2, dtype_in, m, &rest);
      if (rc != SK_OK) return rc;
      *bytes = colmajor_T_result_bytes(S, m) + rest;
      return SK_OK;
    }
    return cols_workspace(S, dtype_in, bytes);
  } else if (op == 1 && (S->kind == SK_GAUSSIAN || trig_kind(S->kind))) {
    // m is the number of rows of A in this orientation; F64 output is the worst case
    return cols_dense_workspace(S, dtype_in, SK_F64, m, bytes);
  }
  return SK_OK;
}

int apply_workspace_for(const sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, size_t* bytes) {
  *bytes = 0;
  if (S->kind == SK_SPARSESTACK) {
    RowsPlan p;
    int rc = plan_rows(S, dtype_in, m, A, lda, &p);
    if (rc != SK_OK) return rc;
    *bytes = p.partial_bytes + p.plan_bytes;
    return SK_OK;
  }
  return apply_workspace(S, 0, dtype_in, m, bytes);
}

int apply_colmajor(sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, int dtype_out, void* SA,
                   int64_t ldsa, void* ws, size_t ws_bytes, hipStream_t st) {
  size_t need = 0;
  int rc = apply_workspace(S, 2, dtype_in, m, &need);
  if (rc != SK_OK) return rc;
  void* w = ws;
  if (w) {
    if (ws_bytes < need) {
      set_error("sketch_apply: workspace too small for column-major A (see sketch_workspace_size, op 2)");
      return SK_E_INVAL;
    }
  } else {
    rc = handle_workspace(S, need, &w, st);
    if (rc != SK_OK) return rc;
  }
  const size_t cb = colmajor_copy_bytes(S, dtype_in, m);
  const int64_t ldt = colmajor_copy_ld(m);
  rc = launch_colmajor_to_rowmajor(dtype_in, A, lda, S->n, m, w, ldt, st);
  if (rc != SK_OK) return rc;
  return apply_dispatch(S, dtype_in, m, w, ldt, dtype_out, SA, ldsa, (char*)w + cb, need - cb, st);
}

// Y = A S^T for column-major A (rows x n): the n x rows row-major matrix A^T
// is sketched by the row-mode apply into the workspace (d x rows), which is
// then transposed into Y.
int apply_T_colmajor(sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                     int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st) {
  size_t need = 0;
  int rc = apply_workspace_for(S, dtype_in, rows, A, lda, &need);
  if (rc != SK_OK) return rc;
  const size_t rb = colmajor_T_result_bytes(S, rows);
  need += rb;
  void* w = ws;
  if (w) {
    if (ws_bytes < need) {
      set_error("sketch_apply_T: workspace too small for column-major A (see sketch_workspace_size, op 3)");
      return SK_E_INVAL;
    }
  } else {
    rc = handle_workspace(S, need, &w, st);
    if (rc != SK_OK) return rc;
  }
  rc = apply_dispatch(S, dtype_in, rows, A, lda, dtype_out, w, rows, (char*)w + rb, need - rb, st);
  if (rc != SK_OK) return rc;
  // S A^T is d x rows row-major, i.e. the column-major rows x d matrix Y
  return launch_colmajor_to_rowmajor(dtype_out, w, rows, rows, S->d, Y, ldy, st);
}

int apply_dispatch(sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, int dtype_out, void* SA,
                   int64_t ldsa, void* ws, size_t ws_bytes, hipStream_t st) {
  switch (S->kind) {
    case SK_IDENTITY_TEST:
      return launch_convert(dtype_in, A, lda, dtype_out, SA, ldsa, S->n, m, st);
    case SK_SPARSESTACK: {
      RowsPlan p;
      int rc = plan_rows(S, dtype_in, m, A, lda, &p);
      if (rc != SK_OK) return rc;
      void* w = ws;
      if (w) {
        if (ws_bytes < p.partial_bytes + p.plan_bytes) {
          set_error("sketch_apply: workspace too small (see sketch_workspace_size)");
          return SK_E_INVAL;
        }
      } else {
        rc = handle_workspace(S, p.partial_bytes + p.plan_bytes, &w, st);
        if (rc != SK_OK) return rc;
      }
      return launch_rows_apply(S, p, dtype_in, m, A, lda, dtype_out, SA, ldsa, w, st);
    }
    case SK_GAUSSIAN: {
      if (dtype_in == SK_F32) {
        const size_t need = gauss_rows_f32_workspace(S, m, dtype_out);
        void* w = ws;
        if (w) {
          if (ws_bytes < need) {
            set_error("sketch_apply: workspace too small (see sketch_workspace_size)");
            return SK_E_INVAL;
          }
        } else {
          int rc = handle_workspace(S, need, &w, st);
          if (rc != SK_OK) return rc;
        }
        return launch_gauss_rows_f32(S, m, (const float*)A, lda, dtype_out, SA, ldsa, w, need, st);
      }
      if (dtype_in != SK_F64 || dtype_out != SK_F64) {
        set_error("sketch_apply: the Gaussian sketch takes F64 (F64 output) or F32 input");
        return SK_E_NOTSUP;
      }
      const size_t need = gauss_workspace(S, (int)m);
      void* w = ws;
      if (w) {
        if (ws_bytes < need) {
          set_error("sketch_apply: workspace too small (see sketch_workspace_size)");
          return SK_E_INVAL;
        }
      } else {
        int rc = handle_workspace(S, need, &w, st);
        if (rc != SK_OK) return rc;
      }
      return launch_gauss_rows(S, m, (const double*)A, lda, nullptr, (double*)SA, ldsa, nullptr, w, need, st);
    }
    case SK_SRTT:
    case SK_SPARSERTT: {
      if (dtype_in != SK_F64 || dtype_out != SK_F64) {
        set_error("sketch_apply: the SRTT and SparseRTT sketches take and return F64");
        return SK_E_NOTSUP;
      }
      const size_t need = srtt_workspace(S, (int)m);
      void* w = ws;
      if (w) {
        if (ws_bytes < need) {
          set_error("sketch_apply: workspace too small (see sketch_workspace_size)");
          return SK_E_INVAL;
        }
      } else {
        int rc = handle_workspace(S, need, &w, st);
        if (rc != SK_OK) return rc;
      }
      return launch_srtt_rows(S, m, (const double*)A, lda, nullptr, (double*)SA, ldsa, nullptr, w, need, st);
    }
    default:
      set_error("sketch_apply: this sketch kind is not available yet");
      return SK_E_NOTSUP;
  }
}

// Y = A S^T for row-major A with more buckets per block than the column
// kernel holds: row-major A is the column-major n x rows matrix A^T, which
// sketch_apply's column-major path (a tiled transpose into the workspace, then
// the row-mode apply) turns into S A^T (d x rows), transposed into Y.
static int apply_T_via_rows(sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out,
                            void* Y, int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st) {
  size_t rest = 0;
  int rc = apply_workspace(S, 2, dtype_in, rows, &rest);
  if (rc != SK_OK) return rc;
  const size_t rb = colmajor_T_result_bytes(S, rows);
  void* w = ws;
  if (w) {
    if (ws_bytes < rb + rest) {
      set_error("sketch_apply_T: workspace too small (see sketch_workspace_size)");
      return SK_E_INVAL;
    }
  } else {
    rc = handle_workspace(S, rb + rest, &w, st);
    if (rc != SK_OK) return rc;
  }
  rc = apply_colmajor(S, dtype_in, rows, A, lda, dtype_out, w, rows, (char*)w + rb, rest, st);
  if (rc != SK_OK) return rc;
  return launch_colmajor_to_rowmajor(dtype_out, w, rows, rows, S->d, Y, ldy, st);
}

int apply_T_dispatch(sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                     int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st) {
  if (S->kind == SK_IDENTITY_TEST) return launch_convert(dtype_in, A, lda, dtype_out, Y, ldy, rows, S->n, st);
  if (S->kind == SK_SPARSESTACK && !cols_kernel_fits(S, dtype_in))
    return apply_T_via_rows(S, dtype_in, rows, A, lda, dtype_out, Y, ldy, ws, ws_bytes, st);
  if (S->kind == SK_SPARSESTACK) {
    size_t need = 0;
    int rc = cols_workspace(S, dtype_in, &need);
    if (rc != SK_OK) return rc;
    void* w = ws;
    if (w) {
      if (ws_bytes < need) {
        set_error("sketch_apply_T: workspace too small (see sketch_workspace_size)");
        return SK_E_INVAL;
      }
    } else {
      rc = handle_workspace(S, need, &w, st);
      if (rc != SK_OK) return rc;
    }
    return launch_cols_apply(S, dtype_in, rows, A, lda, dtype_out, Y, ldy, w, need, st);
  }
  if (S->kind == SK_GAUSSIAN || trig_kind(S->kind)) {
    size_t need = 0;
    int rc = cols_dense_workspace(S, dtype_in, dtype_out, rows, &need);
    if (rc != SK_OK) return rc;
    void* w = ws;
    if (need > 0) {
      if (w) {
        if (ws_bytes < need) {
          set_error("sketch_apply_T: workspace too small (see sketch_workspace_size)");
          return SK_E_INVAL;
        }
      } else {
        rc = handle_workspace(S, need, &w, st);
        if (rc != SK_OK) return rc;
      }
    }
    return launch_cols_dense(S, dtype_in, rows, A, lda, dtype_out, Y, ldy, w, need, st);
  }
  set_error("sketch_apply_T: this sketch kind is not available yet");
  return SK_E_NOTSUP;
}


}  // namespace sk
