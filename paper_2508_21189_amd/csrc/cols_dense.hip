// Column mode (Y = A S^T, A rows x n row-major) for the two comparison
// sketches:
//   * Gaussian (Def. 1.4): S = G is d x n, small enough in this orientation
//     to be written out once (the same Philox + Box-Muller entries as the row
//     mode), after which Y = A G^T is one GEMM on the matrix cores (rocBLAS);
//   * SRTT (eq. 1.1) and SparseRTT (Def. 1.7): every row of A is one
//     length-npad Walsh-Hadamard transform, done in LDS by one workgroup per
//     row (npad <= 2^15 for 32-bit input, 2^14 for 64-bit), followed by the
//     gather of the d sampled entries (SRTT) or the signed sums of xi
//     selected entries per output (SparseRTT). The Rademacher signs are the
//     row mode's (index = column).
#include <algorithm>

#include "sk_drivers.hpp"
#include "sk_lowrank.hpp"

namespace sk {

template <typename T>
__global__ void gauss_fill_kernel(T* __restrict__ G, int64_t d, int64_t n, uint32_t k0, uint32_t k1, double scale) {
  const int64_t pairs = ((d + 1) / 2) * n;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < pairs; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = p / n, i = p - q * n;
    const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)q, kTagGauss}, k0, k1);
    const uint64_t x1 = ((uint64_t)w.x << 20) | (w.y >> 12);
    const uint64_t x2 = ((uint64_t)w.z << 20) | (w.w >> 12);
    const double u1 = ((double)x1 + 0.5) * 0x1p-52;
    const double u2 = ((double)x2 + 0.5) * 0x1p-52;
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    G[(2 * q) * n + i] = (T)(r * c * scale);
    if (2 * q + 1 < d) G[(2 * q + 1) * n + i] = (T)(r * s * scale);
  }
}

__device__ inline uint32_t srtt_word_c(uint64_t i, uint32_t k0, uint32_t k1) {
  const uint64_t blk = i >> 7;
  const U4 w = philox4x32_10(U4{(uint32_t)blk, (uint32_t)(blk >> 32), 0u, kTagSrttSign}, k0, k1);
  return word_of(w, (int)((i & 127) >> 5));
}

template <typename Tin>
__device__ inline float srtt_ld(const Tin* p);
template <>
__device__ inline float srtt_ld<float>(const float* p) {
  return *p;
}
template <>
__device__ inline float srtt_ld<uint16_t>(const uint16_t* p) {
  return bf16_to_f32(*p);
}

// One row per workgroup iteration: x = D a (padded), x = H x in LDS, then
// Y[r][j] = scale * sum_{i < xi} rho_ji x[sample[j*xi + i]] (SRTT: xi = 1,
// no signs, scale 1/sqrt(d)). Tacc: float for 32-bit and 16-bit input,
// double for 64-bit input.
template <typename Tin, typename Tacc>
__global__ void __launch_bounds__(1024) srtt_cols_kernel(const Tin* __restrict__ A, int64_t lda, int64_t rows,
                                                         int64_t n, int p, const int64_t* __restrict__ sample,
                                                         const int8_t* __restrict__ sgn, int xi, int64_t d,
                                                         double scale, uint32_t k0, uint32_t k1,
                                                         void* __restrict__ Y, int64_t ldy, int out_f64) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  Tacc* x = (Tacc*)smem;
  const int64_t npad = 1ll << p;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const Tin* a = A + r * lda;
    for (int64_t i = tid; i < npad; i += nt) {
      Tacc v = 0;
      if (i < n) {
        if constexpr (sizeof(Tin) == 8)
          v = a[i];
        else
          v = srtt_ld<Tin>(a + i);
        if ((srtt_word_c((uint64_t)i, k0, k1) >> (i & 31)) & 1u) v = -v;
      }
      x[i] = v;
    }
    __syncthreads();
    for (int64_t h = 1; h < npad; h <<= 1) {
      for (int64_t t = tid; t < npad / 2; t += nt) {
        const int64_t lo = (t / h) * 2 * h + (t % h);
        const Tacc u = x[lo], w = x[lo + h];
        x[lo] = u + w;
        x[lo + h] = u - w;
      }
      __syncthreads();
    }
    for (int64_t j = tid; j < d; j += nt) {
      Tacc v = 0;
      for (int i = 0; i < xi; ++i) {
        const Tacc u = x[sample[j * xi + i]];
        v += (sgn && sgn[j * xi + i] < 0) ? -u : u;
      }
      if (out_f64)
        ((double*)Y)[r * ldy + j] = (double)v * scale;
      else
        ((float*)Y)[r * ldy + j] = (float)((double)v * scale);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int launch_gauss_fill_f64(const sk_sketch* S, double* G, hipStream_t st) {
  const int64_t pairs = ((S->d + 1) / 2) * S->n;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((pairs + 255) / 256, 16384));
  hipLaunchKernelGGL(gauss_fill_kernel<double>, dim3(blocks), dim3(256), 0, st, G, S->d, S->n, S->k0, S->k1,
                     inv_sqrt_host((double)S->d));
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// Row mode with F32 input (SA = G A, A n x m): G (d x n, F32) is written out
// with the same entries and SA is one rocBLAS SGEMM, F32 accumulation; F64
// output goes through an F32 staging buffer. Used where G is small next to A
// (d x n x 4 bytes <= 8 GB).
size_t gauss_rows_f32_workspace(const sk_sketch* S, int64_t m, int dtype_out) {
  size_t b = ((size_t)S->d * S->n * 4 + 255) & ~(size_t)255;
  if (dtype_out == SK_F64) b += (size_t)S->d * m * 4;
  return b;
}

int launch_gauss_rows_f32(sk_sketch* S, int64_t m, const float* A, int64_t lda, int dtype_out, void* SA, int64_t ldsa,
                          void* ws, size_t ws_bytes, hipStream_t st) {
  if ((double)S->d * (double)S->n * 4.0 > 8.0 * (1ull << 30)) {
    set_error("sketch_apply: the F32 Gaussian row mode writes G out and needs d * n * 4 <= 8 GB");
    return SK_E_NOTSUP;
  }
  if (ws_bytes < gauss_rows_f32_workspace(S, m, dtype_out)) {
    set_error("sketch_apply: workspace too small (see sketch_workspace_size)");
    return SK_E_INVAL;
  }
  const int64_t pairs = ((S->d + 1) / 2) * S->n;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((pairs + 255) / 256, 16384));
  hipLaunchKernelGGL(gauss_fill_kernel<float>, dim3(blocks), dim3(256), 0, st, (float*)ws, S->d, S->n, S->k0, S->k1,
                     inv_sqrt_host((double)S->d));
  SK_HIP(hipGetLastError());
  const size_t gbytes = ((size_t)S->d * S->n * 4 + 255) & ~(size_t)255;
  if (dtype_out == SK_F32) {
    KernelTimer timer(S, st);
    return gemm_rm(S, SK_F32, false, false, S->d, m, S->n, 1.0, ws, S->n, A, lda, 0.0, SA, ldsa, st);
  }
  float* Yf = (float*)((char*)ws + gbytes);
  {
    KernelTimer timer(S, st);
    int rc = gemm_rm(S, SK_F32, false, false, S->d, m, S->n, 1.0, ws, S->n, A, lda, 0.0, Yf, m, st);
    if (rc != SK_OK) return rc;
  }
  return launch_convert(SK_F32, Yf, m, SK_F64, SA, ldsa, S->d, m, st);
}

int cols_dense_workspace(const sk_sketch* S, int dtype_in, int dtype_out, int64_t rows, size_t* bytes) {
  *bytes = 0;
  if (S->kind == SK_GAUSSIAN) {
    const size_t es = dtype_in == SK_F64 ? 8 : 4;
    *bytes = ((S->d * S->n * es + 255) & ~(size_t)255);
    if (dtype_in != SK_F64 && dtype_out == SK_F64) *bytes += (size_t)rows * S->d * 4;
    return SK_OK;
  }
  return SK_OK;  // SRTT column mode needs no workspace
}

int launch_cols_dense(sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                      int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st) {
  if (S->kind == SK_GAUSSIAN) {
    if (dtype_in == SK_BF16) {
      set_error("sketch_apply_T: the Gaussian sketch takes F64 or F32 input");
      return SK_E_NOTSUP;
    }
    size_t need = 0;
    cols_dense_workspace(S, dtype_in, dtype_out, rows, &need);
    if (ws_bytes < need) {
      set_error("sketch_apply_T: workspace too small (see sketch_workspace_size)");
      return SK_E_INVAL;
    }
    const int64_t pairs = ((S->d + 1) / 2) * S->n;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((pairs + 255) / 256, 16384));
    const double scale = inv_sqrt_host((double)S->d);
    if (dtype_in == SK_F64) {
      hipLaunchKernelGGL(gauss_fill_kernel<double>, dim3(blocks), dim3(256), 0, st, (double*)ws, S->d, S->n, S->k0,
                         S->k1, scale);
      SK_HIP(hipGetLastError());
      if (dtype_out != SK_F64) {
        set_error("sketch_apply_T: F64 Gaussian input gives F64 output");
        return SK_E_NOTSUP;
      }
      KernelTimer timer(S, st);
      return gemm_rm(S, SK_F64, false, true, rows, S->d, S->n, 1.0, A, lda, ws, S->n, 0.0, Y, ldy, st);
    }
    hipLaunchKernelGGL(gauss_fill_kernel<float>, dim3(blocks), dim3(256), 0, st, (float*)ws, S->d, S->n, S->k0, S->k1,
                       scale);
    SK_HIP(hipGetLastError());
    const size_t gbytes = ((S->d * S->n * 4 + 255) & ~(size_t)255);
    if (dtype_out == SK_F32) {
      KernelTimer timer(S, st);
      return gemm_rm(S, SK_F32, false, true, rows, S->d, S->n, 1.0, A, lda, ws, S->n, 0.0, Y, ldy, st);
    }
    float* Yf = (float*)((char*)ws + gbytes);
    {
      KernelTimer timer(S, st);
      int rc = gemm_rm(S, SK_F32, false, true, rows, S->d, S->n, 1.0, A, lda, ws, S->n, 0.0, Yf, S->d, st);
      if (rc != SK_OK) return rc;
    }
    return launch_convert(SK_F32, Yf, S->d, SK_F64, Y, ldy, rows, S->d, st);
  }
  // SRTT and SparseRTT
  const int p = S->log2npad;
  const size_t es = dtype_in == SK_F64 ? 8 : 4;
  const size_t lds = ((size_t)1 << p) * es;
  if (lds > 160 * 1024) {
    set_error("sketch_apply_T: SRTT/SparseRTT column mode needs npad * element size <= 160 KB");
    return SK_E_NOTSUP;
  }
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(rows, 4096));
  const double scale = trig_scale(S);
  const int of64 = dtype_out == SK_F64;
  KernelTimer timer(S, st);
  if (dtype_in == SK_F64) {
    auto kern = srtt_cols_kernel<double, double>;
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), lds, st, (const double*)A, lda, rows, S->n, p, S->d_sample, S->d_sgn,
                       S->xi, S->d, scale, S->k0, S->k1, Y, ldy, of64);
  } else if (dtype_in == SK_F32) {
    auto kern = srtt_cols_kernel<float, float>;
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), lds, st, (const float*)A, lda, rows, S->n, p, S->d_sample, S->d_sgn,
                       S->xi, S->d, scale, S->k0, S->k1, Y, ldy, of64);
  } else {
    auto kern = srtt_cols_kernel<uint16_t, float>;
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), lds, st, (const uint16_t*)A, lda, rows, S->n, p, S->d_sample,
                       S->d_sgn, S->xi, S->d, scale, S->k0, S->k1, Y, ldy, of64);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
