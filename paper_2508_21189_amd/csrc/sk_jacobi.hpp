// One-sided (Hestenes) Jacobi SVD of a small square FP64 matrix and the
// rank-truncated solve from it, as device functions run by one whole
// workgroup (blockDim.x a multiple of 64, at most 1024 threads): used by the
// single-problem kernels and by the batched fallback kernel.
#pragma once
#include "sk_common.hpp"

namespace sk {

// Pair of round r (0 <= r < kp-1) for slot i (0 <= i < kp/2), kp even:
// slot 0 pairs r with kp-1; slot i pairs (r+i) and (r-i) mod (kp-1).
__device__ inline void rr_pair(int kp, int r, int i, int* p, int* q) {
  if (i == 0) {
    *p = r;
    *q = kp - 1;
  } else {
    const int m = kp - 1;
    *p = (r + i) % m;
    *q = ((r - i) % m + m) % m;
  }
}

__device__ inline void jacobi_svd_dev(const double* __restrict__ R, int k, double* __restrict__ U,
                                                          double* __restrict__ s, double* __restrict__ V,
                                                          double* __restrict__ Uc, double* __restrict__ Vc) {
  // Uc, Vc: column-major working copies (column j at j*k)
  __shared__ int rotated;
  __shared__ double sig[1024];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  for (int64_t idx = tid; idx < (int64_t)k * k; idx += blockDim.x) {
    const int64_t col = idx / k, row = idx - col * k;
    Uc[idx] = R[row * k + col];
    Vc[idx] = row == col ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kp = k + (k & 1);
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < kp - 1; ++r) {
      for (int i = wave; i < kp / 2; i += nwaves) {
        int p, q;
        rr_pair(kp, r, i, &p, &q);
        if (p >= k || q >= k) continue;
        double* up = Uc + (int64_t)p * k;
        double* uq = Uc + (int64_t)q * k;
        double a = 0, b = 0, g = 0;
        for (int row = lane; row < k; row += 64) {
          const double x = up[row], y = uq[row];
          a += x * x;
          b += y * y;
          g += x * y;
        }
        for (int o = 32; o > 0; o >>= 1) {
          a += __shfl_xor(a, o, 64);
          b += __shfl_xor(b, o, 64);
          g += __shfl_xor(g, o, 64);
        }
        if (fabs(g) > tol * sqrt(a * b) && g != 0.0) {
          const double zeta = (b - a) / (2.0 * g);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          double* vp = Vc + (int64_t)p * k;
          double* vq = Vc + (int64_t)q * k;
          for (int row = lane; row < k; row += 64) {
            const double x = up[row], y = uq[row];
            up[row] = c * x - sn * y;
            uq[row] = sn * x + c * y;
            const double xv = vp[row], yv = vq[row];
            vp[row] = c * xv - sn * yv;
            vq[row] = sn * xv + c * yv;
          }
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // singular values and normalized left vectors
  for (int j = wave; j < k; j += nwaves) {
    double* uj = Uc + (int64_t)j * k;
    double a = 0;
    for (int row = lane; row < k; row += 64) a += uj[row] * uj[row];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    const double sj = sqrt(a);
    if (sj > 0)
      for (int row = lane; row < k; row += 64) uj[row] /= sj;
    if (lane == 0 && j < 1024) sig[j] = sj;
  }
  __syncthreads();
  // rank by descending value (ties by index) and scatter
  for (int j = tid; j < k; j += blockDim.x) {
    const double sj = sig[j];
    int rank = 0;
    for (int i = 0; i < k; ++i) rank += (sig[i] > sj) || (sig[i] == sj && i < j);
    s[rank] = sj;
    for (int row = 0; row < k; ++row) {
      U[(int64_t)row * k + rank] = Uc[(int64_t)j * k + row];
      V[(int64_t)row * k + rank] = Vc[(int64_t)j * k + row];
    }
  }
}

// Rank-truncated solve from the SVD R = U diag(s) V^T (s descending):
// r = #{i : s_i > 5 eps s_1}; x = V_r diag(s_r)^{-1} U_r^T c. One workgroup.
__device__ inline void svd_solve_dev(const double* __restrict__ U, const double* __restrict__ s,
                                                         const double* __restrict__ V, const double* __restrict__ c,
                                                         int k, double eps, double* __restrict__ x,
                                                         double* __restrict__ z, int* __restrict__ rank_out) {
  __shared__ int rank;
  if (threadIdx.x == 0) {
    const double thr = 5.0 * eps * s[0];
    int r = 0;
    while (r < k && s[r] > thr) ++r;
    rank = r;
    *rank_out = r;
  }
  __syncthreads();
  const int r = rank;
  for (int j = threadIdx.x; j < r; j += blockDim.x) {
    double t = 0;
    for (int i = 0; i < k; ++i) t += U[(int64_t)i * k + j] * c[i];
    z[j] = t / s[j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double t = 0;
    for (int j = 0; j < r; ++j) t += V[(int64_t)i * k + j] * z[j];
    x[i] = t;
  }
}

}  // namespace sk
