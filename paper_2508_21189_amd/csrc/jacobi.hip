// One-sided (Hestenes) Jacobi SVD of a small square FP64 matrix, one
// workgroup: columns of U = R are orthogonalized by plane rotations applied
// to U and V (V starts as I) in round-robin order (each round, disjoint pairs
// processed by different waves), until a sweep makes no rotation. Then
// s_j = ||u_j||, u_j /= s_j, and columns are ranked by descending s.
#include "sk_dense.hpp"
#include "sk_jacobi.hpp"

#include <algorithm>

namespace sk {

__global__ void __launch_bounds__(1024) jacobi_svd_kernel(const double* __restrict__ R, int k, double* __restrict__ U,
                                                          double* __restrict__ s, double* __restrict__ V,
                                                          double* __restrict__ Uc, double* __restrict__ Vc) {
  jacobi_svd_dev(R, k, U, s, V, Uc, Vc);
}

__global__ void __launch_bounds__(1024) svd_solve_kernel(const double* __restrict__ U, const double* __restrict__ s,
                                                         const double* __restrict__ V, const double* __restrict__ c,
                                                         int k, double eps, double* __restrict__ x,
                                                         double* __restrict__ z, int* __restrict__ rank_out) {
  svd_solve_dev(U, s, V, c, k, eps, x, z, rank_out);
}

// The rank test of Alg. 3 without an SVD when it certainly passes. For upper
// triangular R (k x k) and X = R^-1, s_1 <= ||R||_F and s_k >= 1 / ||X||_F, so
// ||R||_F ||X||_F < margin / (5 eps) (margin 1e-3 leaves room for the rounding
// of X) implies s_k > 5 eps s_1: the rank is k and the truncated-SVD solution
// is x = R^-1 c = X c. Otherwise *rank_out = -1 and x is not written (the
// caller takes the SVD). Only the upper triangles of R and X are read.
__device__ __forceinline__ void certified_tri_solve_dev(const double* __restrict__ R, const double* __restrict__ X,
                                                        const double* __restrict__ c, int k, double eps,
                                                        double* __restrict__ x, int* __restrict__ rank_out) {
  __shared__ double part[2][16];
  __shared__ int ok;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double r2 = 0, x2 = 0;
  for (int64_t idx = tid; idx < (int64_t)k * k; idx += blockDim.x) {
    const int i = (int)(idx / k), j = (int)(idx - (int64_t)i * k);
    if (j >= i) {
      r2 += R[idx] * R[idx];
      x2 += X[idx] * X[idx];
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    r2 += __shfl_xor(r2, o, 64);
    x2 += __shfl_xor(x2, o, 64);
  }
  if (lane == 0) {
    part[0][wave] = r2;
    part[1][wave] = x2;
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0, tx = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      tr += part[0][w];
      tx += part[1][w];
    }
    const double cond = sqrt(tr) * sqrt(tx);
    ok = (cond == cond && cond < 1e-3 / (5.0 * eps)) ? 1 : 0;  // false for NaN and Inf
    *rank_out = ok ? k : -1;
  }
  __syncthreads();
  if (!ok) return;
  for (int i = tid; i < k; i += blockDim.x) {
    double t = 0;
    for (int j = i; j < k; ++j) t += X[(int64_t)i * k + j] * c[j];
    x[i] = t;
  }
}

__global__ void __launch_bounds__(1024) certified_tri_solve_kernel(const double* __restrict__ R,
                                                                   const double* __restrict__ X,
                                                                   const double* __restrict__ c, int k, double eps,
                                                                   double* __restrict__ x, int* __restrict__ rank_out) {
  certified_tri_solve_dev(R, X, c, k, eps, x, rank_out);
}

__global__ void __launch_bounds__(1024) certified_tri_solve_batched_kernel(const QrBatch* __restrict__ B, double eps) {
  const QrBatch& p = B[blockIdx.x];
  if (p.k == 0) return;
  certified_tri_solve_dev(p.R, p.X, p.c, p.k, eps, p.x, p.rank);
}

__global__ void __launch_bounds__(1024) svd_fallback_batched_kernel(const QrBatch* __restrict__ B, double eps) {
  const QrBatch& p = B[blockIdx.x];
  if (p.k == 0 || !p.Uc) return;
  // (every thread reads the rank before any thread of a problem that goes on
  // can write it: the first write comes after the SVD's barriers)
  if (*p.rank >= 0) return;
  jacobi_svd_dev(p.R, p.k, p.X, p.sv, p.XT, p.Uc, p.Vc);
  __syncthreads();
  svd_solve_dev(p.X, p.sv, p.XT, p.c, p.k, eps, p.x, p.z, p.rank);
}

int svd_fallback_batched(const QrBatch* B, int nprob, double eps, hipStream_t st) {
  if (nprob <= 0) return SK_OK;
  hipLaunchKernelGGL(svd_fallback_batched_kernel, dim3((unsigned)nprob), dim3(1024), 0, st, B, eps);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_certified_tri_solve(const double* R, const double* X, const double* c, int k, double eps, double* x,
                               int* rank_out, hipStream_t st) {
  hipLaunchKernelGGL(certified_tri_solve_kernel, dim3(1), dim3(1024), 0, st, R, X, c, k, eps, x, rank_out);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int certified_tri_solve_batched(const QrBatch* B, int nprob, double eps, hipStream_t st) {
  if (nprob <= 0) return SK_OK;
  hipLaunchKernelGGL(certified_tri_solve_batched_kernel, dim3((unsigned)nprob), dim3(1024), 0, st, B, eps);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_svd_solve(const double* U, const double* s, const double* V, const double* c, int k, double eps, double* x,
                     double* z, int* rank_out, hipStream_t st) {
  hipLaunchKernelGGL(svd_solve_kernel, dim3(1), dim3(1024), 0, st, U, s, V, c, k, eps, x, z, rank_out);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_jacobi_svd(const double* R, int k, double* U, double* s, double* V, double* work, hipStream_t st) {
  if (k > 1024) {
    set_error("Jacobi SVD: at most 1024 columns");
    return SK_E_NOTSUP;
  }
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(1), dim3(1024), 0, st, R, k, U, s, V, work, work + (size_t)k * k);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
