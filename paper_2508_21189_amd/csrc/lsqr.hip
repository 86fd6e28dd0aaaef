// LSQR (Paige & Saunders, ACM TOMS 8, 1982) on the preconditioned operator
// M = A Rinv, with every step on the device:
//   * one fused pass over the row-major FP64 A per iteration computes
//     p = A w + coef * u (w = Rinv v, u the stored left vector), overwrites u
//     with p, and accumulates A^T p and ||p||^2 per workgroup (M v and M^T u
//     of the bidiagonalization in a single sweep of A);
//   * a column reduction sums the workgroup partials in a fixed order;
//   * one small workgroup runs the rest of the iteration on length-m vectors:
//     v = Rinv^T (A^T u) - beta v, the plane rotation, the updates of the
//     solution and the search direction, the stopping test, and w = Rinv v.
// The recurrence scalars live in device memory, so iterations are launched
// back to back; once the stopping test holds, later launches return at once.
#include "sk_lsqr.hpp"

#include <algorithm>

namespace sk {

// p_i = a_i . w + coef * u_i (u_i <- p_i); part[g][j] = sum_i a_ij p_i (j < m),
// part[g][m] = sum_i p_i^2 over the rows of workgroup g. Each wave takes rows
// wave, wave + 4, ...; lanes hold columns (MPL per lane); U rows in flight.
template <int MPL, int U>
__global__ void __launch_bounds__(256) lsqr_pass_kernel(const double* __restrict__ A, int64_t lda, int64_t n, int m,
                                                        const double* __restrict__ w, const double* __restrict__ coefp,
                                                        const int* __restrict__ donep, double* __restrict__ u,
                                                        double* __restrict__ part, int64_t rows_per_wg) {
  if (donep && *donep) return;
  __shared__ double red[4][MPL * 64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double coef = *coefp;
  double wl[MPL], q[MPL];
#pragma unroll
  for (int k = 0; k < MPL; ++k) {
    const int c = lane + 64 * k;
    wl[k] = c < m ? w[c] : 0.0;
    q[k] = 0.0;
  }
  double pp = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(n, r0 + rows_per_wg);
  int64_t i = r0 + wave;
  for (; i + 4 * (U - 1) < r1; i += 4 * U) {
    double x[U][MPL], dt[U], uo[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const double* a = A + (i + 4 * r) * lda;
#pragma unroll
      for (int k = 0; k < MPL; ++k) {
        const int c = lane + 64 * k;
        x[r][k] = c < m ? a[c] : 0.0;
      }
      uo[r] = u[i + 4 * r];
    }
#pragma unroll
    for (int r = 0; r < U; ++r) {
      dt[r] = 0.0;
#pragma unroll
      for (int k = 0; k < MPL; ++k) dt[r] += x[r][k] * wl[k];
    }
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
      for (int r = 0; r < U; ++r) dt[r] += __shfl_xor(dt[r], o, 64);
    }
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const double p = dt[r] + coef * uo[r];
      if (lane == 0) u[i + 4 * r] = p;
#pragma unroll
      for (int k = 0; k < MPL; ++k) q[k] += x[r][k] * p;
      pp += p * p;
    }
  }
  for (; i < r1; i += 4) {
    const double* a = A + i * lda;
    double x0[MPL];
    double d0 = 0;
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
      const int c = lane + 64 * k;
      x0[k] = c < m ? a[c] : 0.0;
      d0 += x0[k] * wl[k];
    }
    for (int o = 32; o > 0; o >>= 1) d0 += __shfl_xor(d0, o, 64);
    const double p0 = d0 + coef * u[i];
    if (lane == 0) u[i] = p0;
#pragma unroll
    for (int k = 0; k < MPL; ++k) q[k] += x0[k] * p0;
    pp += p0 * p0;
  }
  // workgroup partial (waves summed in a fixed order)
#pragma unroll
  for (int k = 0; k < MPL; ++k) red[wave][lane + 64 * k] = q[k];
  if (lane == 0) red[wave][MPL * 64] = pp;
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * (m + 1);
  for (int j = tid; j <= m; j += blockDim.x) {
    const int jj = j < m ? j : MPL * 64;
    out[j] = ((red[0][jj] + red[1][jj]) + red[2][jj]) + red[3][jj];
  }
}

// out[j] = sum_g part[g][j], g in increasing order.
__global__ void reduce_cols_kernel(const double* __restrict__ part, int ngroups, int width, const int* __restrict__ donep,
                                   double* __restrict__ out) {
  if (donep && *donep) return;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < width; j += gridDim.x * blockDim.x) {
    double s = 0;
    for (int g = 0; g < ngroups; ++g) s += part[(int64_t)g * width + j];
    out[j] = s;
  }
}

__device__ inline double wg_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int k = 0; k < nw; ++k) s += red[k];
  return s;
}

// t = Rinv^T x (Rinv upper k x k): t_j = sum_{i <= j} Rinv[i][j] x_i
__device__ inline void rinv_t_apply(const double* Rinv, int k, const double* x, double* t) {
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double s = 0;
    for (int i = 0; i <= j; ++i) s += Rinv[(int64_t)i * k + j] * x[i];
    t[j] = s;
  }
}
// t = Rinv x: t_i = sum_{j >= i} Rinv[i][j] x_j
__device__ inline void rinv_apply(const double* Rinv, int k, const double* x, double* t) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double s = 0;
    for (int j = i; j < k; ++j) s += Rinv[(int64_t)i * k + j] * x[j];
    t[i] = s;
  }
}

// Constants of one solve; coef = -1 makes the first pass form A x0 - b.
__global__ void lsqr_setup_kernel(LsqrDev* st, double tol, int maxit) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->tol = tol;
    st->maxit = maxit;
    st->minus_one = -1.0;
    st->coef = -1.0;
    st->done = 0;
    st->converged = 0;
    st->iters = 0;
  }
}

// After the pass p0 = A x0 - b: q = A^T p0, pp = ||p0||^2 (in qv[m]).
// beta u1 = r0 = -p0; alpha v1 = Rinv^T A^T u1; w = v1; phibar = beta; rhobar = alpha.
__global__ void __launch_bounds__(512) lsqr_init_kernel(LsqrDev* st, const double* __restrict__ qv,
                                                        const double* __restrict__ Rinv, int k, double* __restrict__ v,
                                                        double* __restrict__ wd, double* __restrict__ y,
                                                        double* __restrict__ wv, double* __restrict__ tmp) {
  __shared__ double red[8];
  const double beta = sqrt(qv[k]);
  const double sc = beta > 0 ? -1.0 / beta : 0.0;  // A^T u1 = -q / beta
  for (int j = threadIdx.x; j < k; j += blockDim.x) tmp[j] = qv[j] * sc;
  __syncthreads();
  rinv_t_apply(Rinv, k, tmp, v);
  __syncthreads();
  double part = 0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) part += v[j] * v[j];
  const double alpha = sqrt(wg_sum(part, red));
  const double ia = alpha > 0 ? 1.0 / alpha : 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    v[j] *= ia;
    wd[j] = v[j];
    y[j] = 0.0;
  }
  __syncthreads();
  rinv_apply(Rinv, k, v, wv);
  if (threadIdx.x == 0) {
    st->beta = beta;
    st->alpha = alpha;
    st->bnorm = beta;
    st->phibar = beta;
    st->rhobar = alpha;
    st->anorm2 = 0.0;
    st->rnorm = beta;
    st->arnorm = alpha * beta;
    st->iters = 0;
    st->converged = (beta == 0.0 || alpha == 0.0) ? 1 : 0;
    st->done = (st->converged || st->maxit <= 0) ? 1 : 0;
    st->uscale = sc;                  // u1 = sc * (stored p0)
    st->coef = -alpha * sc;           // next pass: p = A w - alpha u1
  }
}

// One LSQR step after the pass: p = A w - alpha u_k stored, q = A^T p, pp = ||p||^2.
__global__ void __launch_bounds__(512) lsqr_step_kernel(LsqrDev* st, const double* __restrict__ qv,
                                                        const double* __restrict__ Rinv, int k, double* __restrict__ v,
                                                        double* __restrict__ wd, double* __restrict__ y,
                                                        double* __restrict__ wv, double* __restrict__ tmp) {
  __shared__ double red[8];
  __shared__ double sh[4];
  if (st->done) return;
  const double alpha_old = st->alpha;
  const double beta = sqrt(qv[k]);
  const double ib = beta > 0 ? 1.0 / beta : 0.0;
  // v_new = Rinv^T (q / beta) - beta v
  for (int j = threadIdx.x; j < k; j += blockDim.x) tmp[j] = qv[j] * ib;
  __syncthreads();
  rinv_t_apply(Rinv, k, tmp, tmp + k);
  __syncthreads();
  double part = 0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double vn = tmp[k + j] - beta * v[j];
    tmp[k + j] = vn;
    part += vn * vn;
  }
  const double alpha = sqrt(wg_sum(part, red));
  if (threadIdx.x == 0) {
    const double anorm2 = st->anorm2 + alpha_old * alpha_old + beta * beta;
    const double rhobar = st->rhobar, phibar = st->phibar;
    const double rho = hypot(rhobar, beta);
    const double c = rhobar / rho, s = beta / rho;
    const double theta = s * alpha;
    const double phi = c * phibar;
    const double phibar_n = s * phibar;
    sh[0] = phi / rho;
    sh[1] = theta / rho;
    st->rhobar = -c * alpha;
    st->phibar = phibar_n;
    st->anorm2 = anorm2;
    st->alpha = alpha;
    st->beta = beta;
    const double rnorm = phibar_n, arnorm = phibar_n * alpha * fabs(c), anorm = sqrt(anorm2);
    st->rnorm = rnorm;
    st->arnorm = arnorm;
    st->anorm = anorm;
    st->iters += 1;
    const bool conv = rnorm <= st->tol * st->bnorm || arnorm <= st->tol * anorm * rnorm;
    st->done = (conv || st->iters >= st->maxit) ? 1 : 0;
    st->converged = conv ? 1 : 0;
    st->uscale = ib;
    st->coef = -alpha * ib;
  }
  __syncthreads();
  const double f1 = sh[0], f2 = sh[1];
  const double ia = alpha > 0 ? 1.0 / alpha : 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double vn = tmp[k + j] * ia;
    y[j] += f1 * wd[j];
    wd[j] = vn - f2 * wd[j];
    v[j] = vn;
  }
  __syncthreads();
  rinv_apply(Rinv, k, v, wv);
}

// x = x0 + Rinv y
__global__ void lsqr_finish_kernel(const double* __restrict__ Rinv, int k, const double* __restrict__ x0,
                                   const double* __restrict__ y, double* __restrict__ x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    double s = 0;
    for (int j = i; j < k; ++j) s += Rinv[(int64_t)i * k + j] * y[j];
    x[i] = x0[i] + s;
  }
}

// x = Rinv c (the sketch-and-solve warm start)
__global__ void rinv_vec_kernel(const double* __restrict__ Rinv, int k, const double* __restrict__ c,
                                double* __restrict__ x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    double s = 0;
    for (int j = i; j < k; ++j) s += Rinv[(int64_t)i * k + j] * c[j];
    x[i] = s;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int lsqr_pass_groups(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 63) / 64)); }

int launch_lsqr_pass(const double* A, int64_t lda, int64_t n, int m, const double* w, const double* coefp,
                     const int* donep, double* u, double* part, hipStream_t st) {
  const int groups = lsqr_pass_groups(n);
  const int64_t rows = (n + groups - 1) / groups;
  const int mpl = (m + 63) / 64;
#define SK_PASS(MP)                                                                                              \
  hipLaunchKernelGGL((lsqr_pass_kernel<MP, (MP <= 4 ? 4 : 2)>), dim3(groups), dim3(256), 0, st, A, lda, n, m, w,  \
                     coefp, donep, u, part, rows)
  if (mpl <= 1)
    SK_PASS(1);
  else if (mpl <= 2)
    SK_PASS(2);
  else if (mpl <= 4)
    SK_PASS(4);
  else if (mpl <= 8)
    SK_PASS(8);
  else {
    set_error("LSQR: at most 512 columns");
    return SK_E_NOTSUP;
  }
#undef SK_PASS
  SK_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_cols_kernel, dim3((m + 1 + 255) / 256), dim3(256), 0, st, part, groups, m + 1, donep,
                     part + (int64_t)groups * (m + 1));
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_lsqr_setup(LsqrDev* sd, double tol, int maxit, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_setup_kernel, dim3(1), dim3(64), 0, st, sd, tol, maxit);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_lsqr_init(LsqrDev* sd, const double* qv, const double* Rinv, int k, double* v, double* wd, double* y,
                     double* wv, double* tmp, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_init_kernel, dim3(1), dim3(512), 0, st, sd, qv, Rinv, k, v, wd, y, wv, tmp);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_lsqr_step(LsqrDev* sd, const double* qv, const double* Rinv, int k, double* v, double* wd, double* y,
                     double* wv, double* tmp, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_step_kernel, dim3(1), dim3(512), 0, st, sd, qv, Rinv, k, v, wd, y, wv, tmp);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_lsqr_finish(const double* Rinv, int k, const double* x0, const double* y, double* x, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_finish_kernel, dim3((k + 255) / 256), dim3(256), 0, st, Rinv, k, x0, y, x);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_rinv_vec(const double* Rinv, int k, const double* c, double* x, hipStream_t st) {
  hipLaunchKernelGGL(rinv_vec_kernel, dim3((k + 255) / 256), dim3(256), 0, st, Rinv, k, c, x);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
