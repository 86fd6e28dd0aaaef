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
#include <cstdlib>

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
  // U rows per step (rows i, i+4, ...); the next step's rows are loaded
  // before this step's reductions so that two steps of A are in flight.
  auto load_rows = [&](int64_t i0, double (&xx)[U][MPL], double (&uu)[U]) {
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const double* a = A + (i0 + 4 * r) * lda;
#pragma unroll
      for (int k = 0; k < MPL; ++k) {
        const int c = lane + 64 * k;
        xx[r][k] = c < m ? __builtin_nontemporal_load(a + c) : 0.0;
      }
      uu[r] = u[i0 + 4 * r];
    }
  };
  if (i + 4 * (U - 1) < r1) {
    double x[U][MPL], uo[U];
    load_rows(i, x, uo);
    for (;;) {
      const int64_t inext = i + 4 * U;
      const bool more = inext + 4 * (U - 1) < r1;
      double xn[U][MPL], un[U];
      if (more) load_rows(inext, xn, un);
      double dt[U];
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
      i = inext;
      if (!more) break;
#pragma unroll
      for (int r = 0; r < U; ++r) {
        uo[r] = un[r];
#pragma unroll
        for (int k = 0; k < MPL; ++k) x[r][k] = xn[r][k];
      }
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

typedef double v2d __attribute__((ext_vector_type(2)));

// x of the lane n places down this lane's 16-lane DPP row (row_ror:n).
template <int N>
__device__ inline double row_ror(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x120 + N, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x120 + N, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Sum of x over the 16 lanes of this lane's DPP row: every lane ends with
// the same total.
__device__ inline double row16_sum(double x) {
  x += row_ror<8>(x);
  x += row_ror<4>(x);
  x += row_ror<2>(x);
  x += row_ror<1>(x);
  return x;
}

// The same pass for an even number of columns m and 16-byte aligned rows
// (lda even): 16 lanes per row, each loading column pairs 2 (l%16) + 32 k,
// k < MP2, so a wave covers 4 rows per load instruction and a row's dot
// product needs 4 DPP steps inside its 16-lane row. A workgroup takes 16
// consecutive rows per step (row 4 wave + l/16 of the step); the next step's
// rows are loaded before this step's arithmetic. Columns past m load column
// 0 of the same row (w is zero there, and their column sums are dropped);
// rows past the workgroup's range repeat its last row with p = 0.
template <int MP2>
__global__ void __launch_bounds__(256) lsqr_pass16_kernel(const double* __restrict__ A, int64_t lda, int64_t n, int m,
                                                          const double* __restrict__ w,
                                                          const double* __restrict__ coefp,
                                                          const int* __restrict__ donep, double* __restrict__ u,
                                                          double* __restrict__ part, int64_t rows_per_wg) {
  if (donep && *donep) return;
  __shared__ double red[4][MP2 * 32 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, cl = lane & 15;
  const double coef = *coefp;
  v2d wl[MP2], q[MP2];
#pragma unroll
  for (int k = 0; k < MP2; ++k) {
    const int c = 2 * cl + 32 * k;
    const v2d wv = c < m ? v2d{w[c], w[c + 1]} : v2d{0.0, 0.0};
    wl[k] = wv;
    q[k] = v2d{0.0, 0.0};
  }
  double pp = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(n, r0 + rows_per_wg);
  const int64_t nsteps = r1 > r0 ? (r1 - r0 + 15) / 16 : 0;
  auto load = [&](int64_t rb, v2d (&x)[MP2], double& uu) {
    const int64_t i = min(rb + 4 * wave + g, r1 - 1);
    const double* a = A + i * lda;
#pragma unroll
    for (int k = 0; k < MP2; ++k) {
      const int c = 2 * cl + 32 * k;  // past m: column 0 of the same row
      x[k] = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(a + (c < m ? c : 0)));
    }
    uu = u[i];
  };
  v2d x[MP2];
  double uo = 0.0;
  if (nsteps > 0) load(r0, x, uo);
  for (int64_t st = 0; st < nsteps; ++st) {
    const int64_t rb = r0 + 16 * st;
    v2d xn[MP2];
    double un = 0.0;
    const bool more = st + 1 < nsteps;
    if (more) load(rb + 16, xn, un);
    double dt = 0.0;
#pragma unroll
    for (int k = 0; k < MP2; ++k) {
      dt = fma(x[k].x, wl[k].x, dt);
      dt = fma(x[k].y, wl[k].y, dt);
    }
    dt = row16_sum(dt);
    const int64_t i = rb + 4 * wave + g;
    const bool ok = i < r1;
    const double p = ok ? fma(coef, uo, dt) : 0.0;
    if (ok && cl == 0) u[i] = p;
#pragma unroll
    for (int k = 0; k < MP2; ++k) {
      q[k].x = fma(x[k].x, p, q[k].x);
      q[k].y = fma(x[k].y, p, q[k].y);
    }
    pp = fma(p, p, pp);
    if (more) {
#pragma unroll
      for (int k = 0; k < MP2; ++k) x[k] = xn[k];
      uo = un;
    }
  }
  // the wave's column sums: add the 4 rows groups (lanes l, l^16, l^32, l^48)
#pragma unroll
  for (int k = 0; k < MP2; ++k) {
    q[k].x += __shfl_xor(q[k].x, 16, 64);
    q[k].y += __shfl_xor(q[k].y, 16, 64);
    q[k].x += __shfl_xor(q[k].x, 32, 64);
    q[k].y += __shfl_xor(q[k].y, 32, 64);
  }
  pp += __shfl_xor(pp, 16, 64);
  pp += __shfl_xor(pp, 32, 64);
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < MP2; ++k) {
      red[wave][2 * cl + 32 * k] = q[k].x;
      red[wave][2 * cl + 32 * k + 1] = q[k].y;
    }
    if (cl == 0) red[wave][MP2 * 32] = pp;
  }
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * (m + 1);
  for (int j = tid; j <= m; j += blockDim.x) {
    const int jj = j < m ? j : MP2 * 32;
    out[j] = ((red[0][jj] + red[1][jj]) + red[2][jj]) + red[3][jj];
  }
}

// out[j] = sum_g part[g][j]: one workgroup per column j; thread t sums
// g = t, t + 256, ... in order, then a fixed-order tree (deterministic).
__global__ void __launch_bounds__(256) reduce_cols_kernel(const double* __restrict__ part, int ngroups, int width,
                                                          const int* __restrict__ donep, double* __restrict__ out) {
  if (donep && *donep) return;
  __shared__ double red[4];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double s = 0;
  for (int g = tid; g < ngroups; g += 256) s += part[(int64_t)g * width + j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (tid == 0) out[j] = ((red[0] + red[1]) + red[2]) + red[3];
}

// out_j = sum_i M[i][j] x_i for a triangular k x k row-major M (k <= 512):
// UPPER: M[i][j] = 0 for i > j; else M[i][j] = 0 for i < j. Waves take
// rows i = wave, wave + 16, ...; lanes take columns; the per-wave partial
// sums are added in wave order. xs and part live in LDS; out may be global.
template <bool UPPER>
__device__ inline void tri_cols(const double* __restrict__ M, int k, const double* xs, double* out, double* part) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  double acc[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) acc[p] = 0;
  // rows are independent: unrolled so that several rows' loads are in flight
#pragma unroll 4
  for (int i = wave; i < k; i += nw) {
    const double xi = xs[i];
    const double* row = M + (int64_t)i * k;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int j = lane + 64 * p;
      const bool in = UPPER ? (j >= i && j < k) : (j <= i);
      if (in) acc[p] += row[j] * xi;
    }
  }
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int j = lane + 64 * p;
    if (j < k) part[wave * k + j] = acc[p];
  }
  __syncthreads();
  for (int j = tid; j < k; j += blockDim.x) {
    double sum = 0;
    for (int w = 0; w < nw; ++w) sum += part[w * k + j];
    out[j] = sum;
  }
  __syncthreads();
}

__device__ inline double wg_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int q = 0; q < nw; ++q) s += red[q];
  return s;
}

// LDS of the init / step kernels: part[16][k], xs[k], t1[k]
inline size_t lsqr_step_lds(int k) { return (size_t)(16 * k + 2 * k) * sizeof(double); }

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

// After the pass p0 = A x0 - b: q = A^T p0, pp = ||p0||^2 (in qv[k]).
// beta u1 = r0 = -p0; alpha v1 = Rinv^T A^T u1; w = v1; phibar = beta; rhobar = alpha.
__global__ void __launch_bounds__(1024) lsqr_init_kernel(LsqrDev* st, const double* __restrict__ qv,
                                                         const double* __restrict__ Rinv,
                                                         const double* __restrict__ RinvT, int k,
                                                         double* __restrict__ v, double* __restrict__ wd,
                                                         double* __restrict__ y, double* __restrict__ wv) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  double* part = lds;
  double* xs = lds + 16 * k;
  double* t1 = xs + k;
  const double beta = sqrt(qv[k]);
  const double sc = beta > 0 ? -1.0 / beta : 0.0;  // A^T u1 = -q / beta
  for (int j = threadIdx.x; j < k; j += blockDim.x) xs[j] = qv[j] * sc;
  __syncthreads();
  tri_cols<true>(Rinv, k, xs, t1, part);  // Rinv^T (A^T u1)
  double pn = 0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) pn += t1[j] * t1[j];
  const double alpha = sqrt(wg_sum(pn, red));
  const double ia = alpha > 0 ? 1.0 / alpha : 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double vj = t1[j] * ia;
    xs[j] = vj;
    v[j] = vj;
    wd[j] = vj;
    y[j] = 0.0;
  }
  __syncthreads();
  tri_cols<false>(RinvT, k, xs, wv, part);  // Rinv v1
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
    st->uscale = sc;         // u1 = sc * (stored p0)
    st->coef = -alpha * sc;  // next pass: p = A w - alpha u1
  }
}

// One LSQR step after the pass p = A wv - alpha u_k (stored), q = A^T p, ||p||^2.
__global__ void __launch_bounds__(1024) lsqr_step_kernel(LsqrDev* st, const double* __restrict__ qv,
                                                         const double* __restrict__ Rinv,
                                                         const double* __restrict__ RinvT, int k,
                                                         double* __restrict__ v, double* __restrict__ wd,
                                                         double* __restrict__ y, double* __restrict__ wv) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  __shared__ double sh[2];
  if (st->done) return;
  double* part = lds;
  double* xs = lds + 16 * k;
  double* t1 = xs + k;
  const double alpha_old = st->alpha;
  const double beta = sqrt(qv[k]);
  const double ib = beta > 0 ? 1.0 / beta : 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) xs[j] = qv[j] * ib;  // A^T u_{k+1}
  __syncthreads();
  tri_cols<true>(Rinv, k, xs, t1, part);
  double pn = 0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double vn = t1[j] - beta * v[j];
    t1[j] = vn;
    pn += vn * vn;
  }
  const double alpha = sqrt(wg_sum(pn, red));
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
    const double vn = t1[j] * ia;
    y[j] += f1 * wd[j];
    wd[j] = vn - f2 * wd[j];
    v[j] = vn;
    xs[j] = vn;
  }
  __syncthreads();
  tri_cols<false>(RinvT, k, xs, wv, part);  // Rinv v_{k+1}
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
static int env_or(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

int lsqr_pass_groups(int64_t n) {
  static const int cap = env_or("SKETCH_LSQR_GROUPS", 1536);
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + 63) / 64));
}

int launch_lsqr_pass(const double* A, int64_t lda, int64_t n, int m, const double* w, const double* coefp,
                     const int* donep, double* u, double* part, hipStream_t st) {
  const int groups = lsqr_pass_groups(n);
  int64_t rows = (n + groups - 1) / groups;
  // 16 lanes a row for up to 256 columns; wider rows keep 64 lanes a row,
  // whose per-row overhead is already small next to 8 loads a lane
  const bool vec16 = m % 2 == 0 && lda % 2 == 0 && (uintptr_t)A % 16 == 0 && m <= 256;
  static const int use16 = env_or("SKETCH_LSQR_VEC16", 1);
  if (vec16 && use16) {
    rows = ((rows + 15) / 16) * 16;
    const int mp2 = (m + 31) / 32;
#define SK_PASS16(MP)                                                                                           \
  hipLaunchKernelGGL((lsqr_pass16_kernel<MP>), dim3(groups), dim3(256), 0, st, A, lda, n, m, w, coefp, donep, u, \
                     part, rows)
    if (mp2 <= 1)
      SK_PASS16(1);
    else if (mp2 <= 2)
      SK_PASS16(2);
    else if (mp2 <= 4)
      SK_PASS16(4);
    else if (mp2 <= 7)
      SK_PASS16(7);
    else
      SK_PASS16(8);
#undef SK_PASS16
  } else {
    const int mpl = (m + 63) / 64;
    static const int urows = env_or("SKETCH_LSQR_ROWS", 2);
#define SK_PASS(MP, U)                                                                                             \
  hipLaunchKernelGGL((lsqr_pass_kernel<MP, U>), dim3(groups), dim3(256), 0, st, A, lda, n, m, w, coefp, donep, u,  \
                     part, rows)
    if (mpl <= 1)
      SK_PASS(1, 4);
    else if (mpl <= 2)
      SK_PASS(2, 4);
    else if (mpl <= 4) {
      if (urows >= 8)
        SK_PASS(4, 8);
      else if (urows <= 2)
        SK_PASS(4, 2);
      else
        SK_PASS(4, 4);
    } else if (mpl <= 8)
      SK_PASS(8, 2);
    else {
      set_error("LSQR: at most 512 columns");
      return SK_E_NOTSUP;
    }
#undef SK_PASS
  }
  SK_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(m + 1), dim3(256), 0, st, part, groups, m + 1, donep,
                     part + (int64_t)groups * (m + 1));
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_lsqr_setup(LsqrDev* sd, double tol, int maxit, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_setup_kernel, dim3(1), dim3(64), 0, st, sd, tol, maxit);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_lsqr_init(LsqrDev* sd, const double* qv, const double* Rinv, const double* RinvT, int k, double* v,
                     double* wd, double* y, double* wv, hipStream_t st) {
  const size_t lds = lsqr_step_lds(k);
  SK_HIP(hipFuncSetAttribute((const void*)lsqr_init_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(lsqr_init_kernel, dim3(1), dim3(1024), lds, st, sd, qv, Rinv, RinvT, k, v, wd, y, wv);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_lsqr_step(LsqrDev* sd, const double* qv, const double* Rinv, const double* RinvT, int k, double* v,
                     double* wd, double* y, double* wv, hipStream_t st) {
  const size_t lds = lsqr_step_lds(k);
  SK_HIP(hipFuncSetAttribute((const void*)lsqr_step_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(lsqr_step_kernel, dim3(1), dim3(1024), lds, st, sd, qv, Rinv, RinvT, k, v, wd, y, wv);
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
