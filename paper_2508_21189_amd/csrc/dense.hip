// Dense FP64 kernels for the least-squares drivers (gfx950):
//   * blocked Householder QR of a d x k column-major matrix W (the sketched
//     system [SA | Sb] transposed to columns); one workgroup factors a panel
//     and builds the compact-WY factor T; one workgroup per trailing column
//     applies Q_panel^T = I - V T^T V^T;
//   * explicit inverse of the upper-triangular R (the preconditioner);
//   * row-block reductions for LSQR (see lsqr.hip) live in their own file.
#include "sk_dense.hpp"

#include <algorithm>

namespace sk {

constexpr int kPanel = 32;  // panel width of the blocked QR

// Global loads and stores through table pointers (which the compiler would
// otherwise access as flat memory); the loads are made unconditional by the
// callers (clamped addresses) so that they issue back to back.
__device__ inline double gld(const double* p) { return *(const __attribute__((address_space(1))) double*)p; }
__device__ inline void gst(double* p, double v) { *(__attribute__((address_space(1))) double*)p = v; }

// Sums over the wave of N values per lane (N = 8, 16 or 32), returned
// transposed: lane l gets the sum of a[l >> (6 - log2 N)]. Each halving step
// trades half of a lane's values with the lane whose bit differs (the lane
// with the bit set keeps the upper half) and adds, so the N sums cost N - 1
// exchanges and adds instead of N full reductions; the lanes that share an
// entry then finish it with ordinary exchanges.
template <int N>
__device__ inline double wave_sum_transposed(const double* a, int lane) {
  static_assert(N == 8 || N == 16 || N == 32, "N");
  double v[N];
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = a[j];
  int bit = 32;
#pragma unroll
  for (int n = N; n > 1; n /= 2) {
    const bool hi = (lane & bit) != 0;
#pragma unroll
    for (int j = 0; j < n / 2; ++j) {
      const double send = hi ? v[j] : v[n / 2 + j];
      const double keep = hi ? v[n / 2 + j] : v[j];
      v[j] = keep + __shfl_xor(send, bit, 64);
    }
    bit /= 2;
  }
#pragma unroll
  for (int b = 32 / N; b >= 1; b /= 2) v[0] += __shfl_xor(v[0], b, 64);
  return v[0];
}

// Block-wide sum of one double per thread (blockDim.x a multiple of 64, <= 1024).
__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < nw; ++w) s += red[w];  // fixed order: deterministic
  return s;
}

// W (column-major, column c at W + c*ldw) := [M^T-columns | rhs]: column c < k0
// is column c of the row-major d x k0 matrix M, column k0 is the vector r.
__global__ void to_columns_kernel(const double* __restrict__ M, int64_t ldm, const double* __restrict__ r, int64_t d,
                                  int k0, double* __restrict__ W, int64_t ldw) {
  const int64_t total = d * (k0 + (r ? 1 : 0));
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / d, i = idx - c * d;
    W[c * ldw + i] = c < k0 ? M[i * ldm + c] : r[i];
  }
}

// Householder factorization of panel columns [k, k + nbp) of W (d rows), in
// place: R on and above the diagonal, the reflector vectors v (unit leading
// entry implicit) below it. tau[k + j] and T (nbp x nbp, upper, row-major,
// stride kPanel) with Q_panel = H_k ... H_{k+nbp-1} = I - V T V^T. LAPACK's
// sign convention: beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta,
// v = x / (alpha - beta).
// Per column two block-wide reductions: ||x below the diagonal||^2, then in
// one pass over the panel rows all the products the column needs: v^T y for
// the later panel columns (their update) and v_q^T v for the earlier
// reflectors (the Gram entries that build T).
__global__ void __launch_bounds__(1024) hh_panel_kernel(double* __restrict__ W, int64_t ldw, int64_t d, int k,
                                                        int nbp, double* __restrict__ tau, double* __restrict__ T) {
  __shared__ double red[16][kPanel + 1];
  __shared__ double vals[kPanel];
  __shared__ double G[kPanel][kPanel + 1];  // G[q][j] = v_q^T v_j, q < j
  __shared__ double Ts[kPanel][kPanel + 1];
  __shared__ double taus[kPanel];
  __shared__ double sh_scal[4];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (int jj = 0; jj < nbp; ++jj) {
    const int c = k + jj;
    double* x = W + (int64_t)c * ldw;
    double part = 0;
    for (int64_t i = c + 1 + tid; i < d; i += nt) part += x[i] * x[i];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if (lane == 0) red[wave][0] = part;
    __syncthreads();
    if (tid == 0) {
      double sig2 = 0;
      for (int w = 0; w < nw; ++w) sig2 += red[w][0];
      const double alpha = x[c];
      double t = 0, beta = alpha, scale = 0;
      if (sig2 > 0) {
        beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      sh_scal[0] = t;
      sh_scal[1] = beta;
      sh_scal[2] = scale;
      tau[c] = t;
      taus[jj] = t;
    }
    __syncthreads();
    const double t = sh_scal[0], scale = sh_scal[2];
    // v below the diagonal, and all panel products in the same sweep
    double acc[kPanel];
#pragma unroll
    for (int q = 0; q < kPanel; ++q) acc[q] = 0;
    for (int64_t i = c + 1 + tid; i < d; i += nt) {
      double vi = x[i];
      if (t != 0) {
        vi *= scale;
        x[i] = vi;
      }
#pragma unroll
      for (int q = 0; q < kPanel; ++q)
        if (q < nbp && q != jj) acc[q] += vi * W[(int64_t)(k + q) * ldw + i];
    }
#pragma unroll
    for (int q = 0; q < kPanel; ++q) {
      double v = acc[q];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (tid < nbp && tid != jj) {
      double sacc = W[(int64_t)(k + tid) * ldw + c];  // row c: v_c = 1
      for (int w = 0; w < nw; ++w) sacc += red[w][tid];
      vals[tid] = sacc;
      if (tid < jj) G[tid][jj] = sacc;
    }
    if (tid == 0) x[c] = sh_scal[1];
    __syncthreads();
    // apply H_c = I - t v v^T to the later panel columns
    if (t != 0) {
      for (int q = jj + 1; q < nbp; ++q) {
        const double f = t * vals[q];
        double* y = W + (int64_t)(k + q) * ldw;
        for (int64_t i = c + 1 + tid; i < d; i += nt) y[i] -= f * x[i];
        if (tid == 0) y[c] -= f;
      }
    }
    __syncthreads();
  }
  // T: T[i][i] = tau_i; T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
  for (int i = 0; i < nbp; ++i) {
    if (tid < i) {
      double s2 = 0;
      for (int l = tid; l < i; ++l) s2 += Ts[tid][l] * G[l][i];
      Ts[tid][i] = -taus[i] * s2;
    }
    if (tid == i) Ts[i][i] = taus[i];
    if (tid > i && tid < nbp) Ts[tid][i] = 0.0;
    __syncthreads();
  }
  for (int idx = tid; idx < nbp * nbp; idx += nt) {
    const int r = idx / nbp, cc = idx - r * nbp;
    T[r * kPanel + cc] = Ts[r][cc];
  }
}

// Register-resident variant of the panel factorization for panels whose
// rows fit in the workgroup: thread t holds rows k + t + NT*i (i < RPT) of
// the NB panel columns in registers, so each column step touches no memory:
// one block reduction for ||x||^2 (and the pivot), one for all the panel
// products (v^T y for the later columns, v_q^T v for the Gram entries of T),
// then the update in registers. The panel is written back at the end.
template <int NB, int RPT, int NTH>
__device__ __forceinline__ void hh_panel_reg_dev(double* __restrict__ W, int64_t ldw, int64_t d, int k, int nbp,
                                                 double* __restrict__ tau, double* __restrict__ T) {
  __shared__ double red[NTH / 64][NB + 2];
  __shared__ double vals[NB + 2];
  __shared__ double pivot[NB];
  __shared__ double coef[4];  // beta, scale and t of the current column
  __shared__ double G[kPanel][kPanel + 1];
  __shared__ double Ts[kPanel][kPanel + 1];
  __shared__ double taus[kPanel];
  constexpr int NT = NTH;
  constexpr int NW = NTH / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // x[i * NB + q]: row k + tid + NT * i, panel column q (all indices static)
  double x[RPT * NB];
  // unconditional loads (clamped addresses, the value then selected): the
  // panel's loads issue back to back instead of each behind a branch
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = k + tid + (int64_t)NT * i;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const double w = gld(W + (int64_t)(k + min(q, nbp - 1)) * ldw + min(r, d - 1));
      x[i * NB + q] = (r < d && q < nbp) ? w : 0.0;
    }
  }
  // Per column step one reduction and two barriers: D_q = sum over the rows
  // below the pivot of x_jj x_q gives sigma^2 (q = jj) and, with the pivot
  // row x_q[jj] (from the thread that holds it), v^T x_q = x_q[jj] + scale D_q
  // for every other column, v being the reflector scaled to a unit pivot.
  for (int jj = 0; jj < nbp; ++jj) {
    // pivot column jj of this thread's rows (selected with static indices)
    double pc[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      double v = 0;
#pragma unroll
      for (int q = 0; q < NB; ++q) v = (q == jj) ? x[i * NB + q] : v;
      pc[i] = v;
    }
    double acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      double sacc = 0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) sacc += (tid + NT * i > jj ? pc[i] : 0.0) * x[i * NB + q];
      acc[q] = sacc;
    }
    if (tid == jj) {  // row jj is this thread's first (jj < NB <= NT)
#pragma unroll
      for (int q = 0; q < NB; ++q) pivot[q] = x[q];
    }
    {
      // the NB wave sums at once: lane l ends with the sum of entry
      // l >> (6 - log2 NB) (transposed reduction, one exchange per halving)
      const double v = wave_sum_transposed<NB>(acc, lane);
      constexpr int kShift = NB == 32 ? 1 : (NB == 16 ? 2 : 3);
      if ((lane & ((1 << kShift) - 1)) == 0) red[wave][lane >> kShift] = v;
    }
    __syncthreads();
    if (tid < nbp) {
      double sig2 = 0, D = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        sig2 += red[w][jj];
        D += red[w][tid];
      }
      const double alpha = pivot[jj];
      double t = 0, beta = alpha, scale = 0;
      if (sig2 > 0) {
        beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      const double vq = pivot[tid] + scale * D;  // v^T x_tid (x_tid holds v_tid below its pivot for tid < jj)
      if (tid < jj) G[tid][jj] = vq;
      vals[tid] = (t != 0 && tid > jj) ? t * vq : 0.0;
      if (tid == jj) {
        coef[0] = beta;
        coef[1] = scale;
        coef[2] = t;
        tau[k + jj] = t;
        taus[jj] = t;
      }
    }
    __syncthreads();
    const double beta = coef[0], scale = coef[1], t = coef[2];
    // v: scaled below the pivot, the implicit 1 at the pivot
    double vv[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int lr = tid + NT * i;
      if (lr > jj && t != 0) pc[i] *= scale;
      vv[i] = lr > jj ? pc[i] : (lr == jj ? 1.0 : 0.0);
    }
    // H = I - t v v^T on the later panel columns; the pivot column holds v
    // below the pivot and beta at it
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const double f = q < nbp ? vals[q] : 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int lr = tid + NT * i;
        double xv = x[i * NB + q] - f * vv[i];
        if (q == jj) xv = lr > jj ? pc[i] : (lr == jj ? beta : x[i * NB + q]);
        x[i * NB + q] = xv;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = k + tid + (int64_t)NT * i;
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (r < d && q < nbp) gst(W + (int64_t)(k + q) * ldw + r, x[i * NB + q]);
  }
  // T: T[i][i] = tau_i; T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
  for (int i = 0; i < nbp; ++i) {
    if (tid < i) {
      double s2 = 0;
      for (int l = tid; l < i; ++l) s2 += Ts[tid][l] * G[l][i];
      Ts[tid][i] = -taus[i] * s2;
    }
    if (tid == i) Ts[i][i] = taus[i];
    if (tid > i && tid < nbp) Ts[tid][i] = 0.0;
    __syncthreads();
  }
  for (int idx = tid; idx < nbp * nbp; idx += NT) {
    const int r = idx / nbp, cc = idx - r * nbp;
    T[r * kPanel + cc] = Ts[r][cc];
  }
}

template <int NB, int RPT, int NTH>
__global__ void __launch_bounds__(NTH) hh_panel_reg_kernel(double* __restrict__ W, int64_t ldw, int64_t d, int k,
                                                           int nbp, double* __restrict__ tau,
                                                           double* __restrict__ T) {
  hh_panel_reg_dev<NB, RPT, NTH>(W, ldw, d, k, nbp, tau, T);
}

// R (k x k row-major, upper) and c = (Q^T rhs)[0:k] from the factored W.
__device__ __forceinline__ void extract_r_dev(const double* __restrict__ W, int64_t ldw, int k, int has_rhs,
                                              double* __restrict__ R, double* __restrict__ c, unsigned bx, unsigned gx) {
  const int64_t total = (int64_t)k * k;
  for (int64_t idx = bx * (int64_t)blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gx * blockDim.x) {
    const int64_t r = idx / k, col = idx - r * k;
    R[idx] = col >= r ? W[col * ldw + r] : 0.0;
  }
  if (has_rhs)
    for (int64_t r = bx * (int64_t)blockDim.x + threadIdx.x; r < k; r += (int64_t)gx * blockDim.x)
      c[r] = W[(int64_t)k * ldw + r];
}

__global__ void extract_r_kernel(const double* __restrict__ W, int64_t ldw, int k, int has_rhs,
                                 double* __restrict__ R, double* __restrict__ c) {
  extract_r_dev(W, ldw, k, has_rhs, R, c, blockIdx.x, gridDim.x);
}

// X = R^{-1} for upper-triangular R (k x k row-major), and XT = X^T. One
// wave per column j: X[j][j] = 1/R[j][j]; for i = j-1 down to 0,
// X[i][j] = -(sum_{l=i+1..j} R[i][l] X[l][j]) / R[i][i]. The column is built
// in LDS and written to both X (column j) and XT (row j).
__global__ void __launch_bounds__(64) trinv_upper_kernel(const double* __restrict__ R, int k, double* __restrict__ X,
                                                         double* __restrict__ XT) {
  extern __shared__ double col[];
  const int j = blockIdx.x, lane = threadIdx.x;
  for (int i = lane; i < k; i += 64) col[i] = 0.0;
  __syncthreads();
  if (lane == 0) col[j] = 1.0 / R[(int64_t)j * k + j];
  __syncthreads();
  for (int i = j - 1; i >= 0; --i) {
    const double* Ri = R + (int64_t)i * k;
    double s = 0;
    for (int l = i + 1 + lane; l <= j; l += 64) s += Ri[l] * col[l];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) col[i] = -s / Ri[i];
    __syncthreads();
  }
  for (int i = lane; i < k; i += 64) {
    X[(int64_t)i * k + j] = col[i];
    XT[(int64_t)j * k + i] = col[i];
  }
}

// Blocked inverse of an upper-triangular R (k x k row-major, k <= 512), in
// 32 x 32 blocks. First one wave per diagonal block inverts it (lane c holds
// column c; the rows of R come by readlane): X_JJ = R_JJ^{-1}. Then one
// workgroup per column block J forms, for I = J-1 down to 0,
//   X_IJ = -X_II (sum_{L=I+1..J} R_IL X_LJ),
// with the column block of X held in LDS. Writes X (upper, zero below) and
// XT = X^T.
constexpr int kTb = 32;

__device__ inline double rl64d(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ void trinv_diag_dev(const double* __restrict__ R, int k, double* __restrict__ X, unsigned bx) {
  const int c = threadIdx.x;
  const int j0 = bx * kTb;
  const int b = min(kTb, k - j0);
  double col[kTb];  // col[r] = R[j0 + r][j0 + c]
#pragma unroll
  for (int r = 0; r < kTb; ++r) col[r] = (c < b && r < b) ? R[(int64_t)(j0 + r) * k + j0 + c] : 0.0;
  double x[kTb];
#pragma unroll
  for (int i = kTb - 1; i >= 0; --i) {
    x[i] = 0.0;
    if (i < b) {
      double sacc = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < kTb; ++l)
        if (l < b) sacc -= rl64d(col[i], l) * x[l];
      x[i] = sacc / rl64d(col[i], i);
    }
  }
  if (c < b) {
#pragma unroll
    for (int r = 0; r < kTb; ++r)
      if (r < b) X[(int64_t)(j0 + r) * k + j0 + c] = x[r];
  }
}

__global__ void __launch_bounds__(64) trinv_diag_kernel(const double* __restrict__ R, int k, double* __restrict__ X) {
  trinv_diag_dev(R, k, X, blockIdx.x);
}

__device__ __forceinline__ void trinv_cols_dev(const double* __restrict__ R, int k, double* __restrict__ X,
                                               double* __restrict__ XT, double* Xs, unsigned bx) {
  constexpr int XS = kTb + 1;  // LDS row stride of the column block (Xs: [k][XS])
  __shared__ double T[kTb][kTb + 1];
  const int J = (int)bx, j0 = J * kTb, bj = min(kTb, k - j0);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < k * kTb; idx += nt) {
    const int r = idx / kTb, c = idx - r * kTb;
    Xs[r * XS + c] = (r >= j0 && r < j0 + bj && c < bj) ? X[(int64_t)r * k + j0 + c] : 0.0;
  }
  __syncthreads();
  const int r = tid / kTb, c = tid - (tid / kTb) * kTb;  // 1024 threads: one entry of a 32 x 32 block each
  for (int I = J - 1; I >= 0; --I) {
    const int i0 = I * kTb;
    double sacc = 0.0;
    const double* Rrow = R + (int64_t)(i0 + r) * k;
    for (int l = i0 + kTb; l < j0 + bj; ++l) sacc += Rrow[l] * Xs[l * XS + c];
    T[r][c] = sacc;
    __syncthreads();
    double v = 0.0;
    const double* Xii = X + (int64_t)(i0 + r) * k + i0;
    for (int m = r; m < kTb; ++m) v += Xii[m] * T[m][c];
    Xs[(i0 + r) * XS + c] = c < bj ? -v : 0.0;
    __syncthreads();
  }
  for (int idx = tid; idx < k * kTb; idx += nt) {
    const int rr = idx / kTb, cc = idx - rr * kTb;
    if (cc < bj) X[(int64_t)rr * k + j0 + cc] = Xs[rr * XS + cc];
  }
  for (int idx = tid; idx < k * kTb; idx += nt) {
    const int cc = idx / k, rr = idx - cc * k;
    if (cc < bj) XT[(int64_t)(j0 + cc) * k + rr] = Xs[rr * XS + cc];
  }
}

__global__ void __launch_bounds__(1024) trinv_cols_kernel(const double* __restrict__ R, int k, double* __restrict__ X,
                                                          double* __restrict__ XT) {
  extern __shared__ double Xs[];  // [k][kTb + 1]
  trinv_cols_dev(R, k, X, XT, Xs, blockIdx.x);
}

// ---- the same steps for a batch of small problems, one launch per step:
// problem p = blockIdx.y (blockIdx.x for the one-workgroup panel); a problem
// whose k is past the step leaves at once. Every problem has d <= 1024 rows
// (the 32-column register panel) and k <= 512 (the blocked inverse).

__global__ void __launch_bounds__(512) hh_panel_batched_kernel(const QrBatch* __restrict__ B, int c) {
  const QrBatch& p = B[blockIdx.x];
  if (c >= p.k) return;
  hh_panel_reg_dev<32, 2, 512>(p.W, p.ldw, p.d, c, min(kPanel, p.k - c), p.tau, p.T + (int64_t)(c / kPanel) * kPanel * kPanel);
}

// Trailing update by column blocks: workgroup (x, p) applies the panel's
// Q^T = I - V T^T V^T to trailing columns [32 x, 32 x + 32) of problem p,
// over 64-row tiles of V and Y staged in LDS (zero past the matrix):
//   Z = V^T Y  on the FP64 matrix cores, wave w owning the 16 x 16 block
//              (w & 1, w >> 1) of Z;
//   Z2 = T^T Z (T upper triangular; VALU, from LDS);
//   Y -= V Z2  on the matrix cores, wave w owning rows 16 w of each tile.
// v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// item v of the result is row 4 v + l / 16, column l % 16. V is read twice
// and Y read and written once per block of 32 columns.
constexpr int kTrailRows = 64;
typedef double v4d __attribute__((ext_vector_type(4)));
// W: d rows, ncols columns (column-major, ldw); the panel is columns
// [c, c + nbp) with its T; block bx updates columns first + 32 bx onwards.
__device__ __forceinline__ void hh_trail_blk_dev(double* W, int64_t ldw, int64_t d, int ncols, int c, int nbp,
                                                 const double* T, int bx) {
  __shared__ double Vs[kTrailRows][kPanel + 1];
  __shared__ double Ys[kTrailRows][kPanel + 1];
  __shared__ double Zs[kPanel][kPanel + 1];
  const int first = c + nbp;
  const int cb = bx * kPanel;
  const int nc = min(kPanel, ncols - first - cb);  // this block's columns
  if (nc <= 0) return;
  double* Y = W + (int64_t)(first + cb) * ldw;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // Stage rows [r0, r0 + 64) of V (the reflector below its diagonal, 1 on
  // it, 0 above and past nbp) and of Y (0 past nc and d): lanes along the
  // rows (coalesced), unconditional loads from clamped addresses.
  auto stage = [&](int64_t r0) {
    const int rr = tid & 63, g = tid >> 6;
    const int64_t i = r0 + rr, ic = min(i, d - 1);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int q = g + 4 * m;
      const double w = gld(W + (int64_t)(c + min(q, nbp - 1)) * ldw + ic);
      const double y = gld(Y + (int64_t)min(q, nc - 1) * ldw + ic);
      const int64_t diag = c + q;
      Vs[rr][q] = (q < nbp && i < d) ? (i > diag ? w : (i == diag ? 1.0 : 0.0)) : 0.0;
      Ys[rr][q] = (q < nc && i < d) ? y : 0.0;
    }
  };
  // Z = V^T Y
  const int zp = (wave & 1) * 16, zc = (wave >> 1) * 16;
  v4d z = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = c; r0 < d; r0 += kTrailRows) {
    stage(r0);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTrailRows; r += 4)
      z = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[r + lk][zp + li], Ys[r + lk][zc + li], z, 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) Zs[zp + 4 * v + lk][zc + li] = z[v];
  __syncthreads();
  // Z2 = T^T Z (T upper: Z2[p][cc] = sum_{q <= p} T[q][p] Z[q][cc]), negated
  // for the update
  const int cc = tid & 31, pr = tid >> 5;
  double z2[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pp = pr + 8 * j;
    double sum = 0.0;
    if (pp < nbp)
      for (int q = 0; q <= pp; ++q) sum += gld(T + q * kPanel + pp) * Zs[q][cc];
    z2[j] = -sum;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) Zs[pr + 8 * j][cc] = z2[j];
  __syncthreads();
  // Y -= V Z2, tile by tile: wave w updates rows [16 w, 16 w + 16) of the
  // tile in both 16-column blocks, in LDS, then the tile is stored
  const int yr = wave * 16;
  for (int64_t r0 = c; r0 < d; r0 += kTrailRows) {
    stage(r0);
    __syncthreads();
#pragma unroll
    for (int cbk = 0; cbk < 2; ++cbk) {
      const int yc = cbk * 16;
      v4d acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = Ys[yr + 4 * v + lk][yc + li];
#pragma unroll
      for (int s = 0; s < kPanel; s += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[yr + li][s + lk], Zs[s + lk][yc + li], acc, 0, 0, 0);
      // (each wave writes only its own rows of Ys, which no other wave reads)
#pragma unroll
      for (int v = 0; v < 4; ++v) Ys[yr + 4 * v + lk][yc + li] = acc[v];
    }
    __syncthreads();
    {
      const int rr = tid & 63, g = tid >> 6;
      const int64_t i = r0 + rr;
      if (i < d) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int q = g + 4 * m;
          if (q < nc) gst(Y + (int64_t)q * ldw + i, Ys[rr][q]);
        }
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) hh_trail_blk_batched_kernel(const QrBatch* __restrict__ B, int c) {
  const QrBatch& pb = B[blockIdx.y];
  if (c >= pb.k) return;
  hh_trail_blk_dev(pb.W, pb.ldw, pb.d, pb.k + 1, c, min(kPanel, pb.k - c),
                   pb.T + (int64_t)(c / kPanel) * kPanel * kPanel, (int)blockIdx.x);
}

__global__ void __launch_bounds__(256) hh_trail_blk_kernel(double* __restrict__ W, int64_t ldw, int64_t d, int ncols,
                                                           int c, int nbp, const double* __restrict__ T) {
  hh_trail_blk_dev(W, ldw, d, ncols, c, nbp, T, (int)blockIdx.x);
}

__global__ void extract_r_batched_kernel(const QrBatch* __restrict__ B) {
  const QrBatch& p = B[blockIdx.y];
  if (p.k == 0) return;
  extract_r_dev(p.W, p.ldw, p.k, 1, p.R, p.c, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(64) trinv_diag_batched_kernel(const QrBatch* __restrict__ B) {
  const QrBatch& p = B[blockIdx.y];
  if ((int)blockIdx.x * kTb >= p.k) return;
  trinv_diag_dev(p.R, p.k, p.X, blockIdx.x);
}

__global__ void __launch_bounds__(1024) trinv_cols_batched_kernel(const QrBatch* __restrict__ B) {
  extern __shared__ double Xs[];  // [k][kTb + 1], sized for the batch's largest k
  const QrBatch& p = B[blockIdx.y];
  if ((int)blockIdx.x * kTb >= p.k) return;
  trinv_cols_dev(p.R, p.k, p.X, p.XT, Xs, blockIdx.x);
}

__global__ void fill_kernel(double* __restrict__ x, int64_t n, double value) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = value;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int qr_columns(double* W, int64_t ldw, int64_t d, int k, int extra_cols, double* tau, double* Tbuf, hipStream_t st) {
  // panel width: 32 when the panel's rows fit one row per thread, else 16
  // (two rows per thread) while they fit in registers, else the
  // memory-resident panel kernel
  const int nb = d <= 1024 ? 32 : 16;
  for (int c = 0; c < k; c += nb) {
    const int nbp = std::min(nb, k - c);
    double* T = Tbuf + (size_t)(c / nb) * kPanel * kPanel;
    const int64_t rows = d - c;
    if (rows <= 1024 && nb == 32)
      hipLaunchKernelGGL((hh_panel_reg_kernel<32, 2, 512>), dim3(1), dim3(512), 0, st, W, ldw, d, c, nbp, tau, T);
    else if (rows <= 2048)
      hipLaunchKernelGGL((hh_panel_reg_kernel<16, 4, 512>), dim3(1), dim3(512), 0, st, W, ldw, d, c, nbp, tau, T);
    else
      hipLaunchKernelGGL(hh_panel_kernel, dim3(1), dim3(1024), 0, st, W, ldw, d, c, nbp, tau, T);
    SK_HIP(hipGetLastError());
    const int first = c + nbp;
    const int ntrail = k + extra_cols - first;
    if (ntrail > 0) {
      const unsigned nblk = (unsigned)((ntrail + kPanel - 1) / kPanel);
      hipLaunchKernelGGL(hh_trail_blk_kernel, dim3(nblk), dim3(256), 0, st, W, ldw, d, k + extra_cols, c, nbp, T);
      SK_HIP(hipGetLastError());
    }
  }
  return SK_OK;
}

size_t qr_tbuf_doubles(int k) { return (size_t)((k + 15) / 16) * kPanel * kPanel; }

int launch_to_columns(const double* M, int64_t ldm, const double* r, int64_t d, int k0, double* W, int64_t ldw,
                      hipStream_t st) {
  const int64_t total = d * (k0 + (r ? 1 : 0));
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(to_columns_kernel, dim3(blocks), dim3(256), 0, st, M, ldm, r, d, k0, W, ldw);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_extract_r(const double* W, int64_t ldw, int k, int has_rhs, double* R, double* c, hipStream_t st) {
  const int64_t total = (int64_t)k * k;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(extract_r_kernel, dim3(blocks), dim3(256), 0, st, W, ldw, k, has_rhs, R, c);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_fill(double* x, int64_t n, double value, hipStream_t st) {
  if (n <= 0) return SK_OK;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, st, x, n, value);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_trinv(const double* R, int k, double* X, double* XT, hipStream_t st) {
  if (k <= 512) {
    const int nblk = (k + kTb - 1) / kTb;
    hipLaunchKernelGGL(trinv_diag_kernel, dim3(nblk), dim3(64), 0, st, R, k, X);
    SK_HIP(hipGetLastError());
    const size_t lds = (size_t)k * (kTb + 1) * sizeof(double);
    SK_HIP(hipFuncSetAttribute((const void*)trinv_cols_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(trinv_cols_kernel, dim3(nblk), dim3(1024), lds, st, R, k, X, XT);
  } else {
    hipLaunchKernelGGL(trinv_upper_kernel, dim3(k), dim3(64), (size_t)k * sizeof(double), st, R, k, X, XT);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int qr_trinv_batched(const QrBatch* B, int nprob, int kmax, hipStream_t st) {
  if (nprob <= 0 || kmax <= 0) return SK_OK;
  if (kmax > 512) {
    set_error("batched QR: at most 512 columns");
    return SK_E_NOTSUP;
  }
  for (int c = 0; c < kmax; c += kPanel) {
    hipLaunchKernelGGL(hh_panel_batched_kernel, dim3((unsigned)nprob), dim3(512), 0, st, B, c);
    SK_HIP(hipGetLastError());
    const int ntrail = kmax + 1 - c - 1;  // the most trailing columns any problem has at this step
    if (ntrail > 0) {
      const unsigned nblk = (unsigned)((ntrail + kPanel - 1) / kPanel);
      hipLaunchKernelGGL(hh_trail_blk_batched_kernel, dim3(nblk, (unsigned)nprob), dim3(256), 0, st, B, c);
      SK_HIP(hipGetLastError());
    }
  }
  const unsigned eb = (unsigned)std::max(1, std::min(64, (kmax * kmax + 255) / 256));
  hipLaunchKernelGGL(extract_r_batched_kernel, dim3(eb, (unsigned)nprob), dim3(256), 0, st, B);
  SK_HIP(hipGetLastError());
  const unsigned nblk = (unsigned)((kmax + kTb - 1) / kTb);
  hipLaunchKernelGGL(trinv_diag_batched_kernel, dim3(nblk, (unsigned)nprob), dim3(64), 0, st, B);
  SK_HIP(hipGetLastError());
  const size_t lds = (size_t)kmax * (kTb + 1) * sizeof(double);
  SK_HIP(hipFuncSetAttribute((const void*)trinv_cols_batched_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  hipLaunchKernelGGL(trinv_cols_batched_kernel, dim3(nblk, (unsigned)nprob), dim3(1024), lds, st, B);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
