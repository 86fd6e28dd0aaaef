// Dense FP64 kernels of the randomized SVD (Alg. 1):
//   * blocked right-looking Cholesky G = R^T R (upper R, row-major, in
//     place) for the Cholesky-QR orthonormalization of the tall sketch:
//     per 32-column panel one workgroup factors the diagonal block in LDS and
//     inverts it, a column-parallel kernel forms the panel's block row, and a
//     tiled kernel applies the rank-32 update to the trailing upper triangle;
//   * one-sided (Hestenes) Jacobi SVD of a k x k matrix with one workgroup
//     per column pair: each launch is one round of the round-robin ordering
//     (k/2 disjoint pairs), so a sweep is k - 1 launches and every pair of a
//     round runs on its own CU;
//   * small helpers (trace-based shift, transposes, zeroing).
#include "sk_lowrank.hpp"

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdlib>

namespace sk {

constexpr int kCb = 32;  // Cholesky panel width

__device__ inline double wg_reduce_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// G[i][i] += shift, shift = c * trace(G) (the shifted first pass of
// Cholesky QR); one workgroup.
__global__ void __launch_bounds__(1024) add_trace_shift_kernel(double* __restrict__ G, int k, double c) {
  __shared__ double red[16];
  double t = 0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) t += G[(int64_t)i * k + i];
  const double shift = c * wg_reduce_sum(t, red);
  for (int i = threadIdx.x; i < k; i += blockDim.x) G[(int64_t)i * k + i] += shift;
}

__device__ inline double rl64(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Factor the diagonal block [j0, j0 + b) (b <= 32) in one wave; write R_dd
// (upper) back into G and its inverse into Dinv (b x b, stride kCb). Lane c
// holds column c of the block in registers; row jj and the pivots are
// broadcast with readlane, so no step waits on a barrier. *fail = 1 on a
// non-positive pivot.
__global__ void __launch_bounds__(64) chol_diag_kernel(double* __restrict__ G, int k, int j0, int b,
                                                       double* __restrict__ Dinv, int* __restrict__ fail) {
  const int c = threadIdx.x;
  double col[kCb];  // col[r] = entry (r, c) of the block
#pragma unroll
  for (int r = 0; r < kCb; ++r) col[r] = (c < b && r < b) ? G[(int64_t)(j0 + r) * k + j0 + c] : 0.0;
  bool bad = false;
#pragma unroll
  for (int jj = 0; jj < kCb; ++jj) {
    if (jj < b) {
      const double p = rl64(col[jj], jj);
      bad |= !(p > 0.0);
      const double d = p > 0.0 ? sqrt(p) : 1.0;
      if (c == jj)
        col[jj] = d;
      else if (c > jj)
        col[jj] = col[jj] / d;
      // trailing update: entry (i, c) -= R[jj][i] R[jj][c], jj < i <= c
#pragma unroll
      for (int i = jj + 1; i < kCb; ++i) {
        if (i < b) {
          const double rji = rl64(col[jj], i);
          if (c >= i) col[i] -= rji * col[jj];
        }
      }
    }
  }
  if (bad && c == 0) *fail = 1;
  // X = R_dd^{-1} (upper), column c per lane, by rows from the bottom:
  // X[i][c] = (delta_ic - sum_{l > i} R[i][l] X[l][c]) / R[i][i]
  double x[kCb];
#pragma unroll
  for (int i = kCb - 1; i >= 0; --i) {
    x[i] = 0.0;
    if (i < b) {
      double sacc = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int l = i + 1; l < kCb; ++l)
        if (l < b) sacc -= rl64(col[i], l) * x[l];
      x[i] = sacc / rl64(col[i], i);
    }
  }
  if (c < b) {
#pragma unroll
    for (int r = 0; r < kCb; ++r) {
      if (r < b) {
        G[(int64_t)(j0 + r) * k + j0 + c] = c >= r ? col[r] : 0.0;
        Dinv[r * kCb + c] = x[r];
      }
    }
  }
}

// Block row of the panel: R[j0 + l][c] = sum_{l' <= l} Dinv[l'][l] G[j0 + l'][c]
// for c >= j0 + b (R_dd^T x = g). One thread per column c.
__global__ void __launch_bounds__(256) chol_panel_kernel(double* __restrict__ G, int k, int j0, int b,
                                                         const double* __restrict__ Dinv) {
  __shared__ double D[kCb][kCb];
  for (int idx = threadIdx.x; idx < b * kCb; idx += blockDim.x) D[idx / kCb][idx % kCb] = Dinv[idx];
  __syncthreads();
  const int c = j0 + b + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double g[kCb];
#pragma unroll
  for (int l = 0; l < kCb; ++l) g[l] = l < b ? G[(int64_t)(j0 + l) * k + c] : 0.0;
#pragma unroll
  for (int l = 0; l < kCb; ++l) {
    if (l < b) {
      double s = 0;
#pragma unroll
      for (int lp = 0; lp <= l; ++lp) s += D[lp][l] * g[lp];
      G[(int64_t)(j0 + l) * k + c] = s;
    }
  }
}

// Trailing update G[i][c] -= sum_l R[j0+l][i] R[j0+l][c] for t0 <= i <= c < k,
// t0 = j0 + b, in 32 x 32 tiles (only tiles on or above the diagonal).
__global__ void __launch_bounds__(256) chol_trail_kernel(double* __restrict__ G, int k, int j0, int b) {
  __shared__ double Ri[kCb][33], Rc[kCb][33];
  const int t0 = j0 + b;
  const int nt = (k - t0 + 31) / 32;
  // blockIdx.x enumerates (ti, tc) with ti <= tc
  int idx = blockIdx.x, ti = 0;
  while (idx >= nt - ti) {
    idx -= nt - ti;
    ++ti;
  }
  const int tc = ti + idx;
  const int i0 = t0 + 32 * ti, c0 = t0 + 32 * tc;
  for (int e = threadIdx.x; e < b * 32; e += blockDim.x) {
    const int l = e / 32, x = e - l * 32;
    Ri[l][x] = i0 + x < k ? G[(int64_t)(j0 + l) * k + i0 + x] : 0.0;
    Rc[l][x] = c0 + x < k ? G[(int64_t)(j0 + l) * k + c0 + x] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int x = e / 32, y = e - x * 32;
    const int i = i0 + x, c = c0 + y;
    if (i < k && c < k && c >= i) {
      double s = 0;
      for (int l = 0; l < b; ++l) s += Ri[l][x] * Rc[l][y];
      G[(int64_t)i * k + c] -= s;
    }
  }
}

// Zero the strictly lower triangle (k x k row-major).
__global__ void zero_lower_kernel(double* __restrict__ R, int k) {
  const int64_t total = (int64_t)k * k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / k, c = idx - i * k;
    if (c < i) R[idx] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Jacobi SVD, one workgroup per column pair
// ---------------------------------------------------------------------------
// Uc, Vc: column-major working copies (column j at j * k).
// Uc (k columns of length rows) = M (rows x k; row-major, or column-major
// when input_colmajor), Vc (k columns of length k) = I.
__global__ void jacobi_init_kernel(const double* __restrict__ M, int rows, int k, int input_colmajor,
                                   double* __restrict__ Uc, double* __restrict__ Vc) {
  const int64_t total = (int64_t)rows * k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = idx / rows, row = idx - col * rows;
    Uc[idx] = input_colmajor ? M[idx] : M[row * k + col];
  }
  if (!Vc) return;  // left singular vectors only
  const int64_t tv = (int64_t)k * k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tv; idx += (int64_t)gridDim.x * blockDim.x)
    Vc[idx] = (idx / k == idx % k) ? 1.0 : 0.0;
}

__device__ inline void rr_pair_g(int kp, int r, int i, int* p, int* q) {
  if (i == 0) {
    *p = r;
    *q = kp - 1;
  } else {
    const int m = kp - 1;
    *p = (r + i) % m;
    *q = ((r - i) % m + m) % m;
  }
}

// Block one-sided Jacobi. The columns of Uc are cut into blocks of BS; a
// workgroup takes either one block (diagonal visit: every pair inside it, in
// BS - 1 round-robin rounds) or a pair of blocks of the round (cross visit:
// the BS x BS pairs between them, in BS rounds of BS disjoint pairs). It
// holds the visit's columns in LDS, gives each pair of a round to one wave,
// rotates the columns there, and accumulates the same rotations in W
// (2BS x 2BS), so the columns of Vc are updated once at the end, V_J <- V_J W,
// one row of V_J per thread. Rotation and skip test are those of the pairwise
// method: a pair is rotated when |x_p . x_q| > tol sqrt(|x_p|^2 |x_q|^2).
// Columns past k (and blocks past the last) are absent: zero, never rotated,
// never written. Vc = null skips W and the V update (left vectors only).
template <int BS>
__global__ void __launch_bounds__(1024) jacobi_block_kernel(double* __restrict__ Uc, double* __restrict__ Vc, int rows,
                                                            int k, int nbp, int round, int diag, double tol,
                                                            int* __restrict__ rotated) {
  constexpr int NC = 2 * BS;
  extern __shared__ double lds[];
  double* X = lds;                      // [NC][rows]: local column c at X + c rows
  double* W = lds + (size_t)NC * rows;  // [NC][NC]: local column c at W + c NC
  __shared__ int any;
  const int tid = threadIdx.x, lane = tid & 63, nt = blockDim.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int P, Q = -1;
  if (diag)
    P = blockIdx.x;
  else
    rr_pair_g(nbp, round, blockIdx.x, &P, &Q);
  auto gcol = [&](int c) -> int {
    const int b = c < BS ? P : Q;
    const int j = b * BS + (c < BS ? c : c - BS);
    return (b >= 0 && j < k) ? j : -1;
  };
  const int ncols = diag ? BS : NC;
  for (int idx = tid; idx < ncols * rows; idx += nt) {
    const int c = idx / rows, i = idx - c * rows;
    const int j = gcol(c);
    X[idx] = j >= 0 ? Uc[(int64_t)j * rows + i] : 0.0;
  }
  for (int idx = tid; idx < NC * NC; idx += nt) W[idx] = (idx / NC == idx % NC) ? 1.0 : 0.0;
  if (tid == 0) any = 0;
  __syncthreads();

  const int rounds = diag ? BS - 1 : BS;
  const int npairs = diag ? BS / 2 : BS;
  for (int r = 0; r < rounds; ++r) {
    if (wave < npairs) {
      int p, q;
      if (diag) {
        rr_pair_g(BS, r, wave, &p, &q);
      } else {
        p = wave;
        q = BS + (wave + r) % BS;
      }
      double* xp = X + (size_t)p * rows;
      double* xq = X + (size_t)q * rows;
      // the first 8 rows of each lane stay in registers from the dot products
      // to the rotation; rows past 512 are read again
      double xr[8], yr[8];
      double a = 0, b = 0, g = 0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int i = lane + 64 * t;
        xr[t] = i < rows ? xp[i] : 0.0;
        yr[t] = i < rows ? xq[i] : 0.0;
        a += xr[t] * xr[t];
        b += yr[t] * yr[t];
        g += xr[t] * yr[t];
      }
      for (int i = lane + 512; i < rows; i += 64) {
        const double x = xp[i], y = xq[i];
        a += x * x;
        b += y * y;
        g += x * y;
      }
      a = wave_sum_dpp(a);
      b = wave_sum_dpp(b);
      g = wave_sum_dpp(g);
      if (fabs(g) > tol * sqrt(a * b) && g != 0.0) {
        const double zeta = (b - a) / (2.0 * g);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = lane + 64 * u;
          if (i < rows) {
            xp[i] = c * xr[u] - sn * yr[u];
            xq[i] = sn * xr[u] + c * yr[u];
          }
        }
        for (int i = lane + 512; i < rows; i += 64) {
          const double x = xp[i], y = xq[i];
          xp[i] = c * x - sn * y;
          xq[i] = sn * x + c * y;
        }
        if (Vc && lane < NC) {
          const double x = W[p * NC + lane], y = W[q * NC + lane];
          W[p * NC + lane] = c * x - sn * y;
          W[q * NC + lane] = sn * x + c * y;
        }
        if (lane == 0) any = 1;
      }
    }
    __syncthreads();
  }
  if (!any) return;  // nothing rotated: Uc and Vc are unchanged
  for (int idx = tid; idx < ncols * rows; idx += nt) {
    const int c = idx / rows, i = idx - c * rows;
    const int j = gcol(c);
    if (j >= 0) Uc[(int64_t)j * rows + i] = X[idx];
  }
  // V_J <- V_J W: thread i keeps row i of the old V_J in registers
  for (int i = tid; Vc && i < k; i += nt) {
    double v[NC];
#pragma unroll
    for (int r = 0; r < NC; ++r) {
      const int j = r < ncols ? gcol(r) : -1;
      v[r] = j >= 0 ? Vc[(int64_t)j * k + i] : 0.0;
    }
#pragma unroll 1
    for (int c = 0; c < ncols; ++c) {
      const int j = gcol(c);
      if (j < 0) continue;
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < NC; ++r) acc += v[r] * W[c * NC + r];
      Vc[(int64_t)j * k + i] = acc;
    }
  }
  if (tid == 0) *rotated = 1;
}

// s_j = ||u_j||, U = normalized columns; columns ranked by descending s
// (ties by index); U, V written row-major k x k.
__global__ void __launch_bounds__(1024) jacobi_finish_kernel(const double* __restrict__ Uc,
                                                             const double* __restrict__ Vc, int rows, int k,
                                                             double* __restrict__ U, double* __restrict__ s,
                                                             double* __restrict__ V, double* __restrict__ sig) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int j = wave; j < k; j += nw) {
    const double* uj = Uc + (int64_t)j * rows;
    double a = 0;
    for (int i = lane; i < rows; i += 64) a += uj[i] * uj[i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (lane == 0) sig[j] = sqrt(a);
  }
  __syncthreads();
  for (int j = tid; j < k; j += blockDim.x) {
    const double sj = sig[j];
    int rank = 0;
    for (int i = 0; i < k; ++i) rank += (sig[i] > sj) || (sig[i] == sj && i < j);
    s[rank] = sj;
    const double inv = sj > 0 ? 1.0 / sj : 0.0;
    for (int row = 0; row < rows; ++row) U[(int64_t)row * k + rank] = Uc[(int64_t)j * rows + row] * inv;
    if (V)
      for (int row = 0; row < k; ++row) V[(int64_t)row * k + rank] = Vc[(int64_t)j * k + row];
  }
}

__global__ void set_int_kernel(int* __restrict__ p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Y[j][i] = X[i][j] for X r x c row-major.
__global__ void transpose_kernel(const double* __restrict__ X, int64_t r, int64_t c, double* __restrict__ Y) {
  const int64_t total = r * c;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / c, j = idx - i * c;
    Y[j * r + i] = X[idx];
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192));
}

int launch_cholesky_upper(double* G, int k, double shift_coef, double* Dinv, int* fail, hipStream_t st) {
  if (shift_coef > 0) {
    hipLaunchKernelGGL(add_trace_shift_kernel, dim3(1), dim3(1024), 0, st, G, k, shift_coef);
    SK_HIP(hipGetLastError());
  }
  for (int j0 = 0; j0 < k; j0 += kCb) {
    const int b = std::min(kCb, k - j0);
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(64), 0, st, G, k, j0, b, Dinv, fail);
    const int rest = k - j0 - b;
    if (rest > 0) {
      hipLaunchKernelGGL(chol_panel_kernel, dim3((rest + 255) / 256), dim3(256), 0, st, G, k, j0, b,
                         (const double*)Dinv);
      const int nt = (rest + 31) / 32;
      hipLaunchKernelGGL(chol_trail_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, st, G, k, j0, b);
    }
    SK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(zero_lower_kernel, dim3(grid_for((int64_t)k * k)), dim3(256), 0, st, G, k);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, st, p, v);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_transpose(const double* X, int64_t r, int64_t c, double* Y, hipStream_t st) {
  hipLaunchKernelGGL(transpose_kernel, dim3(grid_for(r * c)), dim3(256), 0, st, X, r, c, Y);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

__global__ void sum_partials_kernel(const double* __restrict__ P, int np, int64_t count, double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < np; ++c) acc += P[(int64_t)c * count + e];
    out[e] = acc;
  }
}

int launch_sum_partials(const double* P, int np, int64_t count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(grid_for(count)), dim3(256), 0, st, P, np, count, out);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// Numerical rank r = #{i : s_i > 5 eps s_0} (eps = 2^-52, s descending) and
// the truncated factors: Vs[i][j] = V[i][j] / s_j and Ur[i][j] = U[i][j] for
// j < r, zero for j >= r (V k x k, U p x k, row-major). One workgroup.
__global__ void __launch_bounds__(256) gn_truncate_kernel(const double* __restrict__ s, int k,
                                                          const double* __restrict__ V, double* __restrict__ Vs,
                                                          const double* __restrict__ U, int p, double* __restrict__ Ur,
                                                          int* __restrict__ rank) {
  __shared__ int r_sh;
  if (threadIdx.x == 0) {
    const double thr = 5.0 * 0x1p-52 * s[0];
    int r = 0;
    while (r < k && s[r] > thr) ++r;
    r_sh = r;
    *rank = r;
  }
  __syncthreads();
  const int r = r_sh;
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int j = idx % k;
    Vs[idx] = j < r ? V[idx] / s[j] : 0.0;
  }
  for (int idx = threadIdx.x; idx < p * k; idx += blockDim.x) {
    const int j = idx % k;
    Ur[idx] = j < r ? U[idx] : 0.0;
  }
}

int launch_gn_truncate(const double* s, int k, const double* V, double* Vs, const double* U, int p, double* Ur,
                       int* rank, hipStream_t st) {
  hipLaunchKernelGGL(gn_truncate_kernel, dim3(1), dim3(256), 0, st, s, k, V, Vs, U, p, Ur, rank);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// Nystrom (Alg. 2) helpers --------------------------------------------------

// *nu = coef * sqrt(lambda_max(G)) for a k x k symmetric psd G: power
// iterations from the all-ones vector, stopped when the Rayleigh quotient
// changes by at most 1e-12 relative (at most 100). G is symmetric, so y = G x
// reads G by columns (thread i walks column i: consecutive threads read
// consecutive addresses). One workgroup; x and G x live in LDS.
__global__ void __launch_bounds__(1024) power_norm_kernel(const double* __restrict__ G, int k, double coef,
                                                          double* __restrict__ nu) {
  extern __shared__ double xs[];  // x[k], y[k]
  __shared__ double red[16];
  double* x = xs;
  double* y = xs + k;
  for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] = 1.0;
  __syncthreads();
  double lam = 0.0, lam_prev = -1.0;
  for (int it = 0; it <= 100; ++it) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < k; ++j) acc += G[(int64_t)j * k + i] * x[j];
      y[i] = acc;
    }
    __syncthreads();
    double xy = 0.0, yy = 0.0, xx = 0.0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      xy += x[i] * y[i];
      yy += y[i] * y[i];
      xx += x[i] * x[i];
    }
    xy = wg_reduce_sum(xy, red);
    yy = wg_reduce_sum(yy, red);
    xx = wg_reduce_sum(xx, red);
    lam = xx > 0 ? xy / xx : 0.0;  // Rayleigh quotient of x
    const double inv = yy > 0 ? 1.0 / sqrt(yy) : 0.0;
    __syncthreads();
    // every thread holds the same reduced values: the exit is uniform
    if (fabs(lam - lam_prev) <= 1e-12 * fabs(lam)) break;
    lam_prev = lam;
    for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] = y[i] * inv;
    __syncthreads();
  }
  if (threadIdx.x == 0) *nu = coef * sqrt(fmax(lam, 0.0));
}

// Y (n x k, ld k) += nu Omega with Omega = S^T for a SparseStack S (k x n):
// row i gets rho_it / sqrt(zeta) * nu in column t nb + s_it.
__global__ void add_omega_ss_kernel(double* __restrict__ Y, int64_t n, int k, int zeta, int nb, uint32_t k0, uint32_t k1,
                                    double scale, const double* __restrict__ nup) {
  const double nu = *nup;
  const int ng = (zeta + 3) / 4;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * ng;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / ng;
    const int g = (int)(idx - i * ng);
    const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)g, kTagSparseStack}, k0, k1);
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * g + j;
      if (t < zeta) {
        const uint32_t word = word_of(w, j);
        const double v = (ss_negative(word) ? -scale : scale) * nu;
        Y[i * k + (int64_t)t * nb + ss_bucket(word, (uint32_t)nb)] += v;
      }
    }
  }
}

// Y (n x k) += nu Omega with Omega = G^T, G (k x n, row-major) written out.
__global__ void add_omega_dense_kernel(double* __restrict__ Y, int64_t n, int k, const double* __restrict__ G,
                                       const double* __restrict__ nup) {
  const double nu = *nup;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * k;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / k, j = idx - i * k;
    Y[idx] += nu * G[j * n + i];
  }
}

// B (k x k) <- (B + B^T) / 2
__global__ void symmetrize_kernel(double* __restrict__ B, int k) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)k * k;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / k, j = idx - i * k;
    if (i < j) {
      const double v = 0.5 * (B[i * k + j] + B[j * k + i]);
      B[i * k + j] = v;
      B[j * k + i] = v;
    }
  }
}

// lambda_j = max(0, s_j^2 - nu)
__global__ void remove_shift_kernel(const double* __restrict__ s, int k, const double* __restrict__ nup,
                                    double* __restrict__ lambda) {
  const double nu = *nup;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x)
    lambda[j] = fmax(0.0, s[j] * s[j] - nu);
}

int launch_nystrom_shift(const double* G, int k, int64_t n, double* nu, hipStream_t st) {
  const double coef = std::sqrt((double)n) * 0x1p-52;
  const size_t lds = (size_t)2 * k * sizeof(double);
  SK_HIP(hipFuncSetAttribute((const void*)power_norm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(power_norm_kernel, dim3(1), dim3(1024), lds, st, G, k, coef, nu);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_add_omega_ss(double* Y, int64_t n, int k, int zeta, int nb, uint32_t k0, uint32_t k1, double scale,
                        const double* nu, hipStream_t st) {
  hipLaunchKernelGGL(add_omega_ss_kernel, dim3(grid_for(n * ((zeta + 3) / 4))), dim3(256), 0, st, Y, n, k, zeta, nb,
                     k0, k1, scale, nu);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_add_omega_dense(double* Y, int64_t n, int k, const double* G, const double* nu, hipStream_t st) {
  hipLaunchKernelGGL(add_omega_dense_kernel, dim3(grid_for(n * k)), dim3(256), 0, st, Y, n, k, G, nu);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_symmetrize(double* B, int k, hipStream_t st) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(grid_for((int64_t)k * k)), dim3(256), 0, st, B, k);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_remove_shift(const double* s, int k, const double* nu, double* lambda, hipStream_t st) {
  hipLaunchKernelGGL(remove_shift_kernel, dim3((k + 255) / 256), dim3(256), 0, st, s, k, nu, lambda);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

size_t jacobi_work_doubles(int64_t rows, int k) { return (size_t)rows * k + (size_t)k * k + k; }

int jacobi_svd_rounds(const double* M, int64_t rows, int k, int input_colmajor, double* U, double* s, double* V,
                      double* work, int* flag, int* h_flag, int max_sweeps, int* sweeps, hipStream_t st) {
  if (rows < k || rows > INT_MAX) {
    set_error("Jacobi SVD: need k <= rows");
    return SK_E_INVAL;
  }
  const int nr = (int)rows;
  double* Uc = work;
  double* Vbuf = work + (size_t)nr * k;
  double* sig = Vbuf + (size_t)k * k;
  double* Vc = V ? Vbuf : nullptr;  // V = null: left singular vectors only
  hipLaunchKernelGGL(jacobi_init_kernel, dim3(grid_for((int64_t)nr * k)), dim3(256), 0, st, M, nr, k, input_colmajor,
                     Uc, Vc);
  SK_HIP(hipGetLastError());
  // block size 8 (measured best at k = 512 against 4 and 16: the rounds of a
  // sweep are latency-bound launches, so fewer rounds win until a visit's own
  // work dominates), smaller for tiny k or when a visit (2 BS columns of
  // `rows` doubles + W) would not fit in LDS
  const size_t cap = 160 * 1024;
  static const int bs_env = [] {
    const char* v = std::getenv("SKETCH_JACOBI_BS");
    return v ? std::atoi(v) : 0;
  }();
  int bs = (bs_env == 2 || bs_env == 4 || bs_env == 8 || bs_env == 16) ? bs_env : 8;
  while (bs > 2 && ((bs_env == 0 && 2 * bs > k) || ((size_t)2 * bs * nr + (size_t)4 * bs * bs) * sizeof(double) > cap))
    bs /= 2;
  const size_t lds = ((size_t)2 * bs * nr + (size_t)4 * bs * bs) * sizeof(double);
  if (lds > cap) {
    set_error("Jacobi SVD: columns too long for the block visits");
    return SK_E_NOTSUP;
  }
  const int nblk = (k + bs - 1) / bs;
  const int nbp = nblk + (nblk & 1);
  // rotation threshold sqrt(rows) u (u = 2^-53), the rounding level of the
  // computed column dot products (as in one-sided Jacobi codes such as
  // LAPACK's): a stricter threshold only rotates pairs whose computed product
  // is rounding noise and adds sweeps
  const double tol = std::sqrt((double)nr) * 0x1p-53;
  auto visit = [&](int grid, int round, int diag) -> int {
    switch (bs) {
#define SK_JB(B)                                                                                                  \
  case B:                                                                                                       \
    SK_HIP(hipFuncSetAttribute((const void*)jacobi_block_kernel<B>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                               (int)lds));                                                                      \
    hipLaunchKernelGGL(jacobi_block_kernel<B>, dim3(grid), dim3(64 * B), lds, st, Uc, Vc, nr, k, nbp, round,    \
                       diag, tol, flag);                                                                            \
    break;
      SK_JB(16)
      SK_JB(8)
      SK_JB(4)
      SK_JB(2)
#undef SK_JB
      default:
        return SK_E_NOTSUP;
    }
    SK_HIP(hipGetLastError());
    return SK_OK;
  };
  int sw = 0;
  for (; sw < max_sweeps; ++sw) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, st, flag, 0);
    int rc = visit(nblk, 0, 1);
    if (rc != SK_OK) return rc;
    for (int r = 0; r < nbp - 1; ++r) {
      rc = visit(nbp / 2, r, 0);
      if (rc != SK_OK) return rc;
    }
    SK_HIP(hipMemcpyAsync(h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    SK_HIP(hipStreamSynchronize(st));
    if (*h_flag == 0) {
      ++sw;
      break;
    }
  }
  if (sweeps) *sweeps = sw;
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(1024), 0, st, (const double*)Uc, (const double*)Vc, nr, k, U,
                     s, V, sig);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
