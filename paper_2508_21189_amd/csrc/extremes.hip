// Injectivity and dilation of a SparseStack on the coordinate basis (the
// experiment of Fig. 2): for Q = [e_1 ... e_n], alpha = sigma_min(S Q)^2 and
// beta = sigma_max(S Q)^2 (Prop. 1.9), i.e. the extreme eigenvalues of the
// Gram matrix G = S^T S of the sketch's n columns.
//
// They are estimated by the Lanczos method on G (three-term recurrence from
// a seeded Gaussian start, no reorthogonalization): the extreme
// eigenvalues of the k x k tridiagonal T_k lie inside [lambda_min(G),
// lambda_max(G)] and converge to its ends; lost orthogonality only adds
// copies of converged values. The eigenvalues of T_k come from Sturm-count
// bisection on the host (T_k is tiny).
//
// G v = S^T (S v) without forming G:
//  * S v (d x n times n): a CSR form of S built once per call: the n*zeta
//    (row, column) pairs from the Philox hash, sorted by row with a stable
//    least-significant-digit radix sort (8-bit digits; per-block digit
//    counts, one scan, a scatter in which each wave ranks equal digits by
//    ballot and keeps per-digit running positions, so input order is kept),
//    so each row adds its entries in column order (deterministic), one
//    thread per row;
//  * S^T y: the hash-based adjoint kernel (each column gathers its zeta
//    entries).
// Dot products reduce in a fixed order (per-block partial sums, then every
// block re-adds the partials in order), so the estimate is bitwise
// reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sk_drivers.hpp"

namespace sk {

constexpr uint32_t kTagLanczos = 6;
constexpr int kLzBlocks = 512;
constexpr int kLzThreads = 256;

// Pairs (row t*nb + s_it, column i | negative << 31) for i < n, t < zeta, in
// the order i*zeta + t.
__global__ void ext_pairs_kernel(int64_t n, int zeta, uint32_t nb, uint32_t k0, uint32_t k1, uint32_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals) {
  const int ng = (zeta + 3) / 4;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    for (int g = 0; g < ng; ++g) {
      const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)g, kTagSparseStack}, k0, k1);
      for (int j = 0; j < 4; ++j) {
        const int t = 4 * g + j;
        if (t < zeta) {
          const uint32_t word = word_of(w, j);
          keys[i * zeta + t] = (uint32_t)t * nb + ss_bucket(word, nb);
          vals[i * zeta + t] = (uint32_t)i | (ss_negative(word) << 31);
        }
      }
    }
  }
}

// ---- stable LSD radix sort of (key, value) pairs, 8-bit digits
constexpr int kRsBlocks = 1024;  // element ranges (one workgroup each)

// Elements of range b: [b * per, min(N, (b + 1) * per)).
__global__ void __launch_bounds__(256) rs_count_kernel(int64_t N, int64_t per, const uint32_t* __restrict__ keys,
                                                       int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int b = blockIdx.x;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)b * per, hi = min(N, lo + per);
  for (int64_t e = lo + threadIdx.x; e < hi; e += 256) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
  __syncthreads();
  hist[(int64_t)threadIdx.x * kRsBlocks + b] = h[threadIdx.x];  // digit-major
}

// Exclusive prefix sum of one digit's counts over the ranges (workgroup g
// for digit g; kRsBlocks threads): hist[g][b] becomes the number of
// elements of digit g in ranges before b, tot[g] the digit's total.
__global__ void __launch_bounds__(kRsBlocks) rs_scan_kernel(uint32_t* __restrict__ hist, uint32_t* __restrict__ tot) {
  __shared__ uint32_t s[kRsBlocks];
  const int t = threadIdx.x;
  uint32_t* h = hist + (int64_t)blockIdx.x * kRsBlocks;
  const uint32_t x = h[t];
  s[t] = x;
  __syncthreads();
  for (int off = 1; off < kRsBlocks; off <<= 1) {
    const uint32_t y = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += y;
    __syncthreads();
  }
  h[t] = s[t] - x;
  if (t == kRsBlocks - 1) tot[blockIdx.x] = s[t];
}

// Scatter of range b by one wave, in input order, 64 elements at a time: the
// lanes holding the same digit are found by 8 ballots; a lane's position is
// its digit's running position plus the number of lower lanes with that
// digit, and the highest of them advances the running position.
__global__ void __launch_bounds__(64) rs_scatter_kernel(int64_t N, int64_t per, const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals, int shift,
                                                        const uint32_t* __restrict__ hist,
                                                        const uint32_t* __restrict__ tot,
                                                        uint32_t* __restrict__ okeys, uint32_t* __restrict__ ovals) {
  __shared__ uint32_t run[256];
  const int b = blockIdx.x, lane = threadIdx.x;
  // digits 4 lane .. 4 lane + 3: their start = totals of the lower digits
  uint32_t t4[4], acc = 0;
  for (int j = 0; j < 4; ++j) {
    t4[j] = tot[4 * lane + j];
    acc += t4[j];
  }
  uint32_t incl = acc;  // inclusive scan of the lanes' sums
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  uint32_t start = incl - acc;
  for (int j = 0; j < 4; ++j) {
    const int g = 4 * lane + j;
    run[g] = start + hist[(int64_t)g * kRsBlocks + b];
    start += t4[j];
  }
  __syncthreads();
  const int64_t lo = (int64_t)b * per, hi = min(N, lo + per);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t c = lo; c < hi; c += 64) {
    const int64_t e = c + lane;
    const bool valid = e < hi;
    const uint32_t k = valid ? keys[e] : 0u;
    const uint32_t v = valid ? vals[e] : 0u;
    const uint32_t dg = (k >> shift) & 255u;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t ones = __ballot(valid && ((dg >> bit) & 1u));
      same &= ((dg >> bit) & 1u) ? ones : ~ones;
    }
    if (valid) {
      const uint32_t pos = run[dg] + (uint32_t)__popcll(same & below);
      okeys[pos] = k;
      ovals[pos] = v;
    }
    __syncthreads();  // every lane has read run[] before it advances
    if (valid && (same >> lane) == 1ull) run[dg] += (uint32_t)__popcll(same);
    __syncthreads();
  }
}

// rowptr[r] = first position p with key[p] >= r, for r = 0 .. d (rowptr[d] = N).
__global__ void ext_rowptr_kernel(int64_t N, const uint32_t* __restrict__ key, int64_t d, int64_t* __restrict__ rowptr) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p <= N; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kp = p < N ? (int64_t)key[p] : d;
    const int64_t kprev = p > 0 ? (int64_t)key[p - 1] : -1;
    for (int64_t r = kprev + 1; r <= kp; ++r) rowptr[r] = p;
  }
}

// y[r] = scale * sum over row r's entries of (+-1) v[column], in column order.
__global__ void ext_spmv_kernel(int64_t d, const int64_t* __restrict__ rowptr, const uint32_t* __restrict__ vals,
                                const double* __restrict__ v, double scale, double* __restrict__ y) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < d; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
      const uint32_t e = vals[p];
      const double x = v[e & 0x7fffffffu];
      s += (e >> 31) ? -x : x;
    }
    y[r] = s * scale;
  }
}


// Sum of the block's values in a fixed tree order (blockDim = kLzThreads).
__device__ inline double block_sum(double x, double* sh) {
  const int t = threadIdx.x;
  sh[t] = x;
  __syncthreads();
  for (int s = kLzThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Every block adds the kLzBlocks partials in the same order: the same value
// everywhere.
__device__ inline double sum_partials(const double* __restrict__ part, double* sh) {
  double x = 0.0;
  for (int b = threadIdx.x; b < kLzBlocks; b += kLzThreads) x += part[b];
  return block_sum(x, sh);
}

// Start: w[i] = z_i ~ N(0, 1) (Philox counter (i mod 2^32, i >> 32, 0, TAG)
// under the start seed; Box-Muller on 52-bit uniforms from words (0, 1) and
// (2, 3), the cosine branch), vprev = 0, part2[block] = partial ||w||^2. A
// continuous start has, almost surely, a component along every eigenvector
// (a +-1 start can be orthogonal to one: with zeta = 1, S^T S has eigenvectors
// supported on a few columns).
__global__ void __launch_bounds__(kLzThreads) lz_start_kernel(int64_t n, uint32_t k0, uint32_t k1,
                                                               double* __restrict__ w, double* __restrict__ vprev,
                                                               double* __restrict__ part2) {
  __shared__ double sh[kLzThreads];
  double x = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kLzThreads + threadIdx.x; i < n; i += (int64_t)kLzBlocks * kLzThreads) {
    const U4 q = philox4x32_10(U4{(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, kTagLanczos}, k0, k1);
    const uint64_t x1 = ((uint64_t)q.x << 20) | (q.y >> 12);
    const uint64_t x2 = ((uint64_t)q.z << 20) | (q.w >> 12);
    const double u1 = ((double)x1 + 0.5) * 0x1p-52;
    const double u2 = ((double)x2 + 0.5) * 0x1p-52;
    const double z = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
    w[i] = z;
    vprev[i] = 0.0;
    x += z * z;
  }
  const double s = block_sum(x, sh);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
}

// part[block] = sum over the block's grid-stride share of a[i] * b[i].
__global__ void __launch_bounds__(kLzThreads) lz_dot_kernel(int64_t n, const double* __restrict__ a,
                                                             const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[kLzThreads];
  double x = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kLzThreads + threadIdx.x; i < n; i += (int64_t)kLzBlocks * kLzThreads)
    x += a[i] * b[i];
  const double s = block_sum(x, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// alpha_j = w . v_j (from the partials); w -= alpha_j v_j + beta_j v_{j-1};
// part2[block] = partial ||w||^2.
__global__ void __launch_bounds__(kLzThreads) lz_update_kernel(int64_t n, double* __restrict__ w,
                                                                const double* __restrict__ v,
                                                                const double* __restrict__ vprev,
                                                                const double* __restrict__ part, double* __restrict__ alpha,
                                                                const double* __restrict__ beta, int j,
                                                                double* __restrict__ part2) {
  __shared__ double sh[kLzThreads];
  const double a = sum_partials(part, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) alpha[j] = a;
  const double b = beta[j];
  double x = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kLzThreads + threadIdx.x; i < n; i += (int64_t)kLzBlocks * kLzThreads) {
    const double wi = w[i] - a * v[i] - b * vprev[i];
    w[i] = wi;
    x += wi * wi;
  }
  const double s = block_sum(x, sh);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
}

// beta_{j+1} = ||w||; v_{j+1} = w / beta_{j+1} (written over v_{j-1}, which
// is no longer needed). A breakdown (beta_{j+1} <= tol: an invariant subspace)
// records the step count in *kstop and stops the vectors.
__global__ void __launch_bounds__(kLzThreads) lz_next_kernel(int64_t n, const double* __restrict__ w,
                                                              double* __restrict__ vnext, const double* __restrict__ part2,
                                                              double* __restrict__ beta, int j, double tol,
                                                              int* __restrict__ kstop) {
  __shared__ double sh[kLzThreads];
  const double b = sqrt(sum_partials(part2, sh));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    beta[j + 1] = b;
    if (b <= tol && *kstop > j + 1) *kstop = j + 1;
  }
  const double inv = b > tol ? 1.0 / b : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kLzThreads + threadIdx.x; i < n; i += (int64_t)kLzBlocks * kLzThreads)
    vnext[i] = w[i] * inv;
}

__global__ void lz_init_scalars_kernel(int* kstop, int v, double* beta0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *kstop = v;
    *beta0 = 0.0;
  }
}

// Number of eigenvalues of the symmetric tridiagonal (a[0..k-1], off-diagonal
// b[1..k-1]) below x (Sturm sequence of the LDL^T pivots).
static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, int k, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    const double off = i > 0 ? b[i] * b[i] : 0.0;
    q = a[i] - x - (i > 0 ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// Smallest and largest eigenvalues of the leading k x k tridiagonal, by
// bisection inside the Gershgorin interval.
static void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, int k, double* lo_out,
                             double* hi_out) {
  double glo = a[0], ghi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < k ? std::fabs(b[i + 1]) : 0.0);
    glo = std::min(glo, a[i] - r);
    ghi = std::max(ghi, a[i] + r);
  }
  auto bisect = [&](int target) {  // smallest x with count(x) >= target
    double l = glo - 1e-12 * (1 + std::fabs(glo)), h = ghi + 1e-12 * (1 + std::fabs(ghi));
    for (int it = 0; it < 200 && h - l > 0; ++it) {
      const double mid = 0.5 * (l + h);
      if (mid <= l || mid >= h) break;
      if (sturm_count(a, b, k, mid) >= target)
        h = mid;
      else
        l = mid;
    }
    return 0.5 * (l + h);
  };
  *lo_out = bisect(1);
  *hi_out = bisect(k);
}

namespace {
struct ExtCarve {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + std::max<size_t>(1, count) * sizeof(T);
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

int ext_workspace(sk_sketch* S, size_t bytes, char** out, hipStream_t st) {
  const int rc = grow_buffer(&S->dws, &S->dws_bytes, bytes, st);
  if (rc != SK_OK) return rc;
  *out = static_cast<char*>(S->dws);
  return SK_OK;
}
}  // namespace

}  // namespace sk

using namespace sk;

extern "C" int sketch_sv_extremes(sketch_t S, int steps, uint64_t start_seed, double* alpha_out, double* beta_out,
                                  sk_extremes_info* info, void* stream) {
  if (!S || !alpha_out || !beta_out || steps < 1 || steps > 100000) {
    set_error("sketch_sv_extremes: invalid argument (need a handle, outputs and 1 <= steps <= 100000)");
    return SK_E_INVAL;
  }
  if (S->kind != SK_SPARSESTACK) {
    set_error("sketch_sv_extremes: needs a SparseStack sketch");
    return SK_E_NOTSUP;
  }
  const int64_t n = S->n, d = S->d;
  const int zeta = S->zeta;
  const int64_t N = n * zeta;
  if (n >= (int64_t)1 << 31 || d >= (int64_t)1 << 32 || N >= (int64_t)1 << 31) {
    set_error("sketch_sv_extremes: needs n < 2^31, d < 2^32 and n * zeta < 2^31");
    return SK_E_NOTSUP;
  }
  const int K = (int)std::min<int64_t>(steps, n);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[3] = {};
  for (auto& e : ev) SK_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 3; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  SK_HIP(hipEventRecord(ev[0], st));

  // workspace: the sort's buffers, CSR, Lanczos vectors and scalars
  int end_bit = 1;
  while (end_bit < 32 && ((uint64_t)1 << end_bit) < (uint64_t)d) ++end_bit;
  const size_t sort_tmp = (size_t)256 * (kRsBlocks + 1) * sizeof(uint32_t);
  ExtCarve cv;
  auto carve = [&](ExtCarve& c, uint32_t** k0p, uint32_t** k1p, uint32_t** v0p, uint32_t** v1p, char** tmp,
                   int64_t** rowptr, double** v, double** vp, double** w, double** y, double** part, double** part2,
                   double** al, double** be, int** kstop) {
    *k0p = c.take<uint32_t>(N);
    *k1p = c.take<uint32_t>(N);
    *v0p = c.take<uint32_t>(N);
    *v1p = c.take<uint32_t>(N);
    *tmp = c.take<char>(sort_tmp);
    *rowptr = c.take<int64_t>(d + 1);
    *v = c.take<double>(n);
    *vp = c.take<double>(n);
    *w = c.take<double>(n);
    *y = c.take<double>(d);
    *part = c.take<double>(kLzBlocks);
    *part2 = c.take<double>(kLzBlocks);
    *al = c.take<double>(K + 1);
    *be = c.take<double>(K + 2);
    *kstop = c.take<int>(1);
  };
  uint32_t *keys, *keys2, *vals, *vals2;
  char* tmp;
  int64_t* rowptr;
  double *v, *vp, *w, *y, *part, *part2, *al, *be;
  int* kstop;
  carve(cv, &keys, &keys2, &vals, &vals2, &tmp, &rowptr, &v, &vp, &w, &y, &part, &part2, &al, &be, &kstop);
  char* base = nullptr;
  {
    int rc = ext_workspace(S, cv.off, &base, st);
    if (rc != SK_OK) return rc;
  }
  ExtCarve c2;
  c2.base = base;
  carve(c2, &keys, &keys2, &vals, &vals2, &tmp, &rowptr, &v, &vp, &w, &y, &part, &part2, &al, &be, &kstop);

  // CSR of S
  const unsigned g1 = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
  hipLaunchKernelGGL(ext_pairs_kernel, dim3(g1), dim3(256), 0, st, n, zeta, (uint32_t)S->nb, S->k0, S->k1, keys, vals);
  SK_HIP(hipGetLastError());
  {
    // passes over 8 bits at a time, ping-ponging; the sorted pairs end in
    // keys2 / vals2
    const int passes = (end_bit + 7) / 8;
    const int64_t per = (N + kRsBlocks - 1) / kRsBlocks;
    uint32_t* hist = (uint32_t*)tmp;
    uint32_t* tot = hist + 256 * kRsBlocks;
    // an odd number of passes from keys / vals ends in keys2 / vals2; for
    // an even number the input is first copied to keys2 / vals2 and sorted
    // from there
    uint32_t *ki = keys, *vi = vals, *ko = keys2, *vo = vals2;
    if (passes % 2 == 0) {
      SK_HIP(hipMemcpyAsync(keys2, keys, N * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
      SK_HIP(hipMemcpyAsync(vals2, vals, N * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
      std::swap(ki, ko);
      std::swap(vi, vo);
    }
    for (int p = 0; p < passes; ++p) {
      hipLaunchKernelGGL(rs_count_kernel, dim3(kRsBlocks), dim3(256), 0, st, N, per, (const uint32_t*)ki, 8 * p, hist);
      hipLaunchKernelGGL(rs_scan_kernel, dim3(256), dim3(kRsBlocks), 0, st, hist, tot);
      hipLaunchKernelGGL(rs_scatter_kernel, dim3(kRsBlocks), dim3(64), 0, st, N, per, (const uint32_t*)ki,
                         (const uint32_t*)vi, 8 * p, (const uint32_t*)hist, (const uint32_t*)tot, ko, vo);
      SK_HIP(hipGetLastError());
      std::swap(ki, ko);
      std::swap(vi, vo);
    }
  }
  const unsigned g2 = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + 256) / 256, 16384));
  hipLaunchKernelGGL(ext_rowptr_kernel, dim3(g2), dim3(256), 0, st, N, (const uint32_t*)keys2, d, rowptr);
  SK_HIP(hipGetLastError());
  SK_HIP(hipEventRecord(ev[1], st));

  // Lanczos on G = S^T S
  const double scale = inv_sqrt_host((double)zeta);
  const unsigned gd = (unsigned)std::max<int64_t>(1, std::min<int64_t>((d + 255) / 256, 16384));
  hipLaunchKernelGGL(lz_init_scalars_kernel, dim3(1), dim3(64), 0, st, kstop, K, be);
  hipLaunchKernelGGL(lz_start_kernel, dim3(kLzBlocks), dim3(kLzThreads), 0, st, n, (uint32_t)start_seed,
                     (uint32_t)(start_seed >> 32), w, vp, part2);
  // v_0 = w / ||w|| (the kernel also stores ||w|| in beta[0], which multiplies
  // v_{-1} = 0 and so never enters the recurrence; the tridiagonal uses
  // beta[1..])
  hipLaunchKernelGGL(lz_next_kernel, dim3(kLzBlocks), dim3(kLzThreads), 0, st, n, (const double*)w, v,
                     (const double*)part2, be, -1, 0.0, kstop);
  SK_HIP(hipGetLastError());
  // breakdown threshold: the mean eigenvalue of G is exactly 1 (every column
  // of S has unit norm), so the scale of G is about 1
  const double tol = 1e-12;
  for (int j = 0; j < K; ++j) {
    hipLaunchKernelGGL(ext_spmv_kernel, dim3(gd), dim3(256), 0, st, d, (const int64_t*)rowptr, (const uint32_t*)vals2,
                       (const double*)v, scale, y);
    int rc = launch_adjoint(S, 1, y, 1, w, 1, st);
    if (rc != SK_OK) return rc;
    hipLaunchKernelGGL(lz_dot_kernel, dim3(kLzBlocks), dim3(kLzThreads), 0, st, n, (const double*)w, (const double*)v,
                       part);
    hipLaunchKernelGGL(lz_update_kernel, dim3(kLzBlocks), dim3(kLzThreads), 0, st, n, w, (const double*)v,
                       (const double*)vp, (const double*)part, al, (const double*)be, j, part2);
    hipLaunchKernelGGL(lz_next_kernel, dim3(kLzBlocks), dim3(kLzThreads), 0, st, n, (const double*)w, vp,
                       (const double*)part2, be, j, tol, kstop);
    SK_HIP(hipGetLastError());
    std::swap(v, vp);  // v_{j+1} was written over v_{j-1}
  }
  SK_HIP(hipEventRecord(ev[2], st));
  std::vector<double> a(K + 1), b(K + 2);
  int ks = K;
  SK_HIP(hipMemcpyAsync(a.data(), al, sizeof(double) * K, hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(b.data(), be, sizeof(double) * (K + 1), hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(&ks, kstop, sizeof(int), hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  const int keff = std::max(1, std::min(K, ks));
  double lo = 0, hi = 0;
  tridiag_extremes(a, b, keff, &lo, &hi);
  *alpha_out = lo;
  *beta_out = hi;
  if (info) {
    info->steps = keff;
    double lo2 = lo, hi2 = hi;
    const int kp = std::max(1, (3 * keff) / 4);
    tridiag_extremes(a, b, kp, &lo2, &hi2);
    info->alpha_at_3_4 = lo2;
    info->beta_at_3_4 = hi2;
    float t1 = 0, t2 = 0;
    (void)hipEventElapsedTime(&t1, ev[0], ev[1]);
    (void)hipEventElapsedTime(&t2, ev[1], ev[2]);
    info->t_build_ms = t1;
    info->t_iter_ms = t2;
  }
  return SK_OK;
}
