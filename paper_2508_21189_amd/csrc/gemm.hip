// Dense GEMM on the matrix cores (gfx950): C = alpha op(A) op(B) + beta C for
// row-major FP32 or FP64 operands, op = identity or transpose. The low-rank
// drivers (Alg. 1 and its Nystrom relatives: Y^T Y, Y R^-1, Q^T A, Q U) and
// the materialized Gaussian sketch (Def. 1.4) in column mode multiply through
// it.
//
// Blocking: a workgroup of 4 waves owns a BM x BN tile of C (waves 2 x 2,
// each (BM/2) x (BN/2) built from 16 x 16 matrix-core tiles) and a range of
// K (split-K when the output has too few tiles to fill the chip; partial
// tiles are summed in split order by a second kernel, so the result is
// deterministic). Per step of BK: the next step's tile of op(A) and op(B) is
// read from global memory into registers while the current step's tile is
// multiplied from LDS; both LDS tiles are k-major ([k][m] and [k][n]), so a
// lane's matrix operands (row l % 16, k-step l / 16) are contiguous reads.
//
// v_mfma_f32_16x16x4f32 and v_mfma_f64_16x16x4f64: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the 16 x 16 result's item v sits
// at row 4 (l / 16) + v (FP32) or 4 v + l / 16 (FP64), column l % 16.
#include "sk_gemm.hpp"

#include <algorithm>

namespace sk {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using acc = v4f;
  __device__ static acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // row of item v of the result
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Mfma<double> {
  using acc = v4d;
  __device__ static acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

constexpr int kThreads = 256;

// VEC consecutive elements from an address aligned to VEC elements.
template <typename T, int VEC>
__device__ inline void ldvec(const T* src, T* out) {
  if constexpr (VEC == 4 && sizeof(T) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 v = *(const f4*)src;
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
    out[3] = v[3];
  } else if constexpr (VEC == 2 && sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = *(const d2*)src;
    out[0] = v[0];
    out[1] = v[1];
  } else {
#pragma unroll
    for (int q = 0; q < VEC; ++q) out[q] = src[q];
  }
}

// One workgroup: C tile (m0, n0) of split s; P != nullptr: write the raw
// partial sum there ([split][M][N]) instead of alpha * acc + beta * C.
// VEC consecutive elements along an operand's contiguous dimension are read
// per load when its base and leading dimension allow (VEC = 1 otherwise).
template <typename T, bool TA, bool TB, int BM, int BN, int BK, int VEC>
__global__ void __launch_bounds__(kThreads) gemm_kernel(GemmArgs g) {
  using M = Mfma<T>;
  using Acc = typename M::acc;
  constexpr int WM = BM / 2, WN = BN / 2;        // wave tile
  constexpr int IB = WM / 16, JB = WN / 16;      // 16 x 16 tiles per wave
  constexpr int PAD = 4;                         // LDS row padding (elements)
  constexpr int LA = (BM * BK) / (kThreads * VEC);  // op(A) vector loads of a thread per step
  constexpr int LB = (BK * BN) / (kThreads * VEC);
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = (wave >> 1) * WM, wj = (wave & 1) * WN;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int split = blockIdx.z;
  const int64_t kper = g.k_per_split;
  const int64_t kbeg = (int64_t)split * kper;
  const int64_t kend = min(g.K, kbeg + kper);
  const T* A = (const T*)g.A;
  const T* B = (const T*)g.B;

  // Vector load e of a thread covers (i, kk) .. VEC along the contiguous
  // dimension: k when A is stored row-major M x K (op = identity), i when A
  // is stored K x M (op = transpose); likewise j or k for B.
  auto a_coord = [&](int e, int* i, int* kk) {
    const int q = tid + e * kThreads;
    if constexpr (TA) {
      *kk = q / (BM / VEC);
      *i = (q - *kk * (BM / VEC)) * VEC;
    } else {
      *i = q / (BK / VEC);
      *kk = (q - *i * (BK / VEC)) * VEC;
    }
  };
  auto b_coord = [&](int e, int* kk, int* j) {
    const int q = tid + e * kThreads;
    if constexpr (TB) {
      *j = q / (BK / VEC);
      *kk = (q - *j * (BK / VEC)) * VEC;
    } else {
      *kk = q / (BN / VEC);
      *j = (q - *kk * (BN / VEC)) * VEC;
    }
  };
  T ra[LA][VEC], rb[LB][VEC];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      int i, kk;
      a_coord(e, &i, &kk);
      const int64_t gi = m0 + i, gk = k0 + kk;
      // the VEC elements run along i (TA) or k
      const bool full = TA ? (gk < kend && gi + VEC <= g.M) : (gi < g.M && gk + VEC <= kend);
      const T* src = TA ? A + gk * g.lda + gi : A + gi * g.lda + gk;
      if (full) {
        ldvec<T, VEC>(src, ra[e]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const bool ok = TA ? (gk < kend && gi + v < g.M) : (gi < g.M && gk + v < kend);
          ra[e][v] = ok ? src[v] : (T)0;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      int kk, j;
      b_coord(e, &kk, &j);
      const int64_t gj = n0 + j, gk = k0 + kk;
      const bool full = TB ? (gj < g.N && gk + VEC <= kend) : (gk < kend && gj + VEC <= g.N);
      const T* src = TB ? B + gj * g.ldb + gk : B + gk * g.ldb + gj;
      if (full) {
        ldvec<T, VEC>(src, rb[e]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const bool ok = TB ? (gj < g.N && gk + v < kend) : (gk < kend && gj + v < g.N);
          rb[e][v] = ok ? src[v] : (T)0;
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      int i, kk;
      a_coord(e, &i, &kk);
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        if constexpr (TA)
          As[buf][kk][i + v] = ra[e][v];
        else
          As[buf][kk + v][i] = ra[e][v];
      }
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      int kk, j;
      b_coord(e, &kk, &j);
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        if constexpr (TB)
          Bs[buf][kk + v][j] = rb[e][v];
        else
          Bs[buf][kk][j + v] = rb[e][v];
      }
    }
  };

  Acc acc[IB][JB];
#pragma unroll
  for (int ib = 0; ib < IB; ++ib)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) acc[ib][jb] = Acc{0, 0, 0, 0};

  const int li = lane & 15, lk = lane >> 4;
  int buf = 0;
  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      T av[IB], bv[JB];
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) av[ib] = As[buf][ks + lk][wi + 16 * ib + li];
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) bv[jb] = Bs[buf][ks + lk][wj + 16 * jb + li];
#pragma unroll
      for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) acc[ib][jb] = M::step(av[ib], bv[jb], acc[ib][jb]);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue
  T* P = (T*)g.P;
  T* C = (T*)g.C;
  const T alpha = (T)g.alpha, beta = (T)g.beta;
#pragma unroll
  for (int ib = 0; ib < IB; ++ib)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = m0 + wi + 16 * ib + M::row(lane, v);
        const int64_t c = n0 + wj + 16 * jb + li;
        if (r < g.M && c < g.N) {
          const T s = acc[ib][jb][v];
          if (P) {
            P[((int64_t)split * g.M + r) * g.N + c] = s;
          } else {
            T* cp = C + r * g.ldc + c;
            *cp = beta == (T)0 ? alpha * s : alpha * s + beta * *cp;
          }
        }
      }
}

// C = alpha * (sum over splits of P, in split order) + beta * C.
template <typename T>
__global__ void gemm_splits_kernel(const T* __restrict__ P, int splits, int64_t M, int64_t N, double alpha,
                                   double beta, T* __restrict__ C, int64_t ldc) {
  const int64_t total = M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / N, c = idx - r * N;
    T s = 0;
    for (int q = 0; q < splits; ++q) s += P[q * total + idx];
    T* cp = C + r * ldc + c;
    *cp = beta == 0.0 ? (T)alpha * s : (T)alpha * s + (T)beta * *cp;
  }
}

// Tile shape per type: FP32 128 x 128 x 32 (4-element loads), FP64
// 64 x 64 x 16 (2-element loads): measured against 128 x 128 x 16 (340+
// registers, one wave a SIMD) on the RSVD of 65536 x 16384 with k = 512, the
// Cholesky QR of the sketch takes 8.1 ms against 8.6.
template <typename T>
struct Tile;
template <>
struct Tile<float> {
  static constexpr int BM = 128, BN = 128, BK = 32, VEC = 4;
};
template <>
struct Tile<double> {
  static constexpr int BM = 64, BN = 64, BK = 16, VEC = 2;
};

template <typename T, bool TA, bool TB>
int launch_t(const GemmArgs& g, dim3 grid, hipStream_t st) {
  constexpr int BM = Tile<T>::BM, BN = Tile<T>::BN, BK = Tile<T>::BK, VEC = Tile<T>::VEC;
  // vector loads need the operands' rows aligned to VEC elements
  const uintptr_t al = VEC * sizeof(T);
  const bool vec = (uintptr_t)g.A % al == 0 && (uintptr_t)g.B % al == 0 && g.lda % VEC == 0 && g.ldb % VEC == 0;
  if (vec)
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, BM, BN, BK, VEC>), grid, dim3(kThreads), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, BM, BN, BK, 1>), grid, dim3(kThreads), 0, st, g);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename T>
int launch_ab(const GemmArgs& g, bool ta, bool tb, dim3 grid, hipStream_t st) {
  if (ta) return tb ? launch_t<T, true, true>(g, grid, st) : launch_t<T, true, false>(g, grid, st);
  return tb ? launch_t<T, false, true>(g, grid, st) : launch_t<T, false, false>(g, grid, st);
}

// Splits of K: enough workgroups to fill the chip twice over when the output
// alone has too few tiles, each split at least 256 deep.
int choose_splits(int64_t tiles, int64_t K, int bk) {
  const int64_t target = 512;
  if (tiles >= target) return 1;
  int64_t s = (target + tiles - 1) / tiles;
  s = std::min<int64_t>(s, std::max<int64_t>(1, K / 256));
  s = std::min<int64_t>(s, 64);
  (void)bk;
  return (int)std::max<int64_t>(1, s);
}

}  // namespace

size_t gemm_workspace(int dtype, int64_t M, int64_t N, int64_t K) {
  const int bm = dtype == SK_F64 ? Tile<double>::BM : Tile<float>::BM;
  const int bn = dtype == SK_F64 ? Tile<double>::BN : Tile<float>::BN;
  const int64_t tiles = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  const int s = choose_splits(tiles, K, 16);
  return s > 1 ? (size_t)s * M * N * (dtype == SK_F64 ? 8 : 4) : 0;
}

int gemm_launch(int dtype, bool transA, bool transB, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
                int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* ws,
                size_t ws_bytes, hipStream_t st) {
  if (M <= 0 || N <= 0) return SK_OK;
  if (dtype != SK_F64 && dtype != SK_F32) {
    set_error("gemm: F64 or F32 operands only");
    return SK_E_NOTSUP;
  }
  const int bm = dtype == SK_F64 ? Tile<double>::BM : Tile<float>::BM;
  const int bn = dtype == SK_F64 ? Tile<double>::BN : Tile<float>::BN;
  const int64_t tm = (M + bm - 1) / bm, tn = (N + bn - 1) / bn;
  if (tm > 65535 || tn > (int64_t)INT32_MAX) {
    set_error("gemm: output too tall for the grid");
    return SK_E_NOTSUP;
  }
  const int splits = K > 0 ? choose_splits(tm * tn, K, 16) : 1;
  GemmArgs g;
  g.M = M;
  g.N = N;
  g.K = std::max<int64_t>(K, 0);
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.alpha = alpha;
  g.beta = beta;
  g.P = nullptr;
  // splits start on a K-step boundary (32 covers both types' steps)
  const int64_t kper = ((g.K + splits - 1) / splits + 31) / 32 * 32;
  g.k_per_split = std::max<int64_t>(kper, 32);
  const int ns = (int)std::max<int64_t>(1, (g.K + g.k_per_split - 1) / g.k_per_split);
  if (ns > 1) {
    const size_t need = (size_t)ns * M * N * (dtype == SK_F64 ? 8 : 4);
    if (!ws || ws_bytes < need) {
      set_error("gemm: split-K workspace too small");
      return SK_E_INVAL;
    }
    g.P = ws;
  }
  const dim3 grid((unsigned)tn, (unsigned)tm, (unsigned)ns);
  int rc = dtype == SK_F64 ? launch_ab<double>(g, transA, transB, grid, st) : launch_ab<float>(g, transA, transB, grid, st);
  if (rc != SK_OK || ns == 1) return rc;
  const int64_t total = M * N;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192));
  if (dtype == SK_F64)
    hipLaunchKernelGGL(gemm_splits_kernel<double>, dim3(blocks), dim3(256), 0, st, (const double*)ws, ns, M, N,
                       alpha, beta, (double*)C, ldc);
  else
    hipLaunchKernelGGL(gemm_splits_kernel<float>, dim3(blocks), dim3(256), 0, st, (const float*)ws, ns, M, N, alpha,
                       beta, (float*)C, ldc);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk

using namespace sk;

extern "C" int sk_gemm_workspace_size(int dtype, int64_t M, int64_t N, int64_t K, size_t* bytes) {
  if (!bytes || (dtype != SK_F64 && dtype != SK_F32) || M < 0 || N < 0 || K < 0) {
    set_error("sk_gemm_workspace_size: invalid argument");
    return SK_E_INVAL;
  }
  *bytes = gemm_workspace(dtype, M, N, K);
  return SK_OK;
}

extern "C" int sk_gemm(int dtype, int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha,
                       const void* A, int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                       void* ws, size_t ws_bytes, void* stream) {
  if ((dtype != SK_F64 && dtype != SK_F32) || M < 0 || N < 0 || K < 0 || !C || (K > 0 && (!A || !B))) {
    set_error("sk_gemm: invalid argument");
    return SK_E_INVAL;
  }
  const int64_t acols = transA ? M : K, bcols = transB ? K : N;
  if ((K > 0 && (lda < std::max<int64_t>(1, acols) || ldb < std::max<int64_t>(1, bcols))) ||
      (M > 0 && ldc < std::max<int64_t>(1, N))) {
    set_error("sk_gemm: leading dimension smaller than the row length");
    return SK_E_INVAL;
  }
  return gemm_launch(dtype, transA != 0, transB != 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes,
                     (hipStream_t)stream);
}
