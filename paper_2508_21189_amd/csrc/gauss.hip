// Gaussian test matrix (Def. 1.4) applied on the left: SA = G A with G d x n,
// iid N(0, 1/d), on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// G is never stored. Entry (j, i) comes from Philox4x32-10 with counter
// (i mod 2^32, i >> 32, j / 2, tag 4): the four words give two uniforms
// u = (52 random bits + 1/2) 2^-52, and the Box-Muller transform (Box &
// Muller, 1958) gives r cos(2 pi u2) for even j and r sin(2 pi u2) for odd j,
// r = sqrt(-2 ln u1); G = z / sqrt(d). One Philox call serves two rows of G.
//
// Blocking (split-K GEMM): a workgroup of 4 waves owns a 64-row slice of G
// (16 rows per wave), a slab of 16*BN columns of A (the whole width when it
// fits, so G is generated once per row slice) and one split of the rows of A.
// Per step of 32 rows of A, the workgroup stages the A tile and generates the
// 64 x 32 G tile in LDS, then each wave runs 8 k-steps x BN MFMA blocks into
// register accumulators. Splits write partials [split][d][m]; a second kernel
// adds them in split order (deterministic). Workgroups that share a split are
// given ids 8 apart so they run on one XCD and read the A tile from its L2.
#include "sk_gauss.hpp"

#include <algorithm>
#include <cmath>

namespace sk {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGMT = 64;  // G rows per workgroup
constexpr int kGKT = 32;  // rows of A per step
constexpr double kTwoPi = 6.283185307179586;

// The two Gaussian entries of pair q (rows 2q, 2q+1) of column i, scaled.
__device__ inline void gauss_pair(uint64_t i, uint32_t q, uint32_t k0, uint32_t k1, double scale, double* z0,
                                  double* z1) {
  const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), q, kTagGauss}, k0, k1);
  const uint64_t x1 = ((uint64_t)w.x << 20) | (w.y >> 12);
  const uint64_t x2 = ((uint64_t)w.z << 20) | (w.w >> 12);
  const double u1 = ((double)x1 + 0.5) * 0x1p-52;
  const double u2 = ((double)x2 + 0.5) * 0x1p-52;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(kTwoPi * u2, &s, &c);
  *z0 = r * c * scale;
  *z1 = r * s * scale;
}

struct GaussArgs {
  const double* A;
  int64_t lda;
  const double* rhs;  // optional extra column m (n doubles), or null
  int64_t n;
  int m_eff;  // m (+1 with rhs)
  int m;
  int64_t d;
  uint32_t k0, k1;
  double scale;
  int row_tiles, col_tiles, splits;
  int64_t rows_per_split;
  double* P;  // [split][d][m_eff]
};

template <int BN>
__global__ void __launch_bounds__(256) gauss_rows_kernel(GaussArgs a) {
  constexpr int NT = 16 * BN;
  constexpr int GS = kGKT + 1;  // G tile row stride (doubles)
  constexpr int AS = NT + 1;    // A tile row stride
  extern __shared__ double lds[];
  double* Gs = lds;              // [kGMT][GS]
  double* As = lds + kGMT * GS;  // [kGKT][AS]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = blockIdx.x, xcd = L & 7, q8 = L >> 3;
  const int rt = q8 % a.row_tiles;
  const int ct = (q8 / a.row_tiles) % a.col_tiles;
  const int split = (q8 / (a.row_tiles * a.col_tiles)) * 8 + xcd;
  if (split >= a.splits) return;

  const int64_t r0 = (int64_t)rt * kGMT;  // first G row of the workgroup
  const int c0 = ct * NT;                 // first column of the slab
  const int64_t i_begin = (int64_t)split * a.rows_per_split;
  const int64_t i_end = min(a.n, i_begin + a.rows_per_split);
  const bool wave_rows = r0 + 16 * wave < a.d;

  v4d acc[BN];
#pragma unroll
  for (int b = 0; b < BN; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int64_t kb = i_begin; kb < i_end; kb += kGKT) {
    // A tile [kGKT][NT] (zeros past the split's rows or the matrix's columns)
    for (int idx = tid; idx < kGKT * NT; idx += 256) {
      const int kr = idx / NT, cc = idx - kr * NT;
      const int64_t i = kb + kr;
      const int c = c0 + cc;
      double v = 0.0;
      if (i < i_end) {
        if (c < a.m)
          v = a.A[i * a.lda + c];
        else if (c < a.m_eff)
          v = a.rhs[i];
      }
      As[kr * AS + cc] = v;
    }
    // G tile [kGMT][kGKT]: 32 row pairs x 32 columns, 4 pairs per thread
    for (int p = tid; p < (kGMT / 2) * kGKT; p += 256) {
      const int qq = p / kGKT, kk = p - qq * kGKT;
      const int64_t i = kb + kk;
      double z0 = 0.0, z1 = 0.0;
      if (i < i_end) gauss_pair((uint64_t)i, (uint32_t)(r0 / 2 + qq), a.k0, a.k1, a.scale, &z0, &z1);
      Gs[(2 * qq) * GS + kk] = z0;
      Gs[(2 * qq + 1) * GS + kk] = z1;
    }
    __syncthreads();
    if (wave_rows) {
      const double* gw = Gs + (16 * wave + (lane & 15)) * GS + (lane >> 4);
      const double* aw = As + (lane >> 4) * AS + (lane & 15);
#pragma unroll
      for (int ks = 0; ks < kGKT / 4; ++ks) {
        const double ga = gw[ks * 4];
#pragma unroll
        for (int b = 0; b < BN; ++b) {
          if (c0 + 16 * b < a.m_eff) {
            const double xb = aw[(ks * 4) * AS + 16 * b];
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga, xb, acc[b], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // v_mfma_f64_16x16x4f64 result layout: lane l, item v holds row 4*v + l/16
  // and column l % 16 of the 16 x 16 block (checked on gfx950)
  if (wave_rows) {
    double* P = a.P + (int64_t)split * a.d * a.m_eff;
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      const int c = c0 + 16 * b + (lane & 15);
      if (c < a.m_eff) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = r0 + 16 * wave + 4 * v + (lane >> 4);
          if (row < a.d) P[row * a.m_eff + c] = acc[b][v];
        }
      }
    }
  }
}

// out[j * ldo + c] (c < m) and rhs_out[j] (c = m) = sum over splits, in order.
__global__ void gauss_reduce_kernel(const double* __restrict__ P, int splits, int64_t d, int m, int m_eff,
                                    double* __restrict__ out, int64_t ldo, double* __restrict__ rhs_out) {
  const int64_t total = d * m_eff;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx / m_eff;
    const int c = (int)(idx - j * m_eff);
    double s = 0;
    for (int w = 0; w < splits; ++w) s += P[(int64_t)w * total + idx];
    if (c < m)
      out[j * ldo + c] = s;
    else
      rhs_out[j] = s;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int gauss_bn(int m_eff) {
  const int blocks = (m_eff + 15) / 16;
  if (blocks <= 1) return 1;
  if (blocks <= 4) return 4;
  if (blocks <= 8) return 8;
  return 13;
}

static void gauss_plan(const sk_sketch* S, int m_eff, int* bn, int* row_tiles, int* col_tiles, int* splits,
                       int64_t* rows_per_split) {
  *bn = gauss_bn(m_eff);
  *row_tiles = (int)((S->d + kGMT - 1) / kGMT);
  *col_tiles = (m_eff + 16 * *bn - 1) / (16 * *bn);
  const int per_split = *row_tiles * *col_tiles;
  // about 2048 workgroups (two per CU, four waves each, over several rounds)
  int sp = std::max(1, 2048 / per_split);
  const int64_t max_sp = std::max<int64_t>(1, (S->n + kGKT * 8 - 1) / (kGKT * 8));
  sp = (int)std::min<int64_t>(sp, max_sp);
  int64_t rps = (S->n + sp - 1) / sp;
  rps = ((rps + kGKT - 1) / kGKT) * kGKT;
  *splits = (int)((S->n + rps - 1) / rps);
  *rows_per_split = rps;
}

size_t gauss_workspace(const sk_sketch* S, int m_eff) {
  int bn, rt, ct, sp;
  int64_t rps;
  gauss_plan(S, m_eff, &bn, &rt, &ct, &sp, &rps);
  return (size_t)sp * S->d * m_eff * sizeof(double);
}

template <int BN>
static int launch_gauss_t(const GaussArgs& a, hipStream_t st, const sk_sketch* S) {
  const size_t lds = (size_t)(kGMT * (kGKT + 1) + kGKT * (16 * BN + 1)) * sizeof(double);
  auto kern = gauss_rows_kernel<BN>;
  SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int64_t grid = (int64_t)((a.splits + 7) / 8) * 8 * a.row_tiles * a.col_tiles;
  {
    KernelTimer timer(S, st);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, st, a);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_gauss_rows(const sk_sketch* S, int64_t m, const double* A, int64_t lda, const double* rhs, double* SA,
                      int64_t ldsa, double* Srhs, void* ws, size_t ws_bytes, hipStream_t st) {
  const int m_eff = (int)m + (rhs ? 1 : 0);
  GaussArgs a;
  int bn;
  gauss_plan(S, m_eff, &bn, &a.row_tiles, &a.col_tiles, &a.splits, &a.rows_per_split);
  if (ws_bytes < (size_t)a.splits * S->d * m_eff * sizeof(double)) {
    set_error("Gaussian sketch: workspace too small");
    return SK_E_INVAL;
  }
  a.A = A;
  a.lda = lda;
  a.rhs = rhs;
  a.n = S->n;
  a.m_eff = m_eff;
  a.m = (int)m;
  a.d = S->d;
  a.k0 = S->k0;
  a.k1 = S->k1;
  a.scale = inv_sqrt_host((double)S->d);
  a.P = (double*)ws;
  int rc;
  switch (bn) {
    case 1: rc = launch_gauss_t<1>(a, st, S); break;
    case 4: rc = launch_gauss_t<4>(a, st, S); break;
    case 8: rc = launch_gauss_t<8>(a, st, S); break;
    default: rc = launch_gauss_t<13>(a, st, S); break;
  }
  if (rc != SK_OK) return rc;
  const int64_t total = S->d * m_eff;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(gauss_reduce_kernel, dim3(blocks), dim3(256), 0, st, (const double*)ws, a.splits, S->d, (int)m,
                     m_eff, SA, ldsa, Srhs);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
