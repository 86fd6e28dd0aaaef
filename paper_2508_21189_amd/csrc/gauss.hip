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
// (16 rows per wave), a slab of 16*BN columns of A and one split of the rows
// of A. Per step of 16 rows of A:
//   * the A tile of the next step goes straight from global memory into the
//     other half of a double-buffered LDS tile (global_load_lds, 16 bytes a
//     lane when the rows are 16-byte aligned, else 4), and the columns that
//     are not plain A (a half-filled pair, the right-hand side, zeros) are
//     written by a few lanes;
//   * each wave runs 4 k-steps x BN MFMA blocks on the current tile, with its
//     G operands already in registers, and generates the G operands of the
//     next step in the same stretch of code, so that the generation's vector
//     instructions issue while the matrix cores work. A lane's MFMA operand
//     is G[row 16w + l%16][column 4 ks + l/16]; rows 2q and 2q+1 come from
//     one Box-Muller pair, which lanes l and l^1 share: each lane computes
//     two pairs (k-steps 0,1 on even rows, 2,3 on odd rows) and the two lanes
//     trade the halves they do not use (one DPP move);
//   * one barrier hands the tile buffers over.
// Splits write partials [split][d][m]; a second kernel adds them in split
// order (deterministic). Workgroups that share a split are given ids 8 apart
// so they run on one XCD and read the A tile from its L2.
#include "sk_gauss.hpp"

#include <algorithm>
#include <cmath>

namespace sk {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGMT = 64;  // G rows per workgroup
constexpr int kGKT = 16;  // rows of A per step

// The two Gaussian entries of pair q (rows 2q, 2q+1) of column i, scaled.
__device__ inline void gauss_pair(uint64_t i, uint32_t q, uint32_t k0, uint32_t k1, double scale, double* z0,
                                  double* z1) {
  const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), q, kTagGauss}, k0, k1);
  const uint64_t x1 = ((uint64_t)w.x << 20) | (w.y >> 12);
  const uint64_t x2 = ((uint64_t)w.z << 20) | (w.w >> 12);
  const double u1 = ((double)x1 + 0.5) * 0x1p-52;
  const double u2 = ((double)x2 + 0.5) * 0x1p-52;
  const double r = sqrt(-2.0 * log(u1));
  // cos and sin of 2 pi u2 by the half-turn forms: 2 u2 is exact and needs
  // no large-argument reduction
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  *z0 = r * c * scale;
  *z1 = r * s * scale;
}

// x of lane l ^ 1 (DPP quad permutation 1, 0, 3, 2; all lanes active).
__device__ inline double from_pair_lane(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0xB1, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The wave's G operands of the step at kb: g[ks] = G[row][kb + 4 ks + kq]
// with row = 2 q + parity, zero for columns at or past i_end.
__device__ inline void gauss_operands(int64_t kb, int64_t i_end, uint32_t q, int parity, int kq, uint32_t k0,
                                      uint32_t k1, double scale, double g[4]) {
  const int64_t ia = kb + 8 * parity + kq;  // k-step 2 parity
  const int64_t ib = ia + 4;                // k-step 2 parity + 1
  double a0, a1, b0, b1;
  gauss_pair((uint64_t)ia, q, k0, k1, scale, &a0, &a1);
  gauss_pair((uint64_t)ib, q, k0, k1, scale, &b0, &b1);
  if (ia >= i_end) a0 = a1 = 0.0;
  if (ib >= i_end) b0 = b1 = 0.0;
  const double own_a = parity ? a1 : a0, send_a = parity ? a0 : a1;
  const double own_b = parity ? b1 : b0, send_b = parity ? b0 : b1;
  const double recv_a = from_pair_lane(send_a), recv_b = from_pair_lane(send_b);
  g[0] = parity ? recv_a : own_a;
  g[1] = parity ? recv_b : own_b;
  g[2] = parity ? own_a : recv_a;
  g[3] = parity ? own_b : recv_b;
}

// Direct global->LDS loads: lane l's bytes land at LDS address M0 + l * width
// (inactive lanes leave their slot untouched). Issued from inline assembly so
// that the compiler's memory-counter bookkeeping does not make the MFMA
// operand reads of the other buffer wait for them; the kernel waits for them
// explicitly before the barrier that publishes the tile. M0 is saved and
// restored around the load, with the one wait state the ISA asks for between
// a scalar write of M0 and an LDS-DMA load.
__device__ inline void g_dma16(const void* gsrc, uint32_t lds_addr) {
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(lds_addr), "v"(gsrc)
      : "memory");
}
__device__ inline void g_dma4(const void* gsrc, uint32_t lds_addr) {
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dword %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(lds_addr), "v"(gsrc)
      : "memory");
}
__device__ inline void g_wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

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
  int vec16;  // A rows 16-byte aligned (lda even, A aligned)
  double* P;  // [split][d][m_eff]
};

template <int BN>
__global__ void __launch_bounds__(256, 2) gauss_rows_kernel(GaussArgs a) {
  constexpr int NT = 16 * BN;     // tile columns (row stride of the LDS tile)
  constexpr int TILE = kGKT * NT;  // doubles per tile buffer
  extern __shared__ __attribute__((aligned(16))) double lds[];  // [2][kGKT][NT]

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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
  const int rho = lane & 15, kq = lane >> 4, parity = rho & 1;
  const uint32_t q = (uint32_t)(r0 / 2 + 8 * wave + (rho >> 1));

  // Columns of the slab: [0, acols) are A; the DMA covers [0, dcols) (dcols
  // even on the 16-byte path); tail columns dcols, dcols + 1 hold A, the
  // right-hand side (column m) or zero; later columns stay zero.
  const int acols = max(0, min(NT, a.m - c0));
  const int dcols = a.vec16 ? (acols & ~1) : acols;
  const int rhs_col = (a.rhs && a.m >= c0 && a.m < c0 + NT) ? a.m - c0 : -1;
  const bool tail_lane = wave == 3 && lane < kGKT && dcols < NT && (dcols < acols || rhs_col >= 0);
  const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void*)lds;

  // both buffers start zero (columns past the data are never written)
  for (int idx = tid; idx < TILE; idx += 256) reinterpret_cast<double2*>(lds)[idx] = double2{0.0, 0.0};
  __syncthreads();

  double t0 = 0.0, t1 = 0.0;  // tail values of row `lane` of the tile in flight
  // Issues the loads of the tile at kb into buffer bsel.
  auto issue = [&](int64_t kb, int bsel) {
    const int rows = (int)min<int64_t>(kGKT, i_end - kb);
    double* buf = lds + bsel * TILE;
    if (rows < kGKT) {
      // last step of the matrix: rows past its end are zero
      for (int idx = tid; idx < (kGKT - rows) * NT; idx += 256) buf[rows * NT + idx] = 0.0;
    }
    const uint32_t base = lds0 + (uint32_t)(bsel * TILE * 8);
    if (a.vec16) {
      constexpr int NP = NT / 2;
      constexpr int NI = (kGKT * NP + 63) / 64;
      for (int t = wave; t < NI; t += 4) {
        const int idx = 64 * t + lane;
        const int r = idx / NP, cj = idx - r * NP;
        const uint32_t dst = __builtin_amdgcn_readfirstlane(base + (uint32_t)(t * 1024));
        if (r < rows && 2 * cj < dcols) g_dma16(a.A + (kb + r) * a.lda + c0 + 2 * cj, dst);
      }
    } else {
      constexpr int NW = 2 * NT;  // dwords per tile row
      constexpr int NI = (kGKT * NW + 63) / 64;
      for (int t = wave; t < NI; t += 4) {
        const int idx = 64 * t + lane;
        const int r = idx / NW, dw = idx - r * NW;
        const uint32_t dst = __builtin_amdgcn_readfirstlane(base + (uint32_t)(t * 256));
        if (r < rows && (dw >> 1) < dcols)
          g_dma4(reinterpret_cast<const char*>(a.A + (kb + r) * a.lda + c0 + (dw >> 1)) + 4 * (dw & 1), dst);
      }
    }
    if (tail_lane) {
      t0 = t1 = 0.0;
      if (lane < rows) {
        const int64_t i = kb + lane;
        if (dcols < acols)
          t0 = a.A[i * a.lda + c0 + dcols];
        else if (rhs_col == dcols)
          t0 = a.rhs[i];
        if (dcols + 1 < acols)
          t1 = a.A[i * a.lda + c0 + dcols + 1];
        else if (rhs_col == dcols + 1)
          t1 = a.rhs[i];
      }
    }
  };
  // Completes the tile in buffer bsel and publishes it.
  auto finish = [&](int bsel) {
    if (tail_lane) {
      double* row = lds + bsel * TILE + lane * NT;
      row[dcols] = t0;
      if (dcols + 1 < NT) row[dcols + 1] = t1;
    }
    g_wait_dma();
    __syncthreads();
  };

  v4d acc[BN];
#pragma unroll
  for (int b = 0; b < BN; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
  double g[4] = {0.0, 0.0, 0.0, 0.0};

  if (i_begin < i_end) {
    issue(i_begin, 0);
    if (wave_rows) gauss_operands(i_begin, i_end, q, parity, kq, a.k0, a.k1, a.scale, g);
    finish(0);
  }
  int cur = 0;
  for (int64_t kb = i_begin; kb < i_end; kb += kGKT) {
    const int64_t kn = kb + kGKT;
    const bool more = kn < i_end;
    if (more) issue(kn, cur ^ 1);
    if (wave_rows) {
      const double* aw = lds + cur * TILE + kq * NT + rho;
#pragma unroll
      for (int ks = 0; ks < kGKT / 4; ++ks) {
#pragma unroll
        for (int b = 0; b < BN; ++b)
          acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[ks], aw[4 * ks * NT + 16 * b], acc[b], 0, 0, 0);
      }
      double gn[4];
      gauss_operands(kn, i_end, q, parity, kq, a.k0, a.k1, a.scale, gn);
#pragma unroll
      for (int j = 0; j < 4; ++j) g[j] = gn[j];
    }
    if (more) finish(cur ^ 1);
    cur ^= 1;
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
// Column blocks per workgroup: the instantiated width that needs the fewest
// MFMA blocks in all, counting each extra column slab as two blocks (its G
// operands are generated again).
static int gauss_bn(int m_eff) {
  const int blocks = (m_eff + 15) / 16;
  static const int widths[] = {1, 2, 4, 8, 13};
  int best = 13;
  int64_t best_cost = -1;
  for (int bn : widths) {
    const int64_t slabs = (blocks + bn - 1) / bn;
    const int64_t cost = slabs * (bn + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = bn;
    }
  }
  return best;
}

static void gauss_plan(const sk_sketch* S, int m_eff, int* bn, int* row_tiles, int* col_tiles, int* splits,
                       int64_t* rows_per_split) {
  *bn = gauss_bn(m_eff);
  *row_tiles = (int)((S->d + kGMT - 1) / kGMT);
  *col_tiles = (m_eff + 16 * *bn - 1) / (16 * *bn);
  const int per_split = *row_tiles * *col_tiles;
  // Workgroups of split s run on XCD s mod 8, two per CU (LDS and registers
  // allow two), 64 per XCD at a time. Take the number of splits per XCD that
  // fills four such rounds best, so no XCD is left with a short extra round.
  int per_xcd = std::max(1, (4 * 64) / per_split);
  int sp = 8 * per_xcd;
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
  const size_t lds = (size_t)2 * kGKT * 16 * BN * sizeof(double);
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
  a.vec16 = (lda % 2 == 0) && ((uintptr_t)A % 16 == 0);
  int rc;
  switch (bn) {
    case 1: rc = launch_gauss_t<1>(a, st, S); break;
    case 2: rc = launch_gauss_t<2>(a, st, S); break;
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
