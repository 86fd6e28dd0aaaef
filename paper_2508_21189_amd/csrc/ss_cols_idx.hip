// SparseStack apply, column mode, with bucket-indexed register accumulators:
// Y = A S^T for a wide row-major A (rows x n); Y is rows x d.
//
// Def. 1.5: column i of S carries rho_it / sqrt(zeta) in row t*nb + s_it of
// each block t, so Y[r, t*nb + s] = (1/sqrt(zeta)) * sum_{i: s_it = s}
// rho_it A[r, i].
//
// The row-mode bucket-indexed design (ss_idx.hip) with the roles of rows and
// columns exchanged:
//  * a workgroup owns 64 rows of A (one per lane) and a group of blocks (one
//    wave per block) and sweeps all n columns in tiles of TC columns; each
//    wave keeps the nb accumulators of its block for its 64 rows in the
//    pinned register file and adds column i into the register of bucket
//    s_it (wave-uniform: it depends on the column only) through GPR-index
//    mode, with the sign as a +-1.0 scalar multiplier;
//  * tiles stream into LDS with direct global->LDS dword loads (one 256-byte
//    row segment per load), double buffered; a tile row is padded so that
//    the 64 lanes reading one column hit distinct banks, and the columns of a
//    16-column group sit at immediate offsets;
//  * the codes (bucket register index and sign word of each column and
//    block) come from the row-mode plan kernel over the n columns; every
//    workgroup reads the same codes, so they stay in the caches;
//  * each workgroup sees every column of its rows: the sums run in column
//    order with no partials, so the result is bitwise reproducible.
#include "sk_idx.hpp"
#include "sk_launch.hpp"

#include <algorithm>
#include <cstdlib>

namespace sk {

using namespace idx;

struct ColsIdxArgs {
  const unsigned char* A;
  int64_t lda_bytes;
  int64_t rows, n;
  int zeta, nb, TC;
  int TSB;        // LDS bytes of a tile row
  int buf_bytes;  // LDS bytes of one tile buffer (64 rows)
  int bpg, n_groups;
  int64_t n_tiles;
  void* Y;
  int64_t ldy;
  int out_f64;
  float scale_f;
  double scale_d;
};

// One tile row of SEGS 256-byte segments: SEGS dword loads (64 lanes each)
// from gsrc (this lane's first dword) into LDS at M0 = lds_addr; the
// instruction offset moves the global and the LDS address alike.
template <int SEGS>
__device__ inline void dma_row(const void* gsrc, uint32_t lds_addr) {
  uint32_t saved;
  if constexpr (SEGS == 2)
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %1\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dword %2, off\n\t"
        "global_load_lds_dword %2, off offset:256\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "s"(lds_addr), "v"(gsrc)
        : "memory");
  else
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %1\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dword %2, off\n\t"
        "global_load_lds_dword %2, off offset:256\n\t"
        "global_load_lds_dword %2, off offset:512\n\t"
        "global_load_lds_dword %2, off offset:768\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "s"(lds_addr), "v"(gsrc)
        : "memory");
}

// TC = SEGS * 256 / sizeof(Tin) columns a tile.
template <typename Tin, int NREG, int SEGS>
__global__ void __launch_bounds__(512) ss_cols_idx_kernel(ColsIdxArgs a, const uint32_t* __restrict__ codes_all) {
  using T = IdxT<Tin>;
  using Tacc = typename T::acc;
  constexpr int ES = sizeof(Tin);
  constexpr int GR = 16;  // columns whose codes one scalar group holds
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nwaves = blockDim.x >> 6;
  const int L = blockIdx.x;
  const int group = L % a.n_groups;
  const int64_t r0 = (int64_t)(L / a.n_groups) * 64;
  const int t0 = group * a.bpg;
  const int bpg = min(a.bpg, a.zeta - t0);
  const bool walker = wave < bpg;
  const int nrows = (int)min((int64_t)64, a.rows - r0);

  AccFile f;
  acc_zero<NREG>(f);

  // Tile st into buffer buf: row rr's bytes [c0 ES, c0 ES + tbytes) of A at
  // rr * TSB, one row per wave at a time. A full tile row is SEGS whole
  // segments; the last tile (tbytes a multiple of 4) loads each segment's
  // dwords below tbytes.
  auto issue = [&](int64_t st, int buf) {
    const int64_t c0 = st * a.TC;
    const int tbytes = (int)(min((int64_t)a.TC, a.n - c0) * ES);
    unsigned char* dst = smem + buf * a.buf_bytes;
    const unsigned char* src = a.A + r0 * a.lda_bytes + c0 * ES + lane * 4;
    const bool whole = tbytes == SEGS * 256;
    for (int rr = wave; rr < nrows; rr += nwaves) {
      const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane((int)idx_lds_addr(dst + rr * a.TSB));
      const unsigned char* g = src + rr * a.lda_bytes;
      if (whole) {
        dma_row<SEGS>(g, la);
      } else {
#pragma unroll
        for (int sg = 0; sg < SEGS; ++sg)
          if (sg * 256 + lane * 4 < tbytes) idx_dma4(g + sg * 256, la + sg * 256);
      }
    }
  };

  if (a.n_tiles > 0) issue(0, 0);
  for (int64_t st = 0; st < a.n_tiles; ++st) {
    const int buf = (int)(st & 1);
    idx_wait_vm(0);
    idx_barrier();  // tile st is in LDS; everyone finished tile st - 1
    if (st + 1 < a.n_tiles) issue(st + 1, buf ^ 1);
    if (walker) {
      const int tcv = (int)min((int64_t)a.TC, a.n - st * a.TC);
      // this wave's codes for the tile (uniform address: scalar loads)
      const uint32_t* codes = codes_all + (st * a.zeta + t0 + wave) * (int64_t)(2 * a.TC);
      const uint32_t tbase = idx_lds_addr(smem + buf * a.buf_bytes) + (uint32_t)(lane * a.TSB);
      const int full = tcv & ~(GR - 1);
      for (int g = 0; g < full; g += GR) {
        uint32_t w[GR], h[GR];
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          w[u] = codes[g + u];
          h[u] = codes[a.TC + g + u];
        }
        uint32_t cb = tbase + (uint32_t)(g * ES);
        asm volatile("" : "+v"(cb));
        Tacc v[4], vn[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = idx_val<Tin>(cb + (uint32_t)(u * ES));
#pragma unroll
        for (int k = 0; k < GR; k += 4) {
          if (k + 4 < GR) {
#pragma unroll
            for (int u = 0; u < 4; ++u) vn[u] = idx_val<Tin>(cb + (uint32_t)((k + 4 + u) * ES));
          }
          fma4<NREG>(f, v[0], v[1], v[2], v[3], w[k], w[k + 1], w[k + 2], w[k + 3], idx_pm(h[k], (Tacc*)nullptr),
                     idx_pm(h[k + 1], (Tacc*)nullptr), idx_pm(h[k + 2], (Tacc*)nullptr),
                     idx_pm(h[k + 3], (Tacc*)nullptr));
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = vn[u];
        }
      }
      // the last columns of A (a tile shorter than a multiple of GR)
      for (int c = full; c < tcv; ++c) {
        const uint32_t wc = codes[c], hc = codes[a.TC + c];
        const Tacc v0 = idx_val<Tin>(tbase + (uint32_t)(c * ES));
        fma1<NREG>(f, v0, wc, idx_pm(hc, (Tacc*)nullptr));
      }
    }
  }

  if (walker && lane < nrows) {
    const int64_t base = (r0 + lane) * a.ldy + (int64_t)(t0 + wave) * a.nb;
#pragma unroll
    for (int s = 0; s < NREG / T::rpa; ++s) {
      if (s < a.nb) {
        Tacc val;
        if constexpr (T::rpa == 2) {
          const uint64_t lo = acc_get<NREG>(f, 2 * s), hi = acc_get<NREG>(f, 2 * s + 1);
          val = __builtin_bit_cast(double, lo | (hi << 32));
        } else {
          val = __builtin_bit_cast(float, acc_get<NREG>(f, s));
        }
        if (a.out_f64)
          ((double*)a.Y)[base + s] = (double)val * a.scale_d;
        else
          ((float*)a.Y)[base + s] = (float)(val * (Tacc)(sizeof(Tacc) == 8 ? a.scale_d : a.scale_f));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {
size_t c16(size_t x) { return (x + 15) & ~(size_t)15; }

// Register file for nb accumulators (FP64: two registers each), 0 if none fits.
int cidx_nreg(int dtype_in, int64_t nb) {
  const int64_t regs = nb * (dtype_in == SK_F64 ? 2 : 1);
  if (regs <= 32) return 32;
  if (regs <= 64) return 64;
  if (regs <= 128) return 128;
  if (regs <= 200) return 200;
  return 0;
}
// Waves of that kernel a SIMD holds (the file plus about 40 other registers
// of the 512 a SIMD lane has).
int cidx_waves_per_simd(int nreg) { return nreg <= 32 ? 7 : (nreg <= 64 ? 4 : (nreg <= 128 ? 3 : 2)); }

struct ColsIdxPlan {
  int nreg, bpg, n_groups, segs, TC, TSB, buf_bytes;
  int64_t n_tiles;
  size_t lds, codes_bytes;
};

// LDS bytes of a tile row of 256 * segs bytes: padded so that 64 lanes
// reading the same column (one row each) fall on distinct banks (an odd
// number of 4-byte words, or of 8-byte words for FP64).
int row_bytes(int dtype_in, int segs) { return 256 * segs + (dtype_in == SK_F64 ? 8 : 4); }

int cols_idx_plan(const sk_sketch* S, int dtype_in, ColsIdxPlan* p) {
  p->nreg = cidx_nreg(dtype_in, S->nb);
  if (p->nreg == 0) return SK_E_NOTSUP;
  const int wps = cidx_waves_per_simd(p->nreg);
  p->bpg = std::min(S->zeta, 8);
  p->n_groups = (S->zeta + p->bpg - 1) / p->bpg;
  const int wg_per_cu = std::max(1, std::min(2, (4 * wps) / p->bpg));
  const size_t cap = (size_t)160 * 1024 / wg_per_cu;
  // four segments a row (FP64, 128 columns) where two buffers fit, else two
  p->segs = (dtype_in == SK_F64 && p->nreg >= 128 && 2 * c16((size_t)64 * row_bytes(dtype_in, 4)) <= cap) ? 4 : 2;
  const int TC = p->segs * 256 / (int)dtype_size(dtype_in);
  p->TC = TC;
  p->TSB = row_bytes(dtype_in, p->segs);
  p->buf_bytes = (int)c16((size_t)64 * p->TSB);
  p->lds = 2 * (size_t)p->buf_bytes;
  p->n_tiles = (S->n + TC - 1) / TC;
  p->codes_bytes = c16((size_t)p->n_tiles * S->zeta * 2 * TC * 4);
  return SK_OK;
}

template <typename Tin, int NREG, int SEGS>
int launch_cidx_t(const sk_sketch* S, const ColsIdxPlan& p, int64_t rows, const void* A, int64_t lda, void* Y,
                  int64_t ldy, int out_f64, const uint32_t* codes, hipStream_t st) {
  ColsIdxArgs a;
  a.A = (const unsigned char*)A;
  a.lda_bytes = lda * (int64_t)sizeof(Tin);
  a.rows = rows;
  a.n = S->n;
  a.zeta = S->zeta;
  a.nb = (int)S->nb;
  a.TC = p.TC;
  a.TSB = p.TSB;
  a.buf_bytes = p.buf_bytes;
  a.bpg = p.bpg;
  a.n_groups = p.n_groups;
  a.n_tiles = p.n_tiles;
  a.Y = Y;
  a.ldy = ldy;
  a.out_f64 = out_f64;
  a.scale_d = inv_sqrt_host((double)S->zeta);
  a.scale_f = (float)a.scale_d;
  const int64_t grid = ((rows + 63) / 64) * p.n_groups;
  auto kern = ss_cols_idx_kernel<Tin, NREG, SEGS>;
  SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds));
  {
    KernelTimer timer(S, st);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * p.bpg), p.lds, st, a, codes);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename Tin>
int launch_cidx_n(const sk_sketch* S, const ColsIdxPlan& p, int64_t rows, const void* A, int64_t lda, void* Y,
                  int64_t ldy, int out_f64, const uint32_t* codes, hipStream_t st) {
  if (sizeof(Tin) == 8 && p.segs == 4) {
    if (p.nreg == 128) return launch_cidx_t<Tin, 128, 4>(S, p, rows, A, lda, Y, ldy, out_f64, codes, st);
    if (p.nreg == 200) return launch_cidx_t<Tin, 200, 4>(S, p, rows, A, lda, Y, ldy, out_f64, codes, st);
  }
  switch (p.nreg) {
    case 32:
      return launch_cidx_t<Tin, 32, 2>(S, p, rows, A, lda, Y, ldy, out_f64, codes, st);
    case 64:
      return launch_cidx_t<Tin, 64, 2>(S, p, rows, A, lda, Y, ldy, out_f64, codes, st);
    case 128:
      return launch_cidx_t<Tin, 128, 2>(S, p, rows, A, lda, Y, ldy, out_f64, codes, st);
    default:
      return launch_cidx_t<Tin, 200, 2>(S, p, rows, A, lda, Y, ldy, out_f64, codes, st);
  }
}
}  // namespace

// Whether the bucket-indexed column kernel takes this call: FP64 or FP32
// input, a block's accumulators fit one register file, rows of A are 4-byte
// aligned and each row's n elements end on a 4-byte boundary (whole dword
// loads). BF16 input is switched off: its first run at 65536 x 16384 (d =
// 512, zeta = 8) ended in a GPU memory fault whose cause has not been found
// (small BF16 cases matched the oracle); it keeps the sorted-list kernel.
bool cols_idx_fits(const sk_sketch* S, int dtype_in, const void* A, int64_t lda) {
  const char* e = std::getenv("SKETCH_COLS_IDX");
  if (e && std::atoi(e) == 0) return false;
  if (dtype_in == SK_BF16) return false;
  if (cidx_nreg(dtype_in, S->nb) == 0 || S->n < 1) return false;
  const int64_t es = (int64_t)dtype_size(dtype_in);
  if (!A) return true;  // workspace queries
  return (uintptr_t)A % 4 == 0 && (lda * es) % 4 == 0 && (S->n * es) % 4 == 0;
}

size_t cols_idx_workspace(const sk_sketch* S, int dtype_in) {
  ColsIdxPlan p;
  return cols_idx_plan(S, dtype_in, &p) == SK_OK ? p.codes_bytes : 0;
}

int launch_cols_idx(const sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                    int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st) {
  ColsIdxPlan p;
  if (cols_idx_plan(S, dtype_in, &p) != SK_OK) {
    set_error("sketch_apply_T: bucket register file too small for this block size");
    return SK_E_NOTSUP;
  }
  if (ws_bytes < p.codes_bytes) {
    set_error("sketch_apply_T: workspace too small (see sketch_workspace_size)");
    return SK_E_INVAL;
  }
  uint32_t* codes = (uint32_t*)ws;
  int rc = launch_idx_codes(S, dtype_in, p.n_tiles, p.TC, codes, st);
  if (rc != SK_OK) return rc;
  if (rows == 0) return SK_OK;
  const int of64 = dtype_out == SK_F64;
  if (dtype_in == SK_F64) return launch_cidx_n<double>(S, p, rows, A, lda, Y, ldy, of64, codes, st);
  if (dtype_in == SK_F32) return launch_cidx_n<float>(S, p, rows, A, lda, Y, ldy, of64, codes, st);
  return launch_cidx_n<uint16_t>(S, p, rows, A, lda, Y, ldy, of64, codes, st);
}

}  // namespace sk
