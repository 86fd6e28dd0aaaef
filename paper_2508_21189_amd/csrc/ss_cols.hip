// SparseStack apply, column mode: Y = A S^T (the paper's A Omega) for a wide
// row-major A (rows x n); Y is rows x d.
//
// Y[r, t*nb + s] = (1/sqrt(zeta)) * sum_{i: s_it = s} rho_it A[r, i].
//
// Here the sketched dimension (the columns of A) is contiguous in memory, so
// lanes take rows: a workgroup owns 64 rows of A (one per lane) and sweeps
// their columns in tiles of TC columns. The bucket plans are the row-mode
// plans with the roles of rows and columns exchanged (per tile of columns and
// block: bucket offsets and the columns sorted by bucket), built once per
// call by the plan kernel. Each wave owns one block and a contiguous range of
// its buckets, with one register accumulator per bucket per lane; every list
// entry is a uniform column index, so each read is one conflict-free LDS
// access (tile rows are padded by one element). No partial sums are needed:
// each workgroup sees all columns of its rows, and sums run in list order.
#include "sk_launch.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

namespace sk {

struct ColsArgs {
  const unsigned char* A;
  int64_t lda_bytes;
  int64_t rows, n, d;
  int zeta, nb, TC, bpg, n_groups, H, per_range;
  const unsigned char* plan;
  int rec_bytes, lst_off;
  int64_t n_tiles;
  void* Y;
  int64_t ldy;
  int out_f64;
  float scale_f;
  double scale_d;
  int nu;  // branch-free passes of the prefetching kernel (1 .. 8)
};

template <typename Tin>
struct ColsAcc {
  using type = float;
};
template <>
struct ColsAcc<double> {
  using type = double;
};

template <typename Tin>
__device__ inline typename ColsAcc<Tin>::type cols_load(const unsigned char* p);
template <>
__device__ inline double cols_load<double>(const unsigned char* p) {
  return *(const double*)p;
}
template <>
__device__ inline float cols_load<float>(const unsigned char* p) {
  return *(const float*)p;
}
template <>
__device__ inline float cols_load<uint16_t>(const unsigned char* p) {
  return bf16_to_f32(*(const uint16_t*)p);
}

__device__ inline double flip_c(double v, uint32_t e) {
  return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)(e & 0x80000000u) << 32));
}
__device__ inline float flip_c(float v, uint32_t e) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ (e & 0x80000000u));
}

template <typename Tin, int JB>
__global__ void __launch_bounds__(1024) ss_cols_kernel(ColsArgs a) {
  using Tacc = typename ColsAcc<Tin>::type;
  constexpr int ES = sizeof(Tin);
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int TS = a.TC + 1;  // LDS row stride (elements of Tacc)
  Tacc* T = (Tacc*)smem;    // [64][TS]
  unsigned char* pl = smem + (((size_t)64 * TS * sizeof(Tacc) + 15) & ~(size_t)15);

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x;
  const int L = blockIdx.x;
  const int group = L % a.n_groups;
  const int64_t r0 = (int64_t)(L / a.n_groups) * 64;
  const int t0 = group * a.bpg;
  const int bpg = min(a.bpg, a.zeta - t0);
  const int tl = wave / a.H, hr = wave - (wave / a.H) * a.H;
  const bool walker = tl < bpg;
  const int s_begin = hr * a.per_range;
  const int s_cnt = walker ? max(0, min(a.per_range, a.nb - s_begin)) : 0;
  const int64_t nrows = min((int64_t)64, a.rows - r0);

  Tacc acc[JB];
#pragma unroll
  for (int j = 0; j < JB; ++j) acc[j] = 0;

  for (int64_t tile = 0; tile < a.n_tiles; ++tile) {
    const int64_t c0 = tile * a.TC;
    const int tcv = (int)min((int64_t)a.TC, a.n - c0);
    __syncthreads();  // previous tile fully consumed
    for (int idx = tid; idx < 64 * a.TC; idx += nthreads) {
      const int rr = idx / a.TC, cc = idx - rr * a.TC;
      Tacc v = 0;
      if (rr < nrows && cc < tcv) v = cols_load<Tin>(a.A + (r0 + rr) * a.lda_bytes + (c0 + cc) * ES);
      T[rr * TS + cc] = v;
    }
    const uint4* src = (const uint4*)(a.plan + (tile * a.zeta + t0) * (int64_t)a.rec_bytes);
    uint4* dst = (uint4*)pl;
    for (int idx = tid; idx < bpg * a.rec_bytes / 16; idx += nthreads) dst[idx] = src[idx];
    __syncthreads();
    if (walker) {
      const unsigned char* rec = pl + tl * a.rec_bytes;
      const uint16_t* of = (const uint16_t*)rec;
      const uint32_t* lst = (const uint32_t*)(rec + a.lst_off);
      const Tacc* Tl = T + lane * TS;
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        if (j < s_cnt) {
          const int kb = __builtin_amdgcn_readfirstlane((int)of[s_begin + j]);
          const int ke = __builtin_amdgcn_readfirstlane((int)of[s_begin + j + 1]);
          int k = kb;
          for (; k + 1 < ke; k += 2) {
            const uint32_t ea = lst[k], eb = lst[k + 1];
            const Tacc va = Tl[ea & 0x7fffffffu], vb = Tl[eb & 0x7fffffffu];
            acc[j] += flip_c(va, ea);
            acc[j] += flip_c(vb, eb);
          }
          if (k < ke) {
            const uint32_t ea = lst[k];
            acc[j] += flip_c(Tl[ea & 0x7fffffffu], ea);
          }
        }
      }
    }
  }

  if (walker && lane < nrows) {
    const int64_t col0 = (int64_t)(t0 + tl) * a.nb + s_begin;
    if (a.out_f64) {
      double* Y = (double*)a.Y + (r0 + lane) * a.ldy + col0;
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < s_cnt) Y[j] = (double)acc[j] * a.scale_d;
    } else {
      float* Y = (float*)a.Y + (r0 + lane) * a.ldy + col0;
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < s_cnt) Y[j] = (float)(acc[j] * (Tacc)(sizeof(Tacc) == 8 ? a.scale_d : a.scale_f));
    }
  }
}

// The same walk with the tile loads taken off the critical path: each thread
// fetches its 16-byte chunks of the next tile (and of its plan records) into
// registers before walking the current tile, and stores them to LDS after
// the walk. Needs 16-byte aligned rows and n * element size a multiple of 16
// (a chunk never straddles the end of a row). 8 waves (at most 8 walkers);
// waves past the walkers only load.
template <typename Tin, int JB>
__global__ void __launch_bounds__(512) ss_cols_vec_kernel(ColsArgs a) {
  using Tacc = typename ColsAcc<Tin>::type;
  constexpr int ES = sizeof(Tin);
  constexpr int VPL = 16 / ES;  // values per 16-byte chunk
  constexpr int NCH = 8;        // chunks per thread (tile <= 64 KB, >= 512 threads)
  constexpr int NPL = 2;        // plan chunks per thread
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int TS = a.TC + 1;
  Tacc* T = (Tacc*)smem;  // [64][TS]
  unsigned char* pl = smem + (((size_t)64 * TS * sizeof(Tacc) + 15) & ~(size_t)15);

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x;
  const int L = blockIdx.x;
  const int group = L % a.n_groups;
  const int64_t r0 = (int64_t)(L / a.n_groups) * 64;
  const int t0 = group * a.bpg;
  const int bpg = min(a.bpg, a.zeta - t0);
  const int tl = wave / a.H, hr = wave - (wave / a.H) * a.H;
  const bool walker = tl < bpg;
  const int s_begin = hr * a.per_range;
  const int s_cnt = walker ? max(0, min(a.per_range, a.nb - s_begin)) : 0;
  const int64_t nrows = min((int64_t)64, a.rows - r0);
  const int cpr = a.TC / VPL;       // chunks per tile row
  const int nchunks = 64 * cpr;     // chunks per tile
  const int pchunks = bpg * a.rec_bytes / 16;

  uint4 ra[NCH], rp[NPL];
  uint32_t valid = 0;
  auto fetch = [&](int64_t tile) {
    const int64_t c0 = tile * a.TC;
    valid = 0;
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
      const int f = tid + u * nthreads;
      const int rr = f / cpr, cq = f - (f / cpr) * cpr;
      const int64_t col = c0 + (int64_t)cq * VPL;
      const bool ok = f < nchunks && rr < nrows && col < a.n;
      const unsigned char* src = ok ? a.A + (r0 + rr) * a.lda_bytes + col * ES : a.A;
      ra[u] = *(const uint4*)src;
      valid |= (uint32_t)ok << u;
    }
    const uint4* ps = (const uint4*)(a.plan + (tile * a.zeta + t0) * (int64_t)a.rec_bytes);
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
      const int f = tid + u * nthreads;
      rp[u] = f < pchunks ? ps[f] : uint4{0, 0, 0, 0};
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
      const int f = tid + u * nthreads;
      if (f < nchunks) {
        const int rr = f / cpr, cq = f - (f / cpr) * cpr;
        const bool ok = (valid >> u) & 1u;
        const Tin* v = (const Tin*)&ra[u];
        Tacc* dst = T + rr * TS + cq * VPL;
#pragma unroll
        for (int q = 0; q < VPL; ++q) {
          Tacc x;
          if constexpr (sizeof(Tin) == 2)
            x = bf16_to_f32(v[q]);
          else
            x = (Tacc)v[q];
          dst[q] = ok ? x : (Tacc)0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
      const int f = tid + u * nthreads;
      if (f < pchunks) ((uint4*)pl)[f] = rp[u];
    }
  };

  Tacc acc[JB];
#pragma unroll
  for (int j = 0; j < JB; ++j) acc[j] = 0;

  // the pad column TC of every tile row stays zero (absent list slots read it)
  for (int rr = tid; rr < 64; rr += nthreads) T[rr * TS + a.TC] = (Tacc)0;
  if (a.n_tiles > 0) fetch(0);
  for (int64_t tile = 0; tile < a.n_tiles; ++tile) {
    __syncthreads();  // previous tile fully consumed
    stage();
    __syncthreads();
    if (tile + 1 < a.n_tiles) fetch(tile + 1);
    if (walker) {
      // Lane j describes bucket s_begin + j: its first nu list entries are
      // preloaded (absent ones point at the zero pad column TC), so the first
      // nu passes over all buckets are unrolled and branch-free with their
      // LDS reads independent; buckets with more entries walk the rest. nu
      // (at most NU) is chosen on the host from the expected entries per
      // bucket and tile.
      constexpr int NU = 8;
      const int nu = a.nu;
      const unsigned char* rec = pl + tl * a.rec_bytes;
      const uint16_t* of = (const uint16_t*)rec;
      const uint32_t* lst = (const uint32_t*)(rec + a.lst_off);
      const Tacc* Tl = T + lane * TS;
      uint32_t kbeg = 0, kcnt = 0;
      if (lane < s_cnt) {
        kbeg = of[s_begin + lane];
        kcnt = (uint32_t)of[s_begin + lane + 1] - kbeg;
      }
      uint32_t ev[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) ev[u] = (u < nu && kcnt > (uint32_t)u) ? lst[kbeg + u] : (uint32_t)a.TC;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        if (u >= nu) break;
#pragma unroll
        for (int g = 0; g < JB; g += 8) {
          Tacc v[8];
          uint32_t e[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (g + q < JB) {
              e[q] = (uint32_t)__builtin_amdgcn_readlane((int)ev[u], g + q);
              v[q] = Tl[e[q] & 0x7fffffffu];
            }
          }
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (g + q < JB) acc[g + q] += flip_c(v[q], e[q]);
        }
      }
      const uint64_t more = __ballot(kcnt > (uint32_t)nu);
      if (more) {
#pragma unroll
        for (int j = 0; j < JB; ++j) {
          if ((more >> j) & 1ull) {
            const uint32_t kb = (uint32_t)__builtin_amdgcn_readlane((int)kbeg, j);
            const uint32_t ke = kb + (uint32_t)__builtin_amdgcn_readlane((int)kcnt, j);
            for (uint32_t kk = kb + (uint32_t)nu; kk < ke; ++kk) {
              const uint32_t ea = lst[kk];
              acc[j] += flip_c(Tl[ea & 0x7fffffffu], ea);
            }
          }
        }
      }
    }
  }

  if (walker && lane < nrows) {
    const int64_t col0 = (int64_t)(t0 + tl) * a.nb + s_begin;
    if (a.out_f64) {
      double* Y = (double*)a.Y + (r0 + lane) * a.ldy + col0;
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < s_cnt) Y[j] = (double)acc[j] * a.scale_d;
    } else {
      float* Y = (float*)a.Y + (r0 + lane) * a.ldy + col0;
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < s_cnt) Y[j] = (float)(acc[j] * (Tacc)(sizeof(Tacc) == 8 ? a.scale_d : a.scale_f));
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS of the plan kernel for tiles of R indices (defined with that kernel)
size_t plan_kernel_lds(int R, int zeta, int64_t nb);

// Plan of the column-mode apply; the plan kernel is the row-mode one over the
// n columns (tile = TC columns, entries carry the plain column offset).
struct ColsPlan {
  int TC, JB, bpg, n_groups, H, per_range, W;
  int rec_bytes, lst_off;
  int64_t n_tiles;
  size_t lds, plan_bytes;
};

// The column kernel keeps a block's buckets in the registers of at most 16
// waves: at most 16 * 50 (FP64) or 16 * 64 (FP32 / BF16) buckets per block.
bool cols_kernel_fits(const sk_sketch* S, int dtype_in) {
  const int jmax = dtype_in == SK_F64 ? 50 : 64;
  return S->nb <= 16383 && (S->nb + jmax - 1) / jmax <= 16;
}

static int cols_plan(const sk_sketch* S, int dtype_in, ColsPlan* p) {
  const int accb = dtype_in == SK_F64 ? 8 : 4;
  const int jmax = dtype_in == SK_F64 ? 50 : 64;
  const int64_t nb = S->nb;
  const int Hmin = (int)((nb + jmax - 1) / jmax);
  if (!cols_kernel_fits(S, dtype_in)) {
    set_error("sketch_apply_T: d/zeta too large for the register-resident accumulators");
    return SK_E_NOTSUP;
  }
  if ((int64_t)S->zeta * Hmin <= 16) {
    p->bpg = S->zeta;
    p->n_groups = 1;
    // up to 8 waves (the prefetching kernel's size): with few blocks, split
    // each block's buckets over more waves so that more waves walk
    p->H = std::max<int>(Hmin, (int)std::min<int64_t>(nb, std::max(1, 8 / S->zeta)));
  } else {
    p->bpg = 16 / Hmin;
    p->n_groups = (S->zeta + p->bpg - 1) / p->bpg;
    p->H = Hmin;
  }
  p->W = p->bpg * p->H;
  p->per_range = (int)((nb + p->H - 1) / p->H);
  p->JB = p->per_range <= 16 ? 16 : (p->per_range <= 32 ? 32 : jmax);
  p->TC = dtype_in == SK_F64 ? 128 : 256;
  for (;;) {
    p->lst_off = (int)a16((size_t)(nb + 1) * 2);
    p->rec_bytes = (int)a16((size_t)p->lst_off + (size_t)(p->TC + 1) * 4);
    p->lds = a16((size_t)64 * (p->TC + 1) * accb) + (size_t)p->bpg * p->rec_bytes;
    const size_t plan_lds = plan_kernel_lds(p->TC, S->zeta, nb);
    if ((p->lds <= 160 * 1024 && plan_lds <= 160 * 1024) || p->TC <= 32) break;
    p->TC /= 2;
  }
  p->n_tiles = (S->n + p->TC - 1) / p->TC;
  p->plan_bytes = a16((size_t)p->n_tiles * S->zeta * p->rec_bytes);
  return SK_OK;
}

// Branch-free passes of the prefetching kernel: with lambda = TC / nb entries
// expected per bucket and tile (Poisson), nu passes cost nu loads per bucket
// and the entries past them cost about 3 loads each when walked; nu in 1 .. 8
// minimizes nu + 3 E[(X - nu)+]. SKETCH_COLS_NU overrides.
static int cols_passes(int TC, int64_t nb) {
  static const int env = [] {
    const char* v = std::getenv("SKETCH_COLS_NU");
    return v ? std::atoi(v) : 0;
  }();
  if (env >= 1 && env <= 8) return env;
  const double lam = (double)TC / (double)nb;
  std::vector<double> pmf(64);
  pmf[0] = std::exp(-lam);
  for (int x = 1; x < 64; ++x) pmf[x] = pmf[x - 1] * lam / x;
  int best = 8;
  double best_cost = 1e300;
  for (int nu = 1; nu <= 8; ++nu) {
    double tail = 0.0;
    for (int x = nu + 1; x < 64; ++x) tail += (x - nu) * pmf[x];
    const double cost = nu + 3.0 * tail;
    if (cost < best_cost) {
      best_cost = cost;
      best = nu;
    }
  }
  return best;
}

int cols_workspace(const sk_sketch* S, int dtype_in, size_t* bytes) {
  ColsPlan p;
  int rc = cols_plan(S, dtype_in, &p);
  if (rc != SK_OK) return rc;
  // either kernel's workspace: the bucket-indexed one's codes or the plan
  *bytes = std::max(p.plan_bytes, cols_idx_fits(S, dtype_in, nullptr, 0) ? cols_idx_workspace(S, dtype_in) : 0);
  return SK_OK;
}

int launch_plan_generic(const sk_sketch* S, int R, int rec_bytes, int lst_off, int64_t n_tiles, void* plan,
                        int runit, hipStream_t st);

template <typename Tin, int JB>
static int launch_cols_t(const sk_sketch* S, const ColsPlan& p, int64_t rows, const void* A, int64_t lda, void* Y,
                         int64_t ldy, int out_f64, const void* plan, hipStream_t st) {
  ColsArgs a;
  a.A = (const unsigned char*)A;
  a.lda_bytes = lda * (int64_t)sizeof(Tin);
  a.rows = rows;
  a.n = S->n;
  a.d = S->d;
  a.zeta = S->zeta;
  a.nb = (int)S->nb;
  a.TC = p.TC;
  a.bpg = p.bpg;
  a.n_groups = p.n_groups;
  a.H = p.H;
  a.per_range = p.per_range;
  a.plan = (const unsigned char*)plan;
  a.rec_bytes = p.rec_bytes;
  a.lst_off = p.lst_off;
  a.n_tiles = p.n_tiles;
  a.Y = Y;
  a.ldy = ldy;
  a.out_f64 = out_f64;
  a.scale_d = inv_sqrt_host((double)S->zeta);
  a.scale_f = (float)a.scale_d;
  a.nu = cols_passes(p.TC, S->nb);
  const int64_t grid = ((rows + 63) / 64) * p.n_groups;
  // the prefetching kernel: 16-byte aligned rows, whole chunks per row, the
  // tile within 8 chunks a thread and the plan records within 2
  const int threads = 512;
  const bool vec = p.W <= 8 && ((uintptr_t)A % 16 == 0) && (a.lda_bytes % 16 == 0) && ((S->n * (int64_t)sizeof(Tin)) % 16 == 0) &&
                   (64 * p.TC * (int64_t)sizeof(Tin) / 16 <= 8 * threads) &&
                   ((int64_t)p.bpg * p.rec_bytes / 16 <= 2 * threads);
  KernelTimer timer(S, st);
  if (vec) {
    auto kern = ss_cols_vec_kernel<Tin, JB>;
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), p.lds, st, a);
  } else {
    auto kern = ss_cols_kernel<Tin, JB>;
    SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * p.W), p.lds, st, a);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename Tin>
static int launch_cols_jb(const sk_sketch* S, const ColsPlan& p, int64_t rows, const void* A, int64_t lda, void* Y,
                          int64_t ldy, int out_f64, const void* plan, hipStream_t st) {
  constexpr int JMAX = sizeof(Tin) == 8 ? 50 : 64;
  if (p.JB == 16) return launch_cols_t<Tin, 16>(S, p, rows, A, lda, Y, ldy, out_f64, plan, st);
  if (p.JB == 32) return launch_cols_t<Tin, 32>(S, p, rows, A, lda, Y, ldy, out_f64, plan, st);
  return launch_cols_t<Tin, JMAX>(S, p, rows, A, lda, Y, ldy, out_f64, plan, st);
}

int launch_cols_apply(const sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out,
                      void* Y, int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st) {
  if (cols_idx_fits(S, dtype_in, A, lda))
    return launch_cols_idx(S, dtype_in, rows, A, lda, dtype_out, Y, ldy, ws, ws_bytes, st);
  ColsPlan p;
  int rc = cols_plan(S, dtype_in, &p);
  if (rc != SK_OK) return rc;
  if (ws_bytes < p.plan_bytes) {
    set_error("sketch_apply_T: workspace too small (see sketch_workspace_size)");
    return SK_E_INVAL;
  }
  rc = launch_plan_generic(S, p.TC, p.rec_bytes, p.lst_off, p.n_tiles, ws, 1, st);
  if (rc != SK_OK) return rc;
  const int of64 = dtype_out == SK_F64;
  if (dtype_in == SK_F64) return launch_cols_jb<double>(S, p, rows, A, lda, Y, ldy, of64, ws, st);
  if (dtype_in == SK_F32) return launch_cols_jb<float>(S, p, rows, A, lda, Y, ldy, of64, ws, st);
  return launch_cols_jb<uint16_t>(S, p, rows, A, lda, Y, ldy, of64, ws, st);
}

}  // namespace sk
