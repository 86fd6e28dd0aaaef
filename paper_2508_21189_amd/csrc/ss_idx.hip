// SparseStack apply, row mode, with bucket-indexed register accumulators:
// SA = S A for a tall row-major A (n x m).
//
// Def. 1.5: column i of S carries rho_it / sqrt(zeta) in row t*nb + s_it for
// each block t, so SA[t*nb + s, c] = (1/sqrt(zeta)) * sum_{i: s_it = s} rho_it A[i, c].
//
// Design (gfx950, one HBM pass over A, no sorting):
//  * A workgroup owns a row chunk x a column slab (<= 64 columns, one per
//    lane) x a group of blocks, one wave per block. Each wave keeps the
//    accumulators of all nb buckets of its block in registers: slot s of
//    every lane lives in a fixed VGPR range (v40 upwards), pinned through
//    inline-assembly register constraints.
//  * Rows of a tile are visited in order. For a given row and block the
//    bucket is the same for every lane (it depends on the row only), so the
//    add goes to a register whose number is known only at run time but is
//    wave-uniform: the VALU's GPR-index mode (s_set_gpr_idx_on) offsets the
//    accumulator operand by the bucket's register index, and one FMA with
//    the sign as a +-1.0 scalar multiplier adds the row (exact: the product
//    is the value itself, so the FMA rounds once, like acc +- v).
//  * The work per (row, block) is therefore independent of nb: half an LDS
//    read (two rows per ds_read2st64), one scalar mask, one index switch and
//    one FMA. The earlier sorted design paid a cost per bucket and tile
//    instead, which dominated when buckets held ~1-2 rows per tile.
//  * Each row's code (bucket register index | the sign and exponent bits of
//    +-1.0) is computed once by a plan kernel (Philox hash) into the
//    workspace, [tile][block][row], and read by the sketch waves with scalar
//    loads, 32 rows at a time: moving codes from vector registers with
//    readlane costs more than everything else in the loop together.
//  * Tiles of A stream into LDS with direct global->LDS loads, double
//    buffered.
//  * Partials go to [chunk][d][m]; reduce_partials_kernel sums them in chunk
//    order and scales by 1/sqrt(zeta). No atomics and a fixed order of
//    every sum: bitwise reproducible.
//  * FP64 blocks of more buckets than one register file holds (100) are split
//    into bucket parts, one wave each: every part's wave walks every row,
//    adding rows of its part into their buckets and the others into dump
//    registers that are never stored (rotating over four, so that dumped
//    rows do not queue on one register). Each bucket still receives its rows
//    in row order, so the sums are those of a single register file.
#include "sk_idx.hpp"
#include "sk_launch.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <tuple>
#include <vector>

namespace sk {

using namespace idx;

struct IdxArgs {
  const unsigned char* A;
  int64_t lda_bytes;
  int64_t n, m, d;
  int C, n_slabs, R, bpg, n_groups, n_chunks;
  int64_t rows_per_chunk;
  int zeta, nb;
  uint32_t k0, k1;
  void* P;
  int buf_stride;  // LDS bytes of one tile buffer
  int nbuf;        // tile buffers: loads run nbuf - 1 tiles ahead
  int off_touch;   // LDS scratch (1 KB per wave) that the code prefetch lands in
  const unsigned char* codes_touch;  // the row codes, for that prefetch only
  // bucket parts (more buckets than one register file): parts per block
  // and buckets per part
  int nparts, ps;
  int lb;  // width of the direct loads (16 or 4) where the kernel takes it at run time
};

// Row codes of row i = tile * R + r and block t, at base = (tile * zeta + t)
// * 2R: the bucket's register index bucket * (registers per accumulator) at
// [base + r], and the high word of the +-1.0 multiplier (the sign of the
// entry) at [base + R + r]. The bucket and sign follow Def. 1.5 through the
// Philox reading shared with every other SparseStack kernel.
__global__ void ss_idx_plan_kernel(int64_t n, int64_t n_tiles, int R, int zeta, uint32_t nb, uint32_t one_hi,
                                   uint32_t rpa, uint32_t k0, uint32_t k1, uint32_t* __restrict__ codes) {
  const int ng = (zeta + 3) / 4;
  const int64_t total = n_tiles * R * ng;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tr = idx / ng;  // tile * R + r = the row index i
    const int g = (int)(idx - tr * ng);
    const int64_t tile = tr / R;
    const int r = (int)(tr - tile * R);
    const uint64_t i = (uint64_t)tr;
    U4 w = U4{0u, 0u, 0u, 0u};
    if ((int64_t)i < n) w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)g, kTagSparseStack}, k0, k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * g + j;
      if (t < zeta) {
        const uint32_t word = word_of(w, j);
        uint32_t* c = codes + (tile * zeta + t) * (int64_t)(2 * R);
        c[r] = ss_bucket(word, nb) * rpa;
        c[R + r] = (ss_negative(word) << 31) | one_hi;
      }
    }
  }
}

// Bucket parts: a block whose nb buckets exceed one register file is split
// into nparts parts of ps buckets, one wave each, every wave walking all the
// tile's rows in order. For list (tile, block t, part h), at base =
// ((tile * zeta + t) * nparts + h) * 2R, row r's entry [base + r] is the
// bucket's register index within part h, or, when the bucket lies in another
// part, one of ndump dump slots (registers that are never stored; rotating
// with the row so that consecutive dumped rows do not wait on one register);
// [base + R + r] is the high word of the +-1.0 multiplier. Same Philox
// reading as above.
__global__ void ss_idx_plan_parts_kernel(int64_t n, int64_t n_tiles, int R, int zeta, uint32_t nb, int nparts,
                                         int ps, uint32_t dump0, uint32_t ndump, uint32_t one_hi, uint32_t rpa,
                                         uint32_t k0, uint32_t k1, uint32_t* __restrict__ codes) {
  const int ng = (zeta + 3) / 4;
  const int64_t total = n_tiles * R * ng;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t tr = idx / ng;  // tile * R + r = the row index i
    const int g = (int)(idx - tr * ng);
    const int64_t tile = tr / R;
    const int r = (int)(tr - tile * R);
    const uint64_t i = (uint64_t)tr;
    U4 w = U4{0u, 0u, 0u, 0u};
    if ((int64_t)i < n) w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)g, kTagSparseStack}, k0, k1);
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * g + j;
      if (t >= zeta) break;
      const uint32_t word = word_of(w, j);
      const int b = (int)ss_bucket(word, nb);
      const uint32_t sw = (ss_negative(word) << 31) | one_hi;
      for (int h = 0; h < nparts; ++h) {
        const int rel = b - h * ps;
        uint32_t* c = codes + ((tile * zeta + t) * nparts + h) * (int64_t)(2 * R);
        c[r] = (rel >= 0 && rel < ps ? (uint32_t)rel : dump0 + (uint32_t)r % ndump) * rpa;
        c[R + r] = sw;
      }
    }
  }
}

template <int ES>
struct RawBits;
template <>
struct RawBits<8> {
  using type = uint64_t;
};
template <>
struct RawBits<4> {
  using type = uint32_t;
};
template <>
struct RawBits<2> {
  using type = uint16_t;
};

// Global-memory accesses through pointers that the compiler cannot place
// in the global address space by itself (those read from a table): without
// the cast they become flat accesses, which also count against the LDS
// counter and make the tile's LDS reads wait for them.
template <typename T>
__device__ inline T gload(const void* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ inline void gstore(void* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// The work of workgroup L of the grid that a describes. With HASB the last
// of the a.m columns is not part of the matrix but the vector bcol (stride
// one element): it rides in the lane after the matrix's last column, its
// values loaded to registers by wave 0 and written into the tile's padding
// before the tile is published (two tile buffers only).
template <typename Tin, int NREG, int LB, bool PARTS, bool HASB>
__device__ __forceinline__ void ss_idx_body(const IdxArgs& a, const unsigned char* bcol,
                                            const uint32_t* __restrict__ codes_all, int L) {
  using T = IdxT<Tin>;
  using Tacc = typename T::acc;
  constexpr int ES = sizeof(Tin);
  // Tile rows sit at a fixed stride of one element per lane, so the LDS
  // offsets of the rows of a 64-row group are compile-time immediates.
  constexpr int ROWB = 64 * ES;
  // load width: the template's, or (LB = 0, the batched kernels) the argument's
  const int lb = LB ? LB : a.lb;
  const int CPR = ROWB / lb;  // load chunks per tile row (a power of two)
  constexpr int GR = 16;          // rows whose codes one scalar group holds
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x, nwaves = nthreads >> 6;

  // Work item. Dispatch is round-robin over the 8 XCDs (id L runs on XCD
  // L % 8): all slabs and block groups of one row chunk get ids 8 apart and
  // share one XCD's L2 for the cache lines that straddle slab boundaries.
  const int xcd = L & 7, q8 = L >> 3;
  const int group = q8 % a.n_groups;
  const int slab = (q8 / a.n_groups) % a.n_slabs;
  const int chunk = (q8 / (a.n_groups * a.n_slabs)) * 8 + xcd;
  if (chunk >= a.n_chunks) return;

  const int t0 = group * a.bpg;
  const int bpg = min(a.bpg, a.zeta - t0);
  const int64_t col0 = (int64_t)slab * a.C;
  const int Cw = (int)min((int64_t)a.C, a.m - col0);
  // bytes of the matrix in a tile row of the slab (what the direct loads bring)
  const int slab_bytes = HASB ? (int)max((int64_t)0, min((int64_t)Cw, a.m - 1 - col0)) * ES : Cw * ES;
  const int bl = HASB ? (int)(a.m - 1 - col0) : -1;  // the lane of the b column
  const bool has_b = HASB && bl >= 0 && bl < Cw;
  using Raw = typename RawBits<ES>::type;
  Raw bv[2] = {0, 0};
  const int64_t r_begin = (int64_t)chunk * a.rows_per_chunk;
  const int64_t r_end = min(a.n, r_begin + a.rows_per_chunk);
  const int nsub = r_end > r_begin ? (int)((r_end - r_begin + a.R - 1) / a.R) : 0;
  const int R = a.R, nb = a.nb;
  // this wave's block (and bucket part); the index of its code list in a tile
  int tb = t0 + wave, part = 0;
  if constexpr (PARTS) {
    tb = t0 + wave / a.nparts;
    part = wave - (wave / a.nparts) * a.nparts;
  }
  const bool walker = PARTS ? wave < bpg * a.nparts : wave < bpg;
  auto list_of = [&](int64_t tile) -> int64_t {
    if constexpr (PARTS)
      return (tile * a.zeta + tb) * a.nparts + part;
    else
      return tile * a.zeta + t0 + wave;
  };

  AccFile f;
  acc_zero<NREG>(f);

  // Chunk q of a tile (lb bytes) is row q / CPR, bytes (q % CPR) * lb of it;
  // chunks past the slab's bytes are padding and are not loaded.
  const int n_instr = (R * CPR + 63) / 64;
  auto issue_loads = [&](int st, int buf) {
    const int64_t r0 = r_begin + (int64_t)st * R;
    const int rv = (int)min((int64_t)R, r_end - r0);
    unsigned char* dst = smem + buf * a.buf_stride;
    const unsigned char* tsrc = a.A + r0 * a.lda_bytes + col0 * ES;
    // load k covers chunks [64 k, 64 k + 64): a lane's chunk advances by
    // 64 W chunks per load of its wave. When that is a whole number RSTEP of
    // rows, the lane keeps a fixed byte offset; otherwise (128 chunks a row,
    // FP64 with 4-byte loads, and an odd number of waves) its row and offset
    // are recomputed for every load.
    const int q0 = wave * 64 + lane;
    int cb = (q0 % CPR) * lb;
    const bool whole_rows = (nwaves * 64) % CPR == 0;
    const int rstep = (nwaves * 64) / CPR;
    int row = q0 / CPR;
    const unsigned char* src = tsrc + (int64_t)row * a.lda_bytes + cb;
    const int64_t sstep = (int64_t)rstep * a.lda_bytes;
    // A full tile read with 4-byte loads by 4 or 8 waves: the wave's loads go
    // out 4 (or 2) under one M0 setting, 256 W bytes apart in LDS through the
    // instruction offset (every row of a full tile is valid; a lane skips
    // only chunks past the slab's bytes). This halves the instructions that
    // the loads of such tiles cost.
    const bool grouped = (LB == 0 || LB == 4) && lb == 4 && whole_rows && rv == R && (nwaves == 4 || nwaves == 8);
    if (grouped) {
      const int iters = (n_instr - wave + nwaves - 1) / nwaves;
      int it = 0;
      if (nwaves == 4) {
        for (; it + 4 <= iters; it += 4) {
          const uint32_t la =
              (uint32_t)__builtin_amdgcn_readfirstlane((int)idx_lds_addr(dst + (wave + it * 4) * 256));
          if (cb < slab_bytes) {
            const void* g[4] = {src, src + sstep - 1024, src + 2 * sstep - 2048, src + 3 * sstep - 3072};
            idx_dma4_group<4, 1024>(g, la);
          }
          src += 4 * sstep;
        }
      } else {
        for (; it + 2 <= iters; it += 2) {
          const uint32_t la =
              (uint32_t)__builtin_amdgcn_readfirstlane((int)idx_lds_addr(dst + (wave + it * 8) * 256));
          if (cb < slab_bytes) {
            const void* g[2] = {src, src + sstep - 2048};
            idx_dma4_group<2, 2048>(g, la);
          }
          src += 2 * sstep;
        }
      }
      for (; it < iters; ++it) {
        const uint32_t la =
            (uint32_t)__builtin_amdgcn_readfirstlane((int)idx_lds_addr(dst + (wave + it * nwaves) * 256));
        if (cb < slab_bytes) idx_dma4(src, la);
        src += sstep;
      }
    }
    for (int k = grouped ? n_instr : wave; k < n_instr; k += nwaves) {
      const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane((int)idx_lds_addr(dst + k * 64 * lb));
      if (!whole_rows) {
        const int q = k * 64 + lane;
        row = q / CPR;
        cb = (q % CPR) * lb;
        src = tsrc + (int64_t)row * a.lda_bytes + cb;
      }
      if (row < rv && cb < slab_bytes) {
        if (lb == 16)
          idx_dma16(src, la);
        else
          idx_dma4(src, la);
      }
      row += rstep;
      src += sstep;
    }
    if constexpr (HASB) {
      if (has_b && wave == 0) {
        // unconditional loads (rows past the tile read its last row; they
        // are not written to LDS), so that nothing waits behind a branch
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = gload<Raw>(bcol + (r0 + min(j * 64 + lane, rv - 1)) * ES);
      }
    }
    // Bring this wave's codes of the tile into L2 ahead of their scalar
    // loads: a direct load of them into a scratch LDS area that is never
    // read (the scalar loads would otherwise wait on HBM once per group).
    if (walker) {
      // (the address comes from a second copy of the codes pointer, so that
      // the restrict one never reaches an asm statement)
      const unsigned char* csrc = a.codes_touch + list_of(r0 / R) * (int64_t)R * 8;
      const int cbytes = 8 * R;
      const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane(
          (int)idx_lds_addr(smem + a.off_touch + wave * 1024));
      for (int o = 0; o < cbytes; o += 1024)
        if (o + lane * 16 < cbytes) idx_dma16(csrc + o + lane * 16, la);
    }
  };
  // Loads this wave issues for one full tile: its share of the tile's loads
  // that have an active lane (a load of 64 chunks starting at a row's first
  // chunk always has one; with 128 chunks a row, one starting mid-row has
  // one iff the slab reaches that far), and the code prefetch.
  const int nbuf = a.nbuf;
  int per_tile = walker ? (8 * R + 1023) / 1024 : 0;
  for (int k = wave; k < n_instr; k += nwaves)
    if (((k * 64) % CPR) * lb < slab_bytes) ++per_tile;
  if (HASB && has_b && wave == 0) per_tile += 2;
  for (int p = 0; p < nbuf - 1 && p < nsub; ++p) issue_loads(p, p);
  for (int st = 0; st < nsub; ++st) {
    const int buf = st % nbuf;
    // tile st is complete once only the loads of the later tiles in flight
    // remain; a partial (last) tile among those: wait for everything
    const int later = min(st + nbuf - 2, nsub - 1) - st;
    const bool later_full = later <= 0 || r_begin + (int64_t)(st + later + 1) * R <= r_end;
    idx_wait_vm(later > 0 && later_full ? later * per_tile : 0);
    if constexpr (HASB) {
      // the b values of tile st (loaded with the tile) into its padding lane
      if (has_b && wave == 0) {
        const int64_t r0 = r_begin + (int64_t)st * R;
        const int rv = (int)min((int64_t)R, r_end - r0);
        unsigned char* dst = smem + buf * a.buf_stride + bl * ES;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int brow = j * 64 + lane;
          if (j * 64 < R && brow < rv) *(Raw*)(dst + brow * ROWB) = bv[j];
        }
      }
    }
    idx_barrier();  // tile st is in LDS; everyone finished tile st-1
    if (st + nbuf - 1 < nsub) issue_loads(st + nbuf - 1, (st + nbuf - 1) % nbuf);
    if (walker) {
      const int64_t r0 = r_begin + (int64_t)st * R;
      const int rv = (int)min((int64_t)R, r_end - r0);
      // this wave's codes for the tile (uniform address: scalar loads)
      // (a kernel argument marked restrict, never written here: the
      // compiler reads it with scalar loads)
      const uint32_t* codes = codes_all + list_of(r0 / R) * (int64_t)(2 * R);
      const uint32_t tbase = idx_lds_addr(smem + buf * a.buf_stride) + (uint32_t)(lane * ES);
      const int full = rv & ~(GR - 1);
      // full groups of GR rows: straight-line code, row offsets immediate;
      // the values of batch k + 1 are read before batch k's adds
      for (int g = 0; g < full; g += GR) {
        uint32_t w[GR], h[GR];
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          w[u] = codes[g + u];
          h[u] = codes[R + g + u];
        }
        uint32_t rb = tbase + (uint32_t)(g * ROWB);
        asm volatile("" : "+v"(rb));
        Tacc v[4], vn[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = idx_val<Tin>(rb + (uint32_t)(u * ROWB));
#pragma unroll
        for (int k = 0; k < GR; k += 4) {
          if (k + 4 < GR) {
#pragma unroll
            for (int u = 0; u < 4; ++u) vn[u] = idx_val<Tin>(rb + (uint32_t)((k + 4 + u) * ROWB));
          }
          fma4<NREG>(f, v[0], v[1], v[2], v[3], w[k], w[k + 1], w[k + 2], w[k + 3], idx_pm(h[k], (Tacc*)nullptr),
                     idx_pm(h[k + 1], (Tacc*)nullptr), idx_pm(h[k + 2], (Tacc*)nullptr),
                     idx_pm(h[k + 3], (Tacc*)nullptr));
          // keep the next batch's loads behind this batch's adds (bounded registers)
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = vn[u];
        }
      }
      // the last rows of the matrix (a tile shorter than a multiple of GR)
      for (int r = full; r < rv; ++r) {
        const uint32_t wr = codes[r], hr = codes[R + r];
        const Tacc v0 = idx_val<Tin>(tbase + (uint32_t)(r * ROWB));
        fma1<NREG>(f, v0, wr, idx_pm(hr, (Tacc*)nullptr));
      }
    }
  }

  if (walker && lane < Cw) {
    Tacc* P = (Tacc*)a.P;
    int64_t rowbase = (int64_t)chunk * a.d + (int64_t)(t0 + wave) * nb;
    int nstore = nb;
    if constexpr (PARTS) {
      rowbase = (int64_t)chunk * a.d + (int64_t)tb * nb + (int64_t)part * a.ps;
      nstore = min(a.ps, nb - part * a.ps);
    }
#pragma unroll
    for (int s = 0; s < NREG / T::rpa; ++s) {
      if (s < nstore) {
        Tacc val;
        if constexpr (T::rpa == 2) {
          const uint64_t lo = acc_get<NREG>(f, 2 * s), hi = acc_get<NREG>(f, 2 * s + 1);
          val = __builtin_bit_cast(double, lo | (hi << 32));
        } else {
          val = __builtin_bit_cast(float, acc_get<NREG>(f, s));
        }
        gstore<Tacc>(P + (rowbase + s) * a.m + col0 + lane, val);
      }
    }
  }
}

template <typename Tin, int NREG, int LB, bool PARTS = false>
__global__ void __launch_bounds__(NREG > 64 ? 512 : 1024)
    ss_idx_kernel(IdxArgs a, const uint32_t* __restrict__ codes_all) {
  ss_idx_body<Tin, NREG, LB, PARTS, false>(a, nullptr, codes_all, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Batched sketches: [S_p A_p | S_p b_p] for many independent problems, each
// with its own SparseStack (Def. 1.5). One launch computes the row codes of
// every problem, one launch per kernel variant (input type, register file,
// load width, bucket parts) runs the applies of all its problems, with b_p
// as the column after A_p's last one, and one launch per partial type sums
// the chunks into W_p, column-major d_p x (k_p + 1) (the layout the
// Householder QR takes). Each workgroup finds its problem by a binary
// search over the problems' first workgroups; the arithmetic of every
// problem is that of the single-matrix kernels.
// ---------------------------------------------------------------------------
struct IdxBatchEntry {
  IdxArgs a;                // a.m = k + 1 (column k is b), a.P = the problem's partials
  const unsigned char* b;   // b (k + 1 th column), stride one element
  int64_t codes_off;        // the problem's codes: words from the codes base
  int64_t wg_begin;         // its first workgroup in the launch (a multiple of 8)
};

struct IdxCodesEntry {
  int64_t n, n_tiles, codes_off, blk_begin;
  int R, zeta, nparts, ps;
  uint32_t nb, dump0, ndump, one_hi, rpa, k0, k1;
};

struct IdxReduceEntry {
  const void* P;   // partials [chunk][d][m]
  double* W;       // W[c * ldw + row]
  int64_t d, m, ldw, blk_begin;
  int n_chunks, col_tiles;
  double scale;
};

// The entry whose range [begin, next begin) holds g (entries sorted by begin).
template <typename E, int64_t E::*BEGIN>
__device__ inline int batch_find(const E* __restrict__ tab, int nent, int64_t g) {
  int lo = 0, hi = nent - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].*BEGIN <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename Tin, int NREG, int LB, bool PARTS>
__global__ void __launch_bounds__(NREG > 64 ? 512 : 1024)
    ss_idx_batched_kernel(const IdxBatchEntry* __restrict__ tab, int nent, const uint32_t* __restrict__ codes_all) {
  const int64_t g = blockIdx.x;
  const int e = batch_find<IdxBatchEntry, &IdxBatchEntry::wg_begin>(tab, nent, g);
  // a private copy: the body's asm statements clobber memory, and the
  // fields must not be re-read from the table after each of them
  const IdxArgs a = tab[e].a;
  const unsigned char* bcol = tab[e].b;
  const int64_t off = tab[e].codes_off;
  const int L = (int)(g - tab[e].wg_begin);
  ss_idx_body<Tin, NREG, LB, PARTS, true>(a, bcol, codes_all + off, L);
}

// Codes of every problem, in the layout of the bucket-parts plan kernel
// (with one part, ps = nb, it is the layout of the plain one): block q of
// problem e handles items [q * 1024, (q + 1) * 1024) of its rows x hash
// groups.
constexpr int kCodesPerThread = 4;
__global__ void __launch_bounds__(256)
    ss_idx_plan_batched_kernel(const IdxCodesEntry* __restrict__ tab, int nent, uint32_t* __restrict__ codes_all) {
  const int64_t blk = blockIdx.x;
  const IdxCodesEntry e = tab[batch_find<IdxCodesEntry, &IdxCodesEntry::blk_begin>(tab, nent, blk)];
  const int ng = (e.zeta + 3) / 4;
  const int64_t total = e.n_tiles * e.R * ng;
  uint32_t* codes = codes_all + e.codes_off;
  const int64_t first = (blk - e.blk_begin) * (256 * kCodesPerThread);
  for (int q = 0; q < kCodesPerThread; ++q) {
    const int64_t idx = first + q * 256 + threadIdx.x;
    if (idx >= total) break;
    const int64_t tr = idx / ng;  // tile * R + r = the row index i
    const int g = (int)(idx - tr * ng);
    const int64_t tile = tr / e.R;
    const int r = (int)(tr - tile * e.R);
    const uint64_t i = (uint64_t)tr;
    U4 w = U4{0u, 0u, 0u, 0u};
    if ((int64_t)i < e.n)
      w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)g, kTagSparseStack}, e.k0, e.k1);
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * g + j;
      if (t >= e.zeta) break;
      const uint32_t word = word_of(w, j);
      const int b = (int)ss_bucket(word, e.nb);
      const uint32_t sw = (ss_negative(word) << 31) | e.one_hi;
      for (int h = 0; h < e.nparts; ++h) {
        const int rel = b - h * e.ps;
        uint32_t* c = codes + ((tile * e.zeta + t) * e.nparts + h) * (int64_t)(2 * e.R);
        c[r] = (rel >= 0 && rel < e.ps ? (uint32_t)rel : e.dump0 + (uint32_t)r % e.ndump) * e.rpa;
        c[e.R + r] = sw;
      }
    }
  }
}

// W[c * ldw + row] = scale * (sum over chunks, in chunk order, in FP64, of
// P[chunk][row][c]) for a 64 x 64 tile (row, c) of one problem per block:
// the partials read along c, the tile transposed through LDS, W written
// along the rows.
template <typename Tacc>
__global__ void __launch_bounds__(256) idx_reduce_batched_kernel(const IdxReduceEntry* __restrict__ tab, int nent) {
  __shared__ double tile[64][65];
  const int64_t blk = blockIdx.x;
  const IdxReduceEntry e = tab[batch_find<IdxReduceEntry, &IdxReduceEntry::blk_begin>(tab, nent, blk)];
  const int local = (int)(blk - e.blk_begin);
  const int64_t r0 = (int64_t)(local / e.col_tiles) * 64;
  const int64_t c0 = (int64_t)(local % e.col_tiles) * 64;
  const int j = threadIdx.x & 63, i0 = threadIdx.x >> 6;
  const Tacc* P = (const Tacc*)e.P;
  const int64_t c = c0 + j;
  const int nr = (int)min((int64_t)64, e.d - r0);  // rows of the tile
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  if (c < e.m) {
    // two chunks' loads in flight before their adds (in chunk order); the
    // loads are unconditional (rows past the tile read its last row and are
    // never stored), so that none waits behind a branch
    const int64_t cs = e.d * e.m;  // chunk stride
    const Tacc* Pc = P + r0 * e.m + c;
    int64_t ro[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) ro[q] = (int64_t)min(i0 + 4 * q, nr - 1) * e.m;
    int ch = 0;
    for (; ch + 1 < e.n_chunks; ch += 2, Pc += 2 * cs) {
      Tacc v0[16], v1[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        v0[q] = gload<Tacc>(Pc + ro[q]);
        v1[q] = gload<Tacc>(Pc + cs + ro[q]);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        acc[q] += (double)v0[q];
        acc[q] += (double)v1[q];
      }
    }
    if (ch < e.n_chunks) {
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += (double)gload<Tacc>(Pc + ro[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) tile[j][i0 + 4 * q] = acc[q] * e.scale;
  __syncthreads();
  const int rr = threadIdx.x & 63, cq = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int cc = cq + 4 * q;
    if (r0 + rr < e.d && c0 + cc < e.m) gstore<double>(e.W + (c0 + cc) * e.ldw + r0 + rr, tile[cc][rr]);
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {
size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }
int env_i(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}
// Dump slots of a parts plan: 8 registers (FP32 accumulators) or 4 register
// pairs (FP64).
int dump_slots(int dtype_in) { return dtype_in == SK_F64 ? 4 : 8; }
// Accumulator register files compiled, and how many waves of each fit a SIMD
// (the pinned file plus the kernel's other registers, 512 per SIMD lane).
int idx_nreg(int dtype_in, int64_t nb) {
  const int64_t regs = nb * (dtype_in == SK_F64 ? 2 : 1);
  if (regs <= 32) return 32;
  if (regs <= 64) return 64;
  if (regs <= 128) return 128;
  if (regs <= 200) return 200;
  return 0;
}
int idx_waves_per_simd(int nreg) { return nreg <= 32 ? 5 : (nreg <= 64 ? 4 : 2); }
// Bucket parts of a block: 1 when its buckets fit one register file, else
// (FP64 only) up to four parts (one wave each) of the 200-register file, the
// last few slots of which are kept as the dump for the rows of the other
// parts. Every part walks every row, so k parts cost k times the adds of one:
// measured on 8388608 x 500 with d = 2000, zeta = 8 (250 buckets), FP64 takes
// 30.1 ms with three parts against 34.6 ms on the sorted kernel, while FP32
// (two parts, 12.1 ms against 11.9) and BF16 (14.4 against 12.2) do not gain
// and stay on the sorted kernel.
constexpr int kMaxParts = 4;
int idx_parts(int dtype_in, int64_t nb) {
  if (idx_nreg(dtype_in, nb) != 0) return 1;
  if (dtype_in != SK_F64) return 0;
  const int64_t cap = (dtype_in == SK_F64 ? 100 : 200) - dump_slots(dtype_in);
  const int64_t np = (nb + cap - 1) / cap;
  return np <= kMaxParts ? (int)np : 0;
}

// Bucket parts of a block in the batched sketch: as idx_parts, and FP32 and
// BF16 blocks of more than 200 buckets are split too (192 buckets a part, the
// last 8 slots of the file being the dump): a batch gains from keeping every
// problem in its one launch more than it loses to the repeated walk.
int batch_parts(int dtype_in, int64_t nb) {
  if (idx_nreg(dtype_in, nb) != 0) return 1;
  const int64_t cap = (dtype_in == SK_F64 ? 100 : 200) - dump_slots(dtype_in);
  const int64_t np = (nb + cap - 1) / cap;
  return np <= kMaxParts ? (int)np : 0;
}
}  // namespace

bool idx_apply_fits(const sk_sketch* S, int dtype_in, int64_t m) {
  if (env_i("SKETCH_IDX", 1) == 0) return false;
  return m > 4 && S->zeta >= 4 && idx_parts(dtype_in, S->nb) != 0;
}

// batch: the plan of one problem of a batched sketch (bucket parts by
// batch_parts, two tile buffers, and row chunks sized for a launch that
// many problems fill together rather than for filling the chip alone).
static int plan_idx_lb(const sk_sketch* S, int dtype_in, int64_t m, int load_bytes, RowsPlan* p,
                       bool batch = false, int chunk_mult = 16) {
  const int es = (int)dtype_size(dtype_in);
  const int zeta = S->zeta;
  const int nparts = batch ? batch_parts(dtype_in, S->nb) : idx_parts(dtype_in, S->nb);
  if (nparts == 0) {
    set_error("sketch_apply: bucket register file too small for this block size");
    return SK_E_NOTSUP;
  }
  const int nreg = nparts == 1 ? idx_nreg(dtype_in, S->nb) : 200;
  p->idx = true;
  p->narrow = false;
  p->jb = nreg;
  p->nparts = nparts;
  p->ps = (int)((S->nb + nparts - 1) / nparts);
  const int wps = idx_waves_per_simd(nreg);
  const int wmax = std::min(16, 4 * wps);
  // one wave per (block, part): the blocks of a group share the tile
  p->bpg = std::min(zeta, std::max(1, wmax / nparts));
  p->n_groups = (zeta + p->bpg - 1) / p->bpg;
  p->W = p->bpg * nparts;
  p->H = 1;
  p->ranges = 1;
  p->per_range = (int)S->nb;
  p->load_bytes = load_bytes;
  const int cal = std::max(1, load_bytes / es);
  int ns = (int)((m + 63) / 64);
  int C = (int)((m + ns - 1) / ns);
  C = ((C + cal - 1) / cal) * cal;
  if (C > 64) C = 64;
  p->C = C;
  p->n_slabs = (int)((m + C - 1) / C);
  p->rowb = 64 * es;  // fixed tile-row stride in LDS

  // LDS: workgroups resident on a CU share its 160 KB: two buffers of R
  // tile rows.
  const int wg_per_cu = std::max(1, std::min(2, (4 * wps) / p->W));
  const size_t cap = std::min<size_t>(160 * 1024, (size_t)(160 * 1024 / wg_per_cu));
  const size_t touch = (size_t)1024 * p->W;
  // two buffers: loading three or four tiles ahead measured slower (F64
  // coherent 2.06 ms with two, 2.40 with three, 2.62 with four)
  const int nbuf = batch ? 2 : std::max(2, std::min(4, env_i("SKETCH_IDX_NBUF", 2)));
  p->nbuf = nbuf;
  int R = (int)((cap - touch - 64) / nbuf / (size_t)p->rowb);
  // at most 128 rows: larger tiles measured slower (F32 m = 200: 128 rows
  // 1.34 ms, 288 rows 1.90 ms), and 128 is the most that fits for F64
  R = std::min(R, env_i("SKETCH_IDX_ROWS", 128));
  // whole 32-row groups take the fast path; only the matrix's last tile
  // may end in a partial group
  R = (R / 32) * 32;
  if (R < 32) {
    set_error("sketch_apply: LDS plan does not fit");
    return SK_E_NOTSUP;
  }
  p->R = R;
  const size_t buf = a16((size_t)R * p->rowb);
  p->lds_bytes = nbuf * buf + touch;
  p->rec_bytes = (int)buf;  // buffer stride
  p->lst_off = 0;

  const int64_t n = S->n;
  const int64_t items = (int64_t)p->n_slabs * p->n_groups;
  int64_t nc;
  if (batch) {
    // chunks of at least chunk_mult d rows (16 by default: the partials
    // then add at most about 1/16 of A's bytes) and 2048 rows; not rounded
    // up to a multiple of 8 (the grid is, and its surplus workgroups exit at
    // once)
    const int64_t rows = std::max<int64_t>(2048, (int64_t)std::max(1, chunk_mult) * S->d);
    nc = std::max<int64_t>(1, (n + rows - 1) / rows);
  } else {
    const int target = env_i("SKETCH_IDX_WG", 256 * wg_per_cu);
    nc = std::max<int64_t>(1, (target + items - 1) / items);
    nc = ((std::max<int64_t>(nc, 8) + 7) / 8) * 8;
  }
  nc = std::min<int64_t>(nc, (n + p->R - 1) / p->R);
  int64_t rpc = (n + nc - 1) / nc;
  rpc = ((rpc + p->R - 1) / p->R) * p->R;
  p->rows_per_chunk = rpc;
  p->n_chunks = (int)((n + rpc - 1) / rpc);
  p->n_tiles = (n + p->R - 1) / p->R;
  const size_t accb = dtype_in == SK_F64 ? 8 : 4;
  p->partial_bytes = a16((size_t)p->n_chunks * S->d * m * accb);
  // codes: 2R words per (tile, block, part)
  p->plan_bytes = a16((size_t)p->n_tiles * p->R * zeta * nparts * 8);
  return SK_OK;
}

// A == NULL asks for the workspace bound of any alignment: the larger of
// the two load widths' partial buffers.
int plan_idx(const sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, RowsPlan* p) {
  const int es = (int)dtype_size(dtype_in);
  if (!A) {
    RowsPlan q;
    int rc = plan_idx_lb(S, dtype_in, m, 4, &q);
    if (rc != SK_OK) return rc;
    rc = plan_idx_lb(S, dtype_in, m, (m * es) % 16 == 0 ? 16 : 4, p);
    if (rc != SK_OK) return rc;
    p->partial_bytes = std::max(p->partial_bytes, q.partial_bytes);
    p->plan_bytes = std::max(p->plan_bytes, q.plan_bytes);
    return SK_OK;
  }
  const uintptr_t ap = (uintptr_t)A;
  if (ap % 16 == 0 && (lda * es) % 16 == 0 && (m * es) % 16 == 0)
    return plan_idx_lb(S, dtype_in, m, 16, p);
  if (ap % 4 == 0 && (lda * es) % 4 == 0 && (m * es) % 4 == 0) return plan_idx_lb(S, dtype_in, m, 4, p);
  set_error("sketch_apply: A must be 4-byte aligned with lda*elsize and m*elsize multiples of 4");
  return SK_E_NOTSUP;
}

template <typename Tin, int NREG, int LB, bool PARTS = false>
static int launch_idx_t(const sk_sketch* S, const RowsPlan& p, int64_t m, const void* A, int64_t lda, void* P,
                        const uint32_t* codes, hipStream_t st) {
  IdxArgs a;
  const int es = sizeof(Tin);
  a.A = (const unsigned char*)A;
  a.lda_bytes = lda * es;
  a.n = S->n;
  a.m = m;
  a.d = S->d;
  a.C = p.C;
  a.n_slabs = p.n_slabs;
  a.R = p.R;
  a.bpg = p.bpg;
  a.n_groups = p.n_groups;
  a.n_chunks = p.n_chunks;
  a.rows_per_chunk = p.rows_per_chunk;
  a.zeta = S->zeta;
  a.nb = (int)S->nb;
  a.P = P;
  a.buf_stride = p.rec_bytes;
  a.nbuf = p.nbuf;
  a.off_touch = p.nbuf * p.rec_bytes;
  a.codes_touch = (const unsigned char*)codes;
  a.nparts = p.nparts;
  a.ps = p.ps;
  a.lb = LB;
  const int64_t grid = ((int64_t)(p.n_chunks + 7) / 8) * 8 * p.n_slabs * p.n_groups;
  auto kern = ss_idx_kernel<Tin, NREG, LB, PARTS>;
  SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes));
  {
    KernelTimer timer(S, st);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * p.W), p.lds_bytes, st, a, codes);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename Tin, int LB>
static int launch_idx_n(const sk_sketch* S, const RowsPlan& p, int64_t m, const void* A, int64_t lda, void* P,
                        const uint32_t* codes, hipStream_t st) {
  switch (p.jb) {
    case 32:
      return launch_idx_t<Tin, 32, LB>(S, p, m, A, lda, P, codes, st);
    case 64:
      return launch_idx_t<Tin, 64, LB>(S, p, m, A, lda, P, codes, st);
    case 128:
      return launch_idx_t<Tin, 128, LB>(S, p, m, A, lda, P, codes, st);
    default:
      if (p.nparts > 1) return launch_idx_t<Tin, 200, LB, true>(S, p, m, A, lda, P, codes, st);
      return launch_idx_t<Tin, 200, LB>(S, p, m, A, lda, P, codes, st);
  }
}

// Codes of the n indices of S in tiles of R (the plan kernel above): used
// by the column-mode kernel, whose tiles run over the columns of A.
int launch_idx_codes(const sk_sketch* S, int dtype_in, int64_t n_tiles, int R, uint32_t* codes, hipStream_t st) {
  const uint32_t one_hi = dtype_in == SK_F64 ? IdxT<double>::one_hi : IdxT<float>::one_hi;
  const uint32_t rpa = dtype_in == SK_F64 ? 2u : 1u;
  const int64_t total = n_tiles * R * ((S->zeta + 3) / 4);
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(ss_idx_plan_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, S->n, n_tiles,
                     R, S->zeta, (uint32_t)S->nb, one_hi, rpa, S->k0, S->k1, codes);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

// Workspace: the partials (partial_bytes), then the row codes (plan_bytes).
int launch_idx_sketch(const sk_sketch* S, const RowsPlan& p, int dtype_in, int64_t m, const void* A, int64_t lda,
                      void* ws, hipStream_t st) {
  uint32_t* codes = (uint32_t*)((unsigned char*)ws + p.partial_bytes);
  const uint32_t one_hi = dtype_in == SK_F64 ? IdxT<double>::one_hi : IdxT<float>::one_hi;
  const uint32_t rpa = dtype_in == SK_F64 ? 2u : 1u;
  if (p.nparts > 1) {
    const int64_t total = p.n_tiles * p.R * ((S->zeta + 3) / 4);
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
    const uint32_t ndump = (uint32_t)dump_slots(dtype_in);
    const uint32_t dump0 = (uint32_t)(200 / (int)rpa) - ndump;
    hipLaunchKernelGGL(ss_idx_plan_parts_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st,
                       S->n, p.n_tiles, p.R, S->zeta, (uint32_t)S->nb, p.nparts, p.ps, dump0, ndump, one_hi, rpa,
                       S->k0, S->k1, codes);
    SK_HIP(hipGetLastError());
  } else {
    const int64_t total = p.n_tiles * p.R * ((S->zeta + 3) / 4);
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(ss_idx_plan_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, S->n,
                       p.n_tiles, p.R, S->zeta, (uint32_t)S->nb, one_hi, rpa, S->k0, S->k1, codes);
    SK_HIP(hipGetLastError());
  }
  void* P = ws;
  if (dtype_in == SK_F64)
    return p.load_bytes == 16 ? launch_idx_n<double, 16>(S, p, m, A, lda, P, codes, st)
                              : launch_idx_n<double, 4>(S, p, m, A, lda, P, codes, st);
  if (dtype_in == SK_F32)
    return p.load_bytes == 16 ? launch_idx_n<float, 16>(S, p, m, A, lda, P, codes, st)
                              : launch_idx_n<float, 4>(S, p, m, A, lda, P, codes, st);
  return p.load_bytes == 16 ? launch_idx_n<uint16_t, 16>(S, p, m, A, lda, P, codes, st)
                            : launch_idx_n<uint16_t, 4>(S, p, m, A, lda, P, codes, st);
}

// ---- batched sketches (host)
#define SK_IDX_TRY(expr)     \
  do {                       \
    const int _rc = (expr);  \
    if (_rc < 0) return _rc; \
  } while (0)
namespace {
// Codes and partials of one launch group: 16 GiB, or SKETCH_BATCH_AREA_MB
// (a smaller area splits a batch into more groups; the results do not change).
size_t batch_area_cap() {
  const int mb = env_i("SKETCH_BATCH_AREA_MB", 0);
  return mb > 0 ? (size_t)mb << 20 : (size_t)16 << 30;
}
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int batch_load_bytes(int dtype_in, int64_t k, const void* A, int64_t lda) {
  const int es = (int)dtype_size(dtype_in);
  const uintptr_t ap = (uintptr_t)A;
  if (ap % 16 == 0 && (lda * es) % 16 == 0 && (k * es) % 16 == 0) return 16;
  if (ap % 4 == 0 && (lda * es) % 4 == 0 && (k * es) % 4 == 0) return 4;
  return 0;
}

// A kernel variant and its launch shape: the jobs of one apply launch share it.
using BatchKey = std::tuple<int, int, int, int, int, int, size_t>;
struct BatchPlanned {
  RowsPlan p;
  BatchKey key;
  int64_t wg;            // workgroups of its apply
  size_t codes_bytes, partial_bytes;
};

// (the load width is an argument of the batched kernels: both widths share a launch)
BatchKey batch_key(int dtype_in, const RowsPlan& p) {
  return BatchKey(dtype_in, p.jb, 0, p.nparts, p.W, p.R, p.lds_bytes);
}

template <typename Tin, int NREG, int LB, bool PARTS>
int launch_variant(const IdxBatchEntry* tab, int nent, int64_t grid, int threads, size_t lds, const uint32_t* codes,
                   hipStream_t st) {
  auto kern = ss_idx_batched_kernel<Tin, NREG, LB, PARTS>;
  SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, st, tab, nent, codes);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename Tin, int LB, bool PARTS>
int launch_variant_n(int nreg, const IdxBatchEntry* tab, int nent, int64_t grid, int threads, size_t lds,
                     const uint32_t* codes, hipStream_t st) {
  if constexpr (PARTS) {
    return launch_variant<Tin, 200, LB, true>(tab, nent, grid, threads, lds, codes, st);
  } else {
    switch (nreg) {
      case 32:
        return launch_variant<Tin, 32, LB, false>(tab, nent, grid, threads, lds, codes, st);
      case 64:
        return launch_variant<Tin, 64, LB, false>(tab, nent, grid, threads, lds, codes, st);
      case 128:
        return launch_variant<Tin, 128, LB, false>(tab, nent, grid, threads, lds, codes, st);
      default:
        return launch_variant<Tin, 200, LB, false>(tab, nent, grid, threads, lds, codes, st);
    }
  }
}

template <typename Tin>
int launch_variant_t(const RowsPlan& p, const IdxBatchEntry* tab, int nent, int64_t grid, const uint32_t* codes,
                     hipStream_t st) {
  const int threads = 64 * p.W;
  return p.nparts > 1 ? launch_variant_n<Tin, 0, true>(p.jb, tab, nent, grid, threads, p.lds_bytes, codes, st)
                      : launch_variant_n<Tin, 0, false>(p.jb, tab, nent, grid, threads, p.lds_bytes, codes, st);
}

int plan_batch_job(const IdxBatchJob& j, BatchPlanned* out) {
  const int lb = batch_load_bytes(j.dtype, j.k, j.A, j.lda);
  if (lb == 0) {
    set_error("batched sketch: A must be 4-byte aligned with lda*elsize and k*elsize multiples of 4");
    return SK_E_NOTSUP;
  }
  SK_IDX_TRY(plan_idx_lb(j.S, j.dtype, j.k + 1, lb, &out->p, true, j.chunk_mult > 0 ? j.chunk_mult : 16));
  const RowsPlan& p = out->p;
  out->key = batch_key(j.dtype, p);
  out->wg = ((int64_t)(p.n_chunks + 7) / 8) * 8 * p.n_slabs * p.n_groups;
  out->codes_bytes = al256(p.plan_bytes);
  out->partial_bytes = al256(p.partial_bytes);
  return SK_OK;
}

// Consecutive jobs whose codes and partials fit the area together.
std::vector<std::pair<int, int>> batch_groups(const std::vector<BatchPlanned>& pl, size_t area) {
  std::vector<std::pair<int, int>> g;
  int first = 0;
  size_t used = 0;
  for (int i = 0; i < (int)pl.size(); ++i) {
    const size_t need = pl[i].codes_bytes + pl[i].partial_bytes;
    if (i > first && used + need > area) {
      g.push_back({first, i});
      first = i;
      used = 0;
    }
    used += need;
  }
  if (first < (int)pl.size()) g.push_back({first, (int)pl.size()});
  return g;
}

size_t batch_tables_bytes(int njobs) {
  return al256(sizeof(IdxBatchEntry) * (size_t)njobs) + al256(sizeof(IdxCodesEntry) * (size_t)njobs) +
         al256(sizeof(IdxReduceEntry) * (size_t)njobs);
}

int batch_plans(const IdxBatchJob* jobs, int njobs, std::vector<BatchPlanned>* pl, size_t* area) {
  pl->resize((size_t)njobs);
  size_t total = 0, mx = 0;
  for (int i = 0; i < njobs; ++i) {
    SK_IDX_TRY(plan_batch_job(jobs[i], &(*pl)[i]));
    const size_t need = (*pl)[i].codes_bytes + (*pl)[i].partial_bytes;
    total += need;
    mx = std::max(mx, need);
  }
  *area = std::max(std::min(total, batch_area_cap()), mx);
  return SK_OK;
}
}  // namespace

bool idx_batch_fits(const sk_sketch* S, int dtype_in, int64_t k, const void* A, int64_t lda) {
  if (env_i("SKETCH_IDX", 1) == 0) return false;
  return S->kind == SK_SPARSESTACK && k >= 4 && S->zeta >= 1 && batch_parts(dtype_in, S->nb) != 0 &&
         batch_load_bytes(dtype_in, k, A, lda) != 0;
}

int idx_batch_workspace(const IdxBatchJob* jobs, int njobs, size_t* bytes) {
  std::vector<BatchPlanned> pl;
  size_t area = 0;
  SK_IDX_TRY(batch_plans(jobs, njobs, &pl, &area));
  *bytes = batch_tables_bytes(njobs) + area;
  return SK_OK;
}

int idx_batch_prepare(const IdxBatchJob* jobs, int njobs, void* ws, size_t ws_bytes, IdxBatchProgram* prog) {
  prog->tables.clear();
  prog->launches.clear();
  prog->ws = ws;
  prog->njobs = njobs;
  if (njobs <= 0) return SK_OK;
  std::vector<BatchPlanned> pl;
  size_t area = 0;
  SK_IDX_TRY(batch_plans(jobs, njobs, &pl, &area));
  const size_t tables = batch_tables_bytes(njobs);
  if (!ws || ws_bytes < tables + area) {
    set_error("batched sketch: workspace too small");
    return SK_E_INVAL;
  }
  unsigned char* base = (unsigned char*)ws;
  const size_t off_codes_tab = al256(sizeof(IdxBatchEntry) * (size_t)njobs);
  const size_t off_red_tab = off_codes_tab + al256(sizeof(IdxCodesEntry) * (size_t)njobs);
  unsigned char* area_base = base + tables;
  std::vector<unsigned char>* stage = &prog->tables;
  stage->assign(tables, 0);
  IdxBatchEntry* h_ent = (IdxBatchEntry*)stage->data();
  IdxCodesEntry* h_cod = (IdxCodesEntry*)(stage->data() + off_codes_tab);
  IdxReduceEntry* h_red = (IdxReduceEntry*)(stage->data() + off_red_tab);

  // Per group of jobs (consecutive, codes and partials in the area
  // together): one codes launch, the applies by variant, the reductions by
  // partial type. Job i's codes entry is slot i; its apply and reduce
  // entries take slots of the group's range in launch order.
  using Launch = IdxBatchLaunch;
  std::vector<Launch>& launches = prog->launches;
  for (const auto& gr : batch_groups(pl, area)) {
    std::vector<size_t> part_off;
    size_t off = 0;
    int64_t blk = 0;
    for (int i = gr.first; i < gr.second; ++i) {
      const RowsPlan& p = pl[i].p;
      const sk_sketch* S = jobs[i].S;
      const int rpa = jobs[i].dtype == SK_F64 ? 2 : 1;
      IdxCodesEntry& e = h_cod[i];
      e.n = S->n;
      e.n_tiles = p.n_tiles;
      e.codes_off = (int64_t)(off / 4);
      e.blk_begin = blk;
      e.R = p.R;
      e.zeta = S->zeta;
      e.nparts = p.nparts;
      e.ps = p.ps;
      e.nb = (uint32_t)S->nb;
      e.ndump = (uint32_t)dump_slots(jobs[i].dtype);
      e.dump0 = (uint32_t)(200 / rpa) - e.ndump;
      e.one_hi = jobs[i].dtype == SK_F64 ? IdxT<double>::one_hi : IdxT<float>::one_hi;
      e.rpa = (uint32_t)rpa;
      e.k0 = S->k0;
      e.k1 = S->k1;
      const int64_t items = p.n_tiles * p.R * ((S->zeta + 3) / 4);
      blk += (items + 256 * kCodesPerThread - 1) / (256 * kCodesPerThread);
      off += pl[i].codes_bytes;
    }
    launches.push_back(Launch{0, gr.first, gr.second - gr.first, 0, blk, RowsPlan{}});
    for (int i = gr.first; i < gr.second; ++i) {
      part_off.push_back(off);
      off += pl[i].partial_bytes;
    }
    std::vector<int> order;
    for (int i = gr.first; i < gr.second; ++i) order.push_back(i);
    // by variant; within one, the problems with the longest row chunks first
    // (workgroups start in grid order, so the longest ones do not trail)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      if (pl[x].key != pl[y].key) return pl[x].key < pl[y].key;
      return pl[x].p.rows_per_chunk > pl[y].p.rows_per_chunk;
    });
    int slot = gr.first;
    for (size_t q = 0; q < order.size();) {
      const int first = slot;
      const BatchKey key = pl[order[q]].key;
      int64_t wg = 0;
      for (; q < order.size() && pl[order[q]].key == key; ++q) {
        const int i = order[q];
        const RowsPlan& p = pl[i].p;
        const IdxBatchJob& jb = jobs[i];
        IdxBatchEntry& e = h_ent[slot++];
        IdxArgs& a = e.a;
        a.A = (const unsigned char*)jb.A;
        a.lda_bytes = jb.lda * (int64_t)dtype_size(jb.dtype);
        a.n = jb.S->n;
        a.m = jb.k + 1;
        a.d = jb.S->d;
        a.C = p.C;
        a.n_slabs = p.n_slabs;
        a.R = p.R;
        a.bpg = p.bpg;
        a.n_groups = p.n_groups;
        a.n_chunks = p.n_chunks;
        a.rows_per_chunk = p.rows_per_chunk;
        a.zeta = jb.S->zeta;
        a.nb = (int)jb.S->nb;
        a.k0 = jb.S->k0;
        a.k1 = jb.S->k1;
        a.P = area_base + part_off[(size_t)(i - gr.first)];
        a.buf_stride = p.rec_bytes;
        a.nbuf = p.nbuf;
        a.off_touch = p.nbuf * p.rec_bytes;
        a.codes_touch = area_base + (size_t)h_cod[i].codes_off * 4;
        a.nparts = p.nparts;
        a.ps = p.ps;
        a.lb = p.load_bytes;
        e.b = (const unsigned char*)jb.b;
        e.codes_off = h_cod[i].codes_off;
        e.wg_begin = wg;
        wg += pl[i].wg;
      }
      launches.push_back(Launch{1, first, slot - first, jobs[order[first - gr.first]].dtype, wg,
                                pl[order[first - gr.first]].p});
    }
    slot = gr.first;
    for (int kind = 2; kind <= 3; ++kind) {
      const int first = slot;
      int64_t rblk = 0;
      for (int i = gr.first; i < gr.second; ++i) {
        if ((jobs[i].dtype == SK_F64) != (kind == 2)) continue;
        IdxReduceEntry& e = h_red[slot++];
        e.P = area_base + part_off[(size_t)(i - gr.first)];
        e.W = jobs[i].W;
        e.d = jobs[i].S->d;
        e.m = jobs[i].k + 1;
        e.ldw = jobs[i].S->d;
        e.n_chunks = pl[i].p.n_chunks;
        e.col_tiles = (int)((e.m + 63) / 64);
        e.scale = 1.0 / std::sqrt((double)jobs[i].S->zeta);
        e.blk_begin = rblk;
        rblk += ((e.d + 63) / 64) * e.col_tiles;
      }
      if (slot > first) launches.push_back(Launch{kind, first, slot - first, 0, rblk, RowsPlan{}});
    }
  }
  return SK_OK;
}

int idx_batch_enqueue(const IdxBatchProgram& prog, hipStream_t st) {
  if (prog.launches.empty()) return SK_OK;
  const int njobs = prog.njobs;
  unsigned char* base = (unsigned char*)prog.ws;
  const size_t off_codes_tab = al256(sizeof(IdxBatchEntry) * (size_t)njobs);
  const size_t off_red_tab = off_codes_tab + al256(sizeof(IdxCodesEntry) * (size_t)njobs);
  unsigned char* area_base = base + batch_tables_bytes(njobs);
  const IdxBatchEntry* d_ent = (const IdxBatchEntry*)base;
  const IdxCodesEntry* d_cod = (const IdxCodesEntry*)(base + off_codes_tab);
  const IdxReduceEntry* d_red = (const IdxReduceEntry*)(base + off_red_tab);
  uint32_t* codes = (uint32_t*)area_base;
  for (const auto& l : prog.launches) {
    if (l.grid <= 0) continue;
    if (l.kind == 0) {
      hipLaunchKernelGGL(ss_idx_plan_batched_kernel, dim3((unsigned)l.grid), dim3(256), 0, st, d_cod + l.first,
                         l.count, codes);
      SK_HIP(hipGetLastError());
    } else if (l.kind == 1) {
      const IdxBatchEntry* tab = d_ent + l.first;
      if (l.dtype == SK_F64)
        SK_IDX_TRY(launch_variant_t<double>(l.plan, tab, l.count, l.grid, codes, st));
      else if (l.dtype == SK_F32)
        SK_IDX_TRY(launch_variant_t<float>(l.plan, tab, l.count, l.grid, codes, st));
      else
        SK_IDX_TRY(launch_variant_t<uint16_t>(l.plan, tab, l.count, l.grid, codes, st));
    } else {
      if (l.kind == 2)
        hipLaunchKernelGGL(idx_reduce_batched_kernel<double>, dim3((unsigned)l.grid), dim3(256), 0, st,
                           d_red + l.first, l.count);
      else
        hipLaunchKernelGGL(idx_reduce_batched_kernel<float>, dim3((unsigned)l.grid), dim3(256), 0, st,
                           d_red + l.first, l.count);
      SK_HIP(hipGetLastError());
    }
  }
  return SK_OK;
}

int launch_idx_batch(const IdxBatchJob* jobs, int njobs, void* ws, size_t ws_bytes, IdxBatchProgram* prog,
                     hipStream_t st) {
  SK_IDX_TRY(idx_batch_prepare(jobs, njobs, ws, ws_bytes, prog));
  if (prog->launches.empty()) return SK_OK;
  SK_HIP(hipMemcpyAsync(ws, prog->tables.data(), prog->tables.size(), hipMemcpyHostToDevice, st));
  return idx_batch_enqueue(*prog, st);
}

}  // namespace sk
