// SparseStack apply, row mode: SA = S A for a tall row-major A (n x m).
//
// Def. 1.5: column i of S carries rho_it / sqrt(zeta) in row t*nb + s_it for
// each block t, so SA[t*nb + s, c] = (1/sqrt(zeta)) * sum_{i: s_it = s} rho_it A[i, c].
//
// Design (gfx950, one HBM pass over A):
//  * Plan kernel: for every tile of R rows and every block t, the Philox hash
//    gives (bucket, sign) of each row and one wave counting-sorts the rows by
//    bucket (stable, via wave ballots: no atomics). The result, bucket offsets
//    and the sorted row list, is a few KB per tile; it is computed once and
//    read by every workgroup that covers the tile.
//  * Sketch kernel: a workgroup owns a row chunk x a column slab (<= 64
//    columns, one per lane) x a group of blocks. It streams its rows through
//    LDS in tiles of R rows together with the tiles' plans, double-buffered
//    with direct global->LDS loads, so the prefetch of tile k+1 costs no VGPRs
//    and overlaps the work on tile k.
//  * Each wave owns one block and a contiguous range of its buckets and keeps
//    one accumulator per bucket per lane in registers. A block with more
//    buckets than one workgroup's 16 waves hold is split into bucket ranges
//    over several workgroups, each reading the tile. The first row of every
//    bucket is added by fully unrolled, branch-free code (an empty bucket reads
//    a zero row), so the LDS reads are independent and pipeline; the second
//    and third rows of every bucket are preloaded one per lane and added
//    behind scalar bit tests (one readlane each), and only buckets with four
//    or more rows walk the rest of their list. All lanes read one row at
//    consecutive columns: LDS reads are conflict-free.
//  * At the end of the chunk the accumulators go to a partial buffer
//    [chunk][d][m]; a second kernel sums the partials in chunk order and scales
//    by 1/sqrt(zeta). Summation order is fixed, so results are bitwise
//    reproducible.
#include "sk_launch.hpp"

#include <algorithm>
#include <cstdlib>

namespace sk {

__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
__device__ inline void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Direct global->LDS loads: each lane's bytes land at LDS address
// M0 + lane * width. They are issued from inline assembly so that the
// compiler's memory-counter bookkeeping does not make every later LDS access
// wait for them (it cannot tell that they target the other tile buffer); the
// kernel waits for them explicitly (wait_dma) before the barrier that
// publishes the tile. M0 is saved and restored around the load, with the one wait
// state the ISA asks for between a scalar write of M0 and an LDS-DMA load.
__device__ inline void dma_to_lds16(const void* gsrc, uint32_t lds_addr) {
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
__device__ inline void dma_to_lds4(const void* gsrc, uint32_t lds_addr) {
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
__device__ inline uint32_t lds_addr_of(const void* p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void*)p;
}

// ---------------------------------------------------------------------------
// Plan kernel
// ---------------------------------------------------------------------------
struct PlanArgs {
  int64_t n;
  int R, zeta, nb, nbits;
  uint32_t k0, k1;
  unsigned char* out;  // [tiles][zeta] records of rec_bytes
  int rec_bytes, lst_off;
  int runit;           // list entries carry row * runit
};

// Record of (tile, block t): u16 off[nb + 1] (bucket s holds list entries
// [off[s], off[s+1])), then at lst_off u32 lst[R]: the tile's rows sorted by
// bucket, stable, each entry (row * runit) | negative << 31. The row kernel
// uses runit = (LDS bytes of a tile row) / 8, so (entry << 3) is the row's LDS
// byte offset in the tile (the sign bit shifts out); the narrow kernel and
// the column mode use 1.
__global__ void __launch_bounds__(1024) ss_plan_kernel(PlanArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x, nwaves = nthreads >> 6;
  const int R = a.R, nb = a.nb, zeta = a.zeta;
  const int64_t tile = blockIdx.x;
  const int64_t r0 = tile * R;
  const int rv = (int)min((int64_t)R, a.n - r0);
  uint16_t* codes = (uint16_t*)smem;                          // [zeta][R]
  uint16_t* rnk = codes + (size_t)zeta * R;                   // [zeta][R]
  uint32_t* cnts = (uint32_t*)(rnk + (size_t)zeta * R + ((zeta * R) & 1));  // [waves][nb + 1]

  // Hash: one Philox call gives the words of blocks 4g .. 4g+3 of one row.
  const int ng = (zeta + 3) / 4;
  for (int pi = tid; pi < rv * ng; pi += nthreads) {
    const int g = pi / rv, r = pi - g * rv;
    const uint64_t i = (uint64_t)(r0 + r);
    const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)g, kTagSparseStack}, a.k0, a.k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * g + j;
      if (t < zeta) {
        const uint32_t word = word_of(w, j);
        codes[t * R + r] = (uint16_t)((ss_bucket(word, (uint32_t)nb) << 1) | ss_negative(word));
      }
    }
  }
  lds_barrier();

  // Stable counting sort of block t's rows by bucket, one wave per block;
  // a wave reuses its count array for its next block.
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t* cnt = cnts + (size_t)wave * (nb + 1);
  for (int t = wave; t < zeta; t += nwaves) {
    const uint16_t* cd = codes + t * R;
    uint16_t* rk = rnk + t * R;
    for (int s = lane; s <= nb; s += 64) cnt[s] = 0;
    for (int c0 = 0; c0 < rv; c0 += 64) {
      const int r = c0 + lane;
      const bool valid = r < rv;
      const uint32_t s = valid ? (uint32_t)(cd[r] >> 1) : 0u;
      uint64_t mask = __ballot(valid);
      for (int b = 0; b < a.nbits; ++b) {
        const bool bit = (s >> b) & 1u;
        const uint64_t mb = __ballot(bit);
        mask &= bit ? mb : ~mb;
      }
      const uint32_t rank = (uint32_t)__popcll(mask & below);
      const uint32_t base = valid ? cnt[s] : 0u;
      if (valid) rk[r] = (uint16_t)(base + rank);
      if (valid && rank == 0) cnt[s] = base + (uint32_t)__popcll(mask);
    }
    // exclusive scan of the counts
    const int per = (nb + 63) / 64;
    const int sb = lane * per;
    uint32_t loc = 0;
    for (int k = 0; k < per; ++k)
      if (sb + k < nb) loc += cnt[sb + k];
    uint32_t inc = loc;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    unsigned char* rec = a.out + (tile * zeta + t) * (int64_t)a.rec_bytes;
    uint16_t* gof = (uint16_t*)rec;
    uint32_t* glst = (uint32_t*)(rec + a.lst_off);
    uint32_t run = inc - loc;
    for (int k = 0; k < per; ++k) {
      if (sb + k < nb) {
        const uint32_t c = cnt[sb + k];
        cnt[sb + k] = run;
        gof[sb + k] = (uint16_t)run;
        run += c;
      }
    }
    if (lane == 63) gof[nb] = (uint16_t)inc;
    // scatter (stable: rank order = row order within a bucket)
    for (int c0 = 0; c0 < rv; c0 += 64) {
      const int r = c0 + lane;
      if (r < rv) {
        const uint32_t code = cd[r];
        const uint32_t rkr = rk[r];
        glst[cnt[code >> 1] + rkr] = ((uint32_t)r * (uint32_t)a.runit) | ((code & 1u) << 31);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Sketch kernel
// ---------------------------------------------------------------------------
struct RowsArgs {
  const unsigned char* A;
  int64_t lda_bytes;
  int64_t n, m, d;
  int C, n_slabs, R, bpg, n_groups, H, per_range, n_chunks;
  int ranges;  // bucket-range groups per block: group g takes blocks from g / ranges, range g % ranges
  int64_t rows_per_chunk;
  int zeta, nb;
  const unsigned char* plan;
  int rec_bytes, lst_off;
  void* P;
  int buf_stride, off_zero, off_plan, plan_dma_bytes, off_xtra;
  int rowb;  // LDS bytes of a tile row: the slab's columns, rounded up to 16
  // Direct loads: load k of a tile covers tile bytes [k*64*LB, (k+1)*64*LB);
  // a wave issues loads wave, wave + W, ... so from one of its loads to the
  // next every lane advances by step_rows rows and step_cb bytes (step_cb <
  // rowb), with a carry into the row when the byte offset passes rowb.
  int step_rows, step_cb;
  uint32_t rowb_magic;  // ceil(2^32 / rowb): x / rowb = umulhi(x, rowb_magic) for x < 2^23
};

template <typename Tin>
struct InType;
template <>
struct InType<double> {
  using acc = double;
};
template <>
struct InType<float> {
  using acc = float;
};
template <>
struct InType<uint16_t> {  // bf16
  using acc = float;
};

// acc += (+-1) * tile value for a list entry e: the row's LDS address is
// (e << 3) + base, base = buffer address + lane * element size (one
// v_lshl_add); the sign is applied by flipping the value's sign bit (one
// v_xor), and the add rounds once, exactly like acc + (+-v).
typedef __attribute__((address_space(3))) const unsigned char* lds_cptr;

template <typename Tin>
__device__ inline typename InType<Tin>::acc lds_val(uint32_t addr);
template <>
__device__ inline double lds_val<double>(uint32_t addr) {
  return *(const __attribute__((address_space(3))) double*)(lds_cptr)(uintptr_t)addr;
}
template <>
__device__ inline float lds_val<float>(uint32_t addr) {
  return *(const __attribute__((address_space(3))) float*)(lds_cptr)(uintptr_t)addr;
}
template <>
__device__ inline float lds_val<uint16_t>(uint32_t addr) {
  return bf16_to_f32(*(const __attribute__((address_space(3))) uint16_t*)(lds_cptr)(uintptr_t)addr);
}
// (+-1) * v for a list entry e: flip the sign bit of v with bit 31 of e.
__device__ inline double flip(double v, uint32_t e) {
  return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)(e & 0x80000000u) << 32));
}
__device__ inline float flip(float v, uint32_t e) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ (e & 0x80000000u));
}

template <typename Tin, int JB, int LB>
__global__ void __launch_bounds__(1024) ss_rows_kernel(RowsArgs a) {
  using Tacc = typename InType<Tin>::acc;
  constexpr int ES = sizeof(Tin);
  constexpr int ZROWB = 64 * ES;  // LDS bytes of the zero row (one value per lane)
  static_assert(JB <= 64, "one bucket per lane");
  // The kernel declares no static LDS, so this dynamic segment starts at LDS
  // address 0. Tile rows are packed at a stride of a.rowb bytes (the slab's
  // columns only), so a tile holds as many rows as its bytes allow; lanes
  // past the slab read the next row or the zero row, and their sums are
  // never written.
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x, nwaves = nthreads >> 6;

  // Work item. Dispatch is round-robin over the 8 XCDs (id L runs on XCD
  // L % 8), so all column slabs and block groups of one row chunk get ids
  // 8 apart: they run together on one XCD and share its L2 for the plans and
  // the cache lines that straddle slab boundaries.
  const int L = blockIdx.x, xcd = L & 7, q8 = L >> 3;
  const int group = q8 % a.n_groups;
  const int slab = (q8 / a.n_groups) % a.n_slabs;
  const int chunk = (q8 / (a.n_groups * a.n_slabs)) * 8 + xcd;
  if (chunk >= a.n_chunks) return;

  const int rg = group % a.ranges;
  const int t0 = (group / a.ranges) * a.bpg;
  const int bpg = min(a.bpg, a.zeta - t0);
  const int64_t col0 = (int64_t)slab * a.C;
  const int Cw = (int)min((int64_t)a.C, a.m - col0);
  const int slab_bytes = Cw * ES;
  const int64_t r_begin = (int64_t)chunk * a.rows_per_chunk;
  const int64_t r_end = min(a.n, r_begin + a.rows_per_chunk);
  const int nsub = r_end > r_begin ? (int)((r_end - r_begin + a.R - 1) / a.R) : 0;
  const int R = a.R, nb = a.nb;

  const int tl = wave / a.H, hr = wave - (wave / a.H) * a.H;
  const bool walker = tl < bpg;
  const int s_begin = (rg * a.H + hr) * a.per_range;
  const int s_cnt = walker ? max(0, min(a.per_range, nb - s_begin)) : 0;

  Tacc acc[JB];
#pragma unroll
  for (int j = 0; j < JB; ++j) acc[j] = 0;

  // zero rows (empty buckets read them), one after each tile buffer
  for (int i = tid; i < 2 * (ZROWB / 4); i += nthreads) {
    const int b = i / (ZROWB / 4);
    ((uint32_t*)(smem + b * a.buf_stride + a.off_zero))[i - b * (ZROWB / 4)] = 0u;
  }

  const int rowb = a.rowb;
  const int n_instr = (R * rowb + 64 * LB - 1) / (64 * LB);

  auto issue_loads = [&](int st, int buf) {
    const int64_t r0 = r_begin + (int64_t)st * R;
    const int rv = (int)min((int64_t)R, r_end - r0);
    unsigned char* dst = smem + buf * a.buf_stride;
    const unsigned char* tsrc = a.A + r0 * a.lda_bytes + col0 * ES;
    // (row, byte in row) of this lane in the wave's first load; later loads
    // advance incrementally. Recomputed per tile (a multiply-high; the byte
    // offset is below 2^14 and rowb at most 512, so the quotient is exact)
    // rather than kept live across the tile loop.
    uint32_t fb = (uint32_t)(wave * 64 + lane) * LB;
    asm volatile("" : "+v"(fb));
    int row = (int)__umulhi(fb, a.rowb_magic);
    int cb = (int)fb - row * rowb;
    for (int k = wave; k < n_instr; k += nwaves) {
      const unsigned char* src = a.A;  // in-bounds stand-in for padding lanes
      if (row < rv && cb < slab_bytes) src = tsrc + (int64_t)row * a.lda_bytes + cb;
      const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane((int)lds_addr_of(dst + k * 64 * LB));
      // lanes past the tile (row >= R) stay inactive: their slots hold the zero row
      if (row < R) {
        if constexpr (LB == 16)
          dma_to_lds16(src, la);
        else
          dma_to_lds4(src, la);
      }
      row += a.step_rows;
      cb += a.step_cb;
      if (cb >= rowb) {
        cb -= rowb;
        row += 1;
      }
    }
    // the tile's plan records for this group's blocks (contiguous)
    const unsigned char* psrc = a.plan + ((r0 / R) * a.zeta + t0) * (int64_t)a.rec_bytes;
    unsigned char* pdst = dst + a.off_plan;
    // lane * 16 is recomputed here rather than kept live across the tile
    // loop: that would take a register the accumulators need
    int l16 = lane * 16;
    asm volatile("" : "+v"(l16));
    for (int k = wave; k * 1024 < a.plan_dma_bytes; k += nwaves) {
      const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane((int)lds_addr_of(pdst + k * 1024));
      dma_to_lds16(psrc + k * 1024 + l16, la);
    }
  };

  if (nsub > 0) issue_loads(0, 0);
  for (int st = 0; st < nsub; ++st) {
    const int buf = st & 1;
    wait_dma();
    lds_barrier();  // tile st and its plan are in LDS; everyone finished tile st-1
    if (st + 1 < nsub) issue_loads(st + 1, buf ^ 1);

    // Segmented reduction. Wave (block tl, buckets [s_begin, s_begin + s_cnt)):
    // lane j describes bucket s_begin + j.
    if (walker) {
      int sc = s_cnt;
      asm volatile("" : "+s"(sc));
      const unsigned char* pl = smem + buf * a.buf_stride + a.off_plan + tl * a.rec_bytes;
      const uint16_t* of = (const uint16_t*)pl;
      const uint32_t* lst = (const uint32_t*)(pl + a.lst_off);
      uint32_t base = lds_addr_of(smem + buf * a.buf_stride) + (uint32_t)(lane * ES);
      asm volatile("" : "+v"(base));  // one register: keeps the address to one v_lshl_add
      const uint32_t zentry = (uint32_t)a.off_zero >> 3;
      uint32_t kbeg = 0, kcnt = 0;
      if (lane < sc) {
        kbeg = of[s_begin + lane];
        kcnt = (uint32_t)of[s_begin + lane + 1] - kbeg;
      }
      const uint32_t e0 = kcnt >= 1 ? lst[kbeg] : zentry;
      // first rows of all buckets: unrolled and branch-free (lanes past the
      // wave's range, like empty buckets, point at the zero row), GB loads
      // in flight before their adds (GB bounded by the register budget)
      constexpr int GB = 8;
#pragma unroll
      for (int g = 0; g < JB; g += GB) {
        Tacc v[GB];
        uint32_t ev[GB];
#pragma unroll
        for (int u = 0; u < GB; ++u) {
          if (g + u < JB) {
            ev[u] = (uint32_t)__builtin_amdgcn_readlane((int)e0, g + u);
            v[u] = lds_val<Tin>((ev[u] << 3) + base);
          }
        }
#pragma unroll
        for (int u = 0; u < GB; ++u)
          if (g + u < JB) acc[g + u] += flip(v[u], ev[u]);
        // the adds happen here, not sunk into later code
#pragma unroll
        for (int u = 0; u < GB; ++u)
          if (g + u < JB) asm volatile("" : "+v"(acc[g + u]));
        __builtin_amdgcn_sched_barrier(0);
      }

      // further rows. The second and third entries of every bucket are
      // preloaded one per lane (like the first), so the common cases (two or
      // three rows) take one readlane each; buckets with four or more rows
      // walk the rest of their list. Bucket tests are bit tests of ballots
      // kept in scalar registers.
      const uint32_t e1 = kcnt >= 2 ? lst[kbeg + 1] : zentry;
      const uint32_t e2 = kcnt >= 3 ? lst[kbeg + 2] : zentry;
      uint64_t m2 = __ballot(kcnt >= 2), m3 = __ballot(kcnt >= 3), m4 = __ballot(kcnt >= 4);
      asm volatile("" : "+s"(m2), "+s"(m3), "+s"(m4));
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        if (m2 & (1ull << j)) {
          const uint32_t ea = (uint32_t)__builtin_amdgcn_readlane((int)e1, j);
          acc[j] += flip(lds_val<Tin>((ea << 3) + base), ea);
          if (m3 & (1ull << j)) {
            const uint32_t eb = (uint32_t)__builtin_amdgcn_readlane((int)e2, j);
            acc[j] += flip(lds_val<Tin>((eb << 3) + base), eb);
            if (m4 & (1ull << j)) {
              const uint32_t kb = (uint32_t)__builtin_amdgcn_readlane((int)kbeg, j);
              const uint32_t ke = kb + (uint32_t)__builtin_amdgcn_readlane((int)kcnt, j);
              for (uint32_t k = kb + 3; k < ke; ++k) {
                const uint32_t ec = lst[k];
                acc[j] += flip(lds_val<Tin>((ec << 3) + base), ec);
              }
            }
          }
        }
      }
    }
  }

  if (walker && lane < Cw) {
    Tacc* P = (Tacc*)a.P;
    const int64_t rowbase = (int64_t)chunk * a.d + (int64_t)(t0 + tl) * nb + s_begin;
#pragma unroll
    for (int j = 0; j < JB; ++j)
      if (j < s_cnt) P[(rowbase + j) * a.m + col0 + lane] = acc[j];
  }
}

// Narrow inputs (m <= 4 columns, e.g. the right-hand side b): one lane per
// output row of S (bucket s of block t) walks that bucket's list in the
// tile's plan, so no lane idles on absent columns. A workgroup owns a chunk
// of consecutive tiles; per tile it stages the rows' values (converted to
// the accumulation type) and the tile's plan records in LDS. Sums run in
// list order (row order) and chunks are added in order: deterministic.
struct NarrowArgs {
  const unsigned char* A;
  int64_t lda_bytes, n, d;
  int m, R, zeta, nb;
  const unsigned char* plan;
  int rec_bytes, lst_off;
  int64_t n_tiles, tiles_per_chunk;
  void* P;
};

template <typename Tin>
__device__ inline typename InType<Tin>::acc load_in(const unsigned char* p);
template <>
__device__ inline double load_in<double>(const unsigned char* p) { return *(const double*)p; }
template <>
__device__ inline float load_in<float>(const unsigned char* p) { return *(const float*)p; }
template <>
__device__ inline float load_in<uint16_t>(const unsigned char* p) { return bf16_to_f32(*(const uint16_t*)p); }

template <typename Tin, int MV>
__global__ void __launch_bounds__(1024) ss_narrow_kernel(NarrowArgs a) {
  using Tacc = typename InType<Tin>::acc;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  Tacc* vals = (Tacc*)smem;  // [R][MV]
  unsigned char* pl = smem + (((size_t)a.R * MV * sizeof(Tacc) + 15) & ~(size_t)15);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t tb = (int64_t)blockIdx.x * a.tiles_per_chunk;
  const int64_t te = min(a.n_tiles, tb + a.tiles_per_chunk);
  Tacc acc[4][MV];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < MV; ++c) acc[q][c] = 0;
  const int es = (int)sizeof(Tin);
  for (int64_t tile = tb; tile < te; ++tile) {
    const int64_t r0 = tile * a.R;
    const int rv = (int)min((int64_t)a.R, a.n - r0);
    for (int idx = tid; idx < rv * a.m; idx += nt) {
      const int row = idx / a.m, c = idx - row * a.m;
      vals[row * MV + c] = load_in<Tin>(a.A + (r0 + row) * a.lda_bytes + (int64_t)c * es);
    }
    const uint4* src = (const uint4*)(a.plan + tile * a.zeta * (int64_t)a.rec_bytes);
    uint4* dst = (uint4*)pl;
    const int n16 = a.zeta * a.rec_bytes / 16;
    for (int idx = tid; idx < n16; idx += nt) dst[idx] = src[idx];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = tid + (int64_t)q * nt;
      if (j < a.d) {
        const int t = (int)(j / a.nb), s = (int)(j - (int64_t)t * a.nb);
        const unsigned char* rec = pl + t * a.rec_bytes;
        const uint16_t* of = (const uint16_t*)rec;
        const uint32_t* lst = (const uint32_t*)(rec + a.lst_off);
        const int kb = of[s], ke = of[s + 1];
        for (int k = kb; k < ke; ++k) {
          const uint32_t e = lst[k];
          const Tacc* vr = vals + (e & 0x7fffffffu) * MV;
#pragma unroll
          for (int c = 0; c < MV; ++c) acc[q][c] += (e >> 31) ? -vr[c] : vr[c];
        }
      }
    }
    __syncthreads();
  }
  Tacc* P = (Tacc*)a.P;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t j = tid + (int64_t)q * nt;
    if (j < a.d) {
#pragma unroll
      for (int c = 0; c < MV; ++c)
        if (c < a.m) P[((int64_t)blockIdx.x * a.d + j) * a.m + c] = acc[q][c];
    }
  }
}

// SA[j, c] = scale * sum_w P[w][j][c], w in increasing order.
template <typename Tacc, typename Tout>
__global__ void reduce_partials_kernel(const Tacc* __restrict__ P, int n_chunks, int64_t d, int64_t m, Tacc scale,
                                       Tout* __restrict__ out, int64_t ldo) {
  const int64_t total = d * m;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx / m, c = idx - j * m;
    Tacc s = 0;
    for (int w = 0; w < n_chunks; ++w) s += P[((int64_t)w * d + j) * m + c];
    out[j * ldo + c] = (Tout)(s * scale);
  }
}

__global__ void ss_pattern_kernel(int64_t n, int zeta, uint32_t nb, uint32_t k0, uint32_t k1, int32_t* bucket,
                                  int8_t* sign) {
  const int ng = (zeta + 3) / 4;
  const int64_t total = n * ng;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t i = (uint64_t)(idx / ng);
    const int g = (int)(idx % ng);
    const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)g, kTagSparseStack}, k0, k1);
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * g + j;
      if (t < zeta) {
        const uint32_t word = word_of(w, j);
        bucket[i * zeta + t] = (int32_t)ss_bucket(word, nb);
        sign[i * zeta + t] = ss_negative(word) ? (int8_t)-1 : (int8_t)1;
      }
    }
  }
}

// Z[i, c] = sum_t rho_it / sqrt(zeta) * Y[t*nb + s_it, c]  (S^T Y, a test helper)
__global__ void ss_adjoint_kernel(int64_t n, int64_t m, int zeta, uint32_t nb, uint32_t k0, uint32_t k1,
                                  double scale, const double* __restrict__ Y, int64_t ldy, double* __restrict__ Z,
                                  int64_t ldz) {
  const int64_t total = n * m;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t i = (uint64_t)(idx / m);
    const int64_t c = idx % m;
    double s = 0;
    for (int g = 0; g < (zeta + 3) / 4; ++g) {
      const U4 w = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)g, kTagSparseStack}, k0, k1);
      for (int j = 0; j < 4; ++j) {
        const int t = 4 * g + j;
        if (t < zeta) {
          const uint32_t word = word_of(w, j);
          const double y = Y[((int64_t)t * nb + ss_bucket(word, nb)) * ldy + c];
          s += ss_negative(word) ? -y : y;
        }
      }
    }
    Z[(int64_t)i * ldz + c] = s * scale;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }
static size_t align1k(size_t x) { return (x + 1023) & ~(size_t)1023; }

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Plan record of one (tile, block): u16 offsets [nb + 1], then u32 list [R]
// and one spare slot (the row kernel reads entries in pairs).
static void plan_record(int R, int64_t nb, int* rec_bytes, int* lst_off) {
  *lst_off = (int)align16((size_t)(nb + 1) * 2);
  *rec_bytes = (int)align16((size_t)*lst_off + (size_t)(R + 1) * 4);
}

// LDS layout of the sketch kernel. Per buffer (x2): R tile rows, one zero
// row, the plan records of the group's blocks (padded to whole 1 KB load
// instructions).
struct RowsLds {
  size_t tile, zero, plan, plan_dma, buf_stride, xtra, total;
};
static RowsLds rows_lds(int es, int R, int rowb, int bpg, int rec_bytes, int W) {
  RowsLds l;
  l.tile = (size_t)R * rowb;
  l.zero = l.tile;
  l.plan = align16(l.zero + (size_t)64 * es);
  l.plan_dma = align1k((size_t)bpg * rec_bytes);
  l.buf_stride = align16(l.plan + l.plan_dma);
  l.xtra = 2 * l.buf_stride;
  l.total = l.xtra;
  (void)W;
  return l;
}

// Accumulator slots compiled into the kernel variants (per lane, per wave).
static int jb_max(int dtype_in) { return dtype_in == SK_F64 ? 50 : 64; }
static int jb_variant(int dtype_in, int per_range) {
  if (per_range <= 16) return 16;
  if (per_range <= 32) return 32;
  return jb_max(dtype_in);
}

// LDS of the narrow kernel (values + the tile's plan records) and of the plan
// kernel for a tile of R rows.
static size_t narrow_lds(int R, int accb, int zeta, int rec_bytes) {
  return align16((size_t)R * 4 * accb) + (size_t)zeta * rec_bytes;
}
// The plan kernel runs one wave per block (at most 16), fewer where the
// waves' count arrays would not fit in LDS.
static int plan_waves(int R, int zeta, int64_t nb) {
  const size_t fixed = align16((size_t)2 * zeta * R * 2 + 4);
  int nw = std::min(16, zeta);
  while (nw > 1 && fixed + (size_t)nw * (nb + 1) * 4 > 160 * 1024) --nw;
  return nw;
}
size_t plan_kernel_lds(int R, int zeta, int64_t nb) {
  return align16((size_t)2 * zeta * R * 2 + 4) + (size_t)plan_waves(R, zeta, nb) * (nb + 1) * 4;
}
static size_t plan_lds(int R, int zeta, int64_t nb) { return plan_kernel_lds(R, zeta, nb); }

static int plan_narrow(const sk_sketch* S, int dtype_in, int64_t m, RowsPlan* p) {
  const size_t cap = 160 * 1024;
  const int accb = dtype_in == SK_F64 ? 8 : 4;
  int R = 2048;
  for (;;) {
    plan_record(R, S->nb, &p->rec_bytes, &p->lst_off);
    if ((narrow_lds(R, accb, S->zeta, p->rec_bytes) <= cap && plan_lds(R, S->zeta, S->nb) <= cap) || R <= 64) break;
    R /= 2;
  }
  if (narrow_lds(R, accb, S->zeta, p->rec_bytes) > cap || plan_lds(R, S->zeta, S->nb) > cap) {
    set_error("sketch_apply: zeta * (d/zeta) too large for the narrow-input plan");
    return SK_E_NOTSUP;
  }
  p->narrow = true;
  p->R = R;
  p->C = (int)m;
  p->n_slabs = 1;
  p->n_tiles = (S->n + R - 1) / R;
  const int64_t target = env_int("SKETCH_WG_TARGET", 256);
  int64_t tpc = std::max<int64_t>(1, (p->n_tiles + target - 1) / target);
  p->tiles_per_chunk = tpc;
  p->n_chunks = (int)((p->n_tiles + tpc - 1) / tpc);
  p->rows_per_chunk = tpc * R;
  p->lds_bytes = narrow_lds(R, accb, S->zeta, p->rec_bytes);
  p->partial_bytes = align16((size_t)p->n_chunks * S->d * m * accb);
  p->plan_bytes = align16((size_t)p->n_tiles * S->zeta * p->rec_bytes);
  return SK_OK;
}

int plan_rows(const sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, RowsPlan* p) {
  const int es = (int)dtype_size(dtype_in);
  const int zeta = S->zeta;
  const int64_t nb = S->nb;
  if (m <= 4 && S->d <= 4096 && nb <= 16383) return plan_narrow(S, dtype_in, m, p);
  if (idx_apply_fits(S, dtype_in, m)) return plan_idx(S, dtype_in, m, A, lda, p);
  if (nb > 16384) {
    set_error("SparseStack row apply supports at most 16384 buckets per block");
    return SK_E_NOTSUP;
  }
  const int jmax = jb_max(dtype_in);
  const int Hmin = (int)((nb + jmax - 1) / jmax);
  p->ranges = 1;
  if (Hmin > 16) {
    // more buckets than one workgroup's 16 waves hold in registers: each
    // block's buckets are split over `ranges` workgroups (each reads the
    // tile; one block per workgroup)
    p->ranges = (Hmin + 15) / 16;
    p->bpg = 1;
    p->H = 16;
    p->n_groups = zeta * p->ranges;
  } else if ((int64_t)zeta * Hmin <= 16) {
    p->bpg = zeta;
    p->n_groups = 1;
    p->H = std::max(Hmin, (int)std::min<int64_t>(nb, 16 / zeta));
  } else {
    p->bpg = 16 / Hmin;
    p->n_groups = (zeta + p->bpg - 1) / p->bpg;
    p->H = Hmin;
  }
  p->W = p->bpg * p->H;
  p->per_range = (int)((nb + (int64_t)p->H * p->ranges - 1) / ((int64_t)p->H * p->ranges));
  p->jb = jb_variant(dtype_in, p->per_range);

  // direct global->LDS load width
  const uintptr_t ap = (uintptr_t)A;
  if (ap % 16 == 0 && (lda * es) % 16 == 0 && (m * es) % 16 == 0) {
    p->load_bytes = 16;
  } else if (ap % 4 == 0 && (lda * es) % 4 == 0 && (m * es) % 4 == 0) {
    p->load_bytes = 4;
  } else {
    set_error("sketch_apply: A must be 4-byte aligned with lda*elsize and m*elsize multiples of 4");
    return SK_E_NOTSUP;
  }
  // column slabs: at most 64 columns, each slab a whole number of load units
  const int cal = std::max(1, p->load_bytes / es);
  int ns = (int)((m + 63) / 64);
  int C = (int)((m + ns - 1) / ns);
  C = ((C + cal - 1) / cal) * cal;
  if (C > 64) C = 64;
  p->C = C;
  p->n_slabs = (int)((m + C - 1) / C);
  p->rowb = (int)align16((size_t)C * es);

  // tile rows: about 64 KB per buffer, shrunk until the LDS plan of the
  // sketch kernel and that of the plan kernel fit
  int R = env_int("SKETCH_TILE_ROWS", 65536 / p->rowb);
  const size_t lds_cap = 160 * 1024;
  for (;;) {
    plan_record(R, nb, &p->rec_bytes, &p->lst_off);
    if ((rows_lds(es, R, p->rowb, p->bpg, p->rec_bytes, p->W).total <= lds_cap && plan_lds(R, zeta, nb) <= lds_cap) ||
        R <= 16)
      break;
    R = R * 7 / 8;
  }
  p->R = R;
  p->lds_bytes = rows_lds(es, R, p->rowb, p->bpg, p->rec_bytes, p->W).total;
  if (p->lds_bytes > lds_cap || plan_lds(R, zeta, nb) > lds_cap) {
    set_error("sketch_apply: LDS plan does not fit");
    return SK_E_NOTSUP;
  }
  const int64_t n = S->n;
  const int64_t items = (int64_t)p->n_slabs * p->n_groups;
  const int target = env_int("SKETCH_WG_TARGET", 256);
  int64_t nc = std::max<int64_t>(1, (target + items - 1) / items);
  // chunk c runs on XCD c mod 8: at least 8 chunks, a multiple of 8, so that
  // no XCD idles (wide inputs have many slabs and would otherwise get one)
  nc = ((std::max<int64_t>(nc, 8) + 7) / 8) * 8;
  nc = std::min<int64_t>(nc, (n + p->R - 1) / p->R);
  int64_t rpc = (n + nc - 1) / nc;
  rpc = ((rpc + p->R - 1) / p->R) * p->R;
  p->rows_per_chunk = rpc;
  p->n_chunks = (int)((n + rpc - 1) / rpc);
  p->n_tiles = (n + p->R - 1) / p->R;
  const size_t accb = dtype_in == SK_F64 ? 8 : 4;
  p->partial_bytes = align16((size_t)p->n_chunks * S->d * m * accb);
  // the last tile's DMA may read up to one padded record span past its end
  p->plan_bytes = align16((size_t)p->n_tiles * zeta * p->rec_bytes) + align1k((size_t)p->bpg * p->rec_bytes);
  return SK_OK;
}

// Bucket plans of every tile of R consecutive indices (rows of A in row mode,
// columns of A in column mode).
int launch_plan_generic(const sk_sketch* S, int R, int rec_bytes, int lst_off, int64_t n_tiles, void* plan,
                        int runit, hipStream_t st) {
  PlanArgs a;
  a.n = S->n;
  a.R = R;
  a.zeta = S->zeta;
  a.nb = (int)S->nb;
  int nbits = 0;
  while ((1ll << nbits) < S->nb) ++nbits;
  a.nbits = nbits;
  a.k0 = S->k0;
  a.k1 = S->k1;
  a.out = (unsigned char*)plan;
  a.rec_bytes = rec_bytes;
  a.lst_off = lst_off;
  a.runit = runit;
  const int threads = 64 * plan_waves(R, S->zeta, S->nb);
  const size_t lds = plan_lds(R, S->zeta, S->nb);
  SK_HIP(hipFuncSetAttribute((const void*)ss_plan_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(ss_plan_kernel, dim3((unsigned)n_tiles), dim3(threads), lds, st, a);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

static int launch_plan(const sk_sketch* S, const RowsPlan& p, void* plan, int runit, hipStream_t st) {
  return launch_plan_generic(S, p.R, p.rec_bytes, p.lst_off, p.n_tiles, plan, runit, st);
}

template <typename Tin, int JB, int LB>
static int launch_rows_t(const sk_sketch* S, const RowsPlan& p, int64_t m, const void* A, int64_t lda, void* P,
                         const void* plan, hipStream_t st) {
  RowsArgs a;
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
  a.ranges = p.ranges;
  a.H = p.H;
  a.per_range = p.per_range;
  a.n_chunks = p.n_chunks;
  a.rows_per_chunk = p.rows_per_chunk;
  a.zeta = S->zeta;
  a.nb = (int)S->nb;
  a.plan = (const unsigned char*)plan;
  a.rec_bytes = p.rec_bytes;
  a.lst_off = p.lst_off;
  a.P = P;
  const RowsLds l = rows_lds(es, p.R, p.rowb, p.bpg, p.rec_bytes, p.W);
  a.rowb = p.rowb;
  {
    const int step = 64 * p.W * p.load_bytes;
    a.step_rows = step / p.rowb;
    a.step_cb = step % p.rowb;
    a.rowb_magic = (uint32_t)(((1ull << 32) + (uint64_t)p.rowb - 1) / (uint64_t)p.rowb);
  }
  a.buf_stride = (int)l.buf_stride;
  a.off_zero = (int)l.zero;
  a.off_plan = (int)l.plan;
  a.plan_dma_bytes = (int)l.plan_dma;
  a.off_xtra = (int)l.xtra;
  const int64_t grid = ((int64_t)(p.n_chunks + 7) / 8) * 8 * p.n_slabs * p.n_groups;
  auto kern = ss_rows_kernel<Tin, JB, LB>;
  SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes));
  {
    KernelTimer timer(S, st);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * p.W), p.lds_bytes, st, a);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename Tacc, typename Tout>
static int launch_reduce(const RowsPlan& p, const sk_sketch* S, int64_t m, const void* P, void* out, int64_t ldo,
                         hipStream_t st) {
  const int64_t total = S->d * m;
  const int threads = 256;
  const int64_t blocks = std::min<int64_t>((total + threads - 1) / threads, 4096);
  const Tacc scale = (Tacc)inv_sqrt_host((double)S->zeta);
  hipLaunchKernelGGL((reduce_partials_kernel<Tacc, Tout>), dim3((unsigned)std::max<int64_t>(1, blocks)),
                     dim3(threads), 0, st, (const Tacc*)P, p.n_chunks, S->d, m, scale, (Tout*)out, ldo);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename Tin>
static int launch_rows_jb(const sk_sketch* S, const RowsPlan& p, int64_t m, const void* A, int64_t lda, void* P,
                          const void* plan, hipStream_t st) {
  constexpr int JMAX = sizeof(Tin) == 8 ? 50 : 64;
  if (p.load_bytes == 16) {
    if (p.jb == 16) return launch_rows_t<Tin, 16, 16>(S, p, m, A, lda, P, plan, st);
    if (p.jb == 32) return launch_rows_t<Tin, 32, 16>(S, p, m, A, lda, P, plan, st);
    return launch_rows_t<Tin, JMAX, 16>(S, p, m, A, lda, P, plan, st);
  }
  if (p.jb == 16) return launch_rows_t<Tin, 16, 4>(S, p, m, A, lda, P, plan, st);
  if (p.jb == 32) return launch_rows_t<Tin, 32, 4>(S, p, m, A, lda, P, plan, st);
  return launch_rows_t<Tin, JMAX, 4>(S, p, m, A, lda, P, plan, st);
}

template <typename Tin, int MV>
static int launch_narrow_t(const sk_sketch* S, const RowsPlan& p, int64_t m, const void* A, int64_t lda, void* P,
                           const void* plan, hipStream_t st) {
  NarrowArgs a;
  a.A = (const unsigned char*)A;
  a.lda_bytes = lda * (int64_t)sizeof(Tin);
  a.n = S->n;
  a.d = S->d;
  a.m = (int)m;
  a.R = p.R;
  a.zeta = S->zeta;
  a.nb = (int)S->nb;
  a.plan = (const unsigned char*)plan;
  a.rec_bytes = p.rec_bytes;
  a.lst_off = p.lst_off;
  a.n_tiles = p.n_tiles;
  a.tiles_per_chunk = p.tiles_per_chunk;
  a.P = P;
  const int threads = (int)std::min<int64_t>(1024, ((S->d + 63) / 64) * 64);
  auto kern = ss_narrow_kernel<Tin, MV>;
  SK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes));
  {
    KernelTimer timer(S, st);
    hipLaunchKernelGGL(kern, dim3((unsigned)p.n_chunks), dim3(threads), p.lds_bytes, st, a);
  }
  SK_HIP(hipGetLastError());
  return SK_OK;
}

template <typename Tin>
static int launch_narrow(const sk_sketch* S, const RowsPlan& p, int64_t m, const void* A, int64_t lda, void* P,
                         const void* plan, hipStream_t st) {
  if (m == 1) return launch_narrow_t<Tin, 1>(S, p, m, A, lda, P, plan, st);
  if (m == 2) return launch_narrow_t<Tin, 2>(S, p, m, A, lda, P, plan, st);
  return launch_narrow_t<Tin, 4>(S, p, m, A, lda, P, plan, st);
}

// Workspace: partials, then the plan records.
int launch_rows_apply(const sk_sketch* S, const RowsPlan& p, int dtype_in, int64_t m, const void* A, int64_t lda,
                      int dtype_out, void* SA, int64_t ldsa, void* ws, hipStream_t st) {
  void* P = ws;
  void* plan = (unsigned char*)ws + p.partial_bytes;
  if (p.idx) {
    int rc = launch_idx_sketch(S, p, dtype_in, m, A, lda, ws, st);
    if (rc != SK_OK) return rc;
    if (dtype_in == SK_F64) {
      if (dtype_out == SK_F64) return launch_reduce<double, double>(p, S, m, P, SA, ldsa, st);
      return launch_reduce<double, float>(p, S, m, P, SA, ldsa, st);
    }
    if (dtype_out == SK_F64) return launch_reduce<float, double>(p, S, m, P, SA, ldsa, st);
    return launch_reduce<float, float>(p, S, m, P, SA, ldsa, st);
  }
  // wide kernel: entry << 3 is the row's byte offset in the tile (rows of 64 elements)
  const int runit = p.narrow ? 1 : p.rowb / 8;
  int rc = launch_plan(S, p, plan, runit, st);
  if (rc != SK_OK) return rc;
  if (p.narrow) {
    if (dtype_in == SK_F64)
      rc = launch_narrow<double>(S, p, m, A, lda, P, plan, st);
    else if (dtype_in == SK_F32)
      rc = launch_narrow<float>(S, p, m, A, lda, P, plan, st);
    else
      rc = launch_narrow<uint16_t>(S, p, m, A, lda, P, plan, st);
  } else if (dtype_in == SK_F64)
    rc = launch_rows_jb<double>(S, p, m, A, lda, P, plan, st);
  else if (dtype_in == SK_F32)
    rc = launch_rows_jb<float>(S, p, m, A, lda, P, plan, st);
  else
    rc = launch_rows_jb<uint16_t>(S, p, m, A, lda, P, plan, st);
  if (rc != SK_OK) return rc;
  if (dtype_in == SK_F64) {
    if (dtype_out == SK_F64) return launch_reduce<double, double>(p, S, m, P, SA, ldsa, st);
    return launch_reduce<double, float>(p, S, m, P, SA, ldsa, st);
  }
  if (dtype_out == SK_F64) return launch_reduce<float, double>(p, S, m, P, SA, ldsa, st);
  return launch_reduce<float, float>(p, S, m, P, SA, ldsa, st);
}

int launch_pattern(const sk_sketch* S, int32_t* bucket, int8_t* sign, hipStream_t st) {
  const int64_t total = S->n * ((S->zeta + 3) / 4);
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(ss_pattern_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, S->n,
                     S->zeta, (uint32_t)S->nb, S->k0, S->k1, bucket, sign);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int launch_adjoint(const sk_sketch* S, int64_t m, const double* Y, int64_t ldy, double* Z, int64_t ldz,
                   hipStream_t st) {
  const int64_t total = S->n * m;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(ss_adjoint_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, S->n, m,
                     S->zeta, (uint32_t)S->nb, S->k0, S->k1, inv_sqrt_host((double)S->zeta), Y, ldy, Z, ldz);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
