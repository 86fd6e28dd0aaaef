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
#include <cstdlib>

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

template <typename Tin, int NREG, int LB, bool PARTS = false>
__global__ void __launch_bounds__(NREG > 64 ? 512 : 1024)
    ss_idx_kernel(IdxArgs a, const uint32_t* __restrict__ codes_all) {
  using T = IdxT<Tin>;
  using Tacc = typename T::acc;
  constexpr int ES = sizeof(Tin);
  // Tile rows sit at a fixed stride of one element per lane, so the LDS
  // offsets of the rows of a 64-row group are compile-time immediates.
  constexpr int ROWB = 64 * ES;
  constexpr int CPR = ROWB / LB;  // load chunks per tile row (a power of two)
  constexpr int GR = 16;          // rows whose codes one scalar group holds
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x, nwaves = nthreads >> 6;

  // Work item. Dispatch is round-robin over the 8 XCDs (id L runs on XCD
  // L % 8): all slabs and block groups of one row chunk get ids 8 apart and
  // share one XCD's L2 for the cache lines that straddle slab boundaries.
  const int L = blockIdx.x, xcd = L & 7, q8 = L >> 3;
  const int group = q8 % a.n_groups;
  const int slab = (q8 / a.n_groups) % a.n_slabs;
  const int chunk = (q8 / (a.n_groups * a.n_slabs)) * 8 + xcd;
  if (chunk >= a.n_chunks) return;

  const int t0 = group * a.bpg;
  const int bpg = min(a.bpg, a.zeta - t0);
  const int64_t col0 = (int64_t)slab * a.C;
  const int Cw = (int)min((int64_t)a.C, a.m - col0);
  const int slab_bytes = Cw * ES;
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

  // Chunk q of a tile (LB bytes) is row q / CPR, bytes (q % CPR) * LB of it;
  // chunks past the slab's bytes are padding and are not loaded.
  const int n_instr = (R * CPR + 63) / 64;
  auto issue_loads = [&](int st, int buf) {
    const int64_t r0 = r_begin + (int64_t)st * R;
    const int rv = (int)min((int64_t)R, r_end - r0);
    unsigned char* dst = smem + buf * a.buf_stride;
    const unsigned char* tsrc = a.A + r0 * a.lda_bytes + col0 * ES;
    // load k covers chunks [64 k, 64 k + 64): a lane's chunk advances by
    // 64 W chunks = RSTEP rows per load of its wave, at a fixed byte offset
    const int q0 = wave * 64 + lane;
    const int cb = (q0 % CPR) * LB;
    const int rstep = (nwaves * 64) / CPR;
    int row = q0 / CPR;
    const unsigned char* src = tsrc + (int64_t)row * a.lda_bytes + cb;
    const int64_t sstep = (int64_t)rstep * a.lda_bytes;
    for (int k = wave; k < n_instr; k += nwaves) {
      const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane((int)idx_lds_addr(dst + k * 64 * LB));
      if (row < rv && cb < slab_bytes) {
        if constexpr (LB == 16)
          idx_dma16(src, la);
        else
          idx_dma4(src, la);
      }
      row += rstep;
      src += sstep;
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
    if (((k * 64) % CPR) * LB < slab_bytes) ++per_tile;
  for (int p = 0; p < nbuf - 1 && p < nsub; ++p) issue_loads(p, p);
  for (int st = 0; st < nsub; ++st) {
    const int buf = st % nbuf;
    // tile st is complete once only the loads of the later tiles in flight
    // remain; a partial (last) tile among those: wait for everything
    const int later = min(st + nbuf - 2, nsub - 1) - st;
    const bool later_full = later <= 0 || r_begin + (int64_t)(st + later + 1) * R <= r_end;
    idx_wait_vm(later > 0 && later_full ? later * per_tile : 0);
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
        P[(rowbase + s) * a.m + col0 + lane] = val;
      }
    }
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
}  // namespace

bool idx_apply_fits(const sk_sketch* S, int dtype_in, int64_t m) {
  if (env_i("SKETCH_IDX", 1) == 0) return false;
  return m > 4 && S->zeta >= 4 && idx_parts(dtype_in, S->nb) != 0;
}

static int plan_idx_lb(const sk_sketch* S, int dtype_in, int64_t m, int load_bytes, RowsPlan* p) {
  const int es = (int)dtype_size(dtype_in);
  const int zeta = S->zeta;
  const int nparts = idx_parts(dtype_in, S->nb);
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
  const int nbuf = std::max(2, std::min(4, env_i("SKETCH_IDX_NBUF", 2)));
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
  const int target = env_i("SKETCH_IDX_WG", 256 * wg_per_cu);
  int64_t nc = std::max<int64_t>(1, (target + items - 1) / items);
  nc = ((std::max<int64_t>(nc, 8) + 7) / 8) * 8;
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

}  // namespace sk
