// SparseStack apply, row mode: SA = S A for a tall row-major A (n x m).
//
// Def. 1.5: column i of S carries rho_it / sqrt(zeta) in row t*nb + s_it for
// each block t, so SA[t*nb + s, c] = (1/sqrt(zeta)) * sum_{i: s_it = s} rho_it A[i, c].
//
// Design (gfx950, one HBM pass over A):
//  * A workgroup owns a row chunk x a column slab (<= 64 columns, one per lane)
//    x a group of blocks. It streams its rows through LDS in sub-tiles of R
//    rows, double-buffered with direct global->LDS loads, so the prefetch of
//    tile k+1 costs no VGPRs and overlaps the work on tile k.
//  * For each sub-tile the Philox hash gives (bucket, sign) of every row and
//    block; one wave per block counting-sorts the rows by bucket (stable, via
//    wave ballots: no atomics, so the order is deterministic).
//  * Each wave owns one block and a contiguous range of its buckets and keeps
//    one accumulator per bucket per lane in registers. It walks its buckets in
//    order and, for each, the sorted rows of that bucket: all 64 lanes read
//    the same row (a broadcast list entry) at consecutive columns (conflict-free
//    LDS reads) and add +-value into the bucket's register.
//  * At the end of the chunk the accumulators go to a partial buffer
//    [chunk][d][m]; a second kernel sums the partials in chunk order and scales
//    by 1/sqrt(zeta). Summation order is fixed, so results are bitwise
//    reproducible.
#include "sk_launch.hpp"

#include <algorithm>
#include <cstdlib>

namespace sk {

struct RowsArgs {
  const unsigned char* A;
  int64_t lda_bytes;
  int64_t n, m, d;
  int C, n_slabs, R, bpg, n_groups, H, per_range, n_chunks;
  int64_t rows_per_chunk;
  int zeta, nb, nbits;
  uint32_t k0, k1;
  void* P;
  int off_codes, off_rnk, off_off, off_lists, tile_bytes;
};

template <typename Tin>
struct InType;
template <>
struct InType<double> {
  using acc = double;
  __device__ static double load(const unsigned char* p) { return *(const double*)p; }
};
template <>
struct InType<float> {
  using acc = float;
  __device__ static float load(const unsigned char* p) { return *(const float*)p; }
};
template <>
struct InType<uint16_t> {  // bf16
  using acc = float;
  __device__ static float load(const unsigned char* p) { return bf16_to_f32(*(const uint16_t*)p); }
};

__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
__device__ inline void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ inline __attribute__((address_space(3))) void* as_lds(void* p) {
  return (__attribute__((address_space(3))) void*)p;
}

template <typename Tin>
__device__ inline typename InType<Tin>::acc load_signed(const unsigned char* p, uint32_t neg);
template <>
__device__ inline double load_signed<double>(const unsigned char* p, uint32_t neg) {
  uint64_t u = *(const uint64_t*)p;
  u ^= (uint64_t)neg << 63;
  return __builtin_bit_cast(double, u);
}
template <>
__device__ inline float load_signed<float>(const unsigned char* p, uint32_t neg) {
  uint32_t u = *(const uint32_t*)p;
  return __builtin_bit_cast(float, u ^ (neg << 31));
}
template <>
__device__ inline float load_signed<uint16_t>(const unsigned char* p, uint32_t neg) {
  uint32_t u = (uint32_t)(*(const uint16_t*)p) ^ (neg << 15);
  return __builtin_bit_cast(float, u << 16);
}

template <typename Tin, int JB, int LB>
__global__ void __launch_bounds__(1024) ss_rows_kernel(RowsArgs a) {
  using Tacc = typename InType<Tin>::acc;
  constexpr int ES = sizeof(Tin);
  constexpr int ROWB = 64 * ES;  // LDS bytes per tile row (64 columns)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nthreads = blockDim.x, nwaves = nthreads >> 6;

  // Work item. Workgroup ids L, L+8, ... run on the same XCD (dispatch is
  // round-robin over the 8 XCDs), so the n_groups workgroups that share one
  // A tile are given ids 8 apart and find it in the same L2.
  const int L = blockIdx.x, xcd = L & 7, q = L >> 3;
  const int group = q % a.n_groups;
  const int rest = (q / a.n_groups) * 8 + xcd;
  const int slab = rest % a.n_slabs;
  const int chunk = rest / a.n_slabs;
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

  uint16_t* codes = (uint16_t*)(smem + a.off_codes);  // [bpg][R]: bucket << 1 | negative
  uint16_t* rnk = (uint16_t*)(smem + a.off_rnk);      // [bpg][R]: rank of the row in its bucket
  uint32_t* offs = (uint32_t*)(smem + a.off_off);     // [bpg][nb + 1]: counts, then offsets
  uint16_t* lists = (uint16_t*)(smem + a.off_lists);  // [bpg][R]: row << 1 | negative, by bucket

  const int tl = wave / a.H, hr = wave - (wave / a.H) * a.H;
  const bool walker = tl < bpg;
  const int s_begin = hr * a.per_range;
  const int s_cnt = walker ? max(0, min(a.per_range, nb - s_begin)) : 0;

  Tacc acc[JB];
#pragma unroll
  for (int j = 0; j < JB; ++j) acc[j] = 0;

  auto issue_loads = [&](int st, int buf) {
    const int64_t r0 = r_begin + (int64_t)st * R;
    const int rv = (int)min((int64_t)R, r_end - r0);
    unsigned char* dst = smem + buf * a.tile_bytes;
    const int n_instr = R * ROWB / (64 * LB);
    for (int k = wave; k < n_instr; k += nwaves) {
      const int byte = (k * 64 + lane) * LB;
      const int row = byte / ROWB;
      const int cb = byte - row * ROWB;
      const unsigned char* src = a.A;  // in-bounds stand-in for padding lanes
      if (row < rv && cb < slab_bytes) src = a.A + (r0 + row) * a.lda_bytes + col0 * ES + cb;
      if constexpr (LB == 16)
        __builtin_amdgcn_global_load_lds((const void*)src, as_lds(dst + k * 64 * LB), 16, 0, 0);
      else
        __builtin_amdgcn_global_load_lds((const void*)src, as_lds(dst + k * 64 * LB), 4, 0, 0);
    }
  };

  if (nsub > 0) issue_loads(0, 0);
  for (int st = 0; st < nsub; ++st) {
    const int buf = st & 1;
    const int64_t r0 = r_begin + (int64_t)st * R;
    const int rv = (int)min((int64_t)R, r_end - r0);
    wait_dma();
    lds_barrier();  // tile st is in LDS; everyone finished walking tile st-1
    if (st + 1 < nsub) issue_loads(st + 1, buf ^ 1);

    // Hash: one Philox call gives the words of blocks 4g .. 4g+3 of one row.
    {
      const int g0 = t0 >> 2, g1 = (t0 + bpg - 1) >> 2;
      for (int g = g0; g <= g1; ++g) {
        for (int r = tid; r < rv; r += nthreads) {
          const uint64_t i = (uint64_t)(r0 + r);
          const U4 w =
              philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)g, kTagSparseStack}, a.k0, a.k1);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int t = 4 * g + j;
            if (t >= t0 && t < t0 + bpg) {
              const uint32_t word = word_of(w, j);
              codes[(t - t0) * R + r] = (uint16_t)((ss_bucket(word, (uint32_t)nb) << 1) | ss_negative(word));
            }
          }
        }
      }
    }
    lds_barrier();

    // Stable counting sort of the rows of block `wave` by bucket.
    if (wave < bpg) {
      uint32_t* cnt = offs + wave * (nb + 1);
      const uint16_t* cd = codes + wave * R;
      uint16_t* rk = rnk + wave * R;
      for (int s = lane; s <= nb; s += 64) cnt[s] = 0;
      const uint64_t below = (1ull << lane) - 1ull;
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
      uint32_t run = inc - loc;
      for (int k = 0; k < per; ++k) {
        if (sb + k < nb) {
          const uint32_t c = cnt[sb + k];
          cnt[sb + k] = run;
          run += c;
        }
      }
      if (lane == 63) cnt[nb] = inc;
      // scatter list entries
      uint16_t* lst = lists + wave * R;
      for (int c0 = 0; c0 < rv; c0 += 64) {
        const int r = c0 + lane;
        if (r < rv) {
          const uint32_t code = cd[r];
          const uint32_t pos = cnt[code >> 1] + rk[r];
          lst[pos] = (uint16_t)(((uint32_t)r << 1) | (code & 1u));
        }
      }
    }
    lds_barrier();

    // Segmented reduction: wave (block tl, buckets [s_begin, s_begin + s_cnt)).
    // The wave's list entries (<= 128) and bucket offsets (<= 128) are packed
    // two u16 per lane into VGPRs and read back with v_readlane, so a row costs
    // one LDS read (the value) and a few scalar-operand VALU ops.
    if (walker) {
      // Opaque copy: keeps the per-bucket tests below inside the loop instead
      // of letting them be hoisted as 64 live lane masks.
      int s_cnt_l = s_cnt;
      asm volatile("" : "+s"(s_cnt_l));
      const uint16_t* lst = lists + tl * R;
      const uint32_t* of = offs + tl * (nb + 1);
      const unsigned char* tb = smem + buf * a.tile_bytes + lane * ES;
      const int ebase = __builtin_amdgcn_readfirstlane((int)of[s_begin]);
      const int eend = __builtin_amdgcn_readfirstlane((int)of[s_begin + s_cnt_l]);
      const int nw = eend - ebase;
      uint32_t vo, ve;
      {
        const int j0 = 2 * lane, j1 = 2 * lane + 1;
        const uint32_t o0 = j0 <= s_cnt_l ? of[s_begin + j0] - ebase : 0u;
        const uint32_t o1 = j1 <= s_cnt_l ? of[s_begin + j1] - ebase : 0u;
        vo = o0 | (o1 << 16);
      }
      // entry window: entries [wb, wb + 128) of this wave, two per lane
      int wb = 0;
      auto load_window = [&](int from) {
        const int j0 = from + 2 * lane, j1 = j0 + 1;
        const uint32_t e0 = j0 < nw ? lst[ebase + j0] : 0u;
        const uint32_t e1 = j1 < nw ? lst[ebase + j1] : 0u;
        ve = e0 | (e1 << 16);
      };
      load_window(0);
      int kb = 0;
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        if (j < s_cnt_l) {
          const uint32_t wo = (uint32_t)__builtin_amdgcn_readlane((int)vo, (j + 1) >> 1);
          const int ke = (int)(((j + 1) & 1) ? (wo >> 16) : (wo & 0xffffu));
          for (int k = kb; k < ke; ++k) {
            if (k - wb >= 128) {  // rare: more than 128 rows for this wave
              wb = k;
              load_window(wb);
            }
            const int kk = k - wb;
            const uint32_t we = (uint32_t)__builtin_amdgcn_readlane((int)ve, kk >> 1);
            const uint32_t e = (kk & 1) ? (we >> 16) : (we & 0xffffu);
            acc[j] += load_signed<Tin>(tb + (e >> 1) * ROWB, e & 1u);
          }
          kb = ke;
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

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

static int jb_for(int dtype_in) { return dtype_in == SK_F64 ? 50 : 64; }

int plan_rows(const sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, RowsPlan* p) {
  const int es = (int)dtype_size(dtype_in);
  const int zeta = S->zeta;
  const int64_t nb = S->nb;
  if (nb > 16384) {
    set_error("SparseStack row apply supports at most 16384 buckets per block");
    return SK_E_NOTSUP;
  }
  p->jb = jb_for(dtype_in);
  const int Hmin = (int)((nb + p->jb - 1) / p->jb);
  if (Hmin > 16) {
    set_error("SparseStack row apply: d/zeta too large for the register-resident accumulators");
    return SK_E_NOTSUP;
  }
  if ((int64_t)zeta * Hmin <= 16) {
    p->bpg = zeta;
    p->n_groups = 1;
    p->H = std::max(Hmin, (int)std::min<int64_t>(nb, 16 / zeta));
  } else {
    p->bpg = 16 / Hmin;
    p->n_groups = (zeta + p->bpg - 1) / p->bpg;
    p->H = Hmin;
  }
  p->W = p->bpg * p->H;
  p->per_range = (int)((nb + p->H - 1) / p->H);

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

  // sub-tile rows: 64 KB per buffer, shrunk until the LDS plan fits
  int R = env_int("SKETCH_TILE_ROWS", 65536 / (64 * es));
  const int tile_cap = 160 * 1024;
  for (;;) {
    const size_t tile = (size_t)R * 64 * es;
    size_t off = 2 * tile;
    const size_t codes = off;
    off = align16(off + (size_t)p->bpg * R * 2);
    const size_t rk = off;
    off = align16(off + (size_t)p->bpg * R * 2);
    const size_t of = off;
    off = align16(off + (size_t)p->bpg * (nb + 1) * 4);
    const size_t li = off;
    off = align16(off + (size_t)p->bpg * R * 2);
    if (off <= (size_t)tile_cap || R <= 16) {
      p->R = R;
      p->lds_bytes = off;
      (void)codes;
      (void)rk;
      (void)of;
      (void)li;
      break;
    }
    R /= 2;
  }
  if (p->lds_bytes > (size_t)tile_cap) {
    set_error("sketch_apply: LDS plan does not fit");
    return SK_E_NOTSUP;
  }
  const int64_t n = S->n;
  const int64_t items = (int64_t)p->n_slabs * p->n_groups;
  const int target = env_int("SKETCH_WG_TARGET", 256);
  int64_t nc = std::max<int64_t>(1, (target + items - 1) / items);
  nc = std::min<int64_t>(nc, (n + p->R - 1) / p->R);
  int64_t rpc = (n + nc - 1) / nc;
  rpc = ((rpc + p->R - 1) / p->R) * p->R;
  p->rows_per_chunk = rpc;
  p->n_chunks = (int)((n + rpc - 1) / rpc);
  const size_t accb = dtype_in == SK_F64 ? 8 : 4;
  p->partial_bytes = align16((size_t)p->n_chunks * S->d * m * accb);
  return SK_OK;
}

template <typename Tin, int JB, int LB>
static int launch_rows_t(const sk_sketch* S, const RowsPlan& p, int64_t m, const void* A, int64_t lda, void* P,
                         hipStream_t st) {
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
  a.H = p.H;
  a.per_range = p.per_range;
  a.n_chunks = p.n_chunks;
  a.rows_per_chunk = p.rows_per_chunk;
  a.zeta = S->zeta;
  a.nb = (int)S->nb;
  int nbits = 0;
  while ((1ll << nbits) < S->nb) ++nbits;
  a.nbits = nbits;
  a.k0 = S->k0;
  a.k1 = S->k1;
  a.P = P;
  const size_t tile = (size_t)p.R * 64 * es;
  size_t off = 2 * tile;
  a.tile_bytes = (int)tile;
  a.off_codes = (int)off;
  off = align16(off + (size_t)p.bpg * p.R * 2);
  a.off_rnk = (int)off;
  off = align16(off + (size_t)p.bpg * p.R * 2);
  a.off_off = (int)off;
  off = align16(off + (size_t)p.bpg * (S->nb + 1) * 4);
  a.off_lists = (int)off;
  const int64_t pairs = (int64_t)p.n_chunks * p.n_slabs;
  const int64_t grid = ((pairs + 7) / 8) * 8 * p.n_groups;
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

int launch_rows_apply(const sk_sketch* S, const RowsPlan& p, int dtype_in, int64_t m, const void* A, int64_t lda,
                      int dtype_out, void* SA, int64_t ldsa, void* ws, hipStream_t st) {
  int rc;
  if (dtype_in == SK_F64) {
    rc = p.load_bytes == 16 ? launch_rows_t<double, 50, 16>(S, p, m, A, lda, ws, st)
                            : launch_rows_t<double, 50, 4>(S, p, m, A, lda, ws, st);
  } else if (dtype_in == SK_F32) {
    rc = p.load_bytes == 16 ? launch_rows_t<float, 64, 16>(S, p, m, A, lda, ws, st)
                            : launch_rows_t<float, 64, 4>(S, p, m, A, lda, ws, st);
  } else {
    rc = p.load_bytes == 16 ? launch_rows_t<uint16_t, 64, 16>(S, p, m, A, lda, ws, st)
                            : launch_rows_t<uint16_t, 64, 4>(S, p, m, A, lda, ws, st);
  }
  if (rc != SK_OK) return rc;
  if (dtype_in == SK_F64) {
    if (dtype_out == SK_F64) return launch_reduce<double, double>(p, S, m, ws, SA, ldsa, st);
    return launch_reduce<double, float>(p, S, m, ws, SA, ldsa, st);
  }
  if (dtype_out == SK_F64) return launch_reduce<float, double>(p, S, m, ws, SA, ldsa, st);
  return launch_reduce<float, float>(p, S, m, ws, SA, ldsa, st);
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
