// Batched sketch-and-solve: Alg. 3 for many independent least-squares
// problems (problem p: its own SparseStack S_p of Def. 1.5 with d_p =
// d_per_k k_p rows in zeta blocks under key seed_p; x_p the truncated-SVD
// solution of min ||S_p A_p x - S_p b_p|| through the Householder QR
// S_p [A_p b_p] = Q [R c; 0 *]), run as one persistent kernel fed by device
// work queues (gfx950).
//
// One batch is four kernels, captured once into a graph and replayed with
// one launch:
//   init     - zeroes the queue heads and counters (a kernel, not a memset,
//              so that the graph replays cleanly);
//   codes    - the row codes of every problem (bucket register index and
//              sign of each row in each block, the Philox reading shared
//              with the single-matrix apply);
//   worker   - persistent: each workgroup (8 waves) pops items until every
//              problem is solved;
//   fallback - one workgroup per problem the full-rank certificate rejected:
//              the one-sided Jacobi SVD of R and the rank-truncated solve.
//
// Worker items:
//  * sketch: up to 8/W units of one problem, W waves a unit (one wave per
//    block of S, W = zeta rounded up to a power of two, at most 8). A unit
//    is (row chunk, 64-column slab of [A b], bucket part, block group): its
//    waves stream the chunk's rows of the slab through LDS and add each row
//    into the register accumulator of its bucket (the register file of the
//    single-matrix apply, addressed through the VALU's GPR-index mode).
//    Buckets beyond one register file are split into parts; the parts of
//    one slab share a tile in one item, and rows of the other parts add into
//    a dump register that is never stored. The b column rides in the lane
//    after A's last column (or in a slab of its own). Each unit writes its
//    partial sums to [chunk][d][k + 1].
//  * reduce: rows of d of one problem: W = (1/sqrt(zeta)) sum over chunks
//    of the partials, in chunk order (deterministic), F64, row-major with a
//    zero-padded stride.
//  * QR and solve: run by the workgroup that finishes a problem's last
//    reduce item: blocked Householder QR in the workgroup (16-column panels
//    factored in registers; the trailing update Y -= V T^T V^T Y on the FP64
//    matrix cores, V in LDS), then X = R^-1, the certificate
//    ||R||_F ||X||_F < 1e-3 / (5 eps) (it implies s_k > 5 eps s_1, Alg. 3's
//    rank test) and x = X c, or the problem is left to the fallback kernel.
// Sketch items sit in 8 static queues, one per XCD: all the units of a row
// chunk go to one queue, so the cache lines that neighbouring slabs share
// are fetched through one L2; a workgroup drains its own XCD's queue first
// and then steals. Completions feed a ready queue: the workgroup that
// finishes a problem's last sketch unit pushes the problem's reduce items,
// which are popped before any static item. No workgroup ever waits for
// another: the dependent work is run by whoever completes the dependency,
// so the queues cannot deadlock, and every workgroup leaves once all
// problems are solved.
//
// Per-problem timestamps (the device's constant-rate clock) mark the start
// of a problem's first sketch unit and the end of its solve.
#include "sk_batched.hpp"
#include "sk_idx.hpp"
#include "sk_jacobi.hpp"

#include <algorithm>
#include <cmath>

namespace sk {
namespace bt {

using namespace idx;

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Device side
// ---------------------------------------------------------------------------

__device__ inline uint64_t bt_now() { return __builtin_amdgcn_s_memrealtime(); }

__device__ inline int bt_xcc_id() {
  int v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 7;
}

__device__ inline void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ inline void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Codes of every problem: for row i (tile i / R, row i % R of it), block t
// and bucket part h, at ((tile * nparts + h) * zeta + t) * 2R of the
// problem's code area: the register index of the bucket within part h (the
// dump slot when the bucket is in another part) at [r], and the high word of
// the +-1.0 multiplier at [R + r]. rpre: prefix sums of the problems' padded
// row counts (tiles * R).
__global__ void bt_codes_kernel(const BtProb* __restrict__ probs, const int64_t* __restrict__ rpre, int nprob,
                                uint32_t* __restrict__ base) {
  const int64_t total = rpre[nprob];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nprob - 1;  // the problem whose row range holds g
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rpre[mid] <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    const BtProb& P = probs[lo];
    const int64_t i = g - rpre[lo];
    const int R = P.R;
    const int64_t tile = i / R;
    const int r = (int)(i - tile * R);
    const uint32_t rpa = P.dtype == SK_F64 ? 2u : 1u;
    const uint32_t one_hi = P.dtype == SK_F64 ? IdxT<double>::one_hi : IdxT<float>::one_hi;
    const uint32_t dump = (uint32_t)(kNreg / (int)rpa - 1);
    uint32_t* codes = base + P.codes_off / 4;
    for (int g4 = 0; g4 < (P.zeta + 3) / 4; ++g4) {
      U4 w = U4{0u, 0u, 0u, 0u};
      if (i < P.n)
        w = philox4x32_10(U4{(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)g4, kTagSparseStack}, P.k0,
                          P.k1);
      for (int j = 0; j < 4; ++j) {
        const int t = 4 * g4 + j;
        if (t >= P.zeta) break;
        const uint32_t word = word_of(w, j);
        const int bucket = (int)ss_bucket(word, (uint32_t)P.nb);
        const uint32_t sw = (ss_negative(word) << 31) | one_hi;
        for (int h = 0; h < P.nparts; ++h) {
          const int rel = bucket - h * P.ps;
          const uint32_t slot = (rel >= 0 && rel < P.ps) ? (uint32_t)rel : dump;
          uint32_t* c = codes + ((tile * P.nparts + h) * P.zeta + t) * (int64_t)(2 * R);
          c[r] = slot * rpa;
          c[R + r] = sw;
        }
      }
    }
  }
}

__global__ void bt_init_kernel(int* __restrict__ ctl, int nctl, unsigned long long* __restrict__ t_start,
                               unsigned long long* __restrict__ t_end, int nprob,
                               unsigned long long* __restrict__ rq, int rq_cap) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nctl; i += stride) ctl[i] = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nprob; i += stride) {
    t_start[i] = ~0ull;
    t_end[i] = 0ull;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rq_cap; i += stride) rq[i] = 0ull;
}

// Raw element bits of the b column.
template <typename Tin>
struct RawOf;
template <>
struct RawOf<double> {
  using type = uint64_t;
};
template <>
struct RawOf<float> {
  using type = uint32_t;
};
template <>
struct RawOf<uint16_t> {
  using type = uint16_t;
};

// One sketch item: units u_first .. u_first + cnt - 1 of problem P, unit slot
// s = wave / W run by waves [s W, (s + 1) W). LDS: two tile buffers per slot
// (buf_bytes each), then 1 KB per wave for the code prefetch.
template <typename Tin>
__device__ void sketch_item(const BtArgs& a, const BtProb& P, int u_first, int cnt,
                            const uint32_t* __restrict__ codes_base, unsigned char* smem) {
  using T = IdxT<Tin>;
  using Tacc = typename T::acc;
  using Raw = typename RawOf<Tin>::type;
  constexpr int ES = sizeof(Tin);
  constexpr int ROWB = 64 * ES;   // LDS bytes of a tile row (64 columns)
  constexpr int UPR = ROWB / 4;   // dword loads per tile row
  constexpr int GR = 16;          // rows whose codes one scalar group holds
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wu = a.wu;
  const int s = wave / wu, w = wave - s * wu;
  const int per = P.n_slabs * P.n_gp;  // units per chunk
  const int R = P.R;
  const bool active = s < cnt;
  const int u = u_first + s;
  const int chunk = u / per, rem = u - chunk * per;
  const int slab = rem / P.n_gp, gp = rem - slab * P.n_gp;
  const int group = gp / P.nparts, part = gp - group * P.nparts;
  const int t = group * wu + w;  // this wave's block
  const bool walker = active && t < P.zeta;
  // the slot whose buffers hold this unit's tile: the item's first unit of
  // the same chunk and slab
  const int os = max(u_first, chunk * per + slab * P.n_gp) - u_first;
  const bool loader = active && os == s;
  const int col0 = slab * 64;
  const int ncol = P.k + 1;
  const int Cw = min(64, ncol - col0);             // columns of [A b] in the slab
  const int cwa_bytes = max(0, min(64, P.k - col0)) * ES;  // bytes of A in a tile row
  const bool has_b = P.k >= col0 && P.k < col0 + 64;
  const int bl = P.k - col0;
  const int64_t r_begin = (int64_t)chunk * P.rows_per_chunk;
  const int64_t r_end = min(P.n, r_begin + P.rows_per_chunk);
  const int nsub = active ? (int)((r_end - r_begin + R - 1) / R) : 0;
  int nsub_max = 0;  // tiles of the item's longest unit
  for (int q = 0; q < cnt; ++q) {
    const int cq = (u_first + q) / per;
    const int64_t rb = (int64_t)cq * P.rows_per_chunk, re = min(P.n, rb + P.rows_per_chunk);
    nsub_max = max(nsub_max, (int)((re - rb + R - 1) / R));
  }
  const unsigned char* Ab = P.A;
  const unsigned char* bb = P.b;
  const int64_t lda_bytes = P.lda_bytes;
  const uint32_t* pcodes = codes_base + P.codes_off / 4;
  const unsigned char* tcodes = a.ws + P.codes_off;  // the same codes, for the L2 prefetch only

  AccFile f;
  acc_zero<kNreg>(f);
  Raw bv[2] = {0, 0};

  auto buf_ptr = [&](int buf) { return smem + (os * 2 + buf) * a.buf_bytes; };
  auto code_ptr = [&](int64_t tile) { return ((tile * P.nparts + part) * P.zeta + t) * (int64_t)(2 * R); };
  // Loads of tile st into buffer buf: the slot's A rows (direct to LDS), the
  // b values (to registers; written to LDS by finish), and a prefetch of
  // this wave's codes into L2.
  auto issue = [&](int st, int buf) {
    const int64_t r0 = r_begin + (int64_t)st * R;
    const int rv = (int)min((int64_t)R, r_end - r0);
    if (loader) {
      unsigned char* dst = buf_ptr(buf);
      const int n_instr = R * UPR / 64;
      for (int i = w; i < n_instr; i += wu) {
        const int q0 = i * 64 + lane;
        const int row = q0 / UPR, ub = (q0 - row * UPR) * 4;
        const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane((int)idx_lds_addr(dst + i * 256));
        if (row < rv && ub < cwa_bytes) idx_dma4(Ab + (r0 + row) * lda_bytes + col0 * ES + ub, la);
      }
      if (has_b && w == 0) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int row = j * 64 + lane;
          if (j * 64 < R && row < rv) bv[j] = *(const Raw*)(bb + (r0 + row) * ES);
        }
      }
    }
    if (walker) {
      const unsigned char* csrc = tcodes + code_ptr(r0 / R) * 4;
      const int cbytes = 8 * R;
      const uint32_t la = (uint32_t)__builtin_amdgcn_readfirstlane(
          (int)idx_lds_addr(smem + a.off_touch + wave * 1024));
      for (int o = 0; o < cbytes; o += 1024)
        if (o + lane * 16 < cbytes) idx_dma16(csrc + o + lane * 16, la);
    }
  };
  // Completes tile st in buffer buf: the b column, once the loads landed.
  auto finish = [&](int st, int buf) {
    if (loader && has_b && w == 0 && st < nsub) {
      const int64_t r0 = r_begin + (int64_t)st * R;
      const int rv = (int)min((int64_t)R, r_end - r0);
      unsigned char* dst = buf_ptr(buf);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = j * 64 + lane;
        if (j * 64 < R && row < rv) *(Raw*)(dst + row * ROWB + bl * ES) = bv[j];
      }
    }
  };

  if (nsub > 0) issue(0, 0);
  for (int st = 0; st < nsub_max; ++st) {
    const int buf = st & 1;
    idx_wait_vm(0);
    finish(st, buf);
    idx_barrier();  // tile st is in LDS; everyone finished tile st - 1
    if (st + 1 < nsub) issue(st + 1, buf ^ 1);
    if (walker && st < nsub) {
      const int64_t r0 = r_begin + (int64_t)st * R;
      const int rv = (int)min((int64_t)R, r_end - r0);
      const uint32_t* codes = pcodes + code_ptr(r0 / R);
      const uint32_t tbase = idx_lds_addr(buf_ptr(buf)) + (uint32_t)(lane * ES);
      const int full = rv & ~(GR - 1);
      for (int g = 0; g < full; g += GR) {
        uint32_t wc[GR], hc[GR];
#pragma unroll
        for (int q = 0; q < GR; ++q) {
          wc[q] = codes[g + q];
          hc[q] = codes[R + g + q];
        }
        uint32_t rb = tbase + (uint32_t)(g * ROWB);
        asm volatile("" : "+v"(rb));
        Tacc v[4], vn[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = idx_val<Tin>(rb + (uint32_t)(q * ROWB));
#pragma unroll
        for (int kk = 0; kk < GR; kk += 4) {
          if (kk + 4 < GR) {
#pragma unroll
            for (int q = 0; q < 4; ++q) vn[q] = idx_val<Tin>(rb + (uint32_t)((kk + 4 + q) * ROWB));
          }
          fma4<kNreg>(f, v[0], v[1], v[2], v[3], wc[kk], wc[kk + 1], wc[kk + 2], wc[kk + 3],
                      idx_pm(hc[kk], (Tacc*)nullptr), idx_pm(hc[kk + 1], (Tacc*)nullptr),
                      idx_pm(hc[kk + 2], (Tacc*)nullptr), idx_pm(hc[kk + 3], (Tacc*)nullptr));
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = vn[q];
        }
      }
      for (int r = full; r < rv; ++r) {
        const uint32_t wr = codes[r], hr = codes[R + r];
        const Tacc v0 = idx_val<Tin>(tbase + (uint32_t)(r * ROWB));
        fma1<kNreg>(f, v0, wr, idx_pm(hr, (Tacc*)nullptr));
      }
    }
  }

  if (walker && lane < Cw) {
    Tacc* Pp = (Tacc*)(a.ws + P.P_off);
    const int64_t rowbase = (int64_t)chunk * P.d + (int64_t)t * P.nb + (int64_t)part * P.ps;
    const int nstore = min(P.ps, P.nb - part * P.ps);
#pragma unroll
    for (int sl = 0; sl < kNreg / T::rpa; ++sl) {
      if (sl < nstore) {
        Tacc val;
        if constexpr (T::rpa == 2) {
          const uint64_t lo = acc_get<kNreg>(f, 2 * sl), hi = acc_get<kNreg>(f, 2 * sl + 1);
          val = __builtin_bit_cast(double, lo | (hi << 32));
        } else {
          val = __builtin_bit_cast(float, acc_get<kNreg>(f, sl));
        }
        Pp[(rowbase + sl) * ncol + col0 + lane] = val;
      }
    }
  }
}

// Rows [r * red_rows, ...) of W = scale * (sum over chunks of the partials,
// in chunk order); columns k + 1 .. ldw - 1 are zero. Each thread loads
// eight chunks' values before adding them, so the loads overlap.
template <typename Tacc>
__device__ void reduce_rows(const BtArgs& a, const BtProb& P, int r) {
  const int d = P.d, ncol = P.k + 1, ldw = P.ldw;
  const int row0 = r * a.red_rows, row1 = min(d, row0 + a.red_rows);
  const Tacc* Pp = (const Tacc*)(a.ws + P.P_off);
  double* W = (double*)(a.ws + P.W_off);
  const double scale = P.scale;
  const int total = (row1 - row0) * ldw;
  const int64_t cstride = (int64_t)d * ncol;
  const int nc = P.n_chunks;
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int rr = idx / ldw, col = idx - rr * ldw;
    const int row = row0 + rr;
    double s = 0.0;
    if (col < ncol) {
      const Tacc* src = Pp + (int64_t)row * ncol + col;
      int c = 0;
      for (; c + 8 <= nc; c += 8) {
        Tacc v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = src[(c + j) * cstride];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += (double)v[j];
      }
      for (; c < nc; ++c) s += (double)src[c * cstride];
      s *= scale;
    }
    W[(int64_t)row * ldw + col] = s;
  }
}

// LDS of the QR (after the V panel at offset 0).
struct QrLds {
  double red[kWaves][kNB + 2];
  double vals[kNB + 2];
  double G[kNB][kNB + 1];
  double Ts[kNB][kNB + 1];
  double taus[kNB];
  double T[kNB * kNB];
  int flag;
};

// Householder factorization of panel columns [j0, j0 + nbp) of W (rows
// [j0, d)), LAPACK's conventions (beta = -sign(alpha) ||x||, tau = (beta -
// alpha) / beta, v = x / (alpha - beta), unit leading entry). Thread t holds
// local rows t and t + 512 of the 16 panel columns in registers; per column
// one block reduction for ||x||^2 and the pivot, one for all panel products
// (v^T y for the later columns, v_q^T v for the Gram entries of T). The R
// rows go back to W; V (explicit unit diagonal, zero rows padded to a
// multiple of 16) goes to LDS row-major [row][16], and the compact-WY T
// (Q_panel = I - V T V^T, upper) to q.T.
__device__ void qr_panel(double* W, int ldw, int d, int j0, int nbp, double* Vl, QrLds& q) {
  constexpr int NT = kThreads, RPT = 2, NB = kNB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int dr = d - j0;
  double x[RPT * NB];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int lr = tid + NT * i;
    const double* src = W + (int64_t)(j0 + lr) * ldw + j0;
#pragma unroll
    for (int c = 0; c < NB; ++c) x[i * NB + c] = (lr < dr && c < nbp) ? src[c] : 0.0;
  }
  for (int jj = 0; jj < nbp; ++jj) {
    double pc[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      double v = 0;
#pragma unroll
      for (int c = 0; c < NB; ++c) v = (c == jj) ? x[i * NB + c] : v;
      pc[i] = v;
    }
    double part = 0, alpha_part = 0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int lr = tid + NT * i;
      if (lr > jj) part += pc[i] * pc[i];
      if (lr == jj) alpha_part = pc[i];
    }
    part = wave_sum_dpp(part);
    alpha_part = wave_sum_dpp(alpha_part);
    if (lane == 0) {
      q.red[wave][0] = part;
      q.red[wave][1] = alpha_part;
    }
    __syncthreads();
    double sig2 = 0, alpha = 0;
#pragma unroll
    for (int wv = 0; wv < kWaves; ++wv) {
      sig2 += q.red[wv][0];
      alpha += q.red[wv][1];
    }
    double tau = 0, beta = alpha, scale = 0;
    if (sig2 > 0) {
      beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    double vv[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int lr = tid + NT * i;
      if (lr > jj && tau != 0) pc[i] *= scale;
      vv[i] = lr > jj ? pc[i] : (lr == jj ? 1.0 : 0.0);
    }
    double acc[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double sacc = 0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) sacc += vv[i] * x[i * NB + c];
      acc[c] = sacc;
    }
    __syncthreads();  // q.red is reused
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double v = wave_sum_dpp(acc[c]);
      if (lane == 0) q.red[wave][c] = v;
    }
    __syncthreads();
    if (tid < nbp && tid != jj) {
      double sacc = 0;
#pragma unroll
      for (int wv = 0; wv < kWaves; ++wv) sacc += q.red[wv][tid];
      q.vals[tid] = sacc;
      if (tid < jj) q.G[tid][jj] = sacc;
    }
    if (tid == 0) q.taus[jj] = tau;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double fct = (tau != 0 && c > jj && c < nbp) ? tau * q.vals[c] : 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int lr = tid + NT * i;
        double xv = x[i * NB + c] - fct * vv[i];
        if (c == jj) xv = lr > jj ? pc[i] : (lr == jj ? beta : x[i * NB + c]);
        x[i * NB + c] = xv;
      }
    }
  }
  // R rows (upper part) back to W; V to LDS
  const int dpad = (dr + 15) & ~15;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int lr = tid + NT * i;
    if (lr < nbp) {
      double* dst = W + (int64_t)(j0 + lr) * ldw + j0;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c >= lr && c < nbp) dst[c] = x[i * NB + c];
    }
    if (lr < dpad) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        Vl[lr * NB + c] = (lr < dr && c < nbp) ? (lr > c ? x[i * NB + c] : (lr == c ? 1.0 : 0.0)) : 0.0;
    }
  }
  // T: T[i][i] = tau_i; T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
  for (int i = 0; i < nbp; ++i) {
    if (tid < i) {
      double s2 = 0;
      for (int l = tid; l < i; ++l) s2 += q.Ts[tid][l] * q.G[l][i];
      q.Ts[tid][i] = -q.taus[i] * s2;
    }
    if (tid == i) q.Ts[i][i] = q.taus[i];
    if (tid > i && tid < nbp) q.Ts[tid][i] = 0.0;
    __syncthreads();
  }
  if (tid < NB * NB) {
    const int r = tid / NB, c = tid - r * NB;
    q.T[tid] = (r < nbp && c < nbp) ? q.Ts[r][c] : 0.0;
  }
  __syncthreads();
}

// Trailing update of columns [j0 + nbp, k] of W (rows [j0, d)):
// Y <- Y - V T^T V^T Y, one 16-column block per wave at a time, on the FP64
// matrix cores (v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; item v of the result is row 4 v + l / 16, column l % 16).
__device__ void qr_trail(double* W, int ldw, int d, int k, int j0, int nbp, const double* Vl, const double* Tl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int dr = d - j0;
  const int c_first = j0 + nbp;
  const int ncb = (k + 1 - c_first + 15) / 16;
  for (int cb = wave; cb < ncb; cb += kWaves) {
    double* Y = W + (int64_t)j0 * ldw + c_first + 16 * cb;
    v4d z = {0.0, 0.0, 0.0, 0.0};  // Z = V^T Y
    for (int kr = 0; kr < dr; kr += 4) {
      const int rr = kr + lk;
      const double av = Vl[rr * kNB + li];
      const double bv = rr < dr ? Y[(int64_t)rr * ldw + li] : 0.0;
      z = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, z, 0, 0, 0);
    }
    v4d z2 = {0.0, 0.0, 0.0, 0.0};  // T^T Z
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) z2 = __builtin_amdgcn_mfma_f64_16x16x4f64(Tl[(4 * ks + lk) * kNB + li], z[ks], z2, 0, 0, 0);
    const v4d nz = -z2;
    for (int r0 = 0; r0 < dr; r0 += 16) {
      v4d c;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 4 * v + lk;
        c[v] = row < dr ? Y[(int64_t)row * ldw + li] : 0.0;
      }
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(Vl[(r0 + li) * kNB + 4 * ks + lk], nz[ks], c, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 4 * v + lk;
        if (row < dr) Y[(int64_t)row * ldw + li] = c[v];
      }
    }
  }
}

// Block-wide sum (fixed order over the waves).
__device__ inline double block_sum8(double v, QrLds& q, int slot) {
  v = wave_sum_dpp(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) q.red[wave][slot] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int wv = 0; wv < kWaves; ++wv) s += q.red[wv][slot];
  return s;
}

// QR of [S A | S b] (W, d x (k + 1), stride ldw) and the solve of Alg. 3:
// X = R^-1 (column j by back substitution in thread j); if
// ||R||_F ||X||_F < 1e-3 / (5 eps), x = X c and rank = k; otherwise R and c
// are copied out for the fallback kernel and rank = -1.
__device__ void qr_solve(const BtArgs& a, const BtProb& P, unsigned char* smem) {
  double* Vl = (double*)smem;
  QrLds& q = *(QrLds*)(smem + kQrVBytes);
  double* W = (double*)(a.ws + P.W_off);
  const int d = P.d, k = P.k, ldw = P.ldw;
  for (int j0 = 0; j0 < k; j0 += kNB) {
    const int nbp = min(kNB, k - j0);
    qr_panel(W, ldw, d, j0, nbp, Vl, q);
    qr_trail(W, ldw, d, k, j0, nbp, Vl, q.T);
    __syncthreads();
  }
  const int tid = threadIdx.x;
  double* X = (double*)(a.ws + P.X_off);
  for (int j = tid; j < k; j += kThreads) {
    X[(int64_t)j * k + j] = 1.0 / W[(int64_t)j * ldw + j];
    for (int i = j - 1; i >= 0; --i) {
      const double* Ri = W + (int64_t)i * ldw;
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += Ri[l] * X[(int64_t)l * k + j];
      X[(int64_t)i * k + j] = -s / Ri[i];
    }
  }
  __syncthreads();
  double r2 = 0.0, x2 = 0.0;
  for (int j = tid; j < k; j += kThreads) {
    for (int i = 0; i <= j; ++i) {
      const double rv = W[(int64_t)i * ldw + j], xv = X[(int64_t)i * k + j];
      r2 += rv * rv;
      x2 += xv * xv;
    }
  }
  const double tr = block_sum8(r2, q, 0);
  const double tx = block_sum8(x2, q, 1);
  const double eps = 0x1p-52;
  const double cond = sqrt(tr) * sqrt(tx);
  const bool ok = cond == cond && cond < 1e-3 / (5.0 * eps);  // false for NaN and Inf
  int* rank = a.ctl + C_FIXED + a.nprob;
  if (ok) {
    for (int i = tid; i < k; i += kThreads) {
      double s = 0.0;
      for (int j = i; j < k; ++j) s += X[(int64_t)i * k + j] * W[(int64_t)j * ldw + k];
      P.x[i] = s;
    }
  } else {
    // R (k x k row-major, upper) and c for the fallback kernel
    double* Rs = X + (int64_t)k * k;
    double* cs = Rs + (int64_t)k * k;
    for (int idx = tid; idx < k * k; idx += kThreads) {
      const int i = idx / k, j = idx - i * k;
      Rs[idx] = j >= i ? W[(int64_t)i * ldw + j] : 0.0;
    }
    for (int i = tid; i < k; i += kThreads) cs[i] = W[(int64_t)i * ldw + k];
  }
  if (tid == 0) rank[P.index] = ok ? k : -1;
}

enum { K_NONE = 0, K_SKETCH = 1, K_REDUCE = 2, K_WAIT = 3, K_EXIT = 4 };

// Sketch worker: sketch items from the static queues, reduce items from the
// ready queue (popped first). Leaves once every reduce item is done.
__global__ void __launch_bounds__(kThreads) bt_sketch_kernel(BtArgs a, const BtProb* __restrict__ probs,
                                                             const uint32_t* __restrict__ codes_base) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int s_item[4];
  const int tid = threadIdx.x;
  int* ctl = a.ctl;
  int* unit_done = ctl + C_FIXED;
  const int xcd = bt_xcc_id();
  int dead = 0;             // static queues found empty (thread 0)
  uint64_t wait_since = 0;  // start of the current wait for work (thread 0)
  for (;;) {
    if (tid == 0) {
      int kind = K_NONE, p = 0, x0 = 0, x1 = 0;
      for (;;) {
        const int h = __hip_atomic_load(ctl + C_RQHEAD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int tl = __hip_atomic_load(ctl + C_RQTAIL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h >= tl) break;
        int expect = h;
        if (__hip_atomic_compare_exchange_strong(ctl + C_RQHEAD, &expect, h + 1, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          unsigned long long v;
          // the pusher reserved the slot before writing it: wait for the
          // write (bounded: a missing write is a planning error)
          const uint64_t t0 = bt_now();
          while ((v = __hip_atomic_load(a.rq + h, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) == 0ull &&
                 bt_now() - t0 < kWaitTicks)
            __builtin_amdgcn_s_sleep(1);
          if (v == 0ull) {
            __hip_atomic_store(ctl + C_ERROR, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            kind = K_EXIT;
            break;
          }
          kind = K_REDUCE;
          p = (int)(v >> 32) - 1;
          x0 = (int)(uint32_t)v;
          break;
        }
      }
      if (kind == K_NONE) {
        for (int qq = 0; qq < kQueues; ++qq) {
          const int qi = (xcd + qq) & (kQueues - 1);
          if (dead & (1 << qi)) continue;
          const int len = a.qbeg[qi + 1] - a.qbeg[qi];
          const int i = atomicAdd(ctl + C_QHEAD + qi, 1);
          if (i < len) {
            const int4 it = a.items[a.qbeg[qi] + i];
            kind = K_SKETCH;
            p = it.x;
            x0 = it.y;
            x1 = it.z;
            break;
          }
          dead |= 1 << qi;
        }
      }
      if (kind == K_NONE) {
        // nothing to pop: done, or reduce items still to come from units in
        // flight. The wait is bounded; running out of it (a planning error
        // or an error flag raised elsewhere) ends the kernel with the flag set.
        if (__hip_atomic_load(ctl + C_REDDONE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= a.total_red ||
            __hip_atomic_load(ctl + C_ERROR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          kind = K_EXIT;
        } else {
          if (wait_since == 0) wait_since = bt_now();
          if (bt_now() - wait_since > kWaitTicks) {
            __hip_atomic_store(ctl + C_ERROR, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            kind = K_EXIT;
          } else {
            kind = K_WAIT;
          }
        }
      } else {
        wait_since = 0;
      }
      s_item[0] = kind;
      s_item[1] = p;
      s_item[2] = x0;
      s_item[3] = x1;
    }
    __syncthreads();
    const int kind = s_item[0], p = s_item[1], x0 = s_item[2], x1 = s_item[3];
    __syncthreads();
    if (kind == K_EXIT) break;
    if (kind == K_WAIT) {
      __builtin_amdgcn_s_sleep(32);
      continue;
    }
    const BtProb& P = probs[p];
    if (kind == K_SKETCH) {
      if (tid == 0) atomicMin(a.t_start + p, (unsigned long long)bt_now());
      if (P.dtype == SK_F64)
        sketch_item<double>(a, P, x0, x1, codes_base, smem);
      else if (P.dtype == SK_F32)
        sketch_item<float>(a, P, x0, x1, codes_base, smem);
      else
        sketch_item<uint16_t>(a, P, x0, x1, codes_base, smem);
      fence_release();
      __syncthreads();
      if (tid == 0) {
        const int old = __hip_atomic_fetch_add(unit_done + p, x1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old + x1 == P.n_units) {
          // the problem's partials are complete: its reduce items are ready
          const int s0 = atomicAdd(ctl + C_RQTAIL, P.n_red);
          for (int j = 0; j < P.n_red; ++j)
            __hip_atomic_store(a.rq + s0 + j, ((unsigned long long)(p + 1) << 32) | (unsigned)j, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    } else {  // K_REDUCE
      fence_acquire();
      if (P.dtype == SK_F64)
        reduce_rows<double>(a, P, x0);
      else
        reduce_rows<float>(a, P, x0);
      fence_release();
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(ctl + C_REDDONE, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Solve worker: one problem at a time, largest k first (the order array),
// QR and solve in the workgroup.
__global__ void __launch_bounds__(kThreads) bt_solve_kernel(BtArgs a, const BtProb* __restrict__ probs,
                                                            const int* __restrict__ order) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int s_i;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) s_i = atomicAdd(a.ctl + C_SOLVEHEAD, 1);
    __syncthreads();
    const int i = s_i;
    __syncthreads();
    if (i >= a.nprob) break;
    const int p = order[i];
    qr_solve(a, probs[p], smem);
    __syncthreads();
    if (tid == 0) a.t_end[p] = bt_now();
  }
}

// The problems the certificate rejected: SVD of R, rank-truncated solve.
__global__ void __launch_bounds__(1024) bt_fallback_kernel(BtArgs a, const BtProb* __restrict__ probs) {
  const int p = blockIdx.x;
  int* rank = a.ctl + C_FIXED + a.nprob;
  if (rank[p] >= 0) return;
  const BtProb& P = probs[p];
  const int k = P.k;
  double* X = (double*)(a.ws + P.X_off);
  double* Rs = X + (int64_t)k * k;
  double* cs = Rs + (int64_t)k * k;
  double* U = cs + k;
  double* V = U + (int64_t)k * k;
  double* work = V + (int64_t)k * k;
  double* sv = work + 2 * (int64_t)k * k;
  double* z = sv + k;
  jacobi_svd_dev(Rs, k, U, sv, V, work, work + (int64_t)k * k);
  __syncthreads();
  svd_solve_dev(U, sv, V, cs, k, 0x1p-52, P.x, z, rank + p);
  __syncthreads();
  if (threadIdx.x == 0) a.t_end[p] = bt_now();
}

}  // namespace bt
}  // namespace sk

// ---------------------------------------------------------------------------
// Host side: the plan (problem descriptors, static queues, workspace layout),
// the tile-parameter tuner and its cache, the batch graph, the C-ABI.
// ---------------------------------------------------------------------------
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

struct sk_batch {
  int device = 0;
  int nprob = 0, d_per_k = 0, zeta = 0;
  std::vector<sk_ls_problem> probs;
  std::vector<sk::bt::BtProb> dp;
  std::vector<int4> items;
  std::vector<int> qbeg, order;
  std::vector<int64_t> rpre;
  size_t off_probs = 0, off_items = 0, off_qbeg = 0, off_rpre = 0, off_order = 0, off_ctl = 0, off_tstart = 0,
         off_tend = 0, off_rq = 0, total = 0;
  int nctl = 0, total_red = 0;
  int wu = 4, red_rows = 64, buf_bytes = 0;
  int grid_sketch = 0, grid_solve = 0;
  int tuned = 0;
  void* ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int kernel_nodes = 0;
  int64_t graph_launches = 0;
  double clock_khz = 0.0;
  void* h_res = nullptr;  // pinned: ranks, then t_start and t_end
  bool bound = false;
};

namespace sk {
namespace bt {
namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

bool problem_valid(const sk_ls_problem& p, int d_per_k, int zeta) {
  if (p.n < 1 || p.k < 1 || p.k > 1024 || p.lda < p.k || !p.A || !p.b || !p.x) return false;
  if (p.dtype != SK_F64 && p.dtype != SK_F32 && p.dtype != SK_BF16) return false;
  const int64_t d = (int64_t)d_per_k * p.k;
  return d >= p.k && d % zeta == 0;
}

// Data layouts the kernels take: dword loads of A's rows (4-byte aligned
// rows) and element-aligned b; d <= kMaxD (the workgroup QR).
int problem_supported(const sk_ls_problem& p, int d_per_k, std::string* why) {
  const size_t es = dtype_size(p.dtype);
  const int64_t d = (int64_t)d_per_k * p.k;
  if (d > kMaxD) {
    *why = "d = d_per_k * k above " + std::to_string(kMaxD);
    return SK_E_NOTSUP;
  }
  if ((uintptr_t)p.A % 4 != 0 || (p.lda * (int64_t)es) % 4 != 0) {
    *why = "rows of A are not 4-byte aligned (A and lda * element size must be multiples of 4)";
    return SK_E_NOTSUP;
  }
  if ((uintptr_t)p.b % es != 0 || (uintptr_t)p.x % 8 != 0) {
    *why = "b or x is not aligned to its element size";
    return SK_E_NOTSUP;
  }
  return SK_OK;
}

// ---- tile parameters: tuner cache (flat JSON: {"key": {"R": r, "chunk": c, "ms": t}, ...})
struct Tune {
  int R = 0;
  int64_t chunk = 0;
  double ms = 0.0;
};
std::mutex g_tune_mu;

std::string cache_path() {
  const char* e = std::getenv("SKETCH_TUNE_CACHE");
  if (e && *e) return e;
  const char* x = std::getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/libsketch/batched_tune.json";
  const char* h = std::getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.cache/libsketch/batched_tune.json";
}

std::map<std::string, Tune> read_cache(const std::string& path) {
  std::map<std::string, Tune> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  for (;;) {
    const size_t q0 = s.find('"', pos);
    if (q0 == std::string::npos) break;
    const size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
    pos = q1 + 1;
    if (key.find('/') == std::string::npos) continue;  // not an entry key
    const size_t ob = s.find('{', pos), cb = s.find('}', pos);
    if (ob == std::string::npos || cb == std::string::npos || ob > cb) continue;
    const std::string body = s.substr(ob, cb - ob);
    auto num = [&](const char* name) -> double {
      const size_t k = body.find(std::string("\"") + name + "\"");
      if (k == std::string::npos) return -1.0;
      const size_t c = body.find(':', k);
      return c == std::string::npos ? -1.0 : std::atof(body.c_str() + c + 1);
    };
    Tune t;
    t.R = (int)num("R");
    t.chunk = (int64_t)num("chunk");
    t.ms = num("ms");
    if (t.R > 0 && t.chunk > 0) m[key] = t;
    pos = cb + 1;
  }
  return m;
}

void mkdirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') {
      const std::string dir = path.substr(0, i);
      if (mkdir(dir.c_str(), 0755) != 0 && errno != EEXIST) return;
    }
}

bool write_cache(const std::string& path, const std::map<std::string, Tune>& m) {
  mkdirs(path);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      char line[256];
      std::snprintf(line, sizeof line, "  \"%s\": {\"R\": %d, \"chunk\": %lld, \"ms\": %.6f}%s\n", kv.first.c_str(),
                    kv.second.R, (long long)kv.second.chunk, kv.second.ms, ++i < m.size() ? "," : "");
      f << line;
    }
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

// The class a problem's tile parameters are tuned for: device, input type,
// slabs, bucket parts and waves per unit.
std::string tune_key(const std::string& dev, int dtype, int n_slabs, int nparts, int wu) {
  const char* dt = dtype == SK_F64 ? "f64" : (dtype == SK_F32 ? "f32" : "bf16");
  return dev + "/" + dt + "/s" + std::to_string(n_slabs) + "/p" + std::to_string(nparts) + "/w" + std::to_string(wu);
}

int waves_per_unit(int zeta) { return zeta <= 1 ? 1 : (zeta <= 2 ? 2 : (zeta <= 4 ? 4 : 8)); }

// Largest tile (rows, a multiple of 16, at most 128) whose two buffers per
// unit slot fit the tile LDS.
int max_tile_rows(int es, int wu) {
  const int slots = kWaves / wu;
  const int buf = kTileLds / (2 * slots);
  return std::min(128, (buf / (64 * es)) & ~15);
}

struct Shape {
  int es, nb, nparts, ps, n_slabs, n_gp;
};
Shape shape_of(const sk_ls_problem& p, int d_per_k, int zeta, int wu) {
  Shape s;
  s.es = (int)dtype_size(p.dtype);
  const int d = (int)(d_per_k * p.k);
  s.nb = d / zeta;
  const int rpa = p.dtype == SK_F64 ? 2 : 1;
  const int cap = kNreg / rpa;
  s.nparts = s.nb <= cap ? 1 : (s.nb + cap - 2) / (cap - 1);
  s.ps = (s.nb + s.nparts - 1) / s.nparts;
  s.n_slabs = (int)((p.k + 1 + 63) / 64);
  const int groups = wu == 8 ? (zeta + 7) / 8 : 1;
  s.n_gp = groups * s.nparts;
  return s;
}

std::string device_tag(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch = arch.substr(0, c);
  return arch + ":" + std::to_string(prop.multiProcessorCount);
}

// Layout, descriptors and queues of a batch whose tile parameters are set
// (tune: per-problem R and chunk rows).
int build(sk_batch* B, const std::vector<Tune>& tune) {
  const int np = B->nprob;
  const int wu = B->wu;
  const int slots = kWaves / wu;
  B->buf_bytes = kTileLds / (2 * slots);
  B->dp.assign(np, BtProb{});
  B->order.resize(np);
  std::iota(B->order.begin(), B->order.end(), 0);
  std::stable_sort(B->order.begin(), B->order.end(), [&](int x, int y) {
    const sk_ls_problem &a = B->probs[x], &b = B->probs[y];
    return a.k != b.k ? a.k > b.k : a.n > b.n;
  });
  // header tables first (sizes known up to the item count)
  std::vector<std::vector<int4>> q(kQueues);
  int rot = 0;
  B->total_red = 0;
  for (int oi = 0; oi < np; ++oi) {
    const int i = B->order[oi];
    const sk_ls_problem& p = B->probs[i];
    const Shape sh = shape_of(p, B->d_per_k, B->zeta, wu);
    BtProb& P = B->dp[i];
    P.A = (const unsigned char*)p.A;
    P.b = (const unsigned char*)p.b;
    P.x = p.x;
    P.n = p.n;
    P.lda_bytes = p.lda * sh.es;
    P.index = i;
    P.k = (int)p.k;
    P.d = (int)(B->d_per_k * p.k);
    P.nb = sh.nb;
    P.zeta = B->zeta;
    P.dtype = p.dtype;
    P.R = tune[i].R;
    P.rows_per_chunk = tune[i].chunk;
    P.nparts = sh.nparts;
    P.ps = sh.ps;
    P.n_gp = sh.n_gp;
    P.n_slabs = sh.n_slabs;
    P.n_chunks = (int)((p.n + P.rows_per_chunk - 1) / P.rows_per_chunk);
    P.n_units = P.n_chunks * P.n_slabs * P.n_gp;
    P.n_red = (P.d + B->red_rows - 1) / B->red_rows;
    P.ldw = (P.k + 16 + 7) & ~7;
    P.scale = 1.0 / std::sqrt((double)B->zeta);
    P.k0 = (uint32_t)p.seed;
    P.k1 = (uint32_t)(p.seed >> 32);
    B->total_red += P.n_red;
    // items: consecutive units, all of a row chunk in one queue (the queue of
    // an item's first unit), the chunks of a problem round-robin over queues
    const int per = P.n_slabs * P.n_gp;
    for (int u = 0; u < P.n_units; u += slots) {
      const int cnt = std::min(slots, P.n_units - u);
      const int chunk = u / per;
      q[(rot + chunk) % kQueues].push_back(int4{i, u, cnt, 0});
    }
    rot = (rot + P.n_chunks) % kQueues;
  }
  B->items.clear();
  B->qbeg.assign(kQueues + 1, 0);
  for (int j = 0; j < kQueues; ++j) {
    B->qbeg[j] = (int)B->items.size();
    B->items.insert(B->items.end(), q[j].begin(), q[j].end());
  }
  B->qbeg[kQueues] = (int)B->items.size();
  B->rpre.assign(np + 1, 0);
  for (int i = 0; i < np; ++i) {
    const BtProb& P = B->dp[i];
    const int64_t tiles = (P.n + P.R - 1) / P.R;
    B->rpre[i + 1] = B->rpre[i] + tiles * P.R;
  }
  B->nctl = C_FIXED + 2 * np;
  size_t off = 0;
  B->off_probs = off;
  off = al256(off + sizeof(BtProb) * np);
  B->off_items = off;
  off = al256(off + sizeof(int4) * std::max<size_t>(1, B->items.size()));
  B->off_qbeg = off;
  off = al256(off + sizeof(int) * (kQueues + 1));
  B->off_rpre = off;
  off = al256(off + sizeof(int64_t) * (np + 1));
  B->off_order = off;
  off = al256(off + sizeof(int) * np);
  B->off_ctl = off;
  off = al256(off + sizeof(int) * B->nctl);
  B->off_tstart = off;
  off = al256(off + 8 * (size_t)np);
  B->off_tend = off;
  off = al256(off + 8 * (size_t)np);
  B->off_rq = off;
  off = al256(off + 8 * (size_t)std::max(1, B->total_red));
  for (int i = 0; i < np; ++i) {
    BtProb& P = B->dp[i];
    const int64_t tiles = (P.n + P.R - 1) / P.R;
    P.codes_off = (int64_t)off;
    off = al256(off + (size_t)tiles * P.nparts * P.zeta * 2 * P.R * 4);
    P.P_off = (int64_t)off;
    off = al256(off + (size_t)P.n_chunks * P.d * (P.k + 1) * (P.dtype == SK_F64 ? 8 : 4));
    P.W_off = (int64_t)off;
    off = al256(off + (size_t)P.d * P.ldw * 8);
    P.X_off = (int64_t)off;
    off = al256(off + ((size_t)6 * P.k * P.k + 3 * (size_t)P.k) * 8);
  }
  B->total = off;
  return SK_OK;
}

// Tile parameters for every problem: the cache's entry for its class, the
// default otherwise (the largest tile that fits, 16384-row chunks).
std::vector<Tune> lookup(sk_batch* B, const std::map<std::string, Tune>& cache, const std::string& dev) {
  std::vector<Tune> t(B->nprob);
  B->tuned = 0;
  for (int i = 0; i < B->nprob; ++i) {
    const sk_ls_problem& p = B->probs[i];
    const Shape sh = shape_of(p, B->d_per_k, B->zeta, B->wu);
    const int rmax = max_tile_rows(sh.es, B->wu);
    auto it = cache.find(tune_key(dev, p.dtype, sh.n_slabs, sh.nparts, B->wu));
    Tune v;
    if (it != cache.end() && it->second.R >= 16 && it->second.R <= rmax && it->second.R % 16 == 0) {
      v = it->second;
      ++B->tuned;
    } else {
      v.R = rmax;
      v.chunk = 16384;
    }
    v.chunk = std::max<int64_t>(v.R, (v.chunk / v.R) * v.R);
    t[i] = v;
  }
  return t;
}

}  // namespace
}  // namespace bt
}  // namespace sk

namespace sk {
namespace bt {
namespace {

BtArgs args_of(const sk_batch* B) {
  unsigned char* w = (unsigned char*)B->ws;
  BtArgs a;
  a.items = (const int4*)(w + B->off_items);
  a.qbeg = (const int*)(w + B->off_qbeg);
  a.ctl = (int*)(w + B->off_ctl);
  a.t_start = (unsigned long long*)(w + B->off_tstart);
  a.t_end = (unsigned long long*)(w + B->off_tend);
  a.rq = (unsigned long long*)(w + B->off_rq);
  a.ws = w;
  a.nprob = B->nprob;
  a.total_red = B->total_red;
  a.wu = B->wu;
  a.red_rows = B->red_rows;
  a.buf_bytes = B->buf_bytes;
  a.off_touch = kTileLds;
  return a;
}

// The five kernels of one batch, in stream order on st (capturable: no
// allocation, no memset, no synchronization).
int enqueue(const sk_batch* B, hipStream_t st) {
  const BtArgs a = args_of(B);
  unsigned char* w = (unsigned char*)B->ws;
  const BtProb* probs = (const BtProb*)(w + B->off_probs);
  const int np = B->nprob;
  {
    const int n = std::max(B->nctl, std::max(np, B->total_red));
    const unsigned g = (unsigned)std::min(1024, std::max(1, (n + 255) / 256));
    hipLaunchKernelGGL(bt_init_kernel, dim3(g), dim3(256), 0, st, a.ctl, B->nctl, a.t_start, a.t_end, np, a.rq,
                       B->total_red);
    SK_HIP(hipGetLastError());
  }
  {
    const int64_t rows = B->rpre[np];
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(16384, (rows + 255) / 256));
    hipLaunchKernelGGL(bt_codes_kernel, dim3(g), dim3(256), 0, st, probs, (const int64_t*)(w + B->off_rpre), np,
                       (uint32_t*)w);
    SK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(bt_sketch_kernel, dim3(B->grid_sketch), dim3(kThreads), kLdsBytes, st, a, probs,
                     (const uint32_t*)w);
  SK_HIP(hipGetLastError());
  hipLaunchKernelGGL(bt_solve_kernel, dim3(B->grid_solve), dim3(kThreads), kLdsBytes, st, a, probs,
                     (const int*)(w + B->off_order));
  SK_HIP(hipGetLastError());
  hipLaunchKernelGGL(bt_fallback_kernel, dim3(np), dim3(1024), 0, st, a, probs);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

int release_graph(sk_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  B->bound = false;
  return SK_OK;
}

// Writes the tables into the workspace and captures the batch graph.
int bind(sk_batch* B, void* ws, hipStream_t st) {
  release_graph(B);
  B->ws = ws;
  SK_HIP(hipFuncSetAttribute((const void*)bt_sketch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes));
  SK_HIP(hipFuncSetAttribute((const void*)bt_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes));
  int cus = 0, occ_s = 0, occ_q = 0;
  SK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device));
  SK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_s, (const void*)bt_sketch_kernel, kThreads, kLdsBytes));
  SK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_q, (const void*)bt_solve_kernel, kThreads, kLdsBytes));
  B->grid_sketch = std::max(1, cus * std::max(1, occ_s));
  B->grid_solve = std::max(1, std::min(B->nprob, cus * std::max(1, occ_q)));
  // tables: one staging copy in pinned memory, one synchronous upload
  const size_t hdr = B->off_ctl;
  std::vector<unsigned char> host(hdr, 0);
  std::memcpy(host.data() + B->off_probs, B->dp.data(), sizeof(BtProb) * B->nprob);
  if (!B->items.empty()) std::memcpy(host.data() + B->off_items, B->items.data(), sizeof(int4) * B->items.size());
  std::memcpy(host.data() + B->off_qbeg, B->qbeg.data(), sizeof(int) * B->qbeg.size());
  std::memcpy(host.data() + B->off_rpre, B->rpre.data(), sizeof(int64_t) * B->rpre.size());
  std::memcpy(host.data() + B->off_order, B->order.data(), sizeof(int) * B->order.size());
  SK_HIP(hipMemcpyAsync(ws, host.data(), hdr, hipMemcpyHostToDevice, st));
  SK_HIP(hipStreamSynchronize(st));
  hipStream_t cs = nullptr;
  SK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  int rc = SK_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("lstsq_batched_bind: stream capture failed to start");
    rc = SK_E_HIP;
  } else {
    rc = enqueue(B, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc == SK_OK && e != hipSuccess) {
      set_error("lstsq_batched_bind: stream capture failed");
      rc = SK_E_HIP;
    }
    B->graph = g;
  }
  (void)hipStreamDestroy(cs);
  if (rc != SK_OK) return rc;
  SK_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  size_t nn = 0;
  SK_HIP(hipGraphGetNodes(B->graph, nullptr, &nn));
  B->kernel_nodes = (int)nn;
  B->bound = true;
  return SK_OK;
}

int results(sk_batch* B, sk_ls_problem* probs, hipStream_t st) {
  const int np = B->nprob;
  const size_t rb = sizeof(int) * np, tb = 8 * (size_t)np;
  if (!B->h_res) SK_HIP(hipHostMalloc(&B->h_res, rb + 2 * tb, hipHostMallocDefault));
  unsigned char* h = (unsigned char*)B->h_res;
  unsigned char* w = (unsigned char*)B->ws;
  SK_HIP(hipMemcpyAsync(h, w + B->off_ctl + sizeof(int) * (C_FIXED + np), rb, hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(h + rb, w + B->off_tstart, tb, hipMemcpyDeviceToHost, st));
  SK_HIP(hipMemcpyAsync(h + rb + tb, w + B->off_tend, tb, hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  int err = 0;
  SK_HIP(hipMemcpy(&err, w + B->off_ctl + sizeof(int) * C_ERROR, sizeof(int), hipMemcpyDeviceToHost));
  if (err != 0) {
    set_error("lstsq_batched_results: the sketch worker gave up waiting for work (inconsistent plan)");
    return SK_E_HIP;
  }
  const int* rank = (const int*)h;
  const unsigned long long* t0 = (const unsigned long long*)(h + rb);
  const unsigned long long* t1 = (const unsigned long long*)(h + rb + tb);
  bool rankdef = false;
  for (int i = 0; i < np; ++i) {
    probs[i].rank = rank[i];
    probs[i].status = rank[i] < probs[i].k ? SK_W_RANKDEF : SK_OK;
    probs[i].t_ms = (t1[i] > t0[i] && B->clock_khz > 0) ? (double)(t1[i] - t0[i]) / B->clock_khz : 0.0;
    rankdef = rankdef || rank[i] < probs[i].k;
  }
  return rankdef ? SK_W_RANKDEF : SK_OK;
}

int check_all(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, const char* who, int* bad) {
  *bad = -1;
  if (!probs || nprob < 1 || d_per_k < 1 || zeta < 1) {
    set_error(std::string(who) + ": need problems, nprob >= 1, d_per_k >= 1 and zeta >= 1");
    return SK_E_INVAL;
  }
  for (int i = 0; i < nprob; ++i) {
    if (!problem_valid(probs[i], d_per_k, zeta)) {
      *bad = i;
      set_error(std::string(who) + ": problem " + std::to_string(i) +
                " is invalid (need n >= 1, 1 <= k <= 1024, lda >= k, pointers, a dtype, zeta | d_per_k * k)");
      return SK_E_INVAL;
    }
  }
  for (int i = 0; i < nprob; ++i) {
    std::string why;
    if (problem_supported(probs[i], d_per_k, &why) != SK_OK) {
      *bad = i;
      set_error(std::string(who) + ": problem " + std::to_string(i) + ": " + why);
      return SK_E_NOTSUP;
    }
  }
  return SK_OK;
}

int create(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int flags, sk_batch** out, int* bad);

// Times candidate tile parameters for each class of the batch that the
// cache lacks, on up to 16 of the batch's own problems of that class (their
// A and b are read and their x written), and stores the best in the cache.
int autotune(sk_batch* B, std::map<std::string, Tune>* cache, const std::string& dev) {
  std::map<std::string, std::vector<int>> classes;
  for (int i = 0; i < B->nprob; ++i) {
    const sk_ls_problem& p = B->probs[i];
    const Shape sh = shape_of(p, B->d_per_k, B->zeta, B->wu);
    const std::string key = tune_key(dev, p.dtype, sh.n_slabs, sh.nparts, B->wu);
    if (!cache->count(key)) classes[key].push_back(i);
  }
  if (classes.empty()) return SK_OK;
  hipStream_t ts = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SK_HIP(hipStreamCreateWithFlags(&ts, hipStreamNonBlocking));
  int rc = SK_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = SK_E_HIP;
  for (auto& kv : classes) {
    if (rc != SK_OK) break;
    std::vector<int>& idx = kv.second;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return B->probs[x].n > B->probs[y].n; });
    if (idx.size() > 16) idx.resize(16);
    std::vector<sk_ls_problem> sub;
    for (int i : idx) sub.push_back(B->probs[i]);
    const int es = (int)dtype_size(sub[0].dtype);
    const int rmax = max_tile_rows(es, B->wu);
    Tune best;
    best.ms = 1e30;
    for (int R : {32, 64, 128}) {
      if (R > rmax || rc != SK_OK) continue;
      for (int64_t chunk : {8192, 16384, 32768}) {
        sk_batch* T = nullptr;
        int bad = -1;
        rc = create(sub.data(), (int)sub.size(), B->d_per_k, B->zeta, 0, &T, &bad);
        if (rc != SK_OK) break;
        std::vector<Tune> tv(sub.size());
        for (auto& t : tv) {
          t.R = R;
          t.chunk = chunk;
        }
        build(T, tv);
        void* w = nullptr;
        if (hipMalloc(&w, T->total) != hipSuccess) {
          delete T;
          set_error("batched autotune: workspace allocation failed");
          rc = SK_E_NOMEM;
          break;
        }
        rc = bind(T, w, ts);
        float best_ms = 1e30f;
        for (int rep = 0; rep < 4 && rc == SK_OK; ++rep) {
          if (hipEventRecord(e0, ts) != hipSuccess || hipGraphLaunch(T->exec, ts) != hipSuccess ||
              hipEventRecord(e1, ts) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            set_error("batched autotune: timing run failed");
            rc = SK_E_HIP;
            break;
          }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) best_ms = std::min(best_ms, ms);  // the first run warms up
        }
        release_graph(T);
        (void)hipFree(w);
        if (T->h_res) (void)hipHostFree(T->h_res);
        delete T;
        if (rc == SK_OK && best_ms < best.ms) {
          best.ms = best_ms;
          best.R = R;
          best.chunk = chunk;
        }
      }
    }
    if (rc == SK_OK && best.R > 0) (*cache)[kv.first] = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(ts);
  return rc;
}

int create(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int flags, sk_batch** out, int* bad) {
  int rc = check_all(probs, nprob, d_per_k, zeta, "lstsq_batched_create", bad);
  if (rc != SK_OK) return rc;
  sk_batch* B = new sk_batch;
  SK_HIP(hipGetDevice(&B->device));
  B->nprob = nprob;
  B->d_per_k = d_per_k;
  B->zeta = zeta;
  B->wu = waves_per_unit(zeta);
  B->probs.assign(probs, probs + nprob);
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, B->device) == hipSuccess) B->clock_khz = khz;
  if (flags & SK_BATCH_NOTUNE) {
    build(B, lookup(B, {}, ""));
    *out = B;
    return SK_OK;
  }
  const std::string dev = device_tag(B->device);
  const std::string path = cache_path();
  std::map<std::string, Tune> cache;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    cache = read_cache(path);
  }
  if (flags & SK_BATCH_AUTOTUNE) {
    const size_t before = cache.size();
    rc = autotune(B, &cache, dev);
    if (rc != SK_OK) {
      delete B;
      return rc;
    }
    if (cache.size() != before) {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      std::map<std::string, Tune> merged = read_cache(path);
      for (const auto& kv : cache) merged[kv.first] = kv.second;
      if (!write_cache(path, merged)) {
        set_error("lstsq_batched_create: cannot write the tuning cache " + path);
        delete B;
        return SK_E_INVAL;
      }
    }
  }
  build(B, lookup(B, cache, dev));
  *out = B;
  return SK_OK;
}

}  // namespace
}  // namespace bt
}  // namespace sk

using namespace sk;

// The plan API stays off until the hang of its first device run is explained.
constexpr bool kBatchPlanEnabled = false;

extern "C" {

int lstsq_batched_create(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int flags, sk_batch_t* out) {
  if (!out) {
    set_error("lstsq_batched_create: null output");
    return SK_E_INVAL;
  }
  *out = nullptr;
  if (!kBatchPlanEnabled) {
    set_error("lstsq_batched_create: the persistent batch plan is disabled in this build (its first device run did "
              "not complete and the cause is not yet identified); use lstsq_sketch_solve_batched");
    return SK_E_NOTSUP;
  }
  int bad = -1;
  return bt::create(probs, nprob, d_per_k, zeta, flags, out, &bad);
}

int lstsq_batched_workspace(sk_batch_t B, size_t* bytes) {
  if (!B || !bytes) {
    set_error("lstsq_batched_workspace: null argument");
    return SK_E_INVAL;
  }
  *bytes = B->total;
  return SK_OK;
}

int lstsq_batched_bind(sk_batch_t B, void* ws, size_t ws_bytes, void* stream) {
  if (!B || !ws) {
    set_error("lstsq_batched_bind: null argument");
    return SK_E_INVAL;
  }
  if (ws_bytes < B->total || (uintptr_t)ws % 256 != 0) {
    set_error("lstsq_batched_bind: workspace too small or not 256-byte aligned (see lstsq_batched_workspace)");
    return SK_E_INVAL;
  }
  int dev = -1;
  SK_HIP(hipGetDevice(&dev));
  if (dev != B->device) {
    set_error("lstsq_batched_bind: the batch was planned on another device");
    return SK_E_INVAL;
  }
  return bt::bind(B, ws, (hipStream_t)stream);
}

int lstsq_batched_launch(sk_batch_t B, void* stream) {
  if (!B || !B->bound) {
    set_error("lstsq_batched_launch: the batch has no workspace bound");
    return SK_E_INVAL;
  }
  SK_HIP(hipGraphLaunch(B->exec, (hipStream_t)stream));
  ++B->graph_launches;
  return SK_OK;
}

int lstsq_batched_enqueue(sk_batch_t B, void* stream) {
  if (!B || !B->bound) {
    set_error("lstsq_batched_enqueue: the batch has no workspace bound");
    return SK_E_INVAL;
  }
  return bt::enqueue(B, (hipStream_t)stream);
}

int lstsq_batched_results(sk_batch_t B, sk_ls_problem* probs, void* stream) {
  if (!B || !probs || !B->bound) {
    set_error("lstsq_batched_results: null argument or no workspace bound");
    return SK_E_INVAL;
  }
  return bt::results(B, probs, (hipStream_t)stream);
}

int lstsq_batched_info(sk_batch_t B, sk_batch_info* info) {
  if (!B || !info) {
    set_error("lstsq_batched_info: null argument");
    return SK_E_INVAL;
  }
  info->graph_launches = B->graph_launches;
  info->kernel_nodes = B->kernel_nodes;
  info->sketch_workgroups = B->grid_sketch;
  info->solve_workgroups = B->grid_solve;
  info->sketch_items = (int)B->items.size();
  info->reduce_items = B->total_red;
  info->tuned = B->tuned;
  info->workspace_bytes = B->total;
  return SK_OK;
}

int lstsq_batched_destroy(sk_batch_t B) {
  if (!B) return SK_OK;
  bt::release_graph(B);
  if (B->h_res) (void)hipHostFree(B->h_res);
  delete B;
  return SK_OK;
}

}  // extern "C"
