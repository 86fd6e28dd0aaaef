// Subsampled randomized trigonometric transform (eq. 1.1, Walsh-Hadamard
// version) applied on the left: SA = (1/sqrt(d)) R H D A_pad, and the
// SparseRTT (Def. 1.7), whose output row j is the signed sum of xi selected
// rows of H D A_pad (the SparseCol factor of Def. 4.1), scaled by
// 1/sqrt(d xi). Both share the transform; only the last step differs.
//
// A (n x m) is padded with zero rows to npad = 2^p, D is a Rademacher
// diagonal (bit i mod 128 of Philox block i / 128, tag 2), H the unnormalized
// Sylvester Hadamard matrix (H[r][r'] = (-1)^popcount(r & r')) and R keeps
// the d sampled rows (sorted, drawn at sketch creation).
//
// H over p index bits factors as H_(top a bits) (x) H_(low q bits) (Kronecker,
// top bits most significant). The low q = 8k bits are transformed by k full
// passes over the matrix, 8 bits each, into a work buffer Z (npad x m); the
// top a = p - q <= 8 bits are applied only at the d sampled rows:
//   Y[hi, low] = sum_{hi'} (-1)^popcount(hi & hi') Z[hi', low].
// A full pass reads 256 rows (one value of the other bits, stride 2^lo) x a
// slab of <= 64 columns (one per lane): each of 8 waves first holds 32
// consecutive tile rows in registers and applies the 5 butterfly stages that
// stay inside them, the tile is exchanged through LDS so that each wave holds
// every 8th row, and the remaining 3 stages run in registers again.
#include "sk_srtt.hpp"

#include <algorithm>

namespace sk {

constexpr int kFw = 8;            // index bits per full pass
constexpr int kFt = 1 << kFw;     // rows per tile
constexpr int kFc = 64;           // LDS row stride (doubles)

// D_ii: bit (i mod 128) of Philox block i / 128, tag 2; true = negative.
__device__ inline uint32_t srtt_word(uint64_t i, uint32_t k0, uint32_t k1) {
  const uint64_t blk = i >> 7;
  const U4 w = philox4x32_10(U4{(uint32_t)blk, (uint32_t)(blk >> 32), 0u, kTagSrttSign}, k0, k1);
  return word_of(w, (int)((i & 127) >> 5));
}

struct SrttPassArgs {
  const double* A;
  int64_t lda;
  const double* rhs;
  int64_t n;
  int m, m_eff;
  double* Z;  // npad x m_eff
  int lo;     // first index bit of this pass
  int first;  // read A (signs, padding) instead of Z
  int C, n_slabs;
  uint32_t k0, k1;
};

__device__ inline void bfly(double& x, double& y) {
  const double s = x + y, t = x - y;
  x = s;
  y = t;
}

__global__ void __launch_bounds__(512) srtt_pass_kernel(SrttPassArgs a) {
  extern __shared__ double T[];  // [kFt][kFc]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tile = blockIdx.x / a.n_slabs;
  const int slab = (int)(blockIdx.x - tile * a.n_slabs);
  const int64_t low = tile & ((1ll << a.lo) - 1);
  const int64_t hi = tile >> a.lo;
  auto row_of = [&](int t) -> int64_t { return (hi << (a.lo + kFw)) | ((int64_t)t << a.lo) | low; };
  const int c = slab * a.C + lane;
  const bool active = lane < a.C && c < a.m_eff;

  double x[32];
  if (a.first) {
    // the first pass has lo = 0: this thread's 32 rows share one sign word
    const int64_t r0 = row_of(32 * wave);
    const uint32_t sw = srtt_word((uint64_t)r0, a.k0, a.k1);
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int64_t r = r0 + k;
      double v = 0.0;
      if (active && r < a.n) v = c < a.m ? a.A[r * a.lda + c] : a.rhs[r];
      x[k] = ((sw >> k) & 1u) ? -v : v;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = active ? a.Z[row_of(32 * wave + k) * a.m_eff + c] : 0.0;
  }
  // tile-row bits 0..4 (inside the thread's 32 consecutive rows)
#pragma unroll
  for (int h = 1; h < 32; h <<= 1)
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if ((k & h) == 0) bfly(x[k], x[k + h]);
#pragma unroll
  for (int k = 0; k < 32; ++k) T[(32 * wave + k) * kFc + lane] = x[k];
  __syncthreads();
  // tile rows wave + 8k: bits 5..7 of the tile row are bits 2..4 of k
#pragma unroll
  for (int k = 0; k < 32; ++k) x[k] = T[(wave + 8 * k) * kFc + lane];
#pragma unroll
  for (int h = 4; h < 32; h <<= 1)
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if ((k & h) == 0) bfly(x[k], x[k + h]);
  if (active) {
#pragma unroll
    for (int k = 0; k < 32; ++k) a.Z[row_of(wave + 8 * k) * a.m_eff + c] = x[k];
  }
}

// Output row j from its selected rows r = sample[j*xi + i] (i < xi; xi = 1
// and no signs for the SRTT), each r = hi * 2^q + low:
// out[j][c] = scale * sum_i rho_i sum_{h' < 2^abits} (-1)^popcount(hi & h') Src[h' * 2^q + low][c],
// Src = Z after the full passes, or D A_pad when there were none (q = 0).
__global__ void __launch_bounds__(256) srtt_sample_kernel(const double* __restrict__ Z, const double* __restrict__ A,
                                                          int64_t lda, const double* __restrict__ rhs, int64_t n,
                                                          int m, int m_eff, const int64_t* __restrict__ sample,
                                                          const int8_t* __restrict__ sgn, int xi, int q, int abits,
                                                          double scale, uint32_t k0, uint32_t k1,
                                                          double* __restrict__ out, int64_t ldo,
                                                          double* __restrict__ rhs_out) {
  const int64_t j = blockIdx.x;
  for (int c = threadIdx.x; c < m_eff; c += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < xi; ++i) {
      const int64_t r = sample[j * xi + i];
      const int64_t hi = r >> q, low = r & ((1ll << q) - 1);
      double t = 0.0;
      for (int64_t hp = 0; hp < (1ll << abits); ++hp) {
        const int64_t src = (hp << q) | low;
        double v;
        if (Z) {
          v = Z[src * m_eff + c];
        } else {
          v = 0.0;
          if (src < n) {
            v = c < m ? A[src * lda + c] : rhs[src];
            if ((srtt_word((uint64_t)src, k0, k1) >> (src & 31)) & 1u) v = -v;
          }
        }
        t += (__popcll((uint64_t)(hi & hp)) & 1) ? -v : v;
      }
      s += (sgn && sgn[j * xi + i] < 0) ? -t : t;
    }
    if (c < m)
      out[j * ldo + c] = s * scale;
    else
      rhs_out[j] = s * scale;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int srtt_full_passes(int p) { return p > kFw ? (p - 1) / kFw : 0; }

size_t srtt_workspace(const sk_sketch* S, int m_eff) {
  if (srtt_full_passes(S->log2npad) == 0) return 0;
  return (size_t)S->npad * m_eff * sizeof(double);
}

int launch_srtt_rows(const sk_sketch* S, int64_t m, const double* A, int64_t lda, const double* rhs, double* SA,
                     int64_t ldsa, double* Srhs, void* ws, size_t ws_bytes, hipStream_t st) {
  const int m_eff = (int)m + (rhs ? 1 : 0);
  const int p = S->log2npad;
  const int np = srtt_full_passes(p);
  const int q = kFw * np;
  const int abits = p - q;
  double* Z = nullptr;
  if (np > 0) {
    if (ws_bytes < srtt_workspace(S, m_eff)) {
      set_error("SRTT sketch: workspace too small");
      return SK_E_INVAL;
    }
    Z = (double*)ws;
    const int ns = (m_eff + 63) / 64;
    const int C = (m_eff + ns - 1) / ns;
    const size_t lds = (size_t)kFt * kFc * sizeof(double);
    SK_HIP(hipFuncSetAttribute((const void*)srtt_pass_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    for (int pass = 0; pass < np; ++pass) {
      SrttPassArgs a;
      a.A = A;
      a.lda = lda;
      a.rhs = rhs;
      a.n = S->n;
      a.m = (int)m;
      a.m_eff = m_eff;
      a.Z = Z;
      a.lo = kFw * pass;
      a.first = pass == 0;
      a.C = C;
      a.n_slabs = ns;
      a.k0 = S->k0;
      a.k1 = S->k1;
      const int64_t tiles = S->npad >> kFw;
      KernelTimer timer(S, st);
      hipLaunchKernelGGL(srtt_pass_kernel, dim3((unsigned)(tiles * ns)), dim3(512), lds, st, a);
    }
    SK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(srtt_sample_kernel, dim3((unsigned)S->d), dim3(256), 0, st, Z, A, lda, rhs, S->n, (int)m, m_eff,
                     S->d_sample, S->d_sgn, S->xi, q, abits, trig_scale(S), S->k0, S->k1, SA, ldsa, Srhs);
  SK_HIP(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
