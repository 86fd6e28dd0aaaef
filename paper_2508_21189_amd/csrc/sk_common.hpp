// Shared definitions for the libsketch HIP sources (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "libsketch.h"

namespace sk {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). One call maps a 128-bit
// counter and a 64-bit key to 128 random bits; entries of every sketch are
// pure functions of (seed, index), so any thread can produce any entry.
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Fourth counter word: separates the independent streams drawn from one seed.
constexpr uint32_t kTagSparseStack = 1;
constexpr uint32_t kTagSrttSign = 2;
constexpr uint32_t kTagSrttSample = 3;
constexpr uint32_t kTagGauss = 4;
constexpr uint32_t kTagSparseCol = 5;

struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
    uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

__host__ __device__ inline uint32_t word_of(const U4& v, int j) {
  return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// SparseStack code of one (column i, block t): bucket in [0, nb) and a sign bit
// (1 = negative). Bits: sign = bit 0 of the word; bucket = ((word >> 1) * nb) >> 31.
__host__ __device__ inline uint32_t ss_bucket(uint32_t word, uint32_t nb) {
  return (uint32_t)(((uint64_t)(word >> 1) * nb) >> 31);
}
__host__ __device__ inline uint32_t ss_negative(uint32_t word) { return word & 1u; }

// ---------------------------------------------------------------------------
// bf16 <-> f32 (bf16 is the upper half of an IEEE f32; widening is exact).
// ---------------------------------------------------------------------------
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// ---------------------------------------------------------------------------
// Host-side helpers shared by the API and the launchers.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define SK_HIP(expr)                                       \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return ::sk::hip_fail(_e, #expr); \
  } while (0)

inline size_t dtype_size(int dt) { return dt == SK_F64 ? 8 : (dt == SK_F32 ? 4 : 2); }
inline double inv_sqrt_host(double x) { return 1.0 / __builtin_sqrt(x); }

}  // namespace sk

// The handle. Immutable after sketch_create except for the cached workspace.
struct sk_sketch {
  int kind = 0;
  int64_t d = 0, n = 0;
  int zeta = 1;
  uint64_t seed = 0;
  int64_t nb = 0;  // SparseStack buckets per block (d / zeta)
  int device = 0;
  uint32_t k0 = 0, k1 = 0;
  // SRTT and SparseRTT: padded length 2^p >= n and the selected rows
  // (device): SRTT d sorted rows (xi = 1, no signs); SparseRTT xi sorted
  // rows per output row j at [j*xi, (j+1)*xi) with signs d_sgn (+1 / -1).
  int64_t npad = 0;
  int log2npad = 0;
  int xi = 1;
  int64_t* d_sample = nullptr;
  int8_t* d_sgn = nullptr;
  std::vector<int64_t> h_sample;
  // internal workspace (used when the caller passes ws = NULL)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // driver workspace (least-squares and low-rank drivers) and a pinned host
  // block for reading back their scalars
  void* dws = nullptr;
  size_t dws_bytes = 0;
  void* h_pinned = nullptr;
  // split-K partial sums of the low-rank drivers' GEMMs (grown on first use)
  void* gws = nullptr;
  size_t gws_bytes = 0;
  // optional timing of the dominant kernel of each call (sketch_timing)
  mutable bool timing = false;
  mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
};

namespace sk {
// Records an event pair around the dominant kernel when timing is enabled.
struct KernelTimer {
  const sk_sketch* S;
  hipStream_t st;
  hipEvent_t e1 = nullptr;
  KernelTimer(const sk_sketch* s, hipStream_t stream) : S(s), st(stream) {
    if (S->timing) {
      hipEvent_t e0;
      if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        (void)hipEventRecord(e0, st);
        S->events.push_back({e0, e1});
      } else {
        e1 = nullptr;
      }
    }
  }
  ~KernelTimer() {
    if (e1) (void)hipEventRecord(e1, st);
  }
};

// 64-bit DPP move of v (dpp_ctrl C, row mask RM); disabled rows give 0.
template <int C, int RM>
__device__ inline double dpp64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, C, RM, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), C, RM, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Sum of v over the wave, returned uniformly (the value that ends in lane 63):
// row_ror 8, 4, 2, 1 inside each 16-lane row, then row_bcast 15 and 31 carry
// the row sums up to the last row.
__device__ inline double wave_sum_dpp(double v) {
  v += dpp64<0x128, 0xF>(v);
  v += dpp64<0x124, 0xF>(v);
  v += dpp64<0x122, 0xF>(v);
  v += dpp64<0x121, 0xF>(v);
  v += dpp64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The two trigonometric-transform sketches share the transform kernels.
inline bool trig_kind(int kind) { return kind == SK_SRTT || kind == SK_SPARSERTT; }
// Scale of a selected-row sum: 1/sqrt(d) (SRTT, eq. 1.1), 1/sqrt(d xi)
// (SparseRTT: (1/sqrt(d)) sqrt(npad/xi) from SparseCol times 1/sqrt(npad)
// from the unitary WHT).
inline double trig_scale(const sk_sketch* S) {
  return inv_sqrt_host((double)S->d * (S->kind == SK_SPARSERTT ? (double)S->xi : 1.0));
}
}  // namespace sk
