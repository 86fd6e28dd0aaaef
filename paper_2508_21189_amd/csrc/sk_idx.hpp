// Device helpers of the bucket-indexed SparseStack apply (register
// accumulators addressed through the VALU's GPR-index mode), shared by the
// row-mode kernels (single-matrix and batched) and the column-mode kernel.
#pragma once
#include "sk_common.hpp"

namespace sk {
namespace idx {

__device__ inline void idx_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// Wait until at most n of this wave's memory loads are outstanding (n is
// capped at 15; a smaller count only waits longer).
__device__ inline void idx_wait_vm(int n) {
  switch (n) {
#define SK_VMW(K) \
  case K:         \
    asm volatile("s_waitcnt vmcnt(" #K ")" ::: "memory"); \
    break;
    SK_VMW(1) SK_VMW(2) SK_VMW(3) SK_VMW(4) SK_VMW(5) SK_VMW(6) SK_VMW(7) SK_VMW(8)
    SK_VMW(9) SK_VMW(10) SK_VMW(11) SK_VMW(12) SK_VMW(13) SK_VMW(14) SK_VMW(15)
#undef SK_VMW
    default:
      if (n >= 16)
        asm volatile("s_waitcnt vmcnt(15)" ::: "memory");
      else
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
}

// Direct global->LDS loads (16 or 4 bytes a lane at LDS address M0 + lane *
// width), issued from inline assembly so that the compiler's counters do not
// make later LDS reads wait for them; the kernel waits explicitly before the
// barrier that publishes a tile. M0 is set, one wait state given, and restored.
__device__ inline void idx_dma16(const void* gsrc, uint32_t lds_addr) {
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
__device__ inline void idx_dma4(const void* gsrc, uint32_t lds_addr) {
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
// G 4-byte direct loads under one M0 setting: load j reads global address
// g[j] + j * STEP and writes LDS at M0 + j * STEP + lane * 4 (the instruction
// offset moves both addresses alike), so the caller passes g[j] already
// lowered by j * STEP. (j * STEP must fit the 13-bit signed offset.)
template <int G, int STEP>
__device__ inline void idx_dma4_group(const void* const* g, uint32_t lds_addr) {
  static_assert((G - 1) * STEP <= 4095, "instruction offset");
  uint32_t saved;
  if constexpr (G == 4)
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %1\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dword %2, off\n\t"
        "global_load_lds_dword %3, off offset:%c6\n\t"
        "global_load_lds_dword %4, off offset:%c7\n\t"
        "global_load_lds_dword %5, off offset:%c8\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "s"(lds_addr), "v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]), "i"(STEP), "i"(2 * STEP), "i"(3 * STEP)
        : "memory");
  else
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %1\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dword %2, off\n\t"
        "global_load_lds_dword %3, off offset:%c4\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "s"(lds_addr), "v"(g[0]), "v"(g[1]), "i"(STEP)
        : "memory");
}
__device__ inline uint32_t idx_lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void*)p;
}

typedef int v32i __attribute__((ext_vector_type(32)));
typedef int v8i __attribute__((ext_vector_type(8)));

// Accumulator registers: NREG 32-bit slots at v[40 .. 40 + NREG). Pieces of
// 32 registers (and one of 8 for the 200-slot file) keep each asm operand a
// legal register tuple; the pieces are adjacent, so slot j is v[40 + j].
struct AccFile {
  v32i p0, p1, p2, p3, p4, p5;
  v8i p6;
};

template <int NREG>
__device__ inline void acc_zero(AccFile& f) {
  f.p0 = 0;
  if constexpr (NREG > 32) f.p1 = 0;
  if constexpr (NREG > 64) {
    f.p2 = 0;
    f.p3 = 0;
  }
  if constexpr (NREG > 128) {
    f.p4 = 0;
    f.p5 = 0;
    f.p6 = 0;
  }
}

template <int NREG>
__device__ inline uint32_t acc_get(const AccFile& f, int j) {
  // j is a compile-time constant after unrolling
  if (j < 32) return (uint32_t)f.p0[j];
  if constexpr (NREG > 32)
    if (j < 64) return (uint32_t)f.p1[j - 32];
  if constexpr (NREG > 64) {
    if (j < 96) return (uint32_t)f.p2[j - 64];
    if (j < 128) return (uint32_t)f.p3[j - 96];
  }
  if constexpr (NREG > 128) {
    if (j < 160) return (uint32_t)f.p4[j - 128];
    if (j < 192) return (uint32_t)f.p5[j - 160];
    return (uint32_t)f.p6[j - 192];
  }
  return 0u;
}

// The operand lists that tie the accumulator pieces to their registers.
#define SK_ACC32 "+{v[40:71]}"(f.p0)
#define SK_ACC64 SK_ACC32, "+{v[72:103]}"(f.p1)
#define SK_ACC128 SK_ACC64, "+{v[104:135]}"(f.p2), "+{v[136:167]}"(f.p3)
#define SK_ACC200 SK_ACC128, "+{v[168:199]}"(f.p4), "+{v[200:231]}"(f.p5), "+{v[232:239]}"(f.p6)

#define SK_IDX_ASM(NREG, BODY, ...)                         \
  do {                                                     \
    if constexpr ((NREG) == 32)                            \
      asm volatile(BODY : SK_ACC32 : __VA_ARGS__);          \
    else if constexpr ((NREG) == 64)                       \
      asm volatile(BODY : SK_ACC64 : __VA_ARGS__);          \
    else if constexpr ((NREG) == 128)                      \
      asm volatile(BODY : SK_ACC128 : __VA_ARGS__);         \
    else                                                   \
      asm volatile(BODY : SK_ACC200 : __VA_ARGS__);         \
  } while (0)

// Four rows: acc[slot(w_k)] = fma(v_k, +-1, acc[slot(w_k)]) for k = 0..3,
// slot = the bucket's register index (low 8 bits of the code), the +-1.0
// multiplier in the scalar pair pm_k. GPR-index mode offsets only the
// accumulator operands (SRC2 and DST); the values and multipliers are read
// as named.
template <int NREG>
__device__ inline void fma4(AccFile& f, double v0, double v1, double v2, double v3, uint32_t i0, uint32_t i1,
                            uint32_t i2, uint32_t i3, uint64_t s0, uint64_t s1, uint64_t s2, uint64_t s3) {
  SK_IDX_ASM(NREG,
             "s_set_gpr_idx_on %[i0], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f64 v[40:41], %[v0], %[s0], v[40:41]\n\t"
             "s_set_gpr_idx_on %[i1], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f64 v[40:41], %[v1], %[s1], v[40:41]\n\t"
             "s_set_gpr_idx_on %[i2], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f64 v[40:41], %[v2], %[s2], v[40:41]\n\t"
             "s_set_gpr_idx_on %[i3], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f64 v[40:41], %[v3], %[s3], v[40:41]\n\t"
             "s_set_gpr_idx_off",
             [v0] "v"(v0), [v1] "v"(v1), [v2] "v"(v2), [v3] "v"(v3), [i0] "s"(i0), [i1] "s"(i1), [i2] "s"(i2),
             [i3] "s"(i3), [s0] "s"(s0), [s1] "s"(s1), [s2] "s"(s2), [s3] "s"(s3));
}
template <int NREG>
__device__ inline void fma4(AccFile& f, float v0, float v1, float v2, float v3, uint32_t i0, uint32_t i1,
                            uint32_t i2, uint32_t i3, uint32_t s0, uint32_t s1, uint32_t s2, uint32_t s3) {
  SK_IDX_ASM(NREG,
             "s_set_gpr_idx_on %[i0], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f32 v40, %[v0], %[s0], v40\n\t"
             "s_set_gpr_idx_on %[i1], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f32 v40, %[v1], %[s1], v40\n\t"
             "s_set_gpr_idx_on %[i2], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f32 v40, %[v2], %[s2], v40\n\t"
             "s_set_gpr_idx_on %[i3], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f32 v40, %[v3], %[s3], v40\n\t"
             "s_set_gpr_idx_off",
             [v0] "v"(v0), [v1] "v"(v1), [v2] "v"(v2), [v3] "v"(v3), [i0] "s"(i0), [i1] "s"(i1), [i2] "s"(i2),
             [i3] "s"(i3), [s0] "s"(s0), [s1] "s"(s1), [s2] "s"(s2), [s3] "s"(s3));
}
template <int NREG>
__device__ inline void fma1(AccFile& f, double v0, uint32_t i0, uint64_t s0) {
  SK_IDX_ASM(NREG,
             "s_set_gpr_idx_on %[i0], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f64 v[40:41], %[v0], %[s0], v[40:41]\n\t"
             "s_set_gpr_idx_off",
             [v0] "v"(v0), [i0] "s"(i0), [s0] "s"(s0));
}
template <int NREG>
__device__ inline void fma1(AccFile& f, float v0, uint32_t i0, uint32_t s0) {
  SK_IDX_ASM(NREG,
             "s_set_gpr_idx_on %[i0], gpr_idx(SRC2,DST)\n\t"
             "v_fma_f32 v40, %[v0], %[s0], v40\n\t"
             "s_set_gpr_idx_off",
             [v0] "v"(v0), [i0] "s"(i0), [s0] "s"(s0));
}

template <typename Tin>
struct IdxT;
template <>
struct IdxT<double> {
  using acc = double;
  using pm = uint64_t;
  static constexpr uint32_t one_hi = 0x3FF00000u;  // high word of 1.0
  static constexpr int rpa = 2;                    // registers per accumulator
};
template <>
struct IdxT<float> {
  using acc = float;
  using pm = uint32_t;
  static constexpr uint32_t one_hi = 0x3F800000u;  // 1.0f
  static constexpr int rpa = 1;
};
template <>
struct IdxT<uint16_t> {  // bf16 input, f32 accumulation
  using acc = float;
  using pm = uint32_t;
  static constexpr uint32_t one_hi = 0x3F800000u;
  static constexpr int rpa = 1;
};

template <typename Tin>
__device__ inline typename IdxT<Tin>::acc idx_val(uint32_t addr);
template <>
__device__ inline double idx_val<double>(uint32_t addr) {
  return *(const __attribute__((address_space(3))) double*)(uintptr_t)addr;
}
template <>
__device__ inline float idx_val<float>(uint32_t addr) {
  return *(const __attribute__((address_space(3))) float*)(uintptr_t)addr;
}
template <>
__device__ inline float idx_val<uint16_t>(uint32_t addr) {
  return bf16_to_f32(*(const __attribute__((address_space(3))) uint16_t*)(uintptr_t)addr);
}

// The +-1.0 multiplier from the high word of +-1.0 in the accumulation type.
__device__ inline uint64_t idx_pm(uint32_t h, double*) { return (uint64_t)h << 32; }
__device__ inline uint32_t idx_pm(uint32_t h, float*) { return h; }


}  // namespace idx
}  // namespace sk
