// Batched sketch-and-solve (batched.hip): device descriptors shared by the
// host planner and the kernels.
#pragma once
#include "sk_common.hpp"

namespace sk {
namespace bt {

constexpr int kWaves = 8;                // waves of a worker workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kNreg = 200;               // accumulator registers of a sketch wave
constexpr int kQueues = 8;               // static queues: one per XCD
constexpr int kNB = 16;                  // QR panel width
constexpr int kMaxD = 1024;              // sketch rows one workgroup factors
constexpr int kTileLds = 128 * 1024;     // LDS of the sketch tile buffers
constexpr int kTouchLds = 1024 * kWaves; // LDS landing area of the code prefetch
constexpr int kQrVBytes = kMaxD * kNB * 8;
constexpr int kLdsBytes = 144 * 1024;    // dynamic LDS of the worker

// Counter block (ints): static queue heads, ready queue head and tail,
// reduce items done, the solve queue head, an error flag, then per
// problem: sketch units done, rank.
enum { C_QHEAD = 0, C_RQHEAD = 8, C_RQTAIL = 9, C_REDDONE = 10, C_SOLVEHEAD = 11, C_ERROR = 12, C_FIXED = 16 };

// Longest wait of a sketch workgroup for work, in ticks of the 100 MHz device
// clock (20 s).
constexpr uint64_t kWaitTicks = 2000000000ull;

// One problem as the kernels see it (offsets are bytes into the workspace).
struct BtProb {
  const unsigned char* A;  // n x k row-major
  const unsigned char* b;  // n
  double* x;               // k (output)
  int64_t n;
  int64_t lda_bytes;
  int64_t rows_per_chunk;  // a multiple of R
  int64_t codes_off;       // row codes: [tile][part][block][2R] uint32
  int64_t P_off;           // partial sums: [chunk][d][k + 1] (F64 for F64 input, else F32)
  int64_t W_off;           // S [A b], d x ldw doubles, row-major
  int64_t X_off;           // R^-1 (k x k), then the fallback's R, c, U, V, work, s, z
  double scale;            // 1 / sqrt(zeta)
  int index;               // position in the batch
  int k, d, nb, zeta, dtype;
  int R;                   // tile rows
  int nparts, ps;          // bucket parts of a block and buckets per part
  int n_gp;                // block groups x parts: units per (chunk, slab)
  int n_slabs;             // 64-column slabs of the k + 1 columns of [A b]
  int n_chunks, n_units, n_red;
  int ldw;
  uint32_t k0, k1;
};

struct BtArgs {
  const int4* items;  // static items {problem, first unit, units, 0}
  const int* qbeg;    // kQueues + 1 offsets into items
  int* ctl;
  unsigned long long* t_start;
  unsigned long long* t_end;
  unsigned long long* rq;  // ready slots: (problem + 1) << 32 | reduce index
  unsigned char* ws;
  int nprob;
  int total_red;  // reduce items of the batch
  int wu;         // waves per unit
  int red_rows;   // rows of d per reduce item
  int buf_bytes;  // LDS bytes of one tile buffer
  int off_touch;  // LDS offset of the prefetch area
};

}  // namespace bt
}  // namespace sk
