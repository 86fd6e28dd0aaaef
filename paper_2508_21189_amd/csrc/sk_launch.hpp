// Kernel launchers shared between translation units (host side).
#pragma once
#include "sk_common.hpp"

#include <vector>

namespace sk {

// Plan of the row-mode SparseStack apply (SA = S A, A row-major n x m).
struct RowsPlan {
  int C = 64;            // columns per slab (lanes per wave that hold data)
  int rowb = 512;        // LDS bytes of a tile row (C columns, rounded up to 16)
  int n_slabs = 1;
  int R = 128;           // rows per LDS sub-tile
  int W = 16;            // waves per workgroup
  int bpg = 1;           // sketch blocks handled by one workgroup
  int n_groups = 1;      // workgroups sharing one A tile (zeta / bpg, rounded up, times ranges)
  int ranges = 1;        // bucket-range groups per block (more buckets than 16 waves hold)
  int H = 1;             // bucket ranges per block (one wave each)
  int per_range = 1;     // buckets per range
  int n_chunks = 1;      // row chunks
  int64_t rows_per_chunk = 0;
  int load_bytes = 16;   // 16 or 4: width of the direct global->LDS loads
  int jb = 64;           // accumulator slots compiled into the kernel
  size_t lds_bytes = 0;
  size_t partial_bytes = 0;  // workspace: per-chunk partial sums
  size_t plan_bytes = 0;     // workspace: per-tile bucket plans
  int64_t n_tiles = 0;
  int rec_bytes = 0, lst_off = 0;
  // narrow inputs (m <= 4): lanes over buckets instead of columns
  bool narrow = false;
  int64_t tiles_per_chunk = 0;
  // bucket-indexed register accumulators (ss_idx.hip): jb is the register
  // file size, rec_bytes the LDS buffer stride; plan_bytes holds the row
  // codes
  bool idx = false;
  int nbuf = 2;  // its tile buffers (loads run nbuf - 1 tiles ahead)
  int nparts = 1, ps = 0;  // bucket parts of a block (one wave each) and buckets per part
};

// Chooses the plan; returns SK_OK or SK_E_NOTSUP (and sets the error).
int plan_rows(const sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, RowsPlan* plan);

// The bucket-indexed apply (ss_idx.hip): whether it takes this input, its
// plan, and the sketch kernel writing the partials P.
bool idx_apply_fits(const sk_sketch* S, int dtype_in, int64_t m);
int launch_idx_codes(const sk_sketch* S, int dtype_in, int64_t n_tiles, int R, uint32_t* codes, hipStream_t st);
int plan_idx(const sk_sketch* S, int dtype_in, int64_t m, const void* A, int64_t lda, RowsPlan* plan);
int launch_idx_sketch(const sk_sketch* S, const RowsPlan& p, int dtype_in, int64_t m, const void* A, int64_t lda,
                      void* ws, hipStream_t st);

// Batched row-mode sketches of many problems (ss_idx.hip): for job j,
// W = [S A | S b] in FP64, column-major d x (k + 1) with leading dimension
// d, S the job's SparseStack (A row-major n x k, b n values, both of the
// job's dtype). idx_batch_fits says whether a job can go into the batched
// launches; the workspace holds the tables, the row codes and the partial
// sums (groups of jobs share one area of at most 16 GiB, or one job's need).
// idx_batch_prepare plans the jobs into the workspace and writes the
// tables (host copy, to be uploaded to the start of ws); idx_batch_enqueue
// queues the kernels only (no copies: it may be captured);
// launch_idx_batch does both with an asynchronous upload, so prog (host
// memory) must stay alive until the stream has run it. chunk_mult: row
// chunks of at least chunk_mult * d rows (0: 16).
struct IdxBatchJob {
  const sk_sketch* S;
  int dtype;
  int64_t k;
  const void* A;
  int64_t lda;
  const void* b;
  double* W;
  int chunk_mult;
};
struct IdxBatchLaunch {
  int kind;  // 0 codes, 1 apply, 2 chunk sums of FP64 partials, 3 of FP32 partials
  int first, count, dtype;
  int64_t grid;
  RowsPlan plan;  // the apply variant's launch shape
};
struct IdxBatchProgram {
  std::vector<unsigned char> tables;
  std::vector<IdxBatchLaunch> launches;
  void* ws = nullptr;
  int njobs = 0;
};
bool idx_batch_fits(const sk_sketch* S, int dtype_in, int64_t k, const void* A, int64_t lda);
int idx_batch_workspace(const IdxBatchJob* jobs, int njobs, size_t* bytes);
int idx_batch_prepare(const IdxBatchJob* jobs, int njobs, void* ws, size_t ws_bytes, IdxBatchProgram* prog);
int idx_batch_enqueue(const IdxBatchProgram& prog, hipStream_t st);
int launch_idx_batch(const IdxBatchJob* jobs, int njobs, void* ws, size_t ws_bytes, IdxBatchProgram* prog,
                     hipStream_t st);

int launch_rows_apply(const sk_sketch* S, const RowsPlan& p, int dtype_in, int64_t m, const void* A,
                      int64_t lda, int dtype_out, void* SA, int64_t ldsa, void* ws, hipStream_t st);

// Column mode (Y = A S^T, A rows x n row-major): workspace bytes and launch.
bool cols_kernel_fits(const sk_sketch* S, int dtype_in);
int cols_workspace(const sk_sketch* S, int dtype_in, size_t* bytes);
int launch_cols_apply(const sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out,
                      void* Y, int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st);
// its bucket-indexed kernel (ss_cols_idx.hip), taken when a block's
// accumulators fit one register file (A == NULL: for workspace queries)
bool cols_idx_fits(const sk_sketch* S, int dtype_in, const void* A, int64_t lda);
size_t cols_idx_workspace(const sk_sketch* S, int dtype_in);
int launch_cols_idx(const sk_sketch* S, int dtype_in, int64_t rows, const void* A, int64_t lda, int dtype_out, void* Y,
                    int64_t ldy, void* ws, size_t ws_bytes, hipStream_t st);

int launch_pattern(const sk_sketch* S, int32_t* bucket, int8_t* sign, hipStream_t st);
int launch_adjoint(const sk_sketch* S, int64_t m, const double* Y, int64_t ldy, double* Z, int64_t ldz,
                   hipStream_t st);

}  // namespace sk
