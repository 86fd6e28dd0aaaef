// C-ABI entry points of libsketch: argument checking, handle management,
// workspace management and dispatch to the HIP launchers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <string>

#include "sk_launch.hpp"
#include "sk_drivers.hpp"

namespace sk {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
  return e == hipErrorOutOfMemory ? SK_E_NOMEM : SK_E_HIP;
}

// Floyd's algorithm: d distinct indices of [0, npad), sorted. For
// j = npad-d .. npad-1 draw u uniform on {0..j} (u = (w * (j+1)) >> 32 with w
// the first word of Philox counter (j, 0, TAG)); insert u, or j if u is taken.
static std::vector<int64_t> srtt_sample_host(int64_t npad, int64_t d, uint32_t k0, uint32_t k1) {
  std::set<int64_t> chosen;
  for (int64_t j = npad - d; j < npad; ++j) {
    const U4 w = philox4x32_10(U4{(uint32_t)j, (uint32_t)((uint64_t)j >> 32), 0u, kTagSrttSample}, k0, k1);
    const int64_t u = (int64_t)(((uint64_t)w.x * (uint64_t)(j + 1)) >> 32);
    if (chosen.count(u))
      chosen.insert(j);
    else
      chosen.insert(u);
  }
  return std::vector<int64_t>(chosen.begin(), chosen.end());
}

// SparseCol selectors (Def. 4.1): for each output row j, xi distinct
// indices of [0, npad) by Floyd's algorithm with Philox counter
// (t, j, TAG) for t = npad-xi .. npad-1: u = (w0 * (t+1)) >> 32 is uniform
// on {0..t}; the index taken is u, or t if u is taken; its sign is -1 iff
// bit 0 of w1 is 1. Each row's selectors are sorted by index.
static void sparsecol_host(int64_t npad, int64_t d, int xi, uint32_t k0, uint32_t k1, std::vector<int64_t>& sel,
                           std::vector<int8_t>& sgn) {
  sel.resize((size_t)d * xi);
  sgn.resize((size_t)d * xi);
  std::vector<std::pair<int64_t, int8_t>> picks;
  std::set<int64_t> taken;
  for (int64_t j = 0; j < d; ++j) {
    picks.clear();
    taken.clear();
    for (int64_t t = npad - xi; t < npad; ++t) {
      const U4 w = philox4x32_10(U4{(uint32_t)t, (uint32_t)((uint64_t)t >> 32), (uint32_t)j, kTagSparseCol}, k0, k1);
      const int64_t u = (int64_t)(((uint64_t)w.x * (uint64_t)(t + 1)) >> 32);
      const int64_t idx = taken.count(u) ? t : u;
      taken.insert(idx);
      picks.push_back({idx, (int8_t)((w.y & 1u) ? -1 : 1)});
    }
    std::sort(picks.begin(), picks.end());
    for (int q = 0; q < xi; ++q) {
      sel[(size_t)j * xi + q] = picks[q].first;
      sgn[(size_t)j * xi + q] = picks[q].second;
    }
  }
}

// Grows a handle-owned buffer to at least `bytes`, ordered on the call's
// stream: the old buffer is released and the new one taken with the
// stream-ordered allocator, so no device-wide synchronization is needed (calls
// that share a handle's buffers are serialized by the caller, per the header).
int grow_buffer(void** buf, size_t* cur, size_t bytes, hipStream_t st) {
  if (*cur >= bytes) return SK_OK;
  if (*buf) {
    SK_HIP(hipFreeAsync(*buf, st));
    *buf = nullptr;
    *cur = 0;
  }
  void* p = nullptr;
  SK_HIP(hipMallocAsync(&p, bytes, st));
  *buf = p;
  *cur = bytes;
  return SK_OK;
}

// The handle-owned workspace (used when the caller passes ws = NULL).
int handle_workspace(sk_sketch* S, size_t bytes, void** out, hipStream_t st) {
  if (bytes == 0) {
    *out = nullptr;
    return SK_OK;
  }
  int rc = grow_buffer(&S->ws, &S->ws_bytes, bytes, st);
  if (rc != SK_OK) return rc;
  *out = S->ws;
  return SK_OK;
}

static bool valid_dtype(int dt) { return dt == SK_F64 || dt == SK_F32 || dt == SK_BF16; }

}  // namespace sk

using namespace sk;

extern "C" {

const char* sketch_last_error(void) { return g_last_error.c_str(); }

sketch_t sketch_create(int kind, int64_t d, int64_t n, int zeta, uint64_t seed) {
  if (d < 1 || n < 1) {
    set_error("sketch_create: need d >= 1 and n >= 1");
    return nullptr;
  }
  if (kind == SK_SPARSESTACK) {
    if (zeta < 1 || zeta > d || d % zeta != 0) {
      set_error("sketch_create: SparseStack needs 1 <= zeta <= d and d % zeta == 0");
      return nullptr;
    }
    if (d / zeta >= ((int64_t)1 << 31)) {
      set_error("sketch_create: SparseStack needs d/zeta < 2^31");
      return nullptr;
    }
  } else if (kind == SK_SRTT) {
    int64_t np = 1;
    while (np < n) np <<= 1;
    if (d > np) {
      set_error("sketch_create: SRTT needs d <= 2^ceil(log2 n)");
      return nullptr;
    }
  } else if (kind == SK_SPARSERTT) {
    int64_t np = 1;
    while (np < n) np <<= 1;
    if (zeta < 0 || zeta > np) {
      set_error("sketch_create: SparseRTT needs 0 <= zeta (column sparsity) <= 2^ceil(log2 n)");
      return nullptr;
    }
    if (d > (int64_t)0xFFFFFFFF) {
      set_error("sketch_create: SparseRTT needs d < 2^32");
      return nullptr;
    }
  } else if (kind == SK_IDENTITY_TEST) {
    if (d != n) {
      set_error("sketch_create: identity sketch needs d == n");
      return nullptr;
    }
  } else if (kind != SK_GAUSSIAN) {
    set_error("sketch_create: unknown kind");
    return nullptr;
  }
  sk_sketch* S = new sk_sketch();
  S->kind = kind;
  S->d = d;
  S->n = n;
  S->zeta = kind == SK_SPARSESTACK ? zeta : 1;
  if (kind == SK_SPARSERTT) {
    int64_t np = 1;
    while (np < n) np <<= 1;
    int64_t xi = zeta;
    if (xi == 0) xi = (int64_t)std::ceil(1.5 * std::log((double)d));
    xi = std::max<int64_t>(1, std::min<int64_t>(xi, np));
    S->xi = (int)xi;
    S->zeta = (int)xi;
  }
  S->seed = seed;
  S->nb = kind == SK_SPARSESTACK ? d / zeta : 0;
  S->k0 = (uint32_t)seed;
  S->k1 = (uint32_t)(seed >> 32);
  if (hipGetDevice(&S->device) != hipSuccess) {
    set_error("sketch_create: no HIP device");
    delete S;
    return nullptr;
  }
  if (trig_kind(kind)) {
    S->npad = 1;
    S->log2npad = 0;
    while (S->npad < n) {
      S->npad <<= 1;
      S->log2npad++;
    }
    std::vector<int8_t> h_sgn;
    if (kind == SK_SRTT)
      S->h_sample = srtt_sample_host(S->npad, d, S->k0, S->k1);
    else
      sparsecol_host(S->npad, d, S->xi, S->k0, S->k1, S->h_sample, h_sgn);
    const size_t cnt = S->h_sample.size();
    bool ok = hipMalloc(&S->d_sample, sizeof(int64_t) * cnt) == hipSuccess &&
              hipMemcpy(S->d_sample, S->h_sample.data(), sizeof(int64_t) * cnt, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && kind == SK_SPARSERTT)
      ok = hipMalloc(&S->d_sgn, cnt) == hipSuccess &&
           hipMemcpy(S->d_sgn, h_sgn.data(), cnt, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
      set_error("sketch_create: device allocation for the transform sketch's selectors failed");
      if (S->d_sample) (void)hipFree(S->d_sample);
      if (S->d_sgn) (void)hipFree(S->d_sgn);
      delete S;
      return nullptr;
    }
  }
  return S;
}

static void drop_events(sketch_t S) {
  for (auto& pr : S->events) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  S->events.clear();
}

int sketch_timing(sketch_t S, int mode, double* total_ms, int64_t* count) {
  if (!S || mode < 0 || mode > 2) {
    set_error("sketch_timing: invalid argument");
    return SK_E_INVAL;
  }
  if (mode == 2) {
    double tot = 0;
    for (auto& pr : S->events) {
      SK_HIP(hipEventSynchronize(pr.second));
      float ms = 0;
      SK_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (count) *count = (int64_t)S->events.size();
    return SK_OK;
  }
  (void)hipDeviceSynchronize();
  drop_events(S);
  S->timing = mode == 1;
  return SK_OK;
}

int sketch_destroy(sketch_t S) {
  if (!S) return SK_OK;
  (void)hipDeviceSynchronize();
  drop_events(S);
  // (the handle's workspaces come from the stream-ordered allocator)
  if (S->ws) (void)hipFreeAsync(S->ws, nullptr);
  if (S->d_sample) (void)hipFree(S->d_sample);
  if (S->d_sgn) (void)hipFree(S->d_sgn);
  drivers_release(S);
  (void)hipStreamSynchronize(nullptr);  // the stream-ordered frees
  delete S;
  return SK_OK;
}

int sketch_info(sketch_t S, int* kind, int64_t* d, int64_t* n, int* zeta, uint64_t* seed) {
  if (!S) {
    set_error("sketch_info: null handle");
    return SK_E_INVAL;
  }
  if (kind) *kind = S->kind;
  if (d) *d = S->d;
  if (n) *n = S->n;
  if (zeta) *zeta = S->zeta;
  if (seed) *seed = S->seed;
  return SK_OK;
}

int sketch_workspace_size(sketch_t S, int op, int dtype_in, int64_t m, size_t* bytes) {
  if (!S || !bytes || m < 1 || !valid_dtype(dtype_in) || op < 0 || op > 3) {
    set_error("sketch_workspace_size: invalid argument");
    return SK_E_INVAL;
  }
  return apply_workspace(S, op, dtype_in, m, bytes);
}

int sketch_apply(sketch_t S, int dtype_in, int layout, int64_t m, const void* A, int64_t lda, int dtype_out, void* SA,
                 int64_t ldsa, void* ws, size_t ws_bytes, void* stream) {
  if (!S || !A || !SA) {
    set_error("sketch_apply: null handle or pointer");
    return SK_E_INVAL;
  }
  if (m < 1 || !valid_dtype(dtype_in) || (dtype_out != SK_F64 && dtype_out != SK_F32)) {
    set_error("sketch_apply: need m >= 1, dtype_in in {F64, F32, BF16}, dtype_out in {F64, F32}");
    return SK_E_INVAL;
  }
  if (layout == SK_COL_MAJOR) {
    if (lda < S->n || ldsa < m) {
      set_error("sketch_apply: column-major A needs lda >= n, and ldsa >= m");
      return SK_E_INVAL;
    }
    return apply_colmajor(S, dtype_in, m, A, lda, dtype_out, SA, ldsa, ws, ws_bytes, (hipStream_t)stream);
  }
  if (layout != SK_ROW_MAJOR) {
    set_error("sketch_apply: layout must be SK_ROW_MAJOR or SK_COL_MAJOR");
    return SK_E_INVAL;
  }
  if (lda < m || ldsa < m) {
    set_error("sketch_apply: need lda >= m and ldsa >= m");
    return SK_E_INVAL;
  }
  return apply_dispatch(S, dtype_in, m, A, lda, dtype_out, SA, ldsa, ws, ws_bytes, (hipStream_t)stream);
}

int sketch_apply_T(sketch_t S, int dtype_in, int layout, int64_t rows, const void* A, int64_t lda, int dtype_out,
                   void* Y, int64_t ldy, void* ws, size_t ws_bytes, void* stream) {
  if (!S || !A || !Y) {
    set_error("sketch_apply_T: null handle or pointer");
    return SK_E_INVAL;
  }
  if (rows < 1 || !valid_dtype(dtype_in) || (dtype_out != SK_F64 && dtype_out != SK_F32)) {
    set_error("sketch_apply_T: need rows >= 1, dtype_in in {F64, F32, BF16}, dtype_out in {F64, F32}");
    return SK_E_INVAL;
  }
  if (layout == SK_COL_MAJOR) {
    if (lda < rows || ldy < S->d) {
      set_error("sketch_apply_T: column-major A needs lda >= rows, and ldy >= d");
      return SK_E_INVAL;
    }
    return apply_T_colmajor(S, dtype_in, rows, A, lda, dtype_out, Y, ldy, ws, ws_bytes, (hipStream_t)stream);
  }
  if (layout != SK_ROW_MAJOR) {
    set_error("sketch_apply_T: layout must be SK_ROW_MAJOR or SK_COL_MAJOR");
    return SK_E_INVAL;
  }
  if (lda < S->n || ldy < S->d) {
    set_error("sketch_apply_T: need lda >= n and ldy >= d");
    return SK_E_INVAL;
  }
  return apply_T_dispatch(S, dtype_in, rows, A, lda, dtype_out, Y, ldy, ws, ws_bytes, (hipStream_t)stream);
}

int sketch_adjoint(sketch_t S, int64_t m, const double* Y, int64_t ldy, double* Z, int64_t ldz, void* stream) {
  if (!S || !Y || !Z || m < 1 || ldy < m || ldz < m) {
    set_error("sketch_adjoint: invalid argument");
    return SK_E_INVAL;
  }
  if (S->kind != SK_SPARSESTACK) {
    set_error("sketch_adjoint: SparseStack only");
    return SK_E_NOTSUP;
  }
  return launch_adjoint(S, m, Y, ldy, Z, ldz, (hipStream_t)stream);
}

int sketch_pattern(sketch_t S, int32_t* bucket, int8_t* sign, void* stream) {
  if (!S || !bucket || !sign) {
    set_error("sketch_pattern: invalid argument");
    return SK_E_INVAL;
  }
  if (S->kind != SK_SPARSESTACK) {
    set_error("sketch_pattern: SparseStack only");
    return SK_E_NOTSUP;
  }
  return launch_pattern(S, bucket, sign, (hipStream_t)stream);
}

}  // extern "C"
