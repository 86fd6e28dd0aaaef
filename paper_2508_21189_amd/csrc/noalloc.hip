// sketch_apply_noalloc: SA = S A for a SparseStack S and a row-major A, with
// every scratch byte (the per-chunk partial sums and the per-row codes) in a
// fixed device array instead of the handle's or the caller's workspace, for
// callers that cannot allocate device memory (code under stream capture,
// serving loops, harnesses that forbid allocation).
//
// The array is a file-scope device variable, so each device the library runs
// on holds its own copy for the life of the process. Host code never names
// it directly: its device address is looked up once per device with
// hipGetSymbolAddress and kept; the kernels receive that address like any
// workspace pointer. Every call on a device shares the array, which keeps
// the last call's contents: the apply writes every partial and code it reads
// before reading it, so nothing needs to start at zero, and calls that
// overlap on one device (other streams, other threads) race on it.
#include <mutex>

#include "sk_drivers.hpp"

namespace sk {

// 128 MB: e.g. n = 2^20 rows of a 50-column A with d = 200, zeta = 4
// (33.6 MB of codes, 5.1 MB of partials) or n = 2^19 rows of 200 columns with
// d = 800, zeta = 8.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of the array (looked up on the
// first call on each device, with that device current).
int scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("sketch_apply_noalloc: device index out of range");
    return SK_E_NOTSUP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("sketch_apply_noalloc: no device address for the scratch array");
      return SK_E_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SK_OK;
}
}  // namespace

}  // namespace sk

using namespace sk;

extern "C" size_t sketch_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int sketch_apply_noalloc(sketch_t S, int dtype_in, int64_t m, const void* A, int64_t lda, int dtype_out,
                                    void* SA, int64_t ldsa, void* stream) {
  if (!S || !A || !SA) {
    set_error("sketch_apply_noalloc: null handle or pointer");
    return SK_E_INVAL;
  }
  if (S->kind != SK_SPARSESTACK) {
    set_error("sketch_apply_noalloc: SparseStack sketches only");
    return SK_E_NOTSUP;
  }
  if (m < 1 || (dtype_in != SK_F64 && dtype_in != SK_F32 && dtype_in != SK_BF16) ||
      (dtype_out != SK_F64 && dtype_out != SK_F32) || lda < m || ldsa < m) {
    set_error("sketch_apply_noalloc: need m >= 1, lda >= m, ldsa >= m, dtype_in in {F64, F32, BF16}, "
              "dtype_out in {F64, F32}");
    return SK_E_INVAL;
  }
  int dev = -1;
  SK_HIP(hipGetDevice(&dev));
  if (dev != S->device) {
    set_error("sketch_apply_noalloc: the handle was created on another device");
    return SK_E_INVAL;
  }
  size_t need = 0;
  int rc = apply_workspace_for(S, dtype_in, m, A, lda, &need);
  if (rc != SK_OK) return rc;
  if (need > kScratchBytes) {
    set_error("sketch_apply_noalloc: this apply needs " + std::to_string(need) +
              " bytes of scratch, more than the fixed " + std::to_string(kScratchBytes) +
              " (use sketch_apply with a workspace)");
    return SK_E_NOTSUP;
  }
  void* ptr = nullptr;
  rc = scratch_ptr(dev, &ptr);
  if (rc != SK_OK) return rc;
  return apply_dispatch(S, dtype_in, m, A, lda, dtype_out, SA, ldsa, ptr, kScratchBytes, (hipStream_t)stream);
}
