// soar_assign_noalloc: the SOAR assignment of soar_assign for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
// Its workspace is a fixed device array of this file; nothing is allocated at run time.
//
// Host code never passes the array's name to a kernel or a copy: in host code that name is a
// host-side stand-in.  The array's device address is taken once per device with
// hipGetSymbolAddress (with that device current) and used everywhere instead.
#include <mutex>

#include "../../include/soar.h"
#include "train.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the array on the current device (null on failure).
void* scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

soar_status soar_assign_noalloc(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                                const soar_assign_opts* opts, int32_t* primary, int32_t* spill,
                                float* primary_dist, float* spill_loss, void* stream) {
  size_t need = 0;
  const soar_status s = soar::assign_validate(X, n, d, C, K, opts, primary, spill, &need);
  if (s != SOAR_OK) return s;
  if (need > kScratchBytes) return SOAR_E_NOMEM;
  void* ws = scratch_ptr();
  if (!ws) return SOAR_E_DEVICE;
  return soar::assign_run(X, n, d, C, K, opts, primary, spill, primary_dist, spill_loss, ws,
                          static_cast<hipStream_t>(stream), nullptr, false);
}

size_t soar_assign_noalloc_limit(void) { return kScratchBytes; }

}  // extern "C"
