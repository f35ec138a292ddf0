// sd_noalloc.hip -- sd_deliver_spikes_noalloc: external spike-list delivery
// whose scratch (the packed list and its count) lives in a file-scope device
// array instead of memory the library allocates, for callers that cannot
// allocate (code under graph capture, serving loops, harnesses that forbid
// it).  The call itself allocates nothing and frees nothing.
//
// The array is one per GPU (each device holds its own copy for the life of
// the process).  In host code its name is only a stand-in: its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept, and only that address is ever handed to
// kernels.  Every call on one GPU shares that GPU's copy, which keeps the
// last call's contents; calls that overlap on one GPU (other streams, other
// threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sd_internal.h"

namespace {

constexpr int64_t kScratchEntries = int64_t(1) << 20;  // packed entries (4 MiB)
constexpr int64_t kScratchWords = kScratchEntries + 64;  // + the count, own 256-byte line

// Packed list entries [0, kScratchEntries), then the entry count at word
// kScratchEntries.  The count is written by the packing kernel of each call
// before anything reads it, so nothing here has to start at zero.
static __device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of the array, looked up on first use.
hipError_t scratch_ptr(int dev, uint32_t** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t e2 = cur != dev ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = (uint32_t*)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

sd_status sd_deliver_spikes_noalloc(sd_ctx* ctx, const uint32_t* d_src, const uint8_t* d_lag,
                                    int64_t n, int64_t t0) {
  if (!ctx) return SD_EINVAL;
  if (n > kScratchEntries)
    return sd::set_error(ctx, SD_EINVAL, "sd_deliver_spikes_noalloc takes at most 2^20 entries");
  const int dev = sd::ctx_device(ctx);
  if (dev < 0 || dev >= kMaxDevices)
    return sd::set_error(ctx, SD_EUNSUPPORTED, "device index beyond the scratch table");
  uint32_t* p = nullptr;
  const hipError_t e = scratch_ptr(dev, &p);
  if (e != hipSuccess) return sd::set_error(ctx, SD_EHIP, hipGetErrorString(e));
  return sd::deliver_external(ctx, d_src, d_lag, n, t0, p, (int32_t*)(p + kScratchEntries),
                              kScratchEntries);
}

}  // extern "C"
