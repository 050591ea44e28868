// Allocation-free sampling: grf_sample with its workspace (the per-field
// constants built from a device theta) in a library-owned device array, for
// callers that cannot allocate device memory during the call.
//
// `scratch` lives in device memory from module load until the process ends,
// one copy per device the library runs on.  In host code its name is only a
// stand-in: the device address of each copy is fetched once per device with
// hipGetSymbolAddress (that device current) and kept in `g_scratch`; only
// that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "grf.h"
#include "grf_common.hpp"
#include "grf_host.hpp"

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kScratchBytes = (size_t)GRF_NOALLOC_MAX_FIELDS * sizeof(grf::FieldRec);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device).
grf_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return grf::host::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return grf::host::fail(GRF_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return grf::host::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr) return grf::host::fail(GRF_EDEVICE, "no device address for the scratch array");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GRF_OK;
}

}  // namespace

extern "C" grf_status grf_sample_noalloc(grf_plan plan, uint64_t seed, int64_t batch, const double* theta, void* out,
                                         void* stream) {
  if (plan == nullptr) return grf::host::fail(GRF_EINVAL, "null plan");
  if (batch < 0) return grf::host::fail(GRF_EINVAL, "negative batch");
  if (theta != nullptr && batch > GRF_NOALLOC_MAX_FIELDS)
    return grf::host::fail(GRF_EINVAL, "grf_sample_noalloc: per-field parameters for at most "
                                       "GRF_NOALLOC_MAX_FIELDS fields per call");
  if (batch == 0) return GRF_OK;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  if (theta != nullptr) {
    grf_status st = scratch_ptr(&ws);
    if (st != GRF_OK) return st;
    ws_bytes = kScratchBytes;
  }
  return grf_sample(plan, seed, batch, theta, out, ws, ws_bytes, stream);
}
