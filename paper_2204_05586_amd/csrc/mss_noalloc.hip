// mss_propagate_noalloc (include/mss.h): the ordered product of
// mss_propagate for callers that cannot allocate device memory.  The scan's
// workspace is `scratch`, a static device array of kNoAllocScratchBytes
// that every GPU the library runs on holds until the process ends.  Its
// device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is handed to the kernels.
// Calls that overlap on one GPU share the array and race.
#include <mutex>

#include "mss_internal.h"

using namespace mss;

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The array's address on the current device (looked up on its first use
// there).
mss_status scratch_on_current(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return api_hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return api_fail(MSS_E_UNSUPPORTED, "device ordinal %d is beyond the %d this entry point serves",
                    dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return api_hip_fail(e, "hipGetSymbolAddress of the scan scratch");
    if (!p) return api_fail(MSS_E_DEVICE, "hipGetSymbolAddress gave a NULL scan scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MSS_OK;
}

}  // namespace

extern "C" {

mss_status mss_propagate_noalloc(int32_t spin_twice, int64_t n_samples, const double* U,
                                 const double* psi0, double* psi, double* psi_final,
                                 void* stream) {
  size_t need = 0;
  mss_status s = mss_propagate_workspace_size(spin_twice, n_samples, &need);
  if (s != MSS_OK) return s;
  if (need > kNoAllocScratchBytes)
    return api_fail(MSS_E_INVALID,
                    "n_samples = %lld needs %zu bytes of scan scratch; mss_propagate_noalloc "
                    "holds %zu (at most %lld spin-1 or %lld spin-1/2 intervals)",
                    (long long)n_samples, need, kNoAllocScratchBytes,
                    (long long)MSS_NOALLOC_MAX_SAMPLES_SPIN_ONE,
                    (long long)MSS_NOALLOC_MAX_SAMPLES_SPIN_HALF);
  void* ws = nullptr;
  if ((s = scratch_on_current(&ws)) != MSS_OK) return s;
  return api_propagate(spin_twice, n_samples, U, psi0, psi, psi_final, ws, kNoAllocScratchBytes,
                       stream);
}

}  // extern "C"
