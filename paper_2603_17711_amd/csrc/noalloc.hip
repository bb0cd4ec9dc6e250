// tenso_apply_generator_noalloc: the effective generator at a center with no
// device allocation inside the call.  The workspace and the launch
// descriptors live in `scratch`, a static device array that every GPU the
// library runs on holds until the process ends.  The host reaches each
// device's copy through hipGetSymbolAddress (the array's name on the host is
// only a stand-in, never a device address).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/tenso.h"

namespace tenso {
int apply_generator_scratch(tenso_plan* p, const void* d_state, int center, const double* drive,
                            void* d_out, void* scratch, size_t scratch_bytes, hipStream_t s);
int set_last_error(int code, const std::string& msg);
}  // namespace tenso

namespace {

constexpr size_t kScratchBytes = (size_t)TENSO_NOALLOC_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's `scratch`, looked up once per device with
// that device current (the caller's current device).
int scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return tenso::set_last_error(TENSO_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return tenso::set_last_error(TENSO_EUNSUPPORTED, "device index beyond 64");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return tenso::set_last_error(TENSO_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                   hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TENSO_OK;
}

}  // namespace

extern "C" int tenso_apply_generator_noalloc(tenso_plan* p, const void* d_state, int center,
                                             const double* drive, void* d_out, hipStream_t s) {
  void* ptr = nullptr;
  int rc = scratch_ptr(&ptr);
  if (rc != TENSO_OK) return rc;
  return tenso::apply_generator_scratch(p, d_state, center, drive, d_out, ptr, kScratchBytes, s);
}
