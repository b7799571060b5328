// Device scratch of the allocation-free forward entry point: one array of
// fixed size in the code object, so that a call can run without the context's
// growable workspace (callers under graph capture, or that may not allocate).
//
// The array is a file-scope __device__ variable.  Its name in host code is a
// host-side stand-in, not a device address: host code takes the device
// address of each GPU's copy with hipGetSymbolAddress once per device (with
// that device current) and uses only that pointer afterwards.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nkf_internal.h"

namespace nkf {

namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];
bool g_done[kMaxDevices];

}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

// Looks up (once per device) the device address of this device's copy of the
// scratch array.  `device` must be the current device.
hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_lock);
  if (!g_done[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  return g_err[device];
}

hipError_t static_scratch_ptr(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_lock);
  if (!g_done[device]) return hipErrorNotInitialized;
  if (g_err[device] != hipSuccess) return g_err[device];
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace nkf
