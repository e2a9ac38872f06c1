// lr_project_adjoint_noalloc: lr_project_adjoint with the sky-gradient
// partial sums in a static device array instead of a caller workspace, for
// callers that cannot allocate (see include/lisaresp.h).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lisaresp.h"
#include "internal.hpp"
#include "trace.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(1) << 20;   // 1 MiB: 65536 sky partial pairs

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: it is a host-side stand-in.  The device address
// comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lr::set_error(LR_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return lr::set_error(LR_E_HIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return lr::set_error(LR_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return LR_OK;
}

}  // namespace

extern "C" {

size_t lr_noalloc_scratch_bytes(void) { return kScratchBytes; }

int lr_project_adjoint_noalloc(const lr_orbits* orb, double t0_h, double dt, int64_t n_h,
                               const double* hp, const double* hc, const double* sky, int order,
                               int64_t y_start, int64_t n_y, const double* g_y, double* g_hp,
                               double* g_hc, double* g_sky, void* stream) {
  LR_CALL_RANGE();
  if (!g_sky) {
    return lr_project_adjoint(orb, t0_h, dt, n_h, hp, hc, sky, order, y_start, n_y, g_y, g_hp,
                              g_hc, nullptr, nullptr, 0, stream);
  }
  if (n_y > 0 && lr_project_adjoint_workspace(n_y) > kScratchBytes)
    return lr::set_error(LR_E_WORKSPACE,
                         "n_y = %lld link samples need %zu bytes of sky-gradient scratch; the "
                         "static scratch holds %zu (at most %lld link samples)",
                         (long long)n_y, lr_project_adjoint_workspace(n_y), kScratchBytes,
                         (long long)(kScratchBytes / (2 * sizeof(double)) * lr::kTile));
  void* ptr = nullptr;
  if (int st = scratch_address(&ptr)) return st;
  return lr_project_adjoint(orb, t0_h, dt, n_h, hp, hc, sky, order, y_start, n_y, g_y, g_hp, g_hc,
                            g_sky, ptr, kScratchBytes, stream);
}

}  // extern "C"
