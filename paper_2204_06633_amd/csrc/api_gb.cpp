// C-ABI host layer of the Galactic-binary polarisations: validation and
// launches.  See include/lisaresp.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/lisaresp.h"
#include "gb_types.hpp"
#include "internal.hpp"
#include "trace.hpp"

namespace {

using lr::set_error;

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

int check_common(int64_t n, int64_t n_h, double dt, int64_t h_stride) {
  if (n < 0 || n_h < 0) return set_error(LR_E_ARG, "negative size");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(LR_E_ARG, "dt must be positive");
  if (h_stride < n_h) return set_error(LR_E_ARG, "row stride %lld < %lld samples",
                                       (long long)h_stride, (long long)n_h);
  if (n > 65535) return set_error(LR_E_UNSUPPORTED, "%lld templates per call (max 65535)",
                                  (long long)n);
  return LR_OK;
}

}  // namespace

extern "C" {

int lr_gb_polarizations(const double* params, int64_t n, int64_t k0, int64_t n_h, double dt,
                        double* hp, double* hc, int64_t h_stride, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_common(n, n_h, dt, h_stride)) return st;
  if (n == 0 || n_h == 0) return LR_OK;
  if (!params || !hp || !hc) return set_error(LR_E_ARG, "null pointer");
  const size_t hb = ((size_t)(n - 1) * h_stride + n_h) * sizeof(double);
  const size_t pb = (size_t)n * 8 * sizeof(double);
  if (overlap(hp, hb, hc, hb) || overlap(hp, hb, params, pb) || overlap(hc, hb, params, pb))
    return set_error(LR_E_ARG, "hp, hc and params overlap");
  lr::GbArgs a{};
  a.params = params;
  a.n_h = n_h;
  a.k0 = k0;
  a.dt = dt;
  a.hp = hp;
  a.hc = hc;
  a.h_stride = h_stride;
  hipError_t e = lr::run_gb_forward(a, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return set_error(LR_E_HIP, "lr_gb_polarizations launch: %s", hipGetErrorString(e));
  return LR_OK;
}

size_t lr_gb_adjoint_workspace(int64_t n, int64_t n_h) {
  if (n < 0 || n_h < 0) return 0;
  return (size_t)n * (size_t)lr::gb_blocks(n_h) * lr::kGbSums * sizeof(double) + 8;
}

int lr_gb_polarizations_adjoint(const double* params, int64_t n, int64_t k0, int64_t n_h,
                                double dt, const double* g_hp, const double* g_hc,
                                int64_t h_stride, double* g_params, void* work,
                                size_t work_bytes, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_common(n, n_h, dt, h_stride)) return st;
  if (n == 0) return LR_OK;
  if (!params || !g_params || !work || (n_h > 0 && (!g_hp || !g_hc)))
    return set_error(LR_E_ARG, "null pointer");
  if (n_h == 0) return set_error(LR_E_ARG, "no samples (the gradient would be zero)");
  if (work_bytes < lr_gb_adjoint_workspace(n, n_h))
    return set_error(LR_E_WORKSPACE, "workspace %zu bytes < %zu", work_bytes,
                     lr_gb_adjoint_workspace(n, n_h));
  const size_t hb = ((size_t)(n - 1) * h_stride + n_h) * sizeof(double);
  const size_t pb = (size_t)n * 8 * sizeof(double);
  if (overlap(g_params, pb, params, pb) || overlap(g_params, pb, work, work_bytes) ||
      overlap(g_params, pb, g_hp, hb) || overlap(g_params, pb, g_hc, hb) ||
      overlap(work, work_bytes, params, pb) || overlap(work, work_bytes, g_hp, hb) ||
      overlap(work, work_bytes, g_hc, hb))
    return set_error(LR_E_ARG, "g_params or the workspace overlaps an input");
  lr::GbArgs a{};
  a.params = params;
  a.n_h = n_h;
  a.k0 = k0;
  a.dt = dt;
  a.g_hp = g_hp;
  a.g_hc = g_hc;
  a.h_stride = h_stride;
  a.g_params = g_params;
  a.part = static_cast<double*>(work);
  hipError_t e = lr::run_gb_adjoint(a, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return set_error(LR_E_HIP, "lr_gb_polarizations_adjoint launch: %s", hipGetErrorString(e));
  return LR_OK;
}

}  // extern "C"
