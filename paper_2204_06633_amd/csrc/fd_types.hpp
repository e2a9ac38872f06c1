// Types shared by the frequency-domain likelihood's host layer and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Extra doubles of a transform line's LDS stride beyond its padded length
// (build-time tuning switch; other small odd extras measured the same).
#ifndef LR_FD_LS_EXTRA
#define LR_FD_LS_EXTRA 1
#endif

namespace lr {

// Transform geometry: N = 2^logN points per signal in `passes` passes of
// 2^q[s] points; signals per template: 1 (A + iE) or 2 (A + iE, T + i0).
struct FdGeometry {
  int64_t n;            // samples per channel series (zero-padded to N)
  int logN, passes, q[3], sig_per_tpl;
};

// Device regions of the caller's workspace.
struct FdBuffers {
  double2* tlo;         // [4096] exp(-2 pi i j / N)
  double2* thi;         // [4096] exp(-2 pi i 4096 j / N)
  double2* dspec;       // [2][N] data spectrum, transform order
  double* wpos;         // [2][N] dt^2-scaled two-sided weights, transform order
  double2* work;        // [max_batch][sig_per_tpl][N]
  double* part;         // [max_batch][sig_per_tpl][N / 4096][3]
};

namespace fd {
struct PassArgs {
  int logN, q, logB, tiles_log, twiddle, sig_per_tpl;
  int64_t n_tpl;        // templates in the launch (the last pass orders its tiles by it)
  double2* x;
  const double2* tlo;
  const double2* thi;
  const double* h;      // real channel series in (first forward pass)
  double* g;            // real channel series out (last inverse pass)
  int64_t t_stride, c_stride, n;
  const double2* dspec;
  const double* wpos;
  double* part;
};
}  // namespace fd

hipError_t run_fd_prepare(const FdGeometry& g, const FdBuffers& b, const double* data,
                          int64_t data_cstride, const double* w_ae, const double* w_t, double dt,
                          hipStream_t s);
hipError_t run_fd_loglike(const FdGeometry& g, const FdBuffers& b, int64_t n_tpl, const double* h,
                          int64_t t_stride, int64_t c_stride, double* stats, double* g_h,
                          hipStream_t s);

}  // namespace lr
