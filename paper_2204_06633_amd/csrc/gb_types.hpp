// Arguments shared by the Galactic-binary polarisation kernels and their
// host layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lr {

constexpr int kGbSums = 7;   // per-template sample sums of the parameter gradient

struct GbArgs {
  const double* params;      // [n][8]: A, f0, fdot, phi0, iota, psi, lam, beta
  int64_t n_h;               // samples per template
  int64_t k0;                // time index of sample 0: t_j = (k0 + j) dt
  double dt;
  double* hp;                // [n] rows of h_stride (forward)
  double* hc;
  int64_t h_stride;
  const double* g_hp;        // adjoint inputs, same layout
  const double* g_hc;
  double* g_params;          // [n][8]
  double* part;              // [n][blocks][kGbSums]
};

int64_t gb_blocks(int64_t n_h);
hipError_t run_gb_forward(const GbArgs& a, int64_t n_tpl, hipStream_t s);
hipError_t run_gb_adjoint(const GbArgs& a, int64_t n_tpl, hipStream_t s);
// g_params [n][8] of a batch in waveform mode from the per-tile sums (see
// gb_batch_finalize_kernel); span and sky_span: [n][3] (first, count, index).
hipError_t run_gb_batch_finalize(const double* gb_part, const int64_t* span,
                                 const double* sky_part, const int64_t* sky_span,
                                 const double* params, int64_t n, double* g_params, hipStream_t s);

}  // namespace lr
