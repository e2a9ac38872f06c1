// Internal interface between the C-ABI host layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace lr {

struct ProjArgs {
  OrbitView orb;
  const double* hp;
  const double* hc;
  int64_t n_h;
  double t_off;      // t0_h - (time of coarse orbit sample 0)
  double dt, inv_dt;
  const double* sky; // device [lam, beta]
  int64_t y_start, n_y;
  double* y;         // [6][n_y]
};

struct TdiArgs {
  OrbitView orb;
  const double* y;   // [6][n_y]
  int64_t n_y;
  double t_off;      // t0_y - (time of coarse orbit sample 0)
  double dt, inv_dt;
  int64_t out_start, n_out;
  int channels;      // LR_XYZ, LR_AET or LR_XYZ_AET
  double* out;       // [3 or 6][n_out]
};

struct TdiAdjArgs {
  OrbitView orb;
  const double* g_out;  // [3 or 6][n_out]
  int channels;
  int64_t n_y;
  double t_off;         // t0_y - (time of coarse orbit sample 0)
  double dt, inv_dt;
  int64_t out_start, n_out;
  double* g_y;          // [6][n_y], zero-filled before the launch
  int rl_cap;           // wave row capacity of the carry kernel (even); 0: atomic kernel
};

struct ProjAdjArgs {
  OrbitView orb;
  const double* hp;     // needed for the sky gradient only
  const double* hc;
  int64_t n_h;
  double t_off;
  double dt, inv_dt;
  const double* sky;    // device [lam, beta]
  int64_t y_start, n_y;
  const double* g_y;    // [6][n_y]
  double* g_hp;         // [n_h], zero-filled before the launch
  double* g_hc;
  double* sky_part;     // [blocks][2] partial sky gradients, or null
  int rl_cap;           // wave row capacity of the carry kernel (even); 0: atomic kernel
  // Waveform mode: h+ / hx are the Galactic-binary waveform of this parameter
  // row at t_j = (k0 + j) dt (hp, hc, g_hp, g_hc unused); the carry kernel
  // writes the tile's seven parameter-gradient sums to gb_part[0..6].
  const double* params;
  int64_t k0;
  double* gb_part;
};

// Per-tap-count launchers (N = order + 1), instantiated in forward_*.hip.
template <int N>
hipError_t launch_project(const ProjArgs& a, hipStream_t s);
template <int N>
hipError_t launch_tdi(const TdiArgs& a, int gen, hipStream_t s);

template <int N>
hipError_t launch_tdi_adjoint(const TdiAdjArgs& a, int gen, hipStream_t s);
template <int N>
hipError_t launch_project_adjoint(const ProjAdjArgs& a, hipStream_t s);

// Records a formatted message for lr_last_error() and returns `status`.
int set_error(int status, const char* fmt, ...);

// Wave row capacity of the carry adjoint kernels for a delay spread of
// `spread` seconds (rows per wave, concurrent carries, further doubles of LDS
// per wave), or 0 if the rows do not fit LDS.
int carry_row_capacity(int order, double spread, double dt, int rows, int ncarry, int extra);

// Workgroup size of the tiled kernels (output samples per workgroup).
constexpr int kTile = 256;

hipError_t run_fill_zero(double* p, int64_t n, hipStream_t s);
hipError_t run_sky_finalize(const double* part, int64_t nblocks, double* g_sky, hipStream_t s);
size_t loglike_workspace_bytes();
hipError_t run_loglike(const double* h, const double* d, int64_t n, double inv_var, double* g,
                       double* part, double* out, hipStream_t s);
hipError_t run_tdi_adjoint(int order, int gen, const TdiAdjArgs& a, hipStream_t s);
hipError_t run_batch_loglike(const double* h, const double* d, const int64_t* items,
                             int64_t n_items, double inv_var, double* g, double* part,
                             const int64_t* span, int64_t n_templates, double* out,
                             hipStream_t s);
hipError_t run_batch_sky_finalize(const double* part, const int64_t* span, int64_t n_templates,
                                  double* g_sky, hipStream_t s);
// Before a fused forward: zero the work counter and tabulate sin, cos of each
// template's sky angles (trig[4k..4k+3] from sky[stride * k + 0, 1]).
hipError_t run_forward_prep(int* counter, const double* sky, int stride, int64_t n,
                            double* trig, hipStream_t s);
hipError_t run_project_adjoint(int order, const ProjAdjArgs& a, hipStream_t s);

// Runtime dispatch on the interpolation order (odd 1..31).
hipError_t run_project_links(int order, const ProjArgs& a, hipStream_t s);
hipError_t run_tdi(int order, int gen, const TdiArgs& a, hipStream_t s);

}  // namespace lr
