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
  Sky sky;
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

// Per-tap-count launchers (N = order + 1), instantiated in forward_*.hip.
template <int N>
hipError_t launch_project(const ProjArgs& a, hipStream_t s);
template <int N>
hipError_t launch_tdi(const TdiArgs& a, int gen, hipStream_t s);

// Runtime dispatch on the interpolation order (odd 1..31).
hipError_t run_project_links(int order, const ProjArgs& a, hipStream_t s);
hipError_t run_tdi(int order, int gen, const TdiArgs& a, hipStream_t s);

}  // namespace lr
