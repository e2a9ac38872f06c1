// Batched adjoint kernels for gfx950 (FP64): the transposes of the batched
// forward, one launch per stage over (template or pair, tile) work items.
#pragma once

#include "adjoint_kernels.hpp"
#include "batch_types.hpp"

namespace lr {

// ---------------------------------------------------------------------------
// Batched adjoints: one work item = (template, tile); the per-tile bodies are
// the single-template ones.
// ---------------------------------------------------------------------------
__device__ __forceinline__ TdiAdjArgs batch_tdi_args(const BatchAdjArgs& a,
                                                     const BatchAdjTemplate& T) {
  TdiAdjArgs x;
  x.orb = a.orb_t;
  x.g_out = a.g_out + T.out_off;
  x.channels = a.channels;
  x.n_y = T.n_y;
  x.t_off = a.t_off_y;
  x.dt = a.dt;
  x.inv_dt = a.inv_dt;
  x.out_start = a.F;
  x.n_out = T.n_out;
  x.g_y = a.g_y + T.gy_off;
  x.rl_cap = 0;
  return x;
}

// Work item = (pair of templates, tile): both templates' scatters reuse each
// interpolation weight set (the TDI delays depend on the orbits only).
template <int N, int GEN>
__global__ __launch_bounds__(kBlock, 4) void batch_tdi_adjoint_kernel(BatchAdjArgs a) {
  __shared__ double acc[2 * 6 * kAdjTdiCap(N)];
  __shared__ int red[2][kBlock / 64];
  const int64_t pr = a.items[2 * blockIdx.x], tile = a.items[2 * blockIdx.x + 1];
  const int64_t b0 = a.pairs[2 * pr], b1 = a.pairs[2 * pr + 1];
  TdiAdjArgs x[2];
  x[0] = batch_tdi_args(a, a.tpl[b0]);
  x[1] = b1 >= 0 ? batch_tdi_args(a, a.tpl[b1]) : x[0];
  const bool live[2] = {true, b1 >= 0 && tile * kBlock < x[1].n_out};
  tdi_adjoint_tile<N, GEN, 2>(x, live, tile, acc, red);
}

// Per-template projection-adjoint arguments of work item b.
__device__ __forceinline__ ProjAdjArgs batch_proj_args(const BatchAdjArgs& a,
                                                       const BatchAdjTemplate& T) {
  ProjAdjArgs x;
  x.orb = a.orb_p;
  x.hp = a.hp ? a.hp + T.h_off : nullptr;
  x.hc = a.hc ? a.hc + T.h_off : nullptr;
  x.n_h = T.n_h;
  x.t_off = T.t_off_h;
  x.dt = a.dt;
  x.inv_dt = a.inv_dt;
  x.sky = a.sky + a.sky_stride * T.index;
  x.y_start = T.y_start;
  x.n_y = T.n_y;
  x.g_y = a.g_y + T.gy_off;
  x.g_hp = a.g_hp ? a.g_hp + T.h_off : nullptr;
  x.g_hc = a.g_hc ? a.g_hc + T.h_off : nullptr;
  x.sky_part = nullptr;
  x.rl_cap = 0;
  x.params = a.params ? a.params + 8 * T.index : nullptr;
  x.k0 = -(T.y_start + a.F);                        // waveform time 0 at output sample 0
  x.gb_part = nullptr;
  return x;
}

template <int N>
__global__ __launch_bounds__(kBlock, LR_PADJ_MIN_WAVES) void batch_project_adjoint_kernel(BatchAdjArgs a) {
  __shared__ double acc[2 * kAdjProjCap(N)];
  __shared__ ProjAdjShared sh_;
  const int64_t b = a.items[2 * blockIdx.x], tile = a.items[2 * blockIdx.x + 1];
  project_adjoint_tile<N>(batch_proj_args(a, a.tpl[b]), tile, acc, sh_);
}

template <int N>
__global__ __launch_bounds__(kBlock, LR_SKY_MIN_WAVES) void batch_project_sky_kernel(BatchAdjArgs a) {
  __shared__ double2 win[kAdjProjCap(N)];
  __shared__ ProjAdjShared sh_;
  const int64_t b = a.sky_items[2 * blockIdx.x], tile = a.sky_items[2 * blockIdx.x + 1];
  project_sky_tile<N>(batch_proj_args(a, a.tpl[b]), tile, win, sh_, a.sky_part + 2 * blockIdx.x);
}

// Carry forms: work item = (pair of templates, tile of kCarryTile outputs) for
// the TDI adjoint (both templates' carries share each weight sequence), and
// (template, tile of kCarryTile link samples) for the projection adjoint.
template <int N, int GEN>
__global__ __launch_bounds__(kBlock, LR_TDI_CARRY_MIN_WAVES) void batch_tdi_adjoint_carry_kernel(BatchAdjArgs a) {
  extern __shared__ double lds_dyn[];
  __shared__ CarryShared cs;
  const int64_t pr = a.items[2 * blockIdx.x], tile = a.items[2 * blockIdx.x + 1];
  const int64_t b0 = a.pairs[2 * pr], b1 = a.pairs[2 * pr + 1];
  const TdiAdjArgs x[2] = {batch_tdi_args(a, a.tpl[b0]),
                           batch_tdi_args(a, a.tpl[b1 >= 0 ? b1 : b0])};
  const bool live[2] = {true, b1 >= 0 && tile * kCarryTile < x[1].n_out};
  tdi_adjoint_carry_tile<N, GEN, 2>(x, live, tile, lds_dyn, a.rl_cap, cs);
}

template <int N>
__global__ __launch_bounds__(kBlock, LR_PADJ_CARRY_MIN_WAVES) void batch_project_adjoint_carry_kernel(BatchAdjArgs a) {
  extern __shared__ double lds_dyn[];
  __shared__ CarryShared cs;
  __shared__ double s_trig[2][2];
  const int64_t b = a.items[2 * blockIdx.x], tile = a.items[2 * blockIdx.x + 1];
  ProjAdjArgs x = batch_proj_args(a, a.tpl[b]);
  if (a.gb_part) x.gb_part = a.gb_part + 7 * blockIdx.x;
  project_adjoint_carry_tile<N>(x, tile, lds_dyn, a.rl_cap, cs, s_trig);
}

// a.items: the carry lists (tiles of kCarryTile) when a.rl_cap > 0, else the
// atomic lists (tiles of kBlock).
template <int N, int GEN>
hipError_t launch_batch_tdi_adjoint(const BatchAdjArgs& a, int64_t n_items, hipStream_t s) {
  if (a.rl_cap > 0) {
    const size_t bytes = carry_lds_doubles(12, a.rl_cap, 4, N) * sizeof(double);
    hipError_t e = allow_dynamic_lds(batch_tdi_adjoint_carry_kernel<N, GEN>, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_tdi_adjoint_carry_kernel<N, GEN>), dim3((unsigned)n_items),
                       dim3(kBlock), bytes, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((batch_tdi_adjoint_kernel<N, GEN>), dim3((unsigned)n_items), dim3(kBlock), 0,
                     s, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_batch_project_adjoint(const BatchAdjArgs& a, int64_t n_items,
                                        int64_t n_sky_items, hipStream_t s) {
  hipError_t e;
  if (a.rl_cap > 0) {
    const size_t bytes = proj_carry_lds_doubles(a.rl_cap, N) * sizeof(double);
    e = allow_dynamic_lds(batch_project_adjoint_carry_kernel<N>, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_project_adjoint_carry_kernel<N>), dim3((unsigned)n_items),
                       dim3(kBlock), bytes, s, a);
  } else {
    hipLaunchKernelGGL((batch_project_adjoint_kernel<N>), dim3((unsigned)n_items), dim3(kBlock),
                       0, s, a);
  }
  e = hipGetLastError();
  if (e == hipSuccess && a.sky_part && n_sky_items > 0) {
    hipLaunchKernelGGL((batch_project_sky_kernel<N>), dim3((unsigned)n_sky_items), dim3(kBlock),
                       0, s, a);
    e = hipGetLastError();
  }
  return e;
}

#define LR_INSTANTIATE_BATCH_ADJ(NT)                                                           \
  template hipError_t launch_batch_tdi_adjoint<NT, 1>(const BatchAdjArgs&, int64_t,             \
                                                      hipStream_t);                            \
  template hipError_t launch_batch_tdi_adjoint<NT, 2>(const BatchAdjArgs&, int64_t,             \
                                                      hipStream_t);                            \
  template hipError_t launch_batch_project_adjoint<NT>(const BatchAdjArgs&, int64_t, int64_t,    \
                                                      hipStream_t);

}  // namespace lr
