// Galactic-binary polarisations (Sec. III; the waveform and its compensated
// phase in gb_device.hpp) and their adjoint with respect to the eight source
// parameters, for batches of templates on one time grid.  t = (k0 + j) dt is
// exact for the sample grids used here.
#include "internal.hpp"
#include "gb_device.hpp"
#include "gb_types.hpp"

namespace lr {
namespace gb {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;                 // samples per lane (forward)

__global__ __launch_bounds__(kThreads) void gb_forward_kernel(GbArgs a) {
  const int64_t tpl = blockIdx.y;
  const Source s = load_source(a.params + 8 * tpl);
  const double ap0 = -(1.0 + s.ci * s.ci) * s.A, ac0 = -2.0 * s.ci * s.A;
  double* hp = a.hp + tpl * a.h_stride;
  double* hc = a.hc + tpl * a.h_stride;
  const int64_t j0 = ((int64_t)blockIdx.x * kThreads * kPerThread) + threadIdx.x;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t j = j0 + (int64_t)i * kThreads;
    if (j >= a.n_h) break;
    double p, c;
    polarizations_at(s, ap0, ac0, (double)(a.k0 + j) * a.dt, p, c);
    hp[j] = p;
    hc[j] = c;
  }
}

// Per-block partial sums of the seven sample sums the parameter gradient
// needs (see gb_finalize_kernel).
__global__ __launch_bounds__(kThreads) void gb_adjoint_kernel(GbArgs a) {
  __shared__ double red[kGbSums][kThreads / 64];
  const int64_t tpl = blockIdx.y;
  const Source s = load_source(a.params + 8 * tpl);
  const double* gp = a.g_hp + tpl * a.h_stride;
  const double* gc = a.g_hc + tpl * a.h_stride;
  double acc[kGbSums];
#pragma unroll
  for (int k = 0; k < kGbSums; ++k) acc[k] = 0.0;
  const int64_t j0 = ((int64_t)blockIdx.x * kThreads * kPerThread) + threadIdx.x;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t j = j0 + (int64_t)i * kThreads;
    if (j >= a.n_h) break;
    adjoint_sums(s, (double)(a.k0 + j) * a.dt, gp[j], gc[j], acc);
  }
  // fixed-order reduction: shuffle tree in each wave, then the waves in order
#pragma unroll
  for (int k = 0; k < kGbSums; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_down(acc[k], off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kGbSums; ++k) red[k][wave] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x < kGbSums) {
    double v = red[threadIdx.x][0];
    for (int w = 1; w < kThreads / 64; ++w) v += red[threadIdx.x][w];
    a.part[(tpl * gridDim.x + blockIdx.x) * kGbSums + threadIdx.x] = v;
  }
}

// g_params[t] from the template's block partials, summed in a fixed order
// (finalize_gradient in gb_device.hpp).
__global__ __launch_bounds__(64) void gb_finalize_kernel(GbArgs a, int64_t blocks) {
  __shared__ double tot[kGbSums];
  const int64_t tpl = blockIdx.x;
  if (threadIdx.x < kGbSums) {
    double v = 0.0;
    for (int64_t b = 0; b < blocks; ++b) v += a.part[(tpl * blocks + b) * kGbSums + threadIdx.x];
    tot[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) finalize_gradient(a.params + 8 * tpl, tot, a.g_params + 8 * tpl);
}

// Batched response adjoint in waveform mode: per template (one block of 64
// lanes), the seven sums over its projection tiles and the two sky partials
// over its sky tiles -- lane L adds the tiles i = L, L + 64, ... in order,
// then a fixed-order tree over the lanes (deterministic) -- then the
// parameter gradient.  span rows: (first item, items, template index).
__global__ __launch_bounds__(64) void gb_batch_finalize_kernel(const double* gb_part,
                                                               const int64_t* span,
                                                               const double* sky_part,
                                                               const int64_t* sky_span,
                                                               const double* params,
                                                               double* g_params) {
  const int64_t r = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t first = span[3 * r], cnt = span[3 * r + 1];
  const int64_t sfirst = sky_span[3 * r], scnt = sky_span[3 * r + 1];
  double v[kGbSums + 2];
#pragma unroll
  for (int c = 0; c < kGbSums + 2; ++c) v[c] = 0.0;
  for (int64_t i = lane; i < cnt; i += 64) {
    const double* row = gb_part + (first + i) * kGbSums;
#pragma unroll
    for (int c = 0; c < kGbSums; ++c) v[c] += row[c];
  }
  for (int64_t i = lane; i < scnt; i += 64) {
    v[kGbSums] += sky_part[2 * (sfirst + i)];
    v[kGbSums + 1] += sky_part[2 * (sfirst + i) + 1];
  }
#pragma unroll
  for (int c = 0; c < kGbSums + 2; ++c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o, 64);
  }
  if (lane == 0) {
    const int64_t k = span[3 * r + 2];
    double* g = g_params + 8 * k;
    if (cnt == 0) {                                   // empty template
      for (int c = 0; c < 8; ++c) g[c] = 0.0;
      return;
    }
    finalize_gradient(params + 8 * k, v, g);
    g[6] = v[kGbSums];
    g[7] = v[kGbSums + 1];
  }
}

}  // namespace gb

int64_t gb_blocks(int64_t n_h) {
  const int64_t per = (int64_t)gb::kThreads * gb::kPerThread;
  return (n_h + per - 1) / per;
}

hipError_t run_gb_forward(const GbArgs& a, int64_t n_tpl, hipStream_t s) {
  const dim3 grid((unsigned)gb_blocks(a.n_h), (unsigned)n_tpl);
  hipLaunchKernelGGL(gb::gb_forward_kernel, grid, dim3(gb::kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t run_gb_adjoint(const GbArgs& a, int64_t n_tpl, hipStream_t s) {
  const int64_t blocks = gb_blocks(a.n_h);
  hipLaunchKernelGGL(gb::gb_adjoint_kernel, dim3((unsigned)blocks, (unsigned)n_tpl),
                     dim3(gb::kThreads), 0, s, a);
  hipLaunchKernelGGL(gb::gb_finalize_kernel, dim3((unsigned)n_tpl), dim3(64), 0, s, a, blocks);
  return hipGetLastError();
}

hipError_t run_gb_batch_finalize(const double* gb_part, const int64_t* span,
                                 const double* sky_part, const int64_t* sky_span,
                                 const double* params, int64_t n, double* g_params, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gb::gb_batch_finalize_kernel, dim3((unsigned)n), dim3(64), 0, s, gb_part, span,
                     sky_part, sky_span, params, g_params);
  return hipGetLastError();
}

}  // namespace lr
