// Galactic-binary polarisations (Sec. III) and their adjoint with respect to
// the eight source parameters, for batches of templates on one time grid.
//
//   Phi(t) = 2 pi (f0 t + fdot t^2 / 2 + fddot t^3 / 6) + phi0,
//   fddot  = 11 fdot^2 / (3 f0)   (gravitational-wave driven evolution),
//   a+ = -(1 + cos^2 iota) A cos Phi,   ax = -2 cos(iota) A sin Phi,
//   h+ = cos(2 psi) a+ - sin(2 psi) ax,  hx = sin(2 psi) a+ + cos(2 psi) ax.
//
// t = (k0 + j) dt is exact for the sample grids used here.  The phase is
// evaluated in cycles with f0 t split into a rounded product and its exact
// error (fma), and the whole cycles are removed before the multiplication by
// 2 pi: over a year f0 t reaches ~4e5 cycles, where plain FP64 would leave
// ~1e-10 rad of rounding in the phase.
#include "internal.hpp"
#include "gb_types.hpp"

namespace lr {
namespace gb {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;                 // samples per lane (forward)
constexpr double kTwoPi = 6.283185307179586;

struct Source {
  double A, f0, fdot, fddot, phi0, ci, si, c2, s2;
};

__device__ __forceinline__ Source load_source(const double* p) {
  Source s;
  s.A = p[0];
  s.f0 = p[1];
  s.fdot = p[2];
  s.fddot = 11.0 / 3.0 * p[2] * p[2] / p[1];
  s.phi0 = p[3];
  sincos(p[4], &s.si, &s.ci);
  sincos(2.0 * p[5], &s.s2, &s.c2);
  return s;
}

// Phase in radians reduced by whole cycles (|result| <~ 2 pi + |phi0| plus
// the chirp's few cycles).  Contraction is off here: fusing f0 t into p - n
// would fold the product's rounding error in twice.
__device__ __forceinline__ double phase(const Source& s, double t) {
#pragma clang fp contract(off)
  const double p = s.f0 * t;
  const double e = fma(s.f0, t, -p);          // f0 t = p + e exactly
  const double n = rint(p);
  const double rest = fma(t * t, fma(s.fddot / 6.0, t, 0.5 * s.fdot), e);
  return kTwoPi * ((p - n) + rest) + s.phi0;
}

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
    double sn, cs;
    sincos(phase(s, (double)(a.k0 + j) * a.dt), &sn, &cs);
    const double ap = ap0 * cs, ac = ac0 * sn;
    hp[j] = s.c2 * ap - s.s2 * ac;
    hc[j] = s.s2 * ap + s.c2 * ac;
  }
}

// Per-block partial sums of the seven sample sums the parameter gradient
// needs (see gb_finalize_kernel).
__global__ __launch_bounds__(kThreads) void gb_adjoint_kernel(GbArgs a) {
  __shared__ double red[kGbSums][kThreads / 64];
  const int64_t tpl = blockIdx.y;
  const Source s = load_source(a.params + 8 * tpl);
  const double A = s.A;
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
    const double t = (double)(a.k0 + j) * a.dt;
    double sn, cs;
    sincos(phase(s, t), &sn, &cs);
    const double g_p = gp[j], g_c = gc[j];
    const double Gp = g_p * s.c2 + g_c * s.s2;          // d/d a+
    const double Gc = -g_p * s.s2 + g_c * s.c2;         // d/d ax
    const double ap = -(1.0 + s.ci * s.ci) * A * cs, ac = -2.0 * s.ci * A * sn;
    const double Q = Gp * (1.0 + s.ci * s.ci) * A * sn - Gc * 2.0 * s.ci * A * cs;   // d/d Phi
    acc[0] += Gp * ap + Gc * ac;                        // x A: d/dA
    acc[1] += 2.0 * s.si * A * (Gp * s.ci * cs + Gc * sn);   // d/d iota
    acc[2] += 2.0 * (ap * Gc - ac * Gp);                // d/d psi
    acc[3] += Q;                                        // d/d phi0
    acc[4] += Q * t;
    acc[5] += Q * t * t;
    acc[6] += Q * t * t * t;
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

// g_params[t] from the template's block partials, summed in a fixed order:
// d/dA = S0 / A, d/diota = S1, d/dpsi = S2, d/dphi0 = S3,
// d/df0 = 2 pi (S4 - fddot / (6 f0) S6), d/dfdot = 2 pi (S5 / 2 + (22/3)
// (fdot / f0) S6 / 6)  (fddot depends on f0 and fdot), d/dlam = d/dbeta = 0.
__global__ __launch_bounds__(64) void gb_finalize_kernel(GbArgs a, int64_t blocks) {
  __shared__ double tot[kGbSums];
  const int64_t tpl = blockIdx.x;
  if (threadIdx.x < kGbSums) {
    double v = 0.0;
    for (int64_t b = 0; b < blocks; ++b) v += a.part[(tpl * blocks + b) * kGbSums + threadIdx.x];
    tot[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double* p = a.params + 8 * tpl;
    const double f0 = p[1], fdot = p[2], fddot = 11.0 / 3.0 * fdot * fdot / f0;
    double* g = a.g_params + 8 * tpl;
    g[0] = tot[0] / p[0];
    g[1] = kTwoPi * (tot[4] - fddot / (6.0 * f0) * tot[6]);
    g[2] = kTwoPi * (0.5 * tot[5] + 22.0 / 3.0 * fdot / f0 * tot[6] / 6.0);
    g[3] = tot[3];
    g[4] = tot[1];
    g[5] = tot[2];
    g[6] = 0.0;
    g[7] = 0.0;
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

}  // namespace lr
