// Forward response kernels for gfx950 (FP64):
//   project_links_kernel  -- link responses y_ij, Sec. IV.B
//   tdi_kernel            -- Michelson TDI-1 / TDI-2 and A, E, T, Sec. IV.C
//
// Both kernels are time-tiled: a workgroup owns kBlock consecutive output
// samples, computes every retarded position of its samples first, reduces the
// extent of all their interpolation stencils, stages exactly that window of
// the input series in LDS with coalesced loads, and then evaluates the
// Lagrange sums from LDS (the paper's shared-memory sub-arrays, Sec. IV.E,
// re-designed around a per-tile stencil window).  One lane owns one output
// sample; stores are link- / channel-major and coalesced.
#pragma once

#include <utility>

#include "device_common.hpp"
#include "internal.hpp"

namespace lr {

constexpr int kBlock = kTile;   // output samples per workgroup
constexpr int kSlack = 64;   // window samples beyond kBlock + taps

// ---------------------------------------------------------------------------
// Shared tile machinery
// ---------------------------------------------------------------------------

// Sky basis from the device angles [lam, beta]: two lanes evaluate the
// trigonometric functions, the workgroup shares them through LDS.
struct SkyTrig {
  double sl, cl, sb, cb;
};

__device__ __forceinline__ SkyTrig load_sky(const double* sky, double (&s_trig)[2][2]) {
  const int tid = threadIdx.x;
  if (tid < 2) {
    double sn, cs;
    sincos(sky[tid], &sn, &cs);
    s_trig[tid][0] = sn;
    s_trig[tid][1] = cs;
  }
  __syncthreads();
  return SkyTrig{s_trig[0][0], s_trig[0][1], s_trig[1][0], s_trig[1][1]};
}

// Workgroup-wide [min(lo), max(hi)] of per-lane int ranges.
template <int BLOCK>
__device__ __forceinline__ void block_range(int lo, int hi, int (&red)[2][BLOCK / 64], int& wlo,
                                            int& whi) {
  const int tid = threadIdx.x;
  lo = wave_min(lo);
  hi = wave_max(hi);
  if ((tid & 63) == 0) { red[0][tid >> 6] = lo; red[1][tid >> 6] = hi; }
  __syncthreads();
  wlo = red[0][0];
  whi = red[1][0];
#pragma unroll
  for (int w = 1; w < BLOCK / 64; ++w) { wlo = min(wlo, red[0][w]); whi = max(whi, red[1][w]); }
}

// ---------------------------------------------------------------------------
// Projection
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kBlock) void project_links_kernel(ProjArgs a) {
  constexpr int H = N / 2;
  constexpr int CAP = kBlock + N + kSlack;
  __shared__ double2 win[CAP];
  __shared__ int red[2][kBlock / 64];
  __shared__ double s_trig[2][2];

  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock;
  const int64_t i = i0 + tid;
  const bool active = i < a.n_y;
  const int rel = active ? tid : (int)(a.n_y - 1 - i0);   // idle lanes mirror the last sample
  const int64_t q = a.y_start + i0 + rel;

  const SkyTrig tr = load_sky(a.sky, s_trig);
  const Sky sk = sky_from_trig(tr.sl, tr.cl, tr.sb, tr.cb);
  double u;
  const double* seg = orbit_segment(a.orb, a.t_off + (double)q * a.dt, u);
  LinkGeom g;
  link_geometry(seg, u, sk, g);

  int sh[9];
  double ep[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) sh[p] = split_delay(position_delay(g, p), a.inv_dt, ep[p]);
  int lo = sh[0], hi = sh[0];
#pragma unroll
  for (int p = 1; p < 9; ++p) { lo = min(lo, sh[p]); hi = max(hi, sh[p]); }
  int wlo, whi;
  block_range<kBlock>(rel + lo - (H - 1), rel + hi + H, red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = a.y_start + i0 + wlo;     // h-index of win[0]
  const int64_t hmax = a.n_h - 1;

  double hv[2][9];
  if (count > 0 && count <= CAP) {
    for (int k = tid; k < count; k += kBlock) {
      int64_t j = base + k;
      j = j < 0 ? 0 : (j > hmax ? hmax : j);
      win[k] = make_double2(a.hp[j], a.hc[j]);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      double w[N];
      lagrange_weights<N>(ep[p], w);
      const double2* src = win + (rel + sh[p] - (H - 1) - wlo);
      double sp = 0.0, sc = 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        double2 v = src[m];
        sp = fma(w[m], v.x, sp);
        sc = fma(w[m], v.y, sc);
      }
      hv[0][p] = sp;
      hv[1][p] = sc;
    }
  } else {
    // Window larger than the LDS tile (very small dt or extreme orbits):
    // read the stencils from global memory, indices clamped.
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      double w[N];
      lagrange_weights<N>(ep[p], w);
      const int64_t j0 = q + sh[p] - (H - 1);
      double sp = 0.0, sc = 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        int64_t j = j0 + m;
        j = j < 0 ? 0 : (j > hmax ? hmax : j);
        sp = fma(w[m], a.hp[j], sp);
        sc = fma(w[m], a.hc[j], sc);
      }
      hv[0][p] = sp;
      hv[1][p] = sc;
    }
  }

  if (!active) return;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const int arm = kArm[l];
    const int pr = kLinkRecv[l] - 1, pe = 3 + l;
    double num = g.xip[arm] * (hv[0][pe] - hv[0][pr]) + g.xic[arm] * (hv[1][pe] - hv[1][pr]);
    a.y[(int64_t)l * a.n_y + i] = num / (2.0 * (1.0 - kDir[l] * g.kn[arm]));
  }
}

// ---------------------------------------------------------------------------
// TDI
// ---------------------------------------------------------------------------
// Write X, Y, Z and/or A = (Z-X)/sqrt2, E = (X-2Y+Z)/sqrt6, T = (X+Y+Z)/sqrt3
// (Sec. IV.C) for sample i; rows are n_out apart.
__device__ __forceinline__ void store_channels(const double (&xyz)[3], int channels, double* out,
                                               int64_t n_out, int64_t i) {
  const double X = xyz[0], Y = xyz[1], Z = xyz[2];
  double* o = out + i;
  if (channels != 1) {            // LR_XYZ or LR_XYZ_AET
    o[0] = X;
    o[n_out] = Y;
    o[2 * n_out] = Z;
    o += 3 * n_out;
  }
  if (channels != 0) {            // LR_AET or LR_XYZ_AET
    o[0] = (Z - X) / 1.4142135623730950488;            // sqrt(2)
    o[n_out] = (X - 2.0 * Y + Z) / 2.4494897427831780982;  // sqrt(6)
    o[2 * n_out] = (X + Y + Z) / 1.7320508075688772935;    // sqrt(3)
  }
}

template <int GEN>
struct TdiTab {
  static constexpr TdiTable<GEN> v = make_tdi_table<GEN>();
};

// Delay of group G at the light times L (compile-time table entry).
template <int GEN, int G>
__device__ __forceinline__ double delay_of(const double (&L)[6]) {
  constexpr DelayGroup grp = TdiTab<GEN>::v.group[G];
  double d = 0.0;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    if (grp.cnt[l] == 1) d += L[l];
    else if (grp.cnt[l] > 1) d = fma((double)grp.cnt[l], L[l], d);
  }
  return d;
}

template <int GEN, int... G>
__device__ __forceinline__ void delay_range(const double (&L)[6], double& dmin, double& dmax,
                                            std::integer_sequence<int, G...>) {
  dmin = INFINITY;
  dmax = -INFINITY;
  ((dmin = fmin(dmin, delay_of<GEN, G>(L)), dmax = fmax(dmax, delay_of<GEN, G>(L))), ...);
}

// Interpolate every series that group G delays and add it to its channel.
template <int N, int GEN, int G, bool LDS>
__device__ __forceinline__ void apply_group(const double (&L)[6], double inv_dt, const double* lds,
                                            int lds_stride, int c0, const double* y, int64_t n_y,
                                            int64_t p, double (&acc)[3]) {
  constexpr int H = N / 2;
  constexpr DelayGroup grp = TdiTab<GEN>::v.group[G];
  double eps;
  const int sh = split_delay(delay_of<GEN, G>(L), inv_dt, eps);
  double w[N];
  lagrange_weights<N>(eps, w);
#pragma unroll
  for (int k = 0; k < grp.nuse; ++k) {
    double s = 0.0;
    if constexpr (LDS) {
      const double* src = lds + grp.use[k].link * lds_stride + (c0 + sh - (H - 1));
#pragma unroll
      for (int m = 0; m < N; ++m) s = fma(w[m], src[m], s);
    } else {
      const int64_t j0 = p + sh - (H - 1);
      const double* ys = y + (int64_t)grp.use[k].link * n_y;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        int64_t j = j0 + m;
        j = j < 0 ? 0 : (j > n_y - 1 ? n_y - 1 : j);
        s = fma(w[m], ys[j], s);
      }
    }
    acc[grp.use[k].chan] += (double)grp.use[k].sign * s;
  }
}

template <int N, int GEN, bool LDS, int... G>
__device__ __forceinline__ void apply_groups(const double (&L)[6], double inv_dt, const double* lds,
                                             int lds_stride, int c0, const double* y, int64_t n_y,
                                             int64_t p, double (&acc)[3],
                                             std::integer_sequence<int, G...>) {
  (apply_group<N, GEN, G, LDS>(L, inv_dt, lds, lds_stride, c0, y, n_y, p, acc), ...);
}

template <int N, int GEN>
__global__ __launch_bounds__(kBlock) void tdi_kernel(TdiArgs a) {
  constexpr int H = N / 2;
  constexpr int CAP = kBlock + N + kSlack;
  constexpr int NG = TdiTab<GEN>::v.ngroup;
  constexpr int ND = TdiTab<GEN>::v.ndirect;
  using Groups = std::make_integer_sequence<int, NG>;
  __shared__ double win[6 * CAP];
  __shared__ int red[2][kBlock / 64];

  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock;
  const int64_t i = i0 + tid;
  const bool active = i < a.n_out;
  const int rel = active ? tid : (int)(a.n_out - 1 - i0);
  const int64_t p = a.out_start + i0 + rel;          // y-index of the output sample

  double u;
  const double* seg = orbit_segment(a.orb, a.t_off + (double)p * a.dt, u);
  double L[6];
#pragma unroll
  for (int l = 0; l < 6; ++l) L[l] = spline_at(seg, 9 + l, u);

  double dmin, dmax;
  delay_range<GEN>(L, dmin, dmax, Groups{});
  double e_unused;
  int lo = min(0, split_delay(dmax, a.inv_dt, e_unused) - (H - 1));
  int hi = max(0, split_delay(dmin, a.inv_dt, e_unused) + H);
  int wlo, whi;
  block_range<kBlock>(rel + lo, rel + hi, red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = a.out_start + i0 + wlo;
  const int64_t ymax = a.n_y - 1;
  const int c0 = rel - wlo;

  double acc[3] = {0.0, 0.0, 0.0};
  if (count > 0 && count <= CAP) {
    for (int k = tid; k < count; k += kBlock) {
      int64_t j = base + k;
      j = j < 0 ? 0 : (j > ymax ? ymax : j);
#pragma unroll
      for (int l = 0; l < 6; ++l) win[l * CAP + k] = a.y[(int64_t)l * a.n_y + j];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const Direct dr = TdiTab<GEN>::v.direct[t];
      acc[dr.chan] += (double)dr.sign * win[dr.link * CAP + c0];
    }
    apply_groups<N, GEN, true>(L, a.inv_dt, win, CAP, c0, a.y, a.n_y, p, acc, Groups{});
  } else {
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const Direct dr = TdiTab<GEN>::v.direct[t];
      acc[dr.chan] += (double)dr.sign * a.y[(int64_t)dr.link * a.n_y + p];
    }
    apply_groups<N, GEN, false>(L, a.inv_dt, win, CAP, c0, a.y, a.n_y, p, acc, Groups{});
  }

  if (!active) return;
  store_channels(acc, a.channels, a.out, a.n_out, i);
}

// ---------------------------------------------------------------------------
// Launchers (explicitly instantiated per tap count in forward_*.hip)
// ---------------------------------------------------------------------------
template <int N>
hipError_t launch_project(const ProjArgs& a, hipStream_t s) {
  const int64_t blocks = (a.n_y + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(project_links_kernel<N>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_tdi(const TdiArgs& a, int gen, hipStream_t s) {
  const int64_t blocks = (a.n_out + kBlock - 1) / kBlock;
  if (gen == 1)
    hipLaunchKernelGGL((tdi_kernel<N, 1>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((tdi_kernel<N, 2>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

#define LR_INSTANTIATE_FORWARD(NT)                                              \
  template hipError_t launch_project<NT>(const ProjArgs&, hipStream_t);         \
  template hipError_t launch_tdi<NT>(const TdiArgs&, int, hipStream_t);

}  // namespace lr
