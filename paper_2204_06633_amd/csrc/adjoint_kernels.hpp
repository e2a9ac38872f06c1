// Adjoint (transpose) kernels of the response for gfx950 (FP64).
//
//   tdi_adjoint_kernel      g_out -> g_y: every delayed term's interpolation
//                           transposed into a scatter of w_m * g onto the
//                           stencil taps (Sec. IV.C terms, Sec. IV.E weights)
//   project_adjoint_kernel  g_y -> g_h+, g_hx (and optionally the gradient with
//                           respect to the ecliptic sky angles lam, beta)
//
// Scatter strategy: a workgroup owns the same output tile as the forward
// kernel, accumulates its contributions to its stencil footprint in LDS with
// FP64 LDS atomics, then adds the footprint to the zero-filled global
// gradient with FP64 global atomics.  Neighbouring footprints overlap by
// about one stencil, so a global entry receives at most two tile sums; with a
// zero-filled destination the result does not depend on their order.
#pragma once

#include "forward_kernels.hpp"

namespace lr {

// Gradient with respect to X, Y, Z at sample i from the gradient of the stored
// channels (transpose of store_channels).
__device__ __forceinline__ void load_channel_grads(const double* g_out, int channels,
                                                   int64_t n_out, int64_t i, double (&g)[3]) {
  const double* o = g_out + i;
  g[0] = g[1] = g[2] = 0.0;
  if (channels != 1) {
    g[0] = o[0];
    g[1] = o[n_out];
    g[2] = o[2 * n_out];
    o += 3 * n_out;
  }
  if (channels != 0) {
    const double gA = o[0] / 1.4142135623730950488;
    const double gE = o[n_out] / 2.4494897427831780982;
    const double gT = o[2 * n_out] / 1.7320508075688772935;
    g[0] += gT + gE - gA;
    g[1] += gT - 2.0 * gE;
    g[2] += gT + gE + gA;
  }
}

// ---------------------------------------------------------------------------
// TDI adjoint
// ---------------------------------------------------------------------------
template <int N, int GEN, int G, bool LDS>
__device__ __forceinline__ void scatter_group(const double (&L)[6], double inv_dt, double* lds,
                                              int lds_stride, int c0, double* gy, int64_t n_y,
                                              int64_t p, const double (&gch)[3]) {
  constexpr int H = N / 2;
  constexpr DelayGroup grp = TdiTab<GEN>::v.group[G];
  double eps;
  const int sh = split_delay(delay_of<GEN, G>(L), inv_dt, eps);
  double w[N];
  lagrange_weights<N>(eps, w);
#pragma unroll
  for (int k = 0; k < grp.nuse; ++k) {
    const double v = (double)grp.use[k].sign * gch[grp.use[k].chan];
    if constexpr (LDS) {
      double* dst = lds + grp.use[k].link * lds_stride + (c0 + sh - (H - 1));
#pragma unroll
      for (int m = 0; m < N; ++m) atomicAdd(dst + m, w[m] * v);
    } else {
      const int64_t j0 = p + sh - (H - 1);
      double* ys = gy + (int64_t)grp.use[k].link * n_y;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        int64_t j = j0 + m;
        j = j < 0 ? 0 : (j > n_y - 1 ? n_y - 1 : j);
        atomicAdd(ys + j, w[m] * v);
      }
    }
  }
}

template <int N, int GEN, bool LDS, int... G>
__device__ __forceinline__ void scatter_groups(const double (&L)[6], double inv_dt, double* lds,
                                               int lds_stride, int c0, double* gy, int64_t n_y,
                                               int64_t p, const double (&gch)[3],
                                               std::integer_sequence<int, G...>) {
  (scatter_group<N, GEN, G, LDS>(L, inv_dt, lds, lds_stride, c0, gy, n_y, p, gch), ...);
}

constexpr int kAdjTdiCap(int N) { return kBlock + N + kSlack; }

// One output tile (kBlock samples) of the TDI adjoint; `acc` and `red` are
// the workgroup's LDS scratch.
template <int N, int GEN>
__device__ __forceinline__ void tdi_adjoint_tile(const TdiAdjArgs& a, int64_t tile, double* acc,
                                                 int (&red)[2][kBlock / 64]) {
  constexpr int H = N / 2;
  constexpr int CAP = kAdjTdiCap(N);
  constexpr int NG = TdiTab<GEN>::v.ngroup;
  constexpr int ND = TdiTab<GEN>::v.ndirect;
  using Groups = std::make_integer_sequence<int, NG>;

  const int tid = threadIdx.x;
  const int64_t i0 = tile * kBlock;
  const int64_t i = i0 + tid;
  const bool active = i < a.n_out;
  const int rel = active ? tid : (int)(a.n_out - 1 - i0);
  const int64_t p = a.out_start + i0 + rel;

  double L[6];
  light_times(a.orb, a.t_off + (double)p * a.dt, L);
  double dmin, dmax;
  delay_range<GEN>(L, dmin, dmax, Groups{});
  double e_unused;
  int lo = min(0, split_delay(dmax, a.inv_dt, e_unused) - (H - 1));
  int hi = max(0, split_delay(dmin, a.inv_dt, e_unused) + H);
  int wlo, whi;
  block_range<kBlock>(rel + lo, rel + hi, red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = a.out_start + i0 + wlo;
  const int c0 = rel - wlo;

  double gch[3] = {0.0, 0.0, 0.0};
  if (active) load_channel_grads(a.g_out, a.channels, a.n_out, i, gch);

  if (count > 0 && count <= CAP) {
    for (int k = tid; k < 6 * CAP; k += kBlock) acc[k] = 0.0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const Direct dr = TdiTab<GEN>::v.direct[t];
      atomicAdd(&acc[dr.link * CAP + c0], (double)dr.sign * gch[dr.chan]);
    }
    scatter_groups<N, GEN, true>(L, a.inv_dt, acc, CAP, c0, a.g_y, a.n_y, p, gch, Groups{});
    __syncthreads();
    for (int k = tid; k < count; k += kBlock) {
      const int64_t j = base + k;
      if (j < 0 || j >= a.n_y) continue;
#pragma unroll
      for (int l = 0; l < 6; ++l) atomicAdd(a.g_y + (int64_t)l * a.n_y + j, acc[l * CAP + k]);
    }
  } else {
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const Direct dr = TdiTab<GEN>::v.direct[t];
      atomicAdd(a.g_y + (int64_t)dr.link * a.n_y + p, (double)dr.sign * gch[dr.chan]);
    }
    scatter_groups<N, GEN, false>(L, a.inv_dt, acc, CAP, c0, a.g_y, a.n_y, p, gch, Groups{});
  }
}

template <int N, int GEN>
__global__ __launch_bounds__(kBlock) void tdi_adjoint_kernel(TdiAdjArgs a) {
  __shared__ double acc[6 * kAdjTdiCap(N)];
  __shared__ int red[2][kBlock / 64];
  tdi_adjoint_tile<N, GEN>(a, blockIdx.x, acc, red);
}

// ---------------------------------------------------------------------------
// Projection adjoint
// ---------------------------------------------------------------------------
constexpr int kAdjProjCap(int N) { return kBlock + N + kSlack; }

struct ProjAdjShared {
  int red[2][kBlock / 64];
  double s_trig[2][2];
  double s_part[2][kBlock / 64];
};

// One link-sample tile (kBlock samples) of the projection adjoint; its sky
// partial pair goes to part[0..1] (if SKY).  acc: 2 * CAP doubles of LDS,
// win: CAP double2 (SKY only).
template <int N, bool SKY>
__device__ __forceinline__ void project_adjoint_tile(const ProjAdjArgs& a, int64_t tile,
                                                     double* acc, double2* win,
                                                     ProjAdjShared& sh_, double* part_out) {
  constexpr int H = N / 2;
  constexpr int CAP = kAdjProjCap(N);
  auto& red = sh_.red;
  auto& s_trig = sh_.s_trig;
  auto& s_part = sh_.s_part;

  const int tid = threadIdx.x;
  const int64_t i0 = tile * kBlock;
  const int64_t i = i0 + tid;
  const bool active = i < a.n_y;
  const int rel = active ? tid : (int)(a.n_y - 1 - i0);
  const int64_t q = a.y_start + i0 + rel;

  const SkyTrig tr = load_sky(a.sky, s_trig);
  const Sky sk = sky_from_trig(tr.sl, tr.cl, tr.sb, tr.cb);
  LinkGeom g;
  link_geometry(a.orb, a.t_off + (double)q * a.dt, sk, g);

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
  const int64_t base = a.y_start + i0 + wlo;
  const int64_t hmax = a.n_h - 1;

  // Upstream gradient scaled by 1/(2(1 - k.n)) per link, then the amplitude
  // each of the nine positions scatters onto h+ and hx.
  double gy[6], c[6];
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    gy[l] = active ? a.g_y[(int64_t)l * a.n_y + i] : 0.0;
    c[l] = gy[l] / (2.0 * (1.0 - kDir[l] * g.kn[kArm[l]]));
  }
  double amp[2][9];
#pragma unroll
  for (int s = 0; s < 3; ++s) { amp[0][s] = 0.0; amp[1][s] = 0.0; }
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const int arm = kArm[l], r = kLinkRecv[l] - 1;
    amp[0][3 + l] = c[l] * g.xip[arm];
    amp[1][3 + l] = c[l] * g.xic[arm];
    amp[0][r] -= c[l] * g.xip[arm];
    amp[1][r] -= c[l] * g.xic[arm];
  }

  double hv[2][9], dh[2][9];
  const bool use_lds = count > 0 && count <= CAP;
  if (use_lds) {
    for (int k = tid; k < 2 * CAP; k += kBlock) acc[k] = 0.0;
    if constexpr (SKY) {
      for (int k = tid; k < count; k += kBlock) {
        int64_t j = base + k;
        j = j < 0 ? 0 : (j > hmax ? hmax : j);
        win[k] = make_double2(a.hp[j], a.hc[j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    double w[N], dw[N];
    if constexpr (SKY) lagrange_weights_d<N>(ep[p], w, dw);
    else lagrange_weights<N>(ep[p], w);
    const int off = rel + sh[p] - (H - 1) - wlo;
    const int64_t j0 = q + sh[p] - (H - 1);
    double sp = 0.0, sc = 0.0, dsp = 0.0, dsc = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      if (use_lds) {
        atomicAdd(&acc[off + m], amp[0][p] * w[m]);
        atomicAdd(&acc[CAP + off + m], amp[1][p] * w[m]);
      } else {
        int64_t j = j0 + m;
        j = j < 0 ? 0 : (j > hmax ? hmax : j);
        atomicAdd(a.g_hp + j, amp[0][p] * w[m]);
        atomicAdd(a.g_hc + j, amp[1][p] * w[m]);
      }
      if constexpr (SKY) {
        double2 v;
        if (use_lds) {
          v = win[off + m];
        } else {
          int64_t j = j0 + m;
          j = j < 0 ? 0 : (j > hmax ? hmax : j);
          v = make_double2(a.hp[j], a.hc[j]);
        }
        sp = fma(w[m], v.x, sp);
        sc = fma(w[m], v.y, sc);
        dsp = fma(dw[m], v.x, dsp);
        dsc = fma(dw[m], v.y, dsc);
      }
    }
    hv[0][p] = sp; hv[1][p] = sc;
    dh[0][p] = dsp; dh[1][p] = dsc;
  }

  if (use_lds) {
    __syncthreads();
    for (int k = tid; k < count; k += kBlock) {
      const int64_t j = base + k;
      if (j < 0 || j > hmax) continue;
      atomicAdd(a.g_hp + j, acc[k]);
      atomicAdd(a.g_hc + j, acc[CAP + k]);
    }
  }

  if constexpr (SKY) {
    // d y_l / d(k, u, v) contracted with g_y, then with d(k, u, v)/d(lam, beta).
    double Gk[3] = {0.0, 0.0, 0.0}, Gu[3] = {0.0, 0.0, 0.0}, Gv[3] = {0.0, 0.0, 0.0};
    const double inv_cdt = a.inv_dt / kC;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const int arm = kArm[l], r = kLinkRecv[l] - 1, e = kLinkEmit[l] - 1, pe = 3 + l;
      const double dir = kDir[l];
      const double inv = 1.0 / (2.0 * (1.0 - dir * g.kn[arm]));
      const double dp = hv[0][pe] - hv[0][r], dc = hv[1][pe] - hv[1][r];
      const double yl = inv * (g.xip[arm] * dp + g.xic[arm] * dc);
      const double He = g.xip[arm] * dh[0][pe] + g.xic[arm] * dh[1][pe];
      const double Hr = g.xip[arm] * dh[0][r] + g.xic[arm] * dh[1][r];
      const double sn = 2.0 * inv * yl * dir;          // through 1/(2(1 - k.n))
      const double su = 2.0 * inv * (g.un[arm] * dp + g.vn[arm] * dc);
      const double sv = 2.0 * inv * (g.un[arm] * dc - g.vn[arm] * dp);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const double pos = -inv * inv_cdt * (He * g.x[e][cc] - Hr * g.x[r][cc]);
        Gk[cc] = fma(gy[l], fma(sn, g.n[arm][cc], pos), Gk[cc]);
        Gu[cc] = fma(gy[l], su * g.n[arm][cc], Gu[cc]);
        Gv[cc] = fma(gy[l], sv * g.n[arm][cc], Gv[cc]);
      }
    }
    const SkyDeriv D = sky_derivatives(tr.sl, tr.cl, tr.sb, tr.cb);
    double part[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      double s = 0.0;
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        s += Gk[cc] * D.dk[t][cc] + Gu[cc] * D.du[t][cc] + Gv[cc] * D.dv[t][cc];
      part[t] = s;
    }
    // deterministic block reduction -> one partial pair per workgroup
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) part[t] += __shfl_xor(part[t], o, 64);
    }
    if ((tid & 63) == 0) { s_part[0][tid >> 6] = part[0]; s_part[1][tid >> 6] = part[1]; }
    __syncthreads();
    if (tid == 0) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) { s0 += s_part[0][w]; s1 += s_part[1][w]; }
      part_out[0] = s0;
      part_out[1] = s1;
    }
  }
}

template <int N, bool SKY>
__global__ __launch_bounds__(kBlock) void project_adjoint_kernel(ProjAdjArgs a) {
  __shared__ double acc[2 * kAdjProjCap(N)];
  __shared__ double2 win[SKY ? kAdjProjCap(N) : 1];
  __shared__ ProjAdjShared sh_;
  project_adjoint_tile<N, SKY>(a, blockIdx.x, acc, win, sh_,
                               SKY ? a.sky_part + 2 * blockIdx.x : nullptr);
}

template <int N>
hipError_t launch_tdi_adjoint(const TdiAdjArgs& a, int gen, hipStream_t s) {
  const int64_t blocks = (a.n_out + kBlock - 1) / kBlock;
  if (gen == 1)
    hipLaunchKernelGGL((tdi_adjoint_kernel<N, 1>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((tdi_adjoint_kernel<N, 2>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_project_adjoint(const ProjAdjArgs& a, hipStream_t s) {
  const int64_t blocks = (a.n_y + kBlock - 1) / kBlock;
  if (a.sky_part)
    hipLaunchKernelGGL((project_adjoint_kernel<N, true>), dim3((unsigned)blocks), dim3(kBlock), 0,
                       s, a);
  else
    hipLaunchKernelGGL((project_adjoint_kernel<N, false>), dim3((unsigned)blocks), dim3(kBlock),
                       0, s, a);
  return hipGetLastError();
}

#define LR_INSTANTIATE_ADJOINT(NT)                                                   \
  template hipError_t launch_tdi_adjoint<NT>(const TdiAdjArgs&, int, hipStream_t);   \
  template hipError_t launch_project_adjoint<NT>(const ProjAdjArgs&, hipStream_t);

}  // namespace lr
