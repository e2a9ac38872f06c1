// Adjoint (transpose) kernels of the response for gfx950 (FP64).
//
//   tdi_adjoint_kernel      g_out -> g_y: every delayed term's interpolation
//                           transposed into a scatter of w_m * g onto the
//                           stencil taps (Sec. IV.C terms, Sec. IV.E weights)
//   project_adjoint_kernel  g_y -> g_h+, g_hx
//   project_sky_kernel      g_y, h+, hx -> partial gradients with respect to
//                           the ecliptic sky angles lam, beta
//
// Scatter strategy: a workgroup owns a tile of samples, accumulates its
// contributions to its stencil footprint in LDS with FP64 LDS atomics, then adds the footprint to the zero-filled global
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
constexpr int kAdjTdiCap(int N) { return kBlock + N + kSlack; }

// Fold a lone scatter's value into its weights (saves N multiplies per
// single-use delay group); build-time switch for measurements.
#ifndef LR_TDI_ADJ_FOLD
#define LR_TDI_ADJ_FOLD 1
#endif

// Scatter v * w_m onto N consecutive LDS entries dst[0..N-1].
template <int N>
__device__ __forceinline__ void scatter_lds(double* dst, const double (&w)[N], double v) {
#pragma unroll
  for (int m = 0; m < N; ++m) atomicAdd(dst + m, w[m] * v);
}

// Scatter w_m (already scaled) onto dst[0..N-1].
template <int N>
__device__ __forceinline__ void scatter_lds(double* dst, const double (&w)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) atomicAdd(dst + m, w[m]);
}

// Scatter v * w_m(eps) onto ys[j0 + m], indices clamped to [0, n - 1]; a
// rolled loop computing each weight on its own (rare wide-footprint path).
template <int N>
__device__ __forceinline__ void scatter_global(double* ys, int64_t j0, int64_t n, double eps,
                                               double v) {
#pragma unroll 1
  for (int m = 0; m < N; ++m) {
    int64_t j = j0 + m;
    j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
    atomicAdd(ys + j, lagrange_weight_at<N>(eps, m) * v);
  }
}

// One output tile (kBlock samples) of the TDI adjoint for M templates that
// share the output grid and the TDI orbits (a[k].orb, t_off, dt, out_start
// equal; a[0] the longest): the interpolation weights depend on the orbits
// only, so each weight set serves all M templates' scatters.  live[k] says
// whether template k has outputs in the tile (uniform).  `acc` holds M x 6
// LDS rows of kAdjTdiCap(N); `red` is reduction scratch.  The delay groups
// are walked by a runtime loop over the constant-memory table, so one weight
// set is live at a time.
template <int N, int GEN, int M>
__device__ __forceinline__ void tdi_adjoint_tile(const TdiAdjArgs (&a)[M], const bool (&live)[M],
                                                 int64_t tile, double* acc,
                                                 int (&red)[2][kBlock / 64]) {
  constexpr int H = N / 2;
  constexpr int CAP = kAdjTdiCap(N);
  constexpr int ND = TdiTab<GEN>::v.ndirect;
  const GroupTable<GEN>& GT = group_table<GEN>();
  const TdiAdjArgs& a0 = a[0];

  const int tid = threadIdx.x;
  const int64_t i0 = tile * kBlock;
  const int64_t i = i0 + tid;
  const bool active = i < a0.n_out;
  const int rel = active ? tid : (int)(a0.n_out - 1 - i0);
  const int64_t p = a0.out_start + i0 + rel;

  double L[6];
  light_times(a0.orb, a0.t_off + (double)p * a0.dt, L);
  double dlo, dhi, e_unused;
  group_delay_bounds(L, GT.chain, dlo, dhi);
  const int lo = min(0, split_delay(dhi, a0.inv_dt, e_unused) - (H - 1));
  const int hi = max(0, split_delay(dlo, a0.inv_dt, e_unused) + H);
  int wlo, whi;
  block_range<kBlock>(rel + lo, rel + hi, red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = a0.out_start + i0 + wlo;
  const int c0 = rel - wlo;

  double gch[M][3];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    gch[k][0] = gch[k][1] = gch[k][2] = 0.0;
    if (live[k] && i < a[k].n_out) load_channel_grads(a[k].g_out, a[k].channels, a[k].n_out, i, gch[k]);
  }

  if (count > 0 && count <= CAP) {
    for (int k = tid; k < M * 6 * CAP; k += kBlock) acc[k] = 0.0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const Direct dr = TdiTab<GEN>::v.direct[t];
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (live[k]) atomicAdd(&acc[(k * 6 + dr.link) * CAP + c0], (double)dr.sign * gch[k][dr.chan]);
    }
#pragma unroll 1
    for (int g = 0; g < GT.n; ++g) {
      const GroupRow& G = GT.row[g];
      double eps;
      const int sh = split_delay(row_delay(G, L), a0.inv_dt, eps);
      const int j0 = c0 + sh - (H - 1);
      if (LR_TDI_ADJ_FOLD && M == 1 && G.nuse == 1) {
        // one scatter: fold its value into the weights
        const double v =
            G.sgn[0][0] * gch[0][0] + G.sgn[0][1] * gch[0][1] + G.sgn[0][2] * gch[0][2];
        double w[N];
        lagrange_weights<N>(eps, w, v);
        scatter_lds<N>(acc + G.link[0] * CAP + j0, w);
        continue;
      }
      double w[N];
      lagrange_weights<N>(eps, w);
#pragma unroll 1
      for (int u = 0; u < G.nuse; ++u) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
          if (!live[k]) continue;                       // uniform
          const double v =
              G.sgn[u][0] * gch[k][0] + G.sgn[u][1] * gch[k][1] + G.sgn[u][2] * gch[k][2];
          scatter_lds<N>(acc + (k * 6 + G.link[u]) * CAP + j0, w, v);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (!live[k]) continue;
      for (int e = tid; e < count; e += kBlock) {
        const int64_t j = base + e;
        if (j < 0 || j >= a[k].n_y) continue;
#pragma unroll
        for (int l = 0; l < 6; ++l)
          atomicAdd(a[k].g_y + (int64_t)l * a[k].n_y + j, acc[(k * 6 + l) * CAP + e]);
      }
    }
  } else {
    // stencil footprint wider than the LDS tile: scatter to global memory
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (!live[k] || !(i < a[k].n_out)) continue;
      const TdiAdjArgs& ak = a[k];
#pragma unroll
      for (int t = 0; t < ND; ++t) {
        const Direct dr = TdiTab<GEN>::v.direct[t];
        atomicAdd(ak.g_y + (int64_t)dr.link * ak.n_y + p, (double)dr.sign * gch[k][dr.chan]);
      }
#pragma unroll 1
      for (int g = 0; g < GT.n; ++g) {
        const GroupRow& G = GT.row[g];
        double eps;
        const int sh = split_delay(row_delay(G, L), ak.inv_dt, eps);
#pragma unroll 1
        for (int u = 0; u < G.nuse; ++u) {
          const double v =
              G.sgn[u][0] * gch[k][0] + G.sgn[u][1] * gch[k][1] + G.sgn[u][2] * gch[k][2];
          scatter_global<N>(ak.g_y + (int64_t)G.link[u] * ak.n_y, p + sh - (H - 1), ak.n_y, eps,
                            v);
        }
      }
    }
  }
}

template <int N, int GEN>
__global__ __launch_bounds__(kBlock, 4) void tdi_adjoint_kernel(TdiAdjArgs a) {
  __shared__ double acc[6 * kAdjTdiCap(N)];
  __shared__ int red[2][kBlock / 64];
  const TdiAdjArgs x[1] = {a};
  const bool live[1] = {true};
  tdi_adjoint_tile<N, GEN, 1>(x, live, blockIdx.x, acc, red);
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

// Per link sample of a tile: geometry, the nine retarded positions split into
// shift + fraction, and the window of h indices the tile's stencils touch.
struct ProjAdjSample {
  bool active;
  int rel;              // tile-relative link sample (idle lanes mirror the last)
  int64_t q;            // h index of the link sample
  int sh[9];
  double ep[9];
};

template <int N>
__device__ __forceinline__ void proj_adj_sample(const ProjAdjArgs& a, int64_t tile,
                                                const Sky& sk, LinkGeom& g, ProjAdjSample& s) {
  const int tid = threadIdx.x;
  const int64_t i0 = tile * kBlock;
  s.active = i0 + tid < a.n_y;
  s.rel = s.active ? tid : (int)(a.n_y - 1 - i0);
  s.q = a.y_start + i0 + s.rel;
  link_geometry(a.orb, a.t_off + (double)s.q * a.dt, sk, g);
#pragma unroll
  for (int p = 0; p < 9; ++p) s.sh[p] = split_delay(position_delay(g, p), a.inv_dt, s.ep[p]);
}

// One link-sample tile (kBlock samples) of the projection adjoint: the
// transpose of the nine interpolations, g_y -> g_h+, g_hx.  acc: 2 * CAP
// doubles of LDS.
template <int N>
__device__ __forceinline__ void project_adjoint_tile(const ProjAdjArgs& a, int64_t tile,
                                                     double* acc, ProjAdjShared& sh_) {
  constexpr int H = N / 2;
  constexpr int CAP = kAdjProjCap(N);
  const int tid = threadIdx.x;
  const int64_t i0 = tile * kBlock;

  const SkyTrig tr = load_sky(a.sky, sh_.s_trig);
  const Sky sk = sky_from_trig(tr.sl, tr.cl, tr.sb, tr.cb);
  ProjAdjSample S;
  double amp[2][9];
  {
    LinkGeom g;
    proj_adj_sample<N>(a, tile, sk, g, S);
    // upstream gradient scaled by 1/(2(1 - k.n)) per link, then the amplitude
    // each position scatters onto h+ and hx
#pragma unroll
    for (int s = 0; s < 3; ++s) { amp[0][s] = 0.0; amp[1][s] = 0.0; }
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const double gy = S.active ? a.g_y[(int64_t)l * a.n_y + i0 + tid] : 0.0;
      const double c = gy / (2.0 * (1.0 - kDir[l] * g.kn[kArm[l]]));
      const int arm = kArm[l], r = kLinkRecv[l] - 1;
      amp[0][3 + l] = c * g.xip[arm];
      amp[1][3 + l] = c * g.xic[arm];
      amp[0][r] -= c * g.xip[arm];
      amp[1][r] -= c * g.xic[arm];
    }
  }
  int lo = S.sh[0], hi = S.sh[0];
#pragma unroll
  for (int p = 1; p < 9; ++p) { lo = min(lo, S.sh[p]); hi = max(hi, S.sh[p]); }
  int wlo, whi;
  block_range<kBlock>(S.rel + lo - (H - 1), S.rel + hi + H, sh_.red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = a.y_start + i0 + wlo;
  const int64_t hmax = a.n_h - 1;

  if (count > 0 && count <= CAP) {
    for (int k = tid; k < 2 * CAP; k += kBlock) acc[k] = 0.0;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      double w[N];
      lagrange_weights<N>(S.ep[p], w);
      const int off = S.rel + S.sh[p] - (H - 1) - wlo;
      scatter_lds<N>(acc + off, w, amp[0][p]);
      scatter_lds<N>(acc + CAP + off, w, amp[1][p]);
      __builtin_amdgcn_sched_barrier(0);   // one weight set live at a time
    }
    __syncthreads();
    for (int k = tid; k < count; k += kBlock) {
      const int64_t j = base + k;
      if (j < 0 || j > hmax) continue;
      atomicAdd(a.g_hp + j, acc[k]);
      atomicAdd(a.g_hc + j, acc[CAP + k]);
    }
  } else {
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const int64_t j0 = S.q + S.sh[p] - (H - 1);
      scatter_global<N>(a.g_hp, j0, a.n_h, S.ep[p], amp[0][p]);
      scatter_global<N>(a.g_hc, j0, a.n_h, S.ep[p], amp[1][p]);
    }
  }
}

// One link-sample tile of the sky gradient: sum over links and samples of
// g_y * d y / d(lam, beta), from the interpolated h+, hx at the nine
// positions and their derivatives with respect to the position (streamed,
// no weight arrays).  Writes the tile's partial pair to part_out[0..1].
// win: CAP double2 of LDS.
template <int N>
__device__ __forceinline__ void project_sky_tile(const ProjAdjArgs& a, int64_t tile,
                                                 double2* win, ProjAdjShared& sh_,
                                                 double* part_out) {
  constexpr int H = N / 2;
  constexpr int CAP = kAdjProjCap(N);
  const int tid = threadIdx.x;
  const int64_t i0 = tile * kBlock;

  const SkyTrig tr = load_sky(a.sky, sh_.s_trig);
  const Sky sk = sky_from_trig(tr.sl, tr.cl, tr.sb, tr.cb);
  ProjAdjSample S;
  LinkGeom g;
  proj_adj_sample<N>(a, tile, sk, g, S);
  int lo = S.sh[0], hi = S.sh[0];
#pragma unroll
  for (int p = 1; p < 9; ++p) { lo = min(lo, S.sh[p]); hi = max(hi, S.sh[p]); }
  int wlo, whi;
  block_range<kBlock>(S.rel + lo - (H - 1), S.rel + hi + H, sh_.red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = a.y_start + i0 + wlo;
  const int64_t hmax = a.n_h - 1;

  double hv[2][9], dh[2][9];
  if (count > 0 && count <= CAP) {
    for (int k = tid; k < count; k += kBlock) {
      int64_t j = base + k;
      j = j < 0 ? 0 : (j > hmax ? hmax : j);
      win[k] = make_double2(a.hp[j], a.hc[j]);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      LagrangeStreamD<N> st(S.ep[p]);
      const int off = S.rel + S.sh[p] - (H - 1) - wlo;
      double sp = 0.0, sc = 0.0, dsp = 0.0, dsc = 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const double2 v = win[off + m];
        const double c = st.coef(m), cd = st.coef_d(m);
        st.step(c, cd, v.x, sp, dsp);
        st.step(c, cd, v.y, sc, dsc);
        st.next();
      }
      hv[0][p] = sp; hv[1][p] = sc;
      dh[0][p] = dsp; dh[1][p] = dsc;
    }
  } else {
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      LagrangeStreamD<N> st(S.ep[p]);
      const int64_t j0 = S.q + S.sh[p] - (H - 1);
      double sp = 0.0, sc = 0.0, dsp = 0.0, dsc = 0.0;
#pragma unroll 1
      for (int m = 0; m < N; ++m) {
        int64_t j = j0 + m;
        j = j < 0 ? 0 : (j > hmax ? hmax : j);
        const double c = st.coef(m), cd = st.coef_d(m);
        st.step(c, cd, a.hp[j], sp, dsp);
        st.step(c, cd, a.hc[j], sc, dsc);
        st.next();
      }
      hv[0][p] = sp; hv[1][p] = sc;
      dh[0][p] = dsp; dh[1][p] = dsc;
    }
  }

  // d y_l / d(k, u, v) contracted with g_y, then with d(k, u, v)/d(lam, beta).
  double Gk[3] = {0.0, 0.0, 0.0}, Gu[3] = {0.0, 0.0, 0.0}, Gv[3] = {0.0, 0.0, 0.0};
  const double inv_cdt = a.inv_dt / kC;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const double gy = S.active ? a.g_y[(int64_t)l * a.n_y + i0 + tid] : 0.0;
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
      Gk[cc] = fma(gy, fma(sn, g.n[arm][cc], pos), Gk[cc]);
      Gu[cc] = fma(gy, su * g.n[arm][cc], Gu[cc]);
      Gv[cc] = fma(gy, sv * g.n[arm][cc], Gv[cc]);
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
  if ((tid & 63) == 0) { sh_.s_part[0][tid >> 6] = part[0]; sh_.s_part[1][tid >> 6] = part[1]; }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) { s0 += sh_.s_part[0][w]; s1 += sh_.s_part[1][w]; }
    part_out[0] = s0;
    part_out[1] = s1;
  }
}

// Minimum resident waves per SIMD of the projection-adjoint and sky kernels
// (build-time tuning knobs; 1 leaves the compiler unconstrained).
#ifndef LR_PADJ_MIN_WAVES
#define LR_PADJ_MIN_WAVES 1
#endif
#ifndef LR_SKY_MIN_WAVES
#define LR_SKY_MIN_WAVES 1
#endif

template <int N>
__global__ __launch_bounds__(kBlock, LR_PADJ_MIN_WAVES) void project_adjoint_kernel(ProjAdjArgs a) {
  __shared__ double acc[2 * kAdjProjCap(N)];
  __shared__ ProjAdjShared sh_;
  project_adjoint_tile<N>(a, blockIdx.x, acc, sh_);
}

template <int N>
__global__ __launch_bounds__(kBlock, LR_SKY_MIN_WAVES) void project_sky_kernel(ProjAdjArgs a) {
  __shared__ double2 win[kAdjProjCap(N)];
  __shared__ ProjAdjShared sh_;
  project_sky_tile<N>(a, blockIdx.x, win, sh_, a.sky_part + 2 * blockIdx.x);
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

// Scatter kernel, then (if a.sky_part) the sky-gradient kernel on the same
// tiles.
template <int N>
hipError_t launch_project_adjoint(const ProjAdjArgs& a, hipStream_t s) {
  const int64_t blocks = (a.n_y + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((project_adjoint_kernel<N>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && a.sky_part) {
    hipLaunchKernelGGL((project_sky_kernel<N>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
    e = hipGetLastError();
  }
  return e;
}

#define LR_INSTANTIATE_ADJOINT(NT)                                                   \
  template hipError_t launch_tdi_adjoint<NT>(const TdiAdjArgs&, int, hipStream_t);   \
  template hipError_t launch_project_adjoint<NT>(const ProjAdjArgs&, hipStream_t);

}  // namespace lr
