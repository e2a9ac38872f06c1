// Adjoint (transpose) kernels of the response for gfx950 (FP64).
//
//   tdi_adjoint_kernel      g_out -> g_y: every delayed term's interpolation
//                           transposed into a scatter of w_m * g onto the
//                           stencil taps (Sec. IV.C terms, Sec. IV.E weights)
//   project_adjoint_kernel  g_y -> g_h+, g_hx
//   project_sky_kernel      g_y, h+, hx -> partial gradients with respect to
//                           the ecliptic sky angles lam, beta
//
// Scatter strategy (carry kernels, the default): a workgroup owns 512
// consecutive sources, each wave 128 of them.  Per delay set a wave sums its
// sources' scatters in a register carry (carry.hpp), in a fixed order, and
// adds the result to its own LDS rows; at the end of the tile the four
// waves' rows are summed in wave order and added to the zero-filled global
// gradient with one FP64 atomic per entry.  Neighbouring tiles' footprints
// overlap by about one stencil and never three deep, so every global entry
// receives at most two additions onto zero, and IEEE addition being
// commutative, the result is bitwise reproducible.
//
// When a wave's footprint does not fit the LDS rows (sampling intervals far
// below the light times, or orbits whose positions do not match their light
// times) the atomic kernels take over: LDS atomics inside the tile, then the
// same global additions; their sums depend on the order in which lanes
// arrive, so those results are reproducible to rounding only.
#pragma once

#include "carry.hpp"
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

// Minimum resident waves per SIMD of the carry kernels (register budget;
// build-time tuning knobs).
#ifndef LR_TDI_CARRY_MIN_WAVES
#define LR_TDI_CARRY_MIN_WAVES 2
#endif
#ifndef LR_PADJ_CARRY_MIN_WAVES
#define LR_PADJ_CARRY_MIN_WAVES 2
#endif

// One template per tile: keep the rescaled factors of the suffix pass for
// the prefix pass in the one-channel rows (N more registers, two operations
// less per tap; one year 0.98 -> 0.93 ms); build-time switch for
// measurements.
#ifndef LR_TDI_CARRY_KEEP_NU
#define LR_TDI_CARRY_KEEP_NU 1
#endif

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
// TDI adjoint, carry form
// ---------------------------------------------------------------------------
constexpr int kCarryTile = 4 * kCarrySlots;   // sources per workgroup (4 waves)

struct CarryShared {
  int lo[kBlock / 64];    // per wave: relative index of its row element 0
  int rl[kBlock / 64];    // per wave: row length in use (0: wave took the global path)
  double gb[7][kBlock / 64];   // waveform mode: per-wave parameter-gradient sums
};

// Doubles of dynamic LDS of a carry tile: per wave R rows of rl_cap plus
// NP parked sums per carry of N - 1.
__host__ __device__ constexpr size_t carry_lds_doubles(int rows, int rl_cap, int ncarry, int N) {
  return (size_t)(kBlock / 64) * ((size_t)rows * rl_cap + (size_t)ncarry * (N - 1));
}

// Sum of the waves' rows in wave order for the tile's footprint, added to
// the global rows.  Row r of wave w starts at relative index
// kCarrySlots * w + lo[w]; global index = gbase + relative index, valid in
// [0, n).  `dst(r, n)` gives global row r and sets its length n (null: skip).
template <int NROWS, class Dst>
__device__ __forceinline__ void carry_fold(const double* lds, int rl_cap, const CarryShared& cs,
                                           int64_t gbase, const Dst& dst) {
  constexpr int nrows = NROWS;
  constexpr int W = kBlock / 64;
  const int half = rl_cap / 2;
  int lo_min = 1 << 30, hi_max = -(1 << 30);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    if (cs.rl[w] == 0) continue;
    lo_min = min(lo_min, kCarrySlots * w + cs.lo[w]);
    hi_max = max(hi_max, kCarrySlots * w + cs.lo[w] + cs.rl[w] - 1);
  }
  if (hi_max < lo_min) return;
#pragma unroll
  for (int r = 0; r < nrows; ++r) {
    int64_t n = 0;
    double* g = dst(r, n);
    if (!g) continue;                                  // uniform
    for (int e = lo_min + (int)threadIdx.x; e <= hi_max; e += kBlock) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int idx = e - kCarrySlots * w - cs.lo[w];
        if (idx >= 0 && idx < cs.rl[w])
          s += lds[((size_t)w * nrows + r) * rl_cap + psplit(idx, half)];
      }
      const int64_t j = gbase + e;
      if (j >= 0 && j < n) atomicAdd(g + j, s);
    }
  }
}

// The tile's footprint as values instead of global additions: for every
// relative index with global index j = gbase + e in [0, n), fn(j, v) gets
// the NROWS row sums (waves summed in wave order).  Each lane visits its own
// subset of entries.
template <int NROWS, class Fn>
__device__ __forceinline__ void carry_fold_values(const double* lds, int rl_cap,
                                                  const CarryShared& cs, int64_t gbase, int64_t n,
                                                  const Fn& fn) {
  constexpr int W = kBlock / 64;
  const int half = rl_cap / 2;
  int lo_min = 1 << 30, hi_max = -(1 << 30);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    if (cs.rl[w] == 0) continue;
    lo_min = min(lo_min, kCarrySlots * w + cs.lo[w]);
    hi_max = max(hi_max, kCarrySlots * w + cs.lo[w] + cs.rl[w] - 1);
  }
  for (int e = lo_min + (int)threadIdx.x; e <= hi_max; e += kBlock) {
    const int64_t j = gbase + e;
    if (j < 0 || j >= n) continue;
    double v[NROWS];
#pragma unroll
    for (int r = 0; r < NROWS; ++r) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int idx = e - kCarrySlots * w - cs.lo[w];
        if (idx >= 0 && idx < cs.rl[w])
          s += lds[((size_t)w * NROWS + r) * rl_cap + psplit(idx, half)];
      }
      v[r] = s;
    }
    fn(j, v);
  }
}

// One 512-source tile of the TDI adjoint for M templates sharing the output
// grid and TDI orbits (a[0] the longest; see tdi_adjoint_tile).  lds:
// carry_lds_doubles(M * 6, rl_cap, 2 * M, N) doubles.
template <int N, int GEN, int M>
__device__ __forceinline__ void tdi_adjoint_carry_tile(const TdiAdjArgs (&a)[M],
                                                       const bool (&live)[M], int64_t tile,
                                                       double* lds, int rl_cap, CarryShared& cs) {
  constexpr int H = N / 2;
  constexpr int ND = TdiTab<GEN>::v.ndirect;
  constexpr int NR = M * 6;
  const GroupTable<GEN>& GT = group_table<GEN>();
  const TdiAdjArgs& a0 = a[0];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool lane0 = lane == 0;
  const int half = rl_cap / 2;
  double* rows = lds + (size_t)w * NR * rl_cap;
  double* park = lds + (size_t)(kBlock / 64) * NR * rl_cap + (size_t)w * 2 * M * (N - 1);

  const int64_t i0 = tile * kCarryTile;
  const int64_t ia = i0 + kCarrySlots * w + 2 * lane;     // output index of slot a (b: +1)
  const int64_t last = a0.n_out - 1;
  const int64_t pa = a0.out_start + min(ia, last), pb = a0.out_start + min(ia + 1, last);
  double La[6], Lb[6];
  light_times(a0.orb, a0.t_off + (double)pa * a0.dt, La);
  light_times(a0.orb, a0.t_off + (double)pb * a0.dt, Lb);

  // relative row range of the wave: direct terms at 0..127, delayed terms'
  // carries at [c, c + N + 126] for every shift c = sh - (H - 1)
  double dlo, dhi, dlo_b, dhi_b, e_unused;
  group_delay_bounds(La, GT.chain, dlo, dhi);
  group_delay_bounds(Lb, GT.chain, dlo_b, dhi_b);
  const int c_lo = min(split_delay(dhi, a0.inv_dt, e_unused),
                       split_delay(dhi_b, a0.inv_dt, e_unused)) - (H - 1);
  const int c_hi = max(split_delay(dlo, a0.inv_dt, e_unused),
                       split_delay(dlo_b, a0.inv_dt, e_unused)) - (H - 1);
  const int lo = __builtin_amdgcn_readfirstlane(min(0, wave_min(c_lo)));
  const int hi = __builtin_amdgcn_readfirstlane(max(kCarrySlots - 1, wave_max(c_hi) + N + kCarrySlots - 2));
  const bool fits = hi - lo + 1 <= rl_cap;

  double g[M][2][3];
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      g[k][s][0] = g[k][s][1] = g[k][s][2] = 0.0;
      if (live[k] && ia + s < a[k].n_out)
        load_channel_grads(a[k].g_out, a[k].channels, a[k].n_out, ia + s, g[k][s]);
    }

  if (fits) {
    for (int j = lane; j < NR * rl_cap; j += 64) rows[j] = 0.0;
    // undelayed terms: the lane's own samples
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const Direct dr = TdiTab<GEN>::v.direct[t];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        double* row = rows + (k * 6 + dr.link) * rl_cap;
        row[psplit(2 * lane - lo, half)] += (double)dr.sign * g[k][0][dr.chan];
        row[psplit(2 * lane + 1 - lo, half)] += (double)dr.sign * g[k][1][dr.chan];
      }
    }
    // delayed terms: the streams' common scale goes into the values
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) g[k][s][c] *= LagrangeStream<N>::kScale;

    // one carry per template per shift value present in the wave (almost
    // always one); values of slots with another shift are masked to zero
    // rows that feed one channel: one use, or two uses of one channel whose
    // second link receives the same carry times the sign ratio
#pragma unroll 1
    for (int gi = 0; gi < GT.first[3]; ++gi) {
      const GroupRow& G = GT.row[gi];
      double ea, eb;
      const int sa = split_delay(row_delay(G, La), a0.inv_dt, ea);
      const int sb = split_delay(row_delay(G, Lb), a0.inv_dt, eb);
      int s_lo, s_hi;
      shift_range(sa, sb, s_lo, s_hi);
      const bool two = G.nuse == 2;                   // uniform
      for (int sg = s_lo; sg <= s_hi; ++sg) {
        double va[M], vb[M], A[M], B[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const double xa = G.sgn[0][0] * g[k][0][0] + G.sgn[0][1] * g[k][0][1] +
                            G.sgn[0][2] * g[k][0][2];
          const double xb = G.sgn[0][0] * g[k][1][0] + G.sgn[0][1] * g[k][1][1] +
                            G.sgn[0][2] * g[k][1][2];
          va[k] = sa == sg ? xa : 0.0;
          vb[k] = sb == sg ? xb : 0.0;
        }
        carry_scatter<N, M, M == 1 && LR_TDI_CARRY_KEEP_NU>(ea, eb, va, vb, A, B, park, lane0);
        const int o = sg - (H - 1) - lo;
#pragma unroll
        for (int k = 0; k < M; ++k) {
          carry_add<N>(rows + (k * 6 + G.link[0]) * rl_cap, half, o, lane, 1.0, A[k], B[k],
                       park + k * (N - 1));
          if (two)
            carry_add<N>(rows + (k * 6 + G.link[1]) * rl_cap, half, o, lane, G.ratio, A[k],
                         B[k], park + k * (N - 1));
        }
      }
    }
    // two-link groups whose uses feed different channels
#pragma unroll 1
    for (int gi = GT.first[3]; gi < GT.n; ++gi) {
      const GroupRow& G = GT.row[gi];
      double ea, eb;
      const int sa = split_delay(row_delay(G, La), a0.inv_dt, ea);
      const int sb = split_delay(row_delay(G, Lb), a0.inv_dt, eb);
      int s_lo, s_hi;
      shift_range(sa, sb, s_lo, s_hi);
      for (int sg = s_lo; sg <= s_hi; ++sg) {
        double va[2 * M], vb[2 * M], A[2 * M], B[2 * M];
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const double xa = G.sgn[u][0] * g[k][0][0] + G.sgn[u][1] * g[k][0][1] +
                              G.sgn[u][2] * g[k][0][2];
            const double xb = G.sgn[u][0] * g[k][1][0] + G.sgn[u][1] * g[k][1][1] +
                              G.sgn[u][2] * g[k][1][2];
            va[2 * k + u] = sa == sg ? xa : 0.0;
            vb[2 * k + u] = sb == sg ? xb : 0.0;
          }
        carry_scatter<N, 2 * M, false>(ea, eb, va, vb, A, B, park, lane0);
        const int o = sg - (H - 1) - lo;
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
          for (int u = 0; u < 2; ++u)
            carry_add<N>(rows + (k * 6 + G.link[u]) * rl_cap, half, o, lane, 1.0, A[2 * k + u],
                         B[2 * k + u], park + (2 * k + u) * (N - 1));
      }
    }
  } else {
    // footprint wider than the rows: scatter straight to global memory
    auto scatter = [&](const TdiAdjArgs& ak, int64_t i, const double (&L)[6],
                       const double (&gs)[3]) {
      if (i >= ak.n_out) return;
      const int64_t p = ak.out_start + i;
#pragma unroll
      for (int t = 0; t < ND; ++t) {
        const Direct dr = TdiTab<GEN>::v.direct[t];
        atomicAdd(ak.g_y + (int64_t)dr.link * ak.n_y + p, (double)dr.sign * gs[dr.chan]);
      }
#pragma unroll 1
      for (int gi = 0; gi < GT.n; ++gi) {
        const GroupRow& G = GT.row[gi];
        double eps;
        const int sh = split_delay(row_delay(G, L), ak.inv_dt, eps);
#pragma unroll 1
        for (int u = 0; u < G.nuse; ++u) {
          const double v = G.sgn[u][0] * gs[0] + G.sgn[u][1] * gs[1] + G.sgn[u][2] * gs[2];
          scatter_global<N>(ak.g_y + (int64_t)G.link[u] * ak.n_y, p + sh - (H - 1), ak.n_y, eps,
                            v);
        }
      }
    };
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (!live[k]) continue;
      scatter(a[k], ia, La, g[k][0]);
      scatter(a[k], ia + 1, Lb, g[k][1]);
    }
  }
  if (lane0) {
    cs.lo[w] = lo;
    cs.rl[w] = fits ? hi - lo + 1 : 0;
  }
  __syncthreads();
  carry_fold<NR>(lds, rl_cap, cs, a0.out_start + i0, [&](int r, int64_t& n) -> double* {
    const int k = r / 6, l = r % 6;
#pragma unroll
    for (int kk = 0; kk < M; ++kk)
      if (kk == k && live[kk]) {
        n = a[kk].n_y;
        return a[kk].g_y + (int64_t)l * a[kk].n_y;
      }
    return nullptr;
  });
}

template <int N, int GEN>
__global__ __launch_bounds__(kBlock, LR_TDI_CARRY_MIN_WAVES) void tdi_adjoint_carry_kernel(TdiAdjArgs a) {
  extern __shared__ double lds_dyn[];
  __shared__ CarryShared cs;
  const TdiAdjArgs x[1] = {a};
  const bool live[1] = {true};
  tdi_adjoint_carry_tile<N, GEN, 1>(x, live, blockIdx.x, lds_dyn, a.rl_cap, cs);
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
  const HSource hs = a.params ? HSource::waveform(a.params, a.k0, a.dt, a.n_h)
                              : HSource::arrays(a.hp, a.hc, a.n_h);
  if (count > 0 && count <= CAP) {
    for (int k = tid; k < count; k += kBlock) {
      int64_t j = base + k;
      j = j < 0 ? 0 : (j > hmax ? hmax : j);
      win[k] = hs.at(j);
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
        const double2 hj = hs.at(j);
        st.step(c, cd, hj.x, sp, dsp);
        st.step(c, cd, hj.y, sc, dsc);
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

// ---------------------------------------------------------------------------
// Projection adjoint, carry form
// ---------------------------------------------------------------------------
// What the nine positions of one link sample need: light times, k.x_s / c,
// antenna patterns and the upstream gradient scaled by 1/(2(1 - k.n)).
// Field f is v[f]; a lane's second slot keeps its copy in LDS ([field][lane]
// rows of the wave), which leaves the registers to the carry.
constexpr int kPcKx = 0, kPcL = 3, kPcXip = 9, kPcXic = 12, kPcCl = 15, kPcFields = 21;

struct ProjCarryRegs {
  double v[kPcFields];
  __device__ __forceinline__ double operator()(int f) const { return v[f]; }
};
struct ProjCarryLds {
  const double* p;   // field 0 of the lane; fields 64 doubles apart
  __device__ __forceinline__ double operator()(int f) const { return p[f * 64]; }
};

__device__ __forceinline__ void proj_carry_slot(const ProjAdjArgs& a, const Sky& sk, int64_t i,
                                                double (&v)[kPcFields]) {
  const int64_t last = a.n_y - 1;
  const int64_t q = a.y_start + min(i, last);
  LinkGeom g;
  link_geometry(a.orb, a.t_off + (double)q * a.dt, sk, g);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[kPcKx + k] = g.kx[k];
    v[kPcXip + k] = g.xip[k];
    v[kPcXic + k] = g.xic[k];
  }
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    v[kPcL + l] = g.L[l];
    const double gy = i <= last ? a.g_y[(int64_t)l * a.n_y + i] : 0.0;
    v[kPcCl + l] = gy / (2.0 * (1.0 - kDir[l] * g.kn[kArm[l]]));
  }
}

// Delay of position P and the amplitudes it scatters onto h+ and hx
// (receptions 0..2 subtract the links received there, emissions 3..8 add).
template <int P, class Slot>
__device__ __forceinline__ double proj_carry_pos(const Slot& s, double& ap, double& ac) {
  if constexpr (P >= 3) {
    constexpr int l = P - 3, arm = kArm[l];
    const double cl = s(kPcCl + l);
    ap = cl * s(kPcXip + arm);
    ac = cl * s(kPcXic + arm);
    return s(kPcL + l) + s(kPcKx + kLinkEmit[l] - 1);
  } else {
    ap = 0.0;
    ac = 0.0;
#pragma unroll
    for (int l = 0; l < 6; ++l)
      if (kLinkRecv[l] - 1 == P) {
        const double cl = s(kPcCl + l);
        ap -= cl * s(kPcXip + kArm[l]);
        ac -= cl * s(kPcXic + kArm[l]);
      }
    return s(kPcKx + P);
  }
}

template <int N, int P>
__device__ __forceinline__ void proj_carry_position(const ProjAdjArgs& a, const ProjCarryRegs& sa,
                                                    const ProjCarryLds& sb, int lo, int lane,
                                                    bool lane0, double* rows, int rl_cap,
                                                    double* park) {
  constexpr int H = N / 2;
  const int half = rl_cap / 2;
  double va[2], vb[2], ea, eb;
  const int sha = split_delay(proj_carry_pos<P>(sa, va[0], va[1]), a.inv_dt, ea);
  const int shb = split_delay(proj_carry_pos<P>(sb, vb[0], vb[1]), a.inv_dt, eb);
  int s_lo, s_hi;
  shift_range(sha, shb, s_lo, s_hi);
  // the streams' common scale goes into the values
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    va[c] *= LagrangeStream<N>::kScale;
    vb[c] *= LagrangeStream<N>::kScale;
  }
  for (int sg = s_lo; sg <= s_hi; ++sg) {
    double xa[2], xb[2], A[2], B[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      xa[c] = sha == sg ? va[c] : 0.0;
      xb[c] = shb == sg ? vb[c] : 0.0;
    }
    carry_scatter<N, 2, false>(ea, eb, xa, xb, A, B, park, lane0);
    const int o = sg - (H - 1) - lo;
    carry_add<N>(rows, half, o, lane, 1.0, A[0], B[0], park);
    carry_add<N>(rows + rl_cap, half, o, lane, 1.0, A[1], B[1], park + (N - 1));
  }
}

// One 512-link-sample tile of the projection adjoint (g_y -> g_h+, g_hx).
// lds: proj_carry_lds_doubles(rl_cap, N) doubles.
__host__ __device__ constexpr size_t proj_carry_lds_doubles(int rl_cap, int N) {
  return carry_lds_doubles(2, rl_cap, 2, N) + (size_t)(kBlock / 64) * kPcFields * 64;
}

template <int N>
__device__ __forceinline__ void project_adjoint_carry_tile(const ProjAdjArgs& a, int64_t tile,
                                                           double* lds, int rl_cap,
                                                           CarryShared& cs,
                                                           double (&s_trig)[2][2]) {
  constexpr int H = N / 2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool lane0 = lane == 0;
  double* rows = lds + (size_t)w * 2 * rl_cap;
  double* park = lds + (size_t)(kBlock / 64) * 2 * rl_cap + (size_t)w * 2 * (N - 1);

  const SkyTrig tr = load_sky(a.sky, s_trig);
  const Sky sk = sky_from_trig(tr.sl, tr.cl, tr.sb, tr.cb);
  const int64_t i0 = tile * kCarryTile;
  const int64_t ia = i0 + kCarrySlots * w + 2 * lane;
  ProjCarryRegs sa;
  proj_carry_slot(a, sk, ia, sa.v);
  double* sb_lds = lds + carry_lds_doubles(2, rl_cap, 2, N) + (size_t)w * kPcFields * 64 + lane;
  {
    double v[kPcFields];
    proj_carry_slot(a, sk, ia + 1, v);
#pragma unroll
    for (int f = 0; f < kPcFields; ++f) sb_lds[f * 64] = v[f];
  }
  const ProjCarryLds sb{sb_lds};

  // relative row range: every position's carry covers [c, c + N + 126]
  int c_lo = 1 << 30, c_hi = -(1 << 30);
  {
    double e_unused, u0, u1;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const int x = split_delay(sa(kPcKx + p), a.inv_dt, e_unused);
      const int y = split_delay(sb(kPcKx + p), a.inv_dt, e_unused);
      c_lo = min(c_lo, min(x, y));
      c_hi = max(c_hi, max(x, y));
    }
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const int e = kPcKx + kLinkEmit[l] - 1;
      const int x = split_delay(sa(kPcL + l) + sa(e), a.inv_dt, e_unused);
      const int y = split_delay(sb(kPcL + l) + sb(e), a.inv_dt, e_unused);
      c_lo = min(c_lo, min(x, y));
      c_hi = max(c_hi, max(x, y));
    }
    (void)u0; (void)u1;
  }
  const int lo = __builtin_amdgcn_readfirstlane(wave_min(c_lo) - (H - 1));
  const int hi = __builtin_amdgcn_readfirstlane(wave_max(c_hi) - (H - 1) + N + kCarrySlots - 2);
  const bool fits = hi - lo + 1 <= rl_cap;

  if (fits) {
    for (int j = lane; j < 2 * rl_cap; j += 64) rows[j] = 0.0;
#define LR_PCARRY(P)                                                                          \
    proj_carry_position<N, P>(a, sa, sb, lo, lane, lane0, rows, rl_cap, park);               \
    __builtin_amdgcn_sched_barrier(0);
    LR_PCARRY(0) LR_PCARRY(1) LR_PCARRY(2) LR_PCARRY(3) LR_PCARRY(4) LR_PCARRY(5)
    LR_PCARRY(6) LR_PCARRY(7) LR_PCARRY(8)
#undef LR_PCARRY
  } else if (!a.params) {
    // footprint wider than the rows: scatter straight to global memory
    auto scatter = [&](const auto& S, int64_t i) {
      if (i >= a.n_y) return;
      const int64_t q = a.y_start + i;
#define LR_PGLOBAL(P)                                                                         \
      {                                                                                       \
        double ap, ac, eps;                                                                   \
        const int sh = split_delay(proj_carry_pos<P>(S, ap, ac), a.inv_dt, eps);              \
        scatter_global<N>(a.g_hp, q + sh - (H - 1), a.n_h, eps, ap);                          \
        scatter_global<N>(a.g_hc, q + sh - (H - 1), a.n_h, eps, ac);                          \
      }
      LR_PGLOBAL(0) LR_PGLOBAL(1) LR_PGLOBAL(2) LR_PGLOBAL(3) LR_PGLOBAL(4) LR_PGLOBAL(5)
      LR_PGLOBAL(6) LR_PGLOBAL(7) LR_PGLOBAL(8)
#undef LR_PGLOBAL
    };
    scatter(sa, ia);
    scatter(sb, ia + 1);
  }
  if (lane0) {
    cs.lo[w] = lo;
    cs.rl[w] = fits ? hi - lo + 1 : 0;
  }
  __syncthreads();
  if (!a.params) {
    carry_fold<2>(lds, rl_cap, cs, a.y_start + i0, [&](int r, int64_t& n) -> double* {
      n = a.n_h;
      return r == 0 ? a.g_hp : a.g_hc;
    });
    return;
  }
  // Waveform mode: the tile's share of g_h+, g_hx goes straight into the
  // seven parameter-gradient sums (linear in g_h, so tile shares add up),
  // summed per lane, then over the workgroup in a fixed order.
  const gb::Source src = gb::load_source(a.params);
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (!fits) {
    // a wave whose footprint exceeds its rows: every tap on its own
    auto scatter = [&](const auto& S, int64_t i) {
      if (i >= a.n_y) return;
      const int64_t q = a.y_start + i;
#define LR_PGB(P)                                                                             \
      {                                                                                       \
        double ap, ac, eps;                                                                   \
        const int sh = split_delay(proj_carry_pos<P>(S, ap, ac), a.inv_dt, eps);              \
        const int64_t j0 = q + sh - (H - 1);                                                  \
        for (int m = 0; m < N; ++m) {                                                         \
          const int64_t j = j0 + m;                                                           \
          if (j < 0 || j >= a.n_h) continue;                                                  \
          const double wm = lagrange_weight_at<N>(eps, m);                                    \
          gb::adjoint_sums(src, (double)(a.k0 + j) * a.dt, wm * ap, wm * ac, acc);            \
        }                                                                                     \
      }
      LR_PGB(0) LR_PGB(1) LR_PGB(2) LR_PGB(3) LR_PGB(4) LR_PGB(5) LR_PGB(6) LR_PGB(7) LR_PGB(8)
#undef LR_PGB
    };
    scatter(sa, ia);
    scatter(sb, ia + 1);
  }
  carry_fold_values<2>(lds, rl_cap, cs, a.y_start + i0, a.n_h, [&](int64_t j, const double (&v)[2]) {
    gb::adjoint_sums(src, (double)(a.k0 + j) * a.dt, v[0], v[1], acc);
  });
  // fixed-order reduction: shuffle tree in each wave, then the waves in order
#pragma unroll
  for (int k = 0; k < 7; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_down(acc[k], off);
  }
  if (lane0) {
#pragma unroll
    for (int k = 0; k < 7; ++k) cs.gb[k][w] = acc[k];
  }
  __syncthreads();
  if (tid < 7) {
    double v = cs.gb[tid][0];
#pragma unroll
    for (int ww = 1; ww < kBlock / 64; ++ww) v += cs.gb[tid][ww];
    a.gb_part[tid] = v;
  }
}

template <int N>
__global__ __launch_bounds__(kBlock, LR_PADJ_CARRY_MIN_WAVES) void project_adjoint_carry_kernel(ProjAdjArgs a) {
  extern __shared__ double lds_dyn[];
  __shared__ CarryShared cs;
  __shared__ double s_trig[2][2];
  project_adjoint_carry_tile<N>(a, blockIdx.x, lds_dyn, a.rl_cap, cs, s_trig);
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

// Allow a kernel more than the default 64 KB of dynamic LDS (a per-function
// attribute; set before every such launch, which costs a host call only).
template <class K>
hipError_t allow_dynamic_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int N>
hipError_t launch_tdi_adjoint(const TdiAdjArgs& a, int gen, hipStream_t s) {
  if (a.rl_cap > 0) {
    const int64_t blocks = (a.n_out + kCarryTile - 1) / kCarryTile;
    const size_t bytes = carry_lds_doubles(6, a.rl_cap, 2, N) * sizeof(double);
    if (gen == 1) {
      hipError_t e = allow_dynamic_lds(tdi_adjoint_carry_kernel<N, 1>, bytes);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((tdi_adjoint_carry_kernel<N, 1>), dim3((unsigned)blocks), dim3(kBlock),
                         bytes, s, a);
    } else {
      hipError_t e = allow_dynamic_lds(tdi_adjoint_carry_kernel<N, 2>, bytes);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((tdi_adjoint_carry_kernel<N, 2>), dim3((unsigned)blocks), dim3(kBlock),
                         bytes, s, a);
    }
    return hipGetLastError();
  }
  const int64_t blocks = (a.n_out + kBlock - 1) / kBlock;
  if (gen == 1)
    hipLaunchKernelGGL((tdi_adjoint_kernel<N, 1>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((tdi_adjoint_kernel<N, 2>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Scatter kernel, then (if a.sky_part) the sky-gradient kernel on tiles of
// kBlock link samples.
template <int N>
hipError_t launch_project_adjoint(const ProjAdjArgs& a, hipStream_t s) {
  const int64_t blocks = (a.n_y + kBlock - 1) / kBlock;
  hipError_t e;
  if (a.rl_cap > 0) {
    const size_t bytes = proj_carry_lds_doubles(a.rl_cap, N) * sizeof(double);
    e = allow_dynamic_lds(project_adjoint_carry_kernel<N>, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((project_adjoint_carry_kernel<N>),
                       dim3((unsigned)((a.n_y + kCarryTile - 1) / kCarryTile)), dim3(kBlock),
                       bytes, s, a);
  } else {
    hipLaunchKernelGGL((project_adjoint_kernel<N>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  }
  e = hipGetLastError();
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
