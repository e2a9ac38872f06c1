// Batched response kernels for gfx950 (FP64): many templates (sources or
// MCMC walkers) sharing one output time grid, one launch.
//
// fused_forward_kernel<N, GEN, M, BLOCK, WAVE> is persistent: each workgroup
// takes work items (a group of M templates, a tile of output samples) from an
// atomic counter until the list is exhausted.  For one item it
//   1. computes, template by template, the link series of the tile plus the
//      TDI halo directly into LDS (projection, Sec. IV.B) -- the link series
//      never reaches HBM;
//   2. evaluates TDI (Sec. IV.C) for all M templates at once: the delays
//      depend on the orbits only, so each Lagrange coefficient sequence is
//      generated once per sample and applied to the M templates' series;
//   3. stores X/Y/Z and/or A/E/T of each template.
#pragma once

#include "batch_types.hpp"
#include "forward_kernels.hpp"

namespace lr {

// TDI of the lane's two outputs for M templates from their LDS link windows
// (rows of YT link samples).
template <int N, int GEN, int M, int YT>
__device__ __forceinline__ void fused_tdi(const BatchFwdArgs& a, const double* ylds,
                                          const double (&La)[6], const double (&Lb)[6], int c0,
                                          const bool (&live)[M], double (&acc)[M][2][3]) {
  constexpr int H = N / 2;
  constexpr int ND = TdiTab<GEN>::v.ndirect;
  const GroupTable<GEN>& GT = group_table<GEN>();
  // delayed terms accumulate unscaled streams; the undelayed ones are added
  // after the scale, at the end
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[k][s][c] = 0.0;
  // The padding bound keeps every stored output's stencil inside the tile;
  // the clamp only guards the idle lanes past a template's end.
  const int top = YT - 1 - N;
  auto stencil = [&](const GroupRow& G, double& ea, double& eb, bool& same, int& ja, int& jb) {
    const int sa = split_delay(row_delay(G, La), a.inv_dt, ea);
    const int sb = split_delay(row_delay(G, Lb), a.inv_dt, eb);
    same = __all(sa == sb);
    ja = min(max(c0 + sa - (H - 1), 0), top);
    jb = min(max(c0 + 1 + sb - (H - 1), 0), top);
  };
  // rows that feed one channel c (see GroupTable): one FMA per template and
  // sample; a two-link group of one channel interpolates the signed sum of
  // its link series
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll 1
    for (int g = GT.first[c]; g < GT.comb[c]; ++g) {
      const GroupRow& G = GT.row[g];
      double ea, eb;
      bool same;
      int ja, jb;
      stencil(G, ea, eb, same, ja, jb);
      const double* w[M];
#pragma unroll
      for (int k = 0; k < M; ++k) w[k] = ylds + (k * 6 + G.link[0]) * YT;
      double xa[M], xb[M];
      stream_series<N, YT, M>(ea, eb, same, [&w](int s, int i) { return w[s][i]; },
                              ParStream<YT>(ja), jb, xa, xb);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        acc[k][0][c] = fma(G.sign, xa[k], acc[k][0][c]);
        acc[k][1][c] = fma(G.sign, xb[k], acc[k][1][c]);
      }
    }
#pragma unroll 1
    for (int g = GT.comb[c]; g < GT.first[c + 1]; ++g) {
      const GroupRow& G = GT.row[g];
      double ea, eb;
      bool same;
      int ja, jb;
      stencil(G, ea, eb, same, ja, jb);
      const double* w0[M];
      const double* w1[M];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        w0[k] = ylds + (k * 6 + G.link[0]) * YT;
        w1[k] = ylds + (k * 6 + G.link[1]) * YT;
      }
      const double q = G.ratio;
      double xa[M], xb[M];
      stream_series<N, YT, M>(ea, eb, same,
                              [&w0, &w1, q](int s, int i) { return fma(q, w1[s][i], w0[s][i]); },
                              ParStream<YT>(ja), jb, xa, xb);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        acc[k][0][c] = fma(G.sign, xa[k], acc[k][0][c]);
        acc[k][1][c] = fma(G.sign, xb[k], acc[k][1][c]);
      }
    }
  }
  // two-link groups whose uses feed different channels
#pragma unroll 1
  for (int g = GT.first[3]; g < GT.n; ++g) {
    const GroupRow& G = GT.row[g];
    double ea, eb;
    bool same;
    int ja, jb;
    stencil(G, ea, eb, same, ja, jb);
    const double* w[2 * M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      w[2 * k] = ylds + (k * 6 + G.link[0]) * YT;
      w[2 * k + 1] = ylds + (k * 6 + G.link[1]) * YT;
    }
    double xa[2 * M], xb[2 * M];
    stream_multi<N, YT, 2 * M>(ea, eb, same, w, ParStream<YT>(ja), jb, xa, xb);
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[k][0][c] = fma(G.sgn[0][c], xa[2 * k], fma(G.sgn[1][c], xa[2 * k + 1], acc[k][0][c]));
        acc[k][1][c] = fma(G.sgn[0][c], xb[2 * k], fma(G.sgn[1][c], xb[2 * k + 1], acc[k][1][c]));
      }
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double dir[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    static_for<ND>([&](auto t) {
      constexpr Direct dr = TdiTab<GEN>::v.direct[decltype(t)::value];
      const double* w = ylds + (k * 6 + dr.link) * YT;
      dir[0][dr.chan] += (double)dr.sign * w[par<YT>(c0)];
      dir[1][dr.chan] += (double)dr.sign * w[par<YT>(c0 + 1)];
    });
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        acc[k][s][c] = fma(LagrangeStream<N>::kScale, acc[k][s][c], dir[s][c]);
  }
  (void)live;
}

// Minimum resident waves per SIMD for the fused kernel's register budget
// (build-time tuning knobs; 1 leaves the compiler unconstrained).  Measured
// fastest: two for groups of 1 and 4; three for groups of 2 reading h from
// HBM (whose 49 KB of LDS let three work-groups share a CU; 203 against 206
// ms on the 512-template batch although the third wave costs some spills);
// two for groups of 2 in waveform mode (the synthesis needs more registers:
// 114 against 125 ms on 256 one-year walkers).
#ifndef LR_FUSED_MIN_WAVES
#define LR_FUSED_MIN_WAVES 2
#endif
#ifndef LR_FUSED2_MIN_WAVES
#define LR_FUSED2_MIN_WAVES 3
#endif
#ifndef LR_FUSED2W_MIN_WAVES
#define LR_FUSED2W_MIN_WAVES 2
#endif

// WAVE: h+ / hx synthesised from each template's parameter row (Sec. III)
// instead of read from the caller's arrays.  A compile-time choice: with the
// waveform code in the same kernel the array path's registers spill.
template <int N, int GEN, int M, int BLOCK, bool WAVE>
__global__ __launch_bounds__(BLOCK, M == 2 ? (WAVE ? LR_FUSED2W_MIN_WAVES : LR_FUSED2_MIN_WAVES)
                                           : LR_FUSED_MIN_WAVES)
void fused_forward_kernel(BatchFwdArgs a) {
  constexpr int YT = kPerLane * BLOCK;                // new link samples per tile
  constexpr int HPX = fused_halo_cap(M, BLOCK);       // halo a row can carry
  constexpr int YR = YT + HPX;                        // row length
  constexpr int NST = (M * 6 * HPX + BLOCK - 1) / BLOCK;   // halo values per lane (<= 2)
  constexpr int CAPH = YT + N + kSlack;
  // Template k's h window lives in its own link rows until its projection
  // ends (the rows are written only after a barrier), so the window costs no
  // LDS of its own.
  static_assert(CAPH * sizeof(double2) <= 6 * YR * sizeof(double), "h window fits a row block");
  static_assert(NST <= 2, "two halo values per lane");
  __shared__ __align__(16) double ylds[M * 6 * YR];
  __shared__ int red[2][BLOCK / 64];
  __shared__ int s_item;

  for (;;) {
    // an opaque lane index per item: whatever derives from it (LDS offsets,
    // stencil starts) is recomputed here instead of being hoisted out of the
    // persistent loop and kept in scratch
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (tid == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    // uniform values in scalar registers: the item, its group and segment,
    // and (below) the templates' records come through scalar loads
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= a.n_items) break;
    const int grp = __builtin_amdgcn_readfirstlane(a.items[2 * item]);
    const int seg = __builtin_amdgcn_readfirstlane(a.items[2 * item + 1]);
    const int hp = a.HP;                              // 0: one tile per segment
    const int64_t S = (int64_t)seg * (a.T_out + (int64_t)(a.seg_tiles - 1) * YT);
    const int64_t n_long = a.tpl[grp * M].n_out;      // the group's longest template
    // A segment is seg_tiles consecutive tiles.  Row r of a tile holds link
    // sample rb + r (output-index space, rb = first output - F - ro): the
    // tile's YT new link samples go to rows [hp, hp + YT); from the second
    // tile on, rows [0, hp) hold the previous tile's last hp samples (rows
    // [YT, YT + hp) there), so every tile after the first has YT outputs.
    double halo[NST > 0 ? NST : 1];
#pragma unroll 1
    for (int t = 0; t < a.seg_tiles; ++t) {
      const int64_t o0 = t == 0 ? S : S + a.T_out + (int64_t)(t - 1) * YT;
      if (o0 >= n_long) break;                        // uniform
      const int cnt = t == 0 ? a.T_out : YT;          // outputs of this tile
      const int ro = t == 0 ? hp : 0;
      const int64_t i_new = o0 - a.F + (t == 0 ? 0 : hp);   // link sample of row hp

      // 1. link series of each template of the group into LDS (one copy of the
      // projection code, templates in a rolled loop)
      bool live[M];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const BatchTemplate T = a.tpl[grp * M + k];
        live[k] = T.index >= 0 && o0 < T.n_out;
      }
#pragma unroll 1
      for (int k = 0; k < M; ++k) {
        const BatchTemplate T = a.tpl[grp * M + k];
        if (!(T.index >= 0 && o0 < T.n_out)) continue;  // uniform
        const int64_t n_valid = min((int64_t)cnt, T.n_out - o0);
        // new rows up to the last valid output's stencil (the padding B
        // rounded to the even halo YT - T_out)
        const int r_end =
            (int)min((int64_t)YT, n_valid + (YT - a.T_out) - (t == 0 ? 0 : hp));
        const int last = r_end - 1;
        const bool act_a = 2 * tid <= last, act_b = 2 * tid + 1 <= last;
        const int ra = act_a ? 2 * tid : (last & ~1);
        // sin, cos of the sky angles, tabulated per template before the launch
        // (no trigonometry, and none of its constants, in this loop)
        const double* tr = a.trig + 4 * T.index;
        const Sky sk = sky_from_trig(tr[0], tr[1], tr[2], tr[3]);
        double ya[6], yb[6];
        double2* hwin = reinterpret_cast<double2*>(ylds + k * 6 * YR);
        // h+ / hx: the caller's arrays, or the waveform synthesised into the
        // window from the template's parameter row (waveform time 0 at output
        // sample 0)
        HSource hs;
        if constexpr (WAVE)
          hs = HSource::waveform(a.params + 8 * T.index, -T.out_start, a.dt, T.n_h);
        else
          hs = HSource::arrays(a.hp + T.h_off, a.hc + T.h_off, T.n_h);
        project_pair<N, BLOCK>(a.orb_p, a.t_off_p, i_new, a.dt, a.inv_dt, hs,
                               T.out_start + i_new, sk, ra, hwin, red, ya, yb);
        __syncthreads();                              // the window is read; rows may be written
#pragma unroll
        for (int l = 0; l < 6; ++l) {
          double* row = ylds + (k * 6 + l) * YR;
          if (act_a) row[par<YR>(hp + ra)] = ya[l];
          if (act_b) row[par<YR>(hp + ra + 1)] = yb[l];
        }
        if (t > 0) {
          // the carried halo of this template back into its rows
#pragma unroll
          for (int q = 0; q < NST; ++q) {
            const int e = tid + BLOCK * q, rho = e / max(HPX, 1), j = e - rho * HPX;
            if (rho / 6 == k && rho < M * 6 && j < hp) ylds[rho * YR + par<YR>(j)] = halo[q];
          }
        }
      }
      __syncthreads();

      // 2. TDI of the tile's outputs for all live templates
      const int oa = 2 * tid;                         // tile-relative output of sample a
      const bool out_a = oa < cnt;
      const int ob = out_a ? oa : cnt - 2;            // idle lanes mirror the last pair
      double La[6], Lb[6];
      light_times(a.orb_t, a.t_off_t + (double)(o0 + ob) * a.dt, La);
      light_times(a.orb_t, a.t_off_t + (double)(o0 + ob + 1) * a.dt, Lb);
      double acc[M][2][3];
      fused_tdi<N, GEN, M, YR>(a, ylds, La, Lb, a.F + ro + ob, live, acc);

      // 3. store (the template records read again rather than kept live
      // through the TDI: an opaque copy of the group index stops the compiler
      // from reusing the first loads)
      int grp_s = grp;
      asm volatile("" : "+s"(grp_s));
      if (out_a) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
          if (!live[k]) continue;
          const BatchTemplate T = a.tpl[grp_s * M + k];
          const int64_t i = o0 + oa;
          if (i < T.n_out) store_channels(acc[k][0], a.channels, a.out + T.out_off, T.n_out, i);
          if (i + 1 < T.n_out)
            store_channels(acc[k][1], a.channels, a.out + T.out_off, T.n_out, i + 1);
        }
      }
      if (t + 1 < a.seg_tiles) {
        // the next tile's halo: this tile's rows [YT, YT + hp), read before
        // the next tile's projection windows overwrite them
#pragma unroll
        for (int q = 0; q < NST; ++q) {
          const int e = tid + BLOCK * q, rho = e / max(HPX, 1), j = e - rho * HPX;
          if (rho < M * 6 && j < hp) halo[q] = ylds[rho * YR + par<YR>(YT + j)];
        }
      }
      __syncthreads();                                // LDS free for the next tile
    }
  }
}

template <int N, int GEN, int M, int BLOCK, bool WAVE>
hipError_t launch_fused_forward(const BatchFwdArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((fused_forward_kernel<N, GEN, M, BLOCK, WAVE>), dim3(blocks), dim3(BLOCK),
                     0, s, a);
  return hipGetLastError();
}

// Resident workgroups per CU of the fused kernel (sizes the persistent grid).
template <int N, int GEN, int M, int BLOCK, bool WAVE>
int fused_occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, fused_forward_kernel<N, GEN, M, BLOCK, WAVE>, BLOCK, 0) != hipSuccess)
    nb = 1;
  return nb > 0 ? nb : 1;
}

#define LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, M, BLOCK, WAVE)                              \
  template hipError_t launch_fused_forward<NT, GEN, M, BLOCK, WAVE>(const BatchFwdArgs&, int, \
                                                                    hipStream_t);             \
  template int fused_occupancy<NT, GEN, M, BLOCK, WAVE>();

// Work items of 256, 512 or 1024 link samples (workgroups of 128, 256 or 512
// lanes); groups of 4 at 1024 would need 196 KB of LDS and are left out.
// Waveform mode: groups of 1 and 2 at 512 link samples and of 2 at 1024 (the
// fastest array-mode shapes), which keeps the build time in bounds.
#define LR_INSTANTIATE_BATCH_FWD(NT, GEN)                                                   \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 1, 128, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 1, 256, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 1, 512, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 2, 128, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 2, 256, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 2, 512, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 4, 128, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 4, 256, false)                                        \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 1, 256, true)                                         \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 2, 256, true)                                         \
  LR_INSTANTIATE_BATCH_FWD_M(NT, GEN, 2, 512, true)

}  // namespace lr
