// Deterministic transposed Lagrange interpolation for gfx950 (FP64).
//
// The adjoint of an interpolation y(p) = sum_k w_k(eps_p) f[p + c_p + k]
// (Sec. IV.E weights, taps k = 0..N-1) scatters w_k(eps_p) g_p onto
// f[p + c_p + k].  Instead of one LDS atomic per tap, a wave sums the
// scatters of its 128 consecutive sources (two per lane) in a register carry:
// a shift register over the wave's 128 slots that moves one slot towards
// slot 0 per tap, the cross-lane step being one DPP wave_shl:1 per 32-bit
// half.  After tap k, slot s holds the partial sum of the target
// p_0 + c + s + k, so after the last tap slot s holds the target
// p_0 + c + N - 1 + s complete with respect to the wave's sources; the
// N - 1 partial sums that leave slot 0 on the way (targets p_0 + c + 0 ..
// p_0 + c + N - 2) are parked in LDS by lane 0.  Every sum is formed in a
// fixed order, so the result does not depend on scheduling.
//
// Weights: with nu_m = s_m (eps - x_m) (the rescaled factors of
// LagrangeScaled), w_k = kScale * prod_{m<k} nu_m * prod_{m>k} nu_m.  The
// suffix products are built first (N registers per slot), the prefix
// product runs with the carry.  The second slot of a lane derives its
// factors from the first by one FMA, nu_b = nu_a + s_m (eps_b - eps_a).
#pragma once

#include "device_common.hpp"

namespace lr {

constexpr int kCarrySlots = 128;   // sources per wave (two per lane)

// Lane L receives lane L+1's value; lane 63 receives 0 (DPP wave_shl:1 with
// bound_ctrl, on both 32-bit halves).
__device__ __forceinline__ double lane_down(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Wave-uniform range [lo, hi] of the integer shifts of a wave's slots: one
// ballot when they all agree (all but a few waves), else wave reductions.
__device__ __forceinline__ void shift_range(int sa, int sb, int& lo, int& hi) {
  const int s0 = __builtin_amdgcn_readfirstlane(sa);
  if (__all(sa == s0 && sb == s0)) {
    lo = hi = s0;
    return;
  }
  lo = __builtin_amdgcn_readfirstlane(wave_min(min(sa, sb)));
  hi = __builtin_amdgcn_readfirstlane(wave_max(max(sa, sb)));
}

// Parity-split position of element j in a row of (even) capacity cap: even
// elements first, then odd ones.  Lanes that touch elements o + 2L and
// o + 2L + 1 then read consecutive doubles in each half (no bank conflicts).
__device__ __forceinline__ int psplit(int j, int half) { return (j & 1) * half + (j >> 1); }

// NC carries over one delay set: carry c of slot a scatters va[c] * w_k(ea).
// With NC == 1 the value is folded into the suffix products.  On return
// A[c], B[c] hold the targets of slots 2L and 2L+1 (relative index
// N - 1 + slot), and park[c * (N - 1) + j] (wave-private LDS) the target of
// relative index j = 0..N-2.  The scale kScale is not applied.  KEEP_NU keeps
// slot a's factors from the suffix pass for the prefix pass (N more
// registers, two operations less per tap).
template <int N, int NC, bool KEEP_NU>
__device__ __forceinline__ void carry_scatter(double ea, double eb, const double (&va)[NC],
                                              const double (&vb)[NC], double (&A)[NC],
                                              double (&B)[NC], double* park, bool lane0) {
  constexpr LagrangeScaled<N> S = make_scaled<N>();
  constexpr int H = N / 2;
  // opaque copies: the factors must not be hoisted out of a caller's loop
  // (they would stay live beside the suffix products)
  asm volatile("" : "+v"(ea), "+v"(eb));
  const double de = eb - ea;
  double Sa[N], Sb[N], nu[N];
  Sa[N - 1] = NC == 1 ? va[0] : 1.0;
  Sb[N - 1] = NC == 1 ? vb[0] : 1.0;
  double d = ea + (double)(H - 1) - (double)(N - 1);   // eps_a - x_{N-1}
#pragma unroll
  for (int k = N - 1; k >= 1; --k) {
    const double na = S.s[k] * d;
    const double nb = fma(de, S.s[k], na);
    if (KEEP_NU) nu[k] = na;
    Sa[k - 1] = Sa[k] * na;
    Sb[k - 1] = Sb[k] * nb;
    d += 1.0;
  }
  // d = eps_a - x_0
  if (KEEP_NU) nu[0] = S.s[0] * d;
  double Pa = 1.0, Pb = 1.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) { A[c] = 0.0; B[c] = 0.0; }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k > 0 && lane0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) park[c * (N - 1) + k - 1] = A[c];
    }
    if (NC == 1) {
      const double sh = lane_down(A[0]);
      A[0] = fma(Pa, Sa[k], B[0]);
      B[0] = fma(Pb, Sb[k], sh);
    } else {
      const double wa = Pa * Sa[k], wb = Pb * Sb[k];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double sh = lane_down(A[c]);
        A[c] = fma(wa, va[c], B[c]);
        B[c] = fma(wb, vb[c], sh);
      }
    }
    if (k < N - 1) {
      const double na = KEEP_NU ? nu[k] : S.s[k] * d;
      const double nb = fma(de, S.s[k], na);
      Pa *= na;
      Pb *= nb;
      if (!KEEP_NU) d -= 1.0;
    }
  }
}

// Add a finished carry to a wave-private parity-split row: slots at
// relative index o + N - 1 + 2L (+1), parked sums at o + j (lanes j < N-1).
// o and half are wave-uniform, so both slot positions are a uniform offset
// plus the lane.
template <int N>
__device__ __forceinline__ void carry_add(double* row, int half, int o, int lane, double f,
                                          double A, double B, const double* park) {
  const int base = o + N - 1;
  const int h0 = base >> 1;
  const int pa = (base & 1) ? half + h0 : h0;             // element base + 2L
  const int pb = (base & 1) ? h0 + 1 : half + h0;         // element base + 2L + 1
  row[pa + lane] += f * A;
  row[pb + lane] += f * B;
  if (lane < N - 1) row[psplit(o + lane, half)] += f * park[lane];
}

}  // namespace lr
