// Galactic-binary waveform on the device (Sec. III), shared by the
// polarisation kernels and the fused response kernels that synthesise h+
// and hx in their LDS windows:
//
//   Phi(t) = 2 pi (f0 t + fdot t^2 / 2 + fddot t^3 / 6) + phi0,
//   fddot  = 11 fdot^2 / (3 f0)   (gravitational-wave driven evolution),
//   a+ = -(1 + cos^2 iota) A cos Phi,   ax = -2 cos(iota) A sin Phi,
//   h+ = cos(2 psi) a+ - sin(2 psi) ax,  hx = sin(2 psi) a+ + cos(2 psi) ax.
//
// The phase is evaluated in cycles with f0 t split into a rounded product
// and its exact error (fma), and the whole cycles are removed before the
// multiplication by 2 pi: over a year f0 t reaches ~4e5 cycles, where plain
// FP64 would leave ~1e-10 rad of rounding in the phase.
#pragma once

#include <hip/hip_runtime.h>

namespace lr {
namespace gb {

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

// h+ and hx at time t (ap0 = -(1 + cos^2 iota) A, ac0 = -2 cos(iota) A).
__device__ __forceinline__ void polarizations_at(const Source& s, double ap0, double ac0, double t,
                                                 double& hp, double& hc) {
  double sn, cs;
  sincos(phase(s, t), &sn, &cs);
  const double ap = ap0 * cs, ac = ac0 * sn;
  hp = s.c2 * ap - s.s2 * ac;
  hc = s.s2 * ap + s.c2 * ac;
}

// Seven sample sums of the parameter gradient (the transpose of the
// linearised waveform): for an upstream gradient (g_p, g_c) on (h+, hx) at
// time t, with Gp, Gc its rotation onto (a+, ax) and Q its projection on
// d/d Phi:
//   S0 += Gp a+ + Gc ax            (times 1/A: d/dA)
//   S1 += d/d iota, S2 += d/d psi, S3 += Q (d/d phi0),
//   S4 += Q t, S5 += Q t^2, S6 += Q t^3  (the phase polynomial's powers).
__device__ __forceinline__ void adjoint_sums(const Source& s, double t, double g_p, double g_c,
                                             double (&acc)[7]) {
  const double A = s.A;
  double sn, cs;
  sincos(phase(s, t), &sn, &cs);
  const double Gp = g_p * s.c2 + g_c * s.s2;            // d/d a+
  const double Gc = -g_p * s.s2 + g_c * s.c2;           // d/d ax
  const double ap = -(1.0 + s.ci * s.ci) * A * cs, ac = -2.0 * s.ci * A * sn;
  const double Q = Gp * (1.0 + s.ci * s.ci) * A * sn - Gc * 2.0 * s.ci * A * cs;   // d/d Phi
  acc[0] += Gp * ap + Gc * ac;
  acc[1] += 2.0 * s.si * A * (Gp * s.ci * cs + Gc * sn);
  acc[2] += 2.0 * (ap * Gc - ac * Gp);
  acc[3] += Q;
  acc[4] += Q * t;
  acc[5] += Q * t * t;
  acc[6] += Q * t * t * t;
}

// Gradient with respect to (A, f0, fdot, phi0, iota, psi) from the seven
// sums (fddot = 11 fdot^2 / (3 f0) depends on f0 and fdot):
//   d/dA = S0 / A, d/df0 = 2 pi (S4 - fddot / (6 f0) S6),
//   d/dfdot = 2 pi (S5 / 2 + (22/3) (fdot / f0) S6 / 6), d/dphi0 = S3,
//   d/diota = S1, d/dpsi = S2; lam, beta: 0 (they enter through the response).
__device__ __forceinline__ void finalize_gradient(const double* p, const double* tot, double* g) {
  const double f0 = p[1], fdot = p[2], fddot = 11.0 / 3.0 * fdot * fdot / f0;
  g[0] = tot[0] / p[0];
  g[1] = kTwoPi * (tot[4] - fddot / (6.0 * f0) * tot[6]);
  g[2] = kTwoPi * (0.5 * tot[5] + 22.0 / 3.0 * fdot / f0 * tot[6] / 6.0);
  g[3] = tot[3];
  g[4] = tot[1];
  g[5] = tot[2];
  g[6] = 0.0;
  g[7] = 0.0;
}

}  // namespace gb
}  // namespace lr
