// Device building blocks shared by the response kernels (gfx950, FP64).
//
//  * orbit spline evaluation at a sample time          (Sec. IV.E: orbit data
//    interpolated once and evaluated at every time step)
//  * sky basis k, u, v                                  (Sec. IV.A)
//  * centred Lagrange weights of compile-time tap count (Sec. IV.E)
//  * Michelson TDI-1/TDI-2 delay-group tables           (Sec. IV.C)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lr {

constexpr double kC = 299792458.0;
constexpr int kSeries = 15;      // x1 y1 z1 x2 y2 z2 x3 y3 z3, L12 L23 L31 L13 L32 L21
constexpr int kSegStride = 64;   // doubles per coarse segment: 16 series x 4 coefficients

// Links l = 0..5: (receiver, emitter) = 12, 23, 31, 13, 32, 21 (spacecraft 1..3).
constexpr int kLinkRecv[6] = {1, 2, 3, 1, 3, 2};
constexpr int kLinkEmit[6] = {2, 3, 1, 3, 2, 1};

struct OrbitView {
  const double* coef;  // [nseg][16][4], ascending powers of u = tau - k*dt
  double dt;           // coarse spacing
  double inv_dt;
  int64_t nseg;
};

// Segment of the coarse grid holding tau (seconds since coarse sample 0),
// and the local abscissa.  Out-of-grid times are clamped to the end
// segments; the host rejects calls that would need them.
__device__ __forceinline__ const double* orbit_segment(const OrbitView& o, double tau, double& u) {
  double s = floor(tau * o.inv_dt);
  s = fmin(fmax(s, 0.0), (double)(o.nseg - 1));
  u = tau - s * o.dt;
  return o.coef + (int64_t)s * kSegStride;
}

__device__ __forceinline__ double spline_at(const double* seg, int series, double u) {
  const double* c = seg + 4 * series;
  return fma(fma(fma(c[3], u, c[2]), u, c[1]), u, c[0]);
}

struct Sky {
  double k[3], u[3], v[3];
};

// k = -e_r, u = -e_phi, v = -e_theta for ecliptic longitude lam, latitude beta.
__host__ __device__ inline Sky sky_basis(double lam, double beta) {
  double cb = cos(beta), sb = sin(beta), cl = cos(lam), sl = sin(lam);
  Sky s;
  s.k[0] = -cb * cl; s.k[1] = -cb * sl; s.k[2] = -sb;
  s.u[0] = sl;       s.u[1] = -cl;      s.u[2] = 0.0;
  s.v[0] = -sb * cl; s.v[1] = -sb * sl; s.v[2] = cb;
  return s;
}

// ---------------------------------------------------------------------------
// Lagrange weights, N = order + 1 taps on nodes x_m = m - (N/2 - 1).
//   w_m(eps) = c_m * prod_{j<m}(eps - x_j) * prod_{j>m}(eps - x_j),
//   c_m = 1 / prod_{j != m}(x_m - x_j),
// evaluated with one prefix and one suffix product (about 5N FP64 ops).
// ---------------------------------------------------------------------------
template <int N>
struct LagrangeDenoms {
  double c[N];
};

template <int N>
constexpr LagrangeDenoms<N> make_denoms() {
  LagrangeDenoms<N> r{};
  for (int m = 0; m < N; ++m) {
    double p = 1.0;
    for (int j = 0; j < N; ++j)
      if (j != m) p *= (double)(m - j);
    r.c[m] = 1.0 / p;
  }
  return r;
}

template <int N>
__device__ __forceinline__ void lagrange_weights(double eps, double (&w)[N]) {
  constexpr LagrangeDenoms<N> C = make_denoms<N>();
  constexpr int H = N / 2;
  double pre = 1.0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    w[m] = pre;
    pre *= eps - (double)(m - (H - 1));
  }
  double suf = 1.0;
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    w[m] *= suf * C.c[m];
    suf *= eps - (double)(m - (H - 1));
  }
}

// Split the retarded position q - d/dt into an integer shift (so that
// j0 = q + shift) and eps in [0, 1), with d a delay in seconds.  The shift is
// clamped to +-2^30 so that non-finite delays stay in integer range.
__device__ __forceinline__ int split_delay(double d, double inv_dt, double& eps) {
  double a = -d * inv_dt;
  double f = floor(a);
  f = fmin(fmax(f, -1073741824.0), 1073741824.0);
  eps = a - f;
  return (int)f;
}

// ---------------------------------------------------------------------------
// TDI tables.  X1 / X2 written from eqs. (tdi1) / (tdi2) as (sign, delay
// chain, measured link); Y and Z by the cyclic relabelling 1->2->3->1.
// Delayed terms whose chained delays have the same multiset of link light
// times share one set of interpolation weights ("delay group").
// ---------------------------------------------------------------------------
struct XTerm {
  int sign;
  int len;        // spacecraft in the chain
  int path[8];    // spacecraft 1..3
  int meas_r, meas_e;
};

constexpr XTerm kXTerms[16] = {
    // eq. (tdi1): y13 + D13 y31 + D131 y12 + D1312 y21 - [y12 + D12 y21 + D121 y13 + D1213 y31]
    {+1, 1, {1}, 1, 3},
    {+1, 2, {1, 3}, 3, 1},
    {+1, 3, {1, 3, 1}, 1, 2},
    {+1, 4, {1, 3, 1, 2}, 2, 1},
    {-1, 1, {1}, 1, 2},
    {-1, 2, {1, 2}, 2, 1},
    {-1, 3, {1, 2, 1}, 1, 3},
    {-1, 4, {1, 2, 1, 3}, 3, 1},
    // eq. (tdi2): + D13121 y12 + D131212 y21 + D1312121 y13 + D13121213 y31
    //             - [D12131 y13 + D121313 y31 + D1213131 y12 + D12131312 y21]
    {+1, 5, {1, 3, 1, 2, 1}, 1, 2},
    {+1, 6, {1, 3, 1, 2, 1, 2}, 2, 1},
    {+1, 7, {1, 3, 1, 2, 1, 2, 1}, 1, 3},
    {+1, 8, {1, 3, 1, 2, 1, 2, 1, 3}, 3, 1},
    {-1, 5, {1, 2, 1, 3, 1}, 1, 3},
    {-1, 6, {1, 2, 1, 3, 1, 3}, 3, 1},
    {-1, 7, {1, 2, 1, 3, 1, 3, 1}, 1, 2},
    {-1, 8, {1, 2, 1, 3, 1, 3, 1, 2}, 2, 1},
};

constexpr int link_of(int r, int e) {
  for (int l = 0; l < 6; ++l)
    if (kLinkRecv[l] == r && kLinkEmit[l] == e) return l;
  return -1;
}

constexpr int rot(int s, int times) {
  for (int i = 0; i < times; ++i) s = s % 3 + 1;
  return s;
}

struct GroupUse {
  int chan, sign, link;
};

struct DelayGroup {
  int cnt[6];       // how many times each link light time enters the delay
  int nuse;
  GroupUse use[3];
};

struct Direct {
  int chan, sign, link;
};

template <int GEN>
struct TdiTable {
  static constexpr int kTermsPerChan = GEN == 1 ? 8 : 16;
  DelayGroup group[3 * kTermsPerChan];
  int ngroup;
  Direct direct[6];
  int ndirect;
};

template <int GEN>
constexpr TdiTable<GEN> make_tdi_table() {
  TdiTable<GEN> t{};
  t.ngroup = 0;
  t.ndirect = 0;
  for (int ch = 0; ch < 3; ++ch) {
    for (int i = 0; i < TdiTable<GEN>::kTermsPerChan; ++i) {
      const XTerm& x = kXTerms[i];
      int link = link_of(rot(x.meas_r, ch), rot(x.meas_e, ch));
      if (x.len == 1) {
        t.direct[t.ndirect++] = Direct{ch, x.sign, link};
        continue;
      }
      int cnt[6] = {0, 0, 0, 0, 0, 0};
      for (int s = 0; s + 1 < x.len; ++s) cnt[link_of(rot(x.path[s], ch), rot(x.path[s + 1], ch))] += 1;
      int g = 0;
      for (; g < t.ngroup; ++g) {
        bool same = true;
        for (int l = 0; l < 6; ++l) same = same && (t.group[g].cnt[l] == cnt[l]);
        if (same) break;
      }
      if (g == t.ngroup) {
        for (int l = 0; l < 6; ++l) t.group[g].cnt[l] = cnt[l];
        t.group[g].nuse = 0;
        t.ngroup++;
      }
      t.group[g].use[t.group[g].nuse++] = GroupUse{ch, x.sign, link};
    }
  }
  return t;
}

// Delay of a group: sum of its link light times (s).
__device__ __forceinline__ double group_delay(const DelayGroup& g, const double (&L)[6]) {
  double d = 0.0;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    if (g.cnt[l] == 1) d += L[l];
    else if (g.cnt[l] > 1) d = fma((double)g.cnt[l], L[l], d);
  }
  return d;
}

// Wave (64 lanes) and workgroup min / max of an int.
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace lr
