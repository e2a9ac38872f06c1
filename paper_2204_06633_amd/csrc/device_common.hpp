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

// Spline series FIRST .. FIRST + COUNT - 1 at time tau.  When the whole wave
// sits in one coarse segment (the usual case: a segment spans thousands of
// samples) the coefficients are read once per wave with scalar loads instead
// of once per lane.
template <int FIRST, int COUNT>
__device__ __forceinline__ void orbit_series(const OrbitView& o, double tau, double (&v)[COUNT]) {
  double s = floor(tau * o.inv_dt);
  s = fmin(fmax(s, 0.0), (double)(o.nseg - 1));
  const double u = tau - s * o.dt;
  const int si = (int)s;
  const int su = __builtin_amdgcn_readfirstlane(si);
  if (__all(si == su)) {
    const double* seg = o.coef + (int64_t)su * kSegStride;
#pragma unroll
    for (int k = 0; k < COUNT; ++k) v[k] = spline_at(seg, FIRST + k, u);
  } else {
    const double* seg = o.coef + (int64_t)si * kSegStride;
#pragma unroll
    for (int k = 0; k < COUNT; ++k) v[k] = spline_at(seg, FIRST + k, u);
  }
}

struct Sky {
  double k[3], u[3], v[3];
};

// k = -e_r, u = -e_phi, v = -e_theta for ecliptic longitude lam, latitude beta
// (Sec. IV.A), from sl = sin(lam), cl = cos(lam), sb = sin(beta), cb = cos(beta).
__host__ __device__ inline Sky sky_from_trig(double sl, double cl, double sb, double cb) {
  Sky s;
  s.k[0] = -cb * cl; s.k[1] = -cb * sl; s.k[2] = -sb;
  s.u[0] = sl;       s.u[1] = -cl;      s.u[2] = 0.0;
  s.v[0] = -sb * cl; s.v[1] = -sb * sl; s.v[2] = cb;
  return s;
}

__host__ __device__ inline Sky sky_basis(double lam, double beta) {
  return sky_from_trig(sin(lam), cos(lam), sin(beta), cos(beta));
}

// Derivatives of (k, u, v) with respect to lam and beta.
struct SkyDeriv {
  double dk[2][3], du[2][3], dv[2][3];   // [lam, beta][xyz]
};

__host__ __device__ inline SkyDeriv sky_derivatives(double sl, double cl, double sb, double cb) {
  SkyDeriv d;
  d.dk[0][0] = cb * sl;  d.dk[0][1] = -cb * cl; d.dk[0][2] = 0.0;
  d.dk[1][0] = sb * cl;  d.dk[1][1] = sb * sl;  d.dk[1][2] = -cb;
  d.du[0][0] = cl;       d.du[0][1] = sl;       d.du[0][2] = 0.0;
  d.du[1][0] = 0.0;      d.du[1][1] = 0.0;      d.du[1][2] = 0.0;
  d.dv[0][0] = sb * sl;  d.dv[0][1] = -sb * cl; d.dv[0][2] = 0.0;
  d.dv[1][0] = -cb * cl; d.dv[1][1] = -cb * sl; d.dv[1][2] = -sb;
  return d;
}

// Per-sample constellation geometry at a reception time (Sec. IV.B):
// light times, k.x/c per spacecraft, antenna patterns and k.n per arm.
// Arms 0, 1, 2 are n12, n23, n31; link l uses arm kArm[l] with direction
// kDir[l] (n_ji = -n_ij, so xi is shared and k.n flips sign).
constexpr int kArm[6] = {0, 1, 2, 2, 1, 0};
constexpr double kDir[6] = {1.0, 1.0, 1.0, -1.0, -1.0, -1.0};

struct LinkGeom {
  double x[3][3];       // spacecraft positions (m)
  double L[6];          // light times (s)
  double kx[3];         // k.x_s / c (s)
  double n[3][3];       // unit arm vectors n12, n23, n31
  double un[3], vn[3];  // u.n, v.n per arm
  double xip[3], xic[3], kn[3];
};

__device__ __forceinline__ void link_geometry(const OrbitView& o, double tau, const Sky& sk,
                                              LinkGeom& g) {
  double v[15];
  orbit_series<0, 15>(o, tau, v);
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) g.x[s][c] = v[3 * s + c];
#pragma unroll
  for (int l = 0; l < 6; ++l) g.L[l] = v[9 + l];
  constexpr double inv_c = 1.0 / kC;
#pragma unroll
  for (int s = 0; s < 3; ++s)
    g.kx[s] = (sk.k[0] * g.x[s][0] + sk.k[1] * g.x[s][1] + sk.k[2] * g.x[s][2]) * inv_c;
#pragma unroll
  for (int arm = 0; arm < 3; ++arm) {
    const int r = arm, e = (arm + 1) % 3;
    double d0 = g.x[r][0] - g.x[e][0], d1 = g.x[r][1] - g.x[e][1], d2 = g.x[r][2] - g.x[e][2];
    const double inrm = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    d0 *= inrm; d1 *= inrm; d2 *= inrm;
    g.n[arm][0] = d0; g.n[arm][1] = d1; g.n[arm][2] = d2;
    double un = sk.u[0] * d0 + sk.u[1] * d1 + sk.u[2] * d2;
    double vn = sk.v[0] * d0 + sk.v[1] * d1 + sk.v[2] * d2;
    g.un[arm] = un;
    g.vn[arm] = vn;
    g.xip[arm] = un * un - vn * vn;
    g.xic[arm] = 2.0 * un * vn;
    g.kn[arm] = sk.k[0] * d0 + sk.k[1] * d1 + sk.k[2] * d2;
  }
}

// Retarded delays (s) of the nine interpolation positions of one link
// sample: 0..2 reception at spacecraft 1..3 (shared by the two links received
// there), 3..8 emission of links 0..5.
__device__ __forceinline__ double position_delay(const LinkGeom& g, int p) {
  return p < 3 ? g.kx[p] : g.L[p - 3] + g.kx[kLinkEmit[p - 3] - 1];
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

// scale multiplies every weight (it starts the suffix product, so a scatter
// of scale * w_m costs no extra multiply).
template <int N>
__device__ __forceinline__ void lagrange_weights(double eps, double (&w)[N], double scale = 1.0) {
  constexpr LagrangeDenoms<N> C = make_denoms<N>();
  constexpr int H = N / 2;
  double pre = 1.0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    w[m] = pre;
    pre *= eps - (double)(m - (H - 1));
  }
  double suf = scale;
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    w[m] *= suf * C.c[m];
    suf *= eps - (double)(m - (H - 1));
  }
}

// Streaming Lagrange interpolation, without materialising the weights.
// With d_k = eps - x_k the interpolant is I = sum_j c_j f_j prod_{i != j} d_i.
// Rescaled factors nu_k = s_k d_k, s_k = K / c_k, turn every weight into a
// pure product: prod_{i != j} nu_i = (K^(N-1) prod_i 1/c_i) c_j prod_{i != j} d_i.
// So with R_0 = 1, R_{k+1} = R_k nu_k and the recurrence
//   T_0 = f_0,   T_k = T_{k-1} nu_k + R_k f_k,
// T_{N-1} = I / kScale, kScale = K prod_i (c_i / K).  K is a power of two
// near the geometric mean of the |c_i|, so that every |s_k| is of order one
// and every partial product stays within ~1e+-20 for N <= 32.
template <int N>
struct LagrangeScaled {
  double s[N];      // s_k = K / c_k = K prod_{j != k} (x_k - x_j)
  double scale;     // kScale
};

template <int N>
constexpr LagrangeScaled<N> make_scaled() {
  LagrangeScaled<N> r{};
  double p[N] = {};
  int esum = 0;
  for (int m = 0; m < N; ++m) {
    p[m] = 1.0;
    for (int j = 0; j < N; ++j)
      if (j != m) p[m] *= (double)(m - j);
    double v = p[m] < 0.0 ? -p[m] : p[m];
    while (v >= 2.0) { v *= 0.5; ++esum; }
  }
  const int e = (esum + N / 2) / N;
  double K = 1.0;
  for (int i = 0; i < e; ++i) K *= 0.5;
  double scale = K;
  for (int m = 0; m < N; ++m) {
    r.s[m] = K * p[m];
    scale /= r.s[m];
  }
  r.scale = scale;
  return r;
}

// One sample.  Per tap: 3 FP64 ops shared by all series on the stencil (the
// product update, eps - x_k by an inline-constant subtraction, nu_k with s_k
// from an SGPR) plus 2 per series, in O(1) registers.  Usage per tap
// k = 0, 1, ...: tap(k), then for every series x = step(x, f_k, k); the
// interpolant is finish(x).
template <int N>
struct LagrangeStream {
  static constexpr double kScale = make_scaled<N>().scale;   // finish() multiplier
  double d, R, nu;
  __device__ __forceinline__ explicit LagrangeStream(double eps)
      : d(eps + (double)(N / 2 - 1)), R(1.0), nu(0.0) {}
  __device__ __forceinline__ void tap(int k) {
    constexpr LagrangeScaled<N> S = make_scaled<N>();
    if (k > 0) {
      R *= nu;
      d -= 1.0;
    }
    nu = S.s[k] * d;
  }
  __device__ __forceinline__ double step(double x, double f, int k) const {
    return k == 0 ? f : fma(R, f, x * nu);
  }
  __device__ __forceinline__ static double finish(double x) { return x * kScale; }
};

// Two samples a and b of one lane, stepped through the same tap index k
// (their stencils may start at different window positions).  Sample b's
// factor comes from sample a's by one FMA, nu_b = nu_a + s_k (eps_b - eps_a),
// whose only scalar operand is s_k; a VOP3 reads at most one, so computing
// s_k (eps_b - x_k) afresh would cost a subtraction and a multiply.  Per tap
// the pair shares 5 FP64 ops (6 for two LagrangeStreams) plus 2 per series.
// Same scale as LagrangeStream: finish() with LagrangeStream<N>::finish.
template <int N>
struct LagrangePair {
  double d, de, Ra, Rb, na, nb;
  __device__ __forceinline__ LagrangePair(double ea, double eb)
      : d(ea + (double)(N / 2 - 1)), de(eb - ea), Ra(1.0), Rb(1.0), na(0.0), nb(0.0) {}
  __device__ __forceinline__ void tap(int k) {
    constexpr LagrangeScaled<N> S = make_scaled<N>();
    if (k > 0) {
      Ra *= na;
      Rb *= nb;
      d -= 1.0;
    }
    na = S.s[k] * d;
    nb = fma(de, S.s[k], na);
  }
  __device__ __forceinline__ double step_a(double x, double f, int k) const {
    return k == 0 ? f : fma(Ra, f, x * na);
  }
  __device__ __forceinline__ double step_b(double x, double f, int k) const {
    return k == 0 ? f : fma(Rb, f, x * nb);
  }
};

// LagrangeStream with the derivative with respect to eps carried along:
// P'_{k+1} = P'_k (eps - x_k) + P_k, and a series follows
// T'_k = T'_{k-1} (eps - x_k) + T_{k-1} + c_k P'_k f_k.
template <int N>
struct LagrangeStreamD {
  double d, P, Pd;
  __device__ __forceinline__ explicit LagrangeStreamD(double eps)
      : d(eps + (double)(N / 2 - 1)), P(1.0), Pd(0.0) {}
  __device__ __forceinline__ double coef(int k) const {
    constexpr LagrangeDenoms<N> C = make_denoms<N>();
    return C.c[k] * P;
  }
  __device__ __forceinline__ double coef_d(int k) const {
    constexpr LagrangeDenoms<N> C = make_denoms<N>();
    return C.c[k] * Pd;
  }
  // one tap of a series: value t and derivative td, sample f
  __device__ __forceinline__ void step(double c, double cd, double f, double& t,
                                       double& td) const {
    td = fma(cd, f, fma(td, d, t));
    t = fma(c, f, t * d);
  }
  __device__ __forceinline__ void next() {
    Pd = fma(Pd, d, P);
    P *= d;
    d -= 1.0;
  }
};

// Weight of tap m alone, O(N) work, for paths that cannot hold a weight
// array (tap index not known at compile time).
template <int N>
__device__ __forceinline__ double lagrange_weight_at(double eps, int m) {
  constexpr int H = N / 2;
  double num = 1.0, den = 1.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool skip = j == m;
    num *= skip ? 1.0 : eps - (double)(j - (H - 1));
    den *= skip ? 1.0 : (double)(m - j);
  }
  return num / den;
}

// Two weight sets at once (two independent product chains).
template <int N>
__device__ __forceinline__ void lagrange_weights2(double ea, double eb, double (&wa)[N],
                                                  double (&wb)[N]) {
  constexpr LagrangeDenoms<N> C = make_denoms<N>();
  constexpr int H = N / 2;
  double pa = 1.0, pb = 1.0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    wa[m] = pa;
    wb[m] = pb;
    const double x = (double)(m - (H - 1));
    pa *= ea - x;
    pb *= eb - x;
  }
  double sa = 1.0, sb = 1.0;
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    wa[m] *= sa * C.c[m];
    wb[m] *= sb * C.c[m];
    const double x = (double)(m - (H - 1));
    sa *= ea - x;
    sb *= eb - x;
  }
}

// Split the retarded position q - d/dt into an integer shift (so that
// j0 = q + shift) and eps in [0, 1), with d a delay in seconds.  The shift is
// clamped to +-2^24 so that non-finite delays keep every index computation in
// int32 range (such samples then take the clamped global-memory path).
__device__ __forceinline__ int split_delay(double d, double inv_dt, double& eps) {
  double a = -d * inv_dt;
  double f = floor(a);
  f = fmin(fmax(f, -16777216.0), 16777216.0);
  eps = a - f;
  return (int)f;
}

// Derivative weights dw_m/deps of the same Lagrange basis (product rule on
// the prefix and suffix products).
template <int N>
__device__ __forceinline__ void lagrange_weights_d(double eps, double (&w)[N], double (&dw)[N]) {
  constexpr LagrangeDenoms<N> C = make_denoms<N>();
  constexpr int H = N / 2;
  double pre = 1.0, dpre = 0.0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    w[m] = pre;
    dw[m] = dpre;
    const double d = eps - (double)(m - (H - 1));
    dpre = fma(dpre, d, pre);
    pre *= d;
  }
  double suf = 1.0, dsuf = 0.0;
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    dw[m] = C.c[m] * fma(dw[m], suf, w[m] * dsuf);
    w[m] *= suf * C.c[m];
    const double d = eps - (double)(m - (H - 1));
    dsuf = fma(dsuf, d, suf);
    suf *= d;
  }
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
// ds_swizzle in bit mode: lane i reads lane i ^ X within its 32-lane half
// (pattern xor_mask << 10 | and_mask 0x1f).  The pattern is an immediate, so
// no lane-address registers have to be kept.
#define LR_SWZ_XOR(v, X) __builtin_amdgcn_ds_swizzle((v), ((X) << 10) | 0x1f)

// xor butterflies within each half-wave, then the two halves; the result is
// wave-uniform.
__device__ __forceinline__ int wave_min(int v) {
  v = min(v, LR_SWZ_XOR(v, 16));
  v = min(v, LR_SWZ_XOR(v, 8));
  v = min(v, LR_SWZ_XOR(v, 4));
  v = min(v, LR_SWZ_XOR(v, 2));
  v = min(v, LR_SWZ_XOR(v, 1));
  return min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 32));
}
__device__ __forceinline__ int wave_max(int v) {
  v = max(v, LR_SWZ_XOR(v, 16));
  v = max(v, LR_SWZ_XOR(v, 8));
  v = max(v, LR_SWZ_XOR(v, 4));
  v = max(v, LR_SWZ_XOR(v, 2));
  v = max(v, LR_SWZ_XOR(v, 1));
  return max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 32));
}

}  // namespace lr
