// Forward response kernels for gfx950 (FP64):
//   project_links_kernel  -- link responses y_ij, Sec. IV.B
//   tdi_kernel            -- Michelson TDI-1 / TDI-2 and A, E, T, Sec. IV.C
//
// Both kernels are time-tiled: a workgroup owns kFwdTile consecutive output
// samples, computes every retarded position of its samples first, reduces the
// extent of all their interpolation stencils, stages exactly that window of
// the input series in LDS with coalesced loads, and then evaluates the
// Lagrange sums from LDS (the paper's shared-memory sub-arrays, Sec. IV.E,
// re-designed around a per-tile stencil window).
//
// Each lane owns two consecutive output samples.  Their retarded positions
// drift by far less than a sample, so for every position the two stencils
// are the same window shifted by one: the lane streams N + 1 values from LDS
// and feeds both Lagrange sums (half the LDS traffic of one sample per lane),
// and the two weight sets are independent product chains (twice the
// instruction-level parallelism).  A wave whose two stencils do not line up
// for some position (an integer crossing) takes a separate-window branch for
// that position.  Stores are link- / channel-major and coalesced.
#pragma once

#include <type_traits>
#include <utility>

#include "device_common.hpp"
#include "gb_device.hpp"
#include "internal.hpp"

namespace lr {

constexpr int kBlock = kTile;          // lanes per workgroup
constexpr int kSlack = 64;             // window samples beyond the tile + taps
constexpr int kPerLane = 2;            // forward kernels: consecutive samples per lane
constexpr int kFwdTile = kBlock * kPerLane;

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

// LDS windows of the two-samples-per-lane kernels are stored split by
// parity: element j of a window of capacity CAP sits at par(j) = (j odd ?
// half : 0) + j/2.  A lane streams from element ra + c (ra = 2*lane, c shared
// by the wave), so for every tap the wave reads 64 consecutive addresses
// instead of every other one (no bank conflicts).
template <int CAP>
__device__ __forceinline__ int par(int j) {
  return (j & 1) * ((CAP + 1) / 2) + (j >> 1);
}

// Addresses of elements j0 and j0 + 1 of a parity-split window: element
// j0 + k is at first + k/2 for even k and at second + (k-1)/2 for odd k.
template <int CAP>
struct ParStream {
  int first, second;
  __device__ __forceinline__ explicit ParStream(int j0)
      : first(par<CAP>(j0)), second(first + ((j0 & 1) ? 1 - (CAP + 1) / 2 : (CAP + 1) / 2)) {}
  __device__ __forceinline__ int at(int k) const { return (k & 1) ? second + (k >> 1) : first + (k >> 1); }
};

// ---------------------------------------------------------------------------
// Projection
// ---------------------------------------------------------------------------

// Positions p = 0..2 (reception at spacecraft p+1) enter the links received
// there with a minus sign; p = 3..8 (emission of link p-3) enter that link
// with a plus sign.  Adds xi+ h+ + xix hx of position p to the numerators.
__device__ __forceinline__ void add_position(int p, const double (&xip)[3],
                                             const double (&xic)[3], double hp, double hc,
                                             double (&num)[6]) {
  if (p >= 3) {
    const int l = p - 3, arm = kArm[l];
    num[l] += xip[arm] * hp + xic[arm] * hc;
  } else {
#pragma unroll
    for (int l = 0; l < 6; ++l)
      if (kLinkRecv[l] - 1 == p) num[l] -= xip[kArm[l]] * hp + xic[kArm[l]] * hc;
  }
}

// add_position for a position index known only at run time: the links are
// selected by comparisons, so the accumulators stay in registers.
__device__ __forceinline__ void add_position_rt(int p, const double (&xip)[3],
                                                const double (&xic)[3], double hp, double hc,
                                                double (&num)[6]) {
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const int arm = kArm[l];
    const double v = xip[arm] * hp + xic[arm] * hc;
    const bool emit = p == 3 + l, recv = p == kLinkRecv[l] - 1;
    num[l] += emit ? v : (recv ? -v : 0.0);
  }
}

// Per-sample state of the projection: what the link assembly needs.
struct ProjSample {
  int sh[9];
  double ep[9];
  double xip[3], xic[3], kn[3];
};

__device__ __forceinline__ void proj_sample(const OrbitView& orb, double tau, double inv_dt,
                                            const Sky& sk, ProjSample& s) {
  LinkGeom g;
  link_geometry(orb, tau, sk, g);
#pragma unroll
  for (int p = 0; p < 9; ++p) s.sh[p] = split_delay(position_delay(g, p), inv_dt, s.ep[p]);
#pragma unroll
  for (int k = 0; k < 3; ++k) { s.xip[k] = g.xip[k]; s.xic[k] = g.xic[k]; s.kn[k] = g.kn[k]; }
}

// Source of the h+ / hx samples a projection reads, by h-index j in
// [0, n_h): arrays in HBM, or the Galactic-binary waveform (Sec. III)
// evaluated at t_j = (k0 + j) dt from one parameter row (the fused batch
// kernels synthesise their LDS windows this way; the waveform's constants
// are set up once per template).
struct HSource {
  const double* hp;
  const double* hc;
  int64_t n_h;
  bool wave;
  gb::Source src;
  double ap0, ac0, dt;
  int64_t k0;

  __device__ __forceinline__ static HSource arrays(const double* hp, const double* hc,
                                                   int64_t n_h) {
    HSource h;
    h.hp = hp;
    h.hc = hc;
    h.n_h = n_h;
    h.wave = false;
    return h;
  }
  // params: A, f0, fdot, phi0, iota, psi (lam, beta unused here)
  __device__ __forceinline__ static HSource waveform(const double* params, int64_t k0, double dt,
                                                     int64_t n_h) {
    HSource h;
    h.hp = h.hc = nullptr;
    h.n_h = n_h;
    h.wave = true;
    h.src = gb::load_source(params);
    h.ap0 = -(1.0 + h.src.ci * h.src.ci) * h.src.A;
    h.ac0 = -2.0 * h.src.ci * h.src.A;
    h.dt = dt;
    h.k0 = k0;
    return h;
  }
  __device__ __forceinline__ double2 at(int64_t j) const {
    if (wave) {                                   // uniform
      double p, c;
      gb::polarizations_at(src, ap0, ac0, (double)(k0 + j) * dt, p, c);
      return make_double2(p, c);
    }
    return make_double2(hp[j], hc[j]);
  }
};

// Window loads kept in flight per stream in project_pair (0: the compiler's
// own schedule).  Build-time tuning knob (sched_group_barrier masks: 0x100
// LDS reads, 0x002 VALU).
#ifndef LR_PROJ_PIPE
#define LR_PROJ_PIPE 2
#endif

// Link responses of one template at the lane's two tile samples ra and ra+1
// (ra even), in a workgroup of BLOCK lanes (a tile of 2 BLOCK samples).  Tile element r has h-index hq0 + r and orbit time
// t_off + (ti0 + r) * dt.  Uses the workgroup's LDS window and reduction
// scratch; contains barriers, so every lane of the workgroup must call it.
template <int N, int BLOCK = kBlock>
__device__ __forceinline__ void project_pair(const OrbitView& orb, double t_off, int64_t ti0,
                                             double dt, double inv_dt, const HSource& hs,
                                             int64_t hq0,
                                             const Sky& sk, int ra, double2* win,
                                             int (&red)[2][BLOCK / 64], double (&ya)[6],
                                             double (&yb)[6]) {
  constexpr int H = N / 2;
  constexpr int CAP = kPerLane * BLOCK + N + kSlack;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));          // not hoisted out of a caller's loop
  ProjSample A, B;
  proj_sample(orb, t_off + (double)(ti0 + ra) * dt, inv_dt, sk, A);
  __builtin_amdgcn_sched_barrier(0);     // one sample's geometry live at a time
  proj_sample(orb, t_off + (double)(ti0 + ra + 1) * dt, inv_dt, sk, B);
  __builtin_amdgcn_sched_barrier(0);

  int lo = min(A.sh[0], B.sh[0] + 1), hi = max(A.sh[0], B.sh[0] + 1);
#pragma unroll
  for (int p = 1; p < 9; ++p) {
    lo = min(lo, min(A.sh[p], B.sh[p] + 1));
    hi = max(hi, max(A.sh[p], B.sh[p] + 1));
  }
  int wlo, whi;
  block_range<BLOCK>(ra + lo - (H - 1), ra + hi + H, red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = hq0 + wlo;                // h-index of window element 0
  const int64_t hmax = hs.n_h - 1;
  const int64_t qa = hq0 + ra;

  double na[6] = {0, 0, 0, 0, 0, 0}, nb[6] = {0, 0, 0, 0, 0, 0};
  if (count > 0 && count <= CAP) {
    for (int k = tid; k < count; k += BLOCK) {
      int64_t j = base + k;
      j = j < 0 ? 0 : (j > hmax ? hmax : j);
      win[par<CAP>(k)] = hs.at(j);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      LagrangePair<N> st(A.ep[p], B.ep[p]);
      const ParStream<CAP> src(ra + A.sh[p] - (H - 1) - wlo);
      double pa = 0.0, ca = 0.0, pb = 0.0, cb = 0.0;
      if (__all(A.sh[p] == B.sh[p])) {
        // sample b's stencil is sample a's shifted by one: N + 1 loads feed both
        double2 cur = win[src.at(0)];
#pragma unroll
        for (int k = 0; k < N; ++k) {
          if (LR_PROJ_PIPE > 0) {
            // at most LR_PROJ_PIPE window loads in flight: bounds the registers
            // the scheduler spends on early loads
            if (k == 0) __builtin_amdgcn_sched_group_barrier(0x100, LR_PROJ_PIPE, 0);
            if (k + LR_PROJ_PIPE <= N) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);
          }
          const double2 nxt = win[src.at(k + 1)];
          st.tap(k);
          pa = st.step_a(pa, cur.x, k);
          ca = st.step_a(ca, cur.y, k);
          pb = st.step_b(pb, nxt.x, k);
          cb = st.step_b(cb, nxt.y, k);
          cur = nxt;
        }
      } else {
        const ParStream<CAP> srb(ra + 1 + B.sh[p] - (H - 1) - wlo);
#pragma unroll
        for (int k = 0; k < N; ++k) {
          if (LR_PROJ_PIPE > 0) {
            if (k == 0) __builtin_amdgcn_sched_group_barrier(0x100, 2 * LR_PROJ_PIPE, 0);
            if (k + LR_PROJ_PIPE < N) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);
          }
          const double2 v = win[src.at(k)], w = win[srb.at(k)];
          st.tap(k);
          pa = st.step_a(pa, v.x, k);
          ca = st.step_a(ca, v.y, k);
          pb = st.step_b(pb, w.x, k);
          cb = st.step_b(cb, w.y, k);
        }
      }
      add_position(p, A.xip, A.xic, pa, ca, na);
      add_position(p, B.xip, B.xic, pb, cb, nb);
      __builtin_amdgcn_sched_barrier(0);   // keep one position's streams live at a time
    }
  } else {
    // Window larger than the LDS tile (very small dt or extreme orbits):
    // read the stencils from global memory, indices clamped.  A rolled loop
    // over copies of the per-sample state (which may then live in scratch):
    // this rare path must not set the register budget of the LDS path.
    const ProjSample Ac = A, Bc = B;
#pragma unroll 1
    for (int p = 0; p < 9; ++p) {
      LagrangePair<N> st(Ac.ep[p], Bc.ep[p]);
      const int64_t ja = qa + Ac.sh[p] - (H - 1), jb = qa + 1 + Bc.sh[p] - (H - 1);
      double pa = 0.0, ca = 0.0, pb = 0.0, cb = 0.0;
#pragma unroll 1
      for (int m = 0; m < N; ++m) {
        int64_t j = ja + m;
        j = j < 0 ? 0 : (j > hmax ? hmax : j);
        int64_t jj = jb + m;
        jj = jj < 0 ? 0 : (jj > hmax ? hmax : jj);
        st.tap(m);
        const double2 va = hs.at(j), vb = hs.at(jj);
        pa = st.step_a(pa, va.x, m);
        ca = st.step_a(ca, va.y, m);
        pb = st.step_b(pb, vb.x, m);
        cb = st.step_b(cb, vb.y, m);
      }
      add_position_rt(p, A.xip, A.xic, pa, ca, na);
      add_position_rt(p, B.xip, B.xic, pb, cb, nb);
    }
  }
  // the streams' common scale folded into the link normalisation
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const int arm = kArm[l];
    ya[l] = LagrangeStream<N>::finish(na[l]) / (2.0 * (1.0 - kDir[l] * A.kn[arm]));
    yb[l] = LagrangeStream<N>::finish(nb[l]) / (2.0 * (1.0 - kDir[l] * B.kn[arm]));
  }
}

// Minimum resident waves per SIMD the compiler must allow (register budget);
// build-time tuning knobs.
#ifndef LR_PROJ_MIN_WAVES
#define LR_PROJ_MIN_WAVES 1
#endif
#ifndef LR_TDI_MIN_WAVES
#define LR_TDI_MIN_WAVES 4
#endif

template <int N>
__global__ __launch_bounds__(kBlock, LR_PROJ_MIN_WAVES)
void project_links_kernel(ProjArgs a) {
  constexpr int CAP = kFwdTile + N + kSlack;
  __shared__ double2 win[CAP];
  __shared__ int red[2][kBlock / 64];
  __shared__ double s_trig[2][2];

  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kFwdTile;
  const int last = (int)min((int64_t)(kFwdTile - 1), a.n_y - 1 - i0);
  const bool act_a = kPerLane * tid <= last, act_b = kPerLane * tid + 1 <= last;
  const int ra = act_a ? kPerLane * tid : last;          // idle lanes mirror the last sample

  const SkyTrig tr = load_sky(a.sky, s_trig);
  const Sky sk = sky_from_trig(tr.sl, tr.cl, tr.sb, tr.cb);
  double ya[6], yb[6];
  project_pair<N>(a.orb, a.t_off, a.y_start + i0, a.dt, a.inv_dt,
                  HSource::arrays(a.hp, a.hc, a.n_h), a.y_start + i0, sk, ra, win, red, ya, yb);

  if (!act_a) return;
  const int64_t i = i0 + ra;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    double* dst = a.y + (int64_t)l * a.n_y + i;
    if (act_b && ((reinterpret_cast<uintptr_t>(dst) & 15) == 0)) {
      *reinterpret_cast<double2*>(dst) = make_double2(ya[l], yb[l]);
    } else {
      dst[0] = ya[l];
      if (act_b) dst[1] = yb[l];
    }
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

// f(std::integral_constant<int, I>) for I = 0 .. COUNT-1: lets a loop body
// read the TDI table as constant expressions (no table loads, no run-time
// signs or channel indices).
template <int COUNT, int I = 0, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < COUNT) {
    f(std::integral_constant<int, I>{});
    static_for<COUNT, I + 1>(f);
  }
}

// Delay groups as a run-time table in constant memory: the kernels loop over
// groups without unrolling, so only one group's state is live at a time.
// Rows are ordered by channel: for channel c, rows [first[c], comb[c]) have
// one use, rows [comb[c], first[c + 1]) two uses of that same channel (their
// two link series are combined before the interpolation); rows [first[3], n)
// feed two different channels.  The general fields (nuse, link, sgn) describe
// every row, for kernels that loop over all rows alike.
struct GroupRow {
  double cnt[6];       // light-time multiplicities of the group's delay
  int nuse;            // 1 or 2 delayed terms share the delay
  int link[2];         // measured link of each use
  double sgn[2][3];    // signed X, Y, Z selector of each use
  double sign;         // one-channel rows: sign of use 0
  double ratio;        // two uses of one channel: sign of use 1 / sign of use 0
};

template <int GEN>
struct GroupTable {
  GroupRow row[3 * TdiTable<GEN>::kTermsPerChan];
  int n;
  int chain;           // longest chain of link delays (3 or 7)
  int first[4];        // see above
  int comb[3];
};

template <int GEN>
constexpr GroupTable<GEN> make_group_table() {
  constexpr TdiTable<GEN> t = make_tdi_table<GEN>();
  GroupTable<GEN> r{};
  r.n = 0;
  r.chain = GEN == 1 ? 3 : 7;
  auto add = [&r, &t](int g) {
    GroupRow& row = r.row[r.n++];
    for (int l = 0; l < 6; ++l) row.cnt[l] = (double)t.group[g].cnt[l];
    row.nuse = t.group[g].nuse;
    for (int k = 0; k < t.group[g].nuse; ++k) {
      row.link[k] = t.group[g].use[k].link;
      for (int c = 0; c < 3; ++c)
        row.sgn[k][c] = t.group[g].use[k].chan == c ? (double)t.group[g].use[k].sign : 0.0;
    }
    row.sign = (double)t.group[g].use[0].sign;
    row.ratio = t.group[g].nuse == 2
                    ? (double)(t.group[g].use[1].sign * t.group[g].use[0].sign) : 0.0;
  };
  auto one_chan = [&t](int g, int c) {
    for (int k = 0; k < t.group[g].nuse; ++k)
      if (t.group[g].use[k].chan != c) return false;
    return true;
  };
  for (int c = 0; c < 3; ++c) {
    r.first[c] = r.n;
    for (int g = 0; g < t.ngroup; ++g)
      if (t.group[g].nuse == 1 && one_chan(g, c)) add(g);
    r.comb[c] = r.n;
    for (int g = 0; g < t.ngroup; ++g)
      if (t.group[g].nuse == 2 && one_chan(g, c)) add(g);
  }
  r.first[3] = r.n;
  for (int g = 0; g < t.ngroup; ++g) {
    bool single = false;
    for (int c = 0; c < 3; ++c) single = single || (t.group[g].nuse <= 2 && one_chan(g, c));
    if (!single) add(g);
  }
  return r;
}

static __constant__ GroupTable<1> kGroups1 = make_group_table<1>();
static __constant__ GroupTable<2> kGroups2 = make_group_table<2>();

template <int GEN>
__device__ __forceinline__ const GroupTable<GEN>& group_table();
template <>
__device__ __forceinline__ const GroupTable<1>& group_table<1>() { return kGroups1; }
template <>
__device__ __forceinline__ const GroupTable<2>& group_table<2>() { return kGroups2; }

__device__ __forceinline__ double row_delay(const GroupRow& g, const double (&L)[6]) {
  double d = 0.0;
#pragma unroll
  for (int l = 0; l < 6; ++l) d = fma(g.cnt[l], L[l], d);
  return d;
}

// Safe bounds of every group delay from the light times: a delay is a sum of
// 1..chain link light times.
__device__ __forceinline__ void group_delay_bounds(const double (&L)[6], int chain, double& dlo,
                                                   double& dhi) {
  double lmin = L[0], lmax = L[0];
#pragma unroll
  for (int l = 1; l < 6; ++l) { lmin = fmin(lmin, L[l]); lmax = fmax(lmax, L[l]); }
  dlo = fmin(lmin, chain * lmin);
  dhi = fmax(lmax, chain * lmax);
}

// S series that share one delay, for both samples of a lane: load(s, i)
// returns series s at window element i (a parity-split LDS position).  sa_
// starts sample a's stencil; if `same`, sample b's stencil is the next window
// position, otherwise it starts at element jb0.  One LagrangePair serves all
// S series of both samples.  Returns the streams' unscaled values
// (LagrangeStream<N>::finish scales).
template <int N, int CAP, int S, class Load>
__device__ __forceinline__ void stream_series(double ea, double eb, bool same, const Load& load,
                                              const ParStream<CAP>& sa_, int jb0,
                                              double (&xa)[S], double (&xb)[S]) {
  LagrangePair<N> P(ea, eb);
#pragma unroll
  for (int s = 0; s < S; ++s) { xa[s] = 0.0; xb[s] = 0.0; }
  if (same) {
    double cur[S];
#pragma unroll
    for (int s = 0; s < S; ++s) cur[s] = load(s, sa_.at(0));
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double nxt[S];
#pragma unroll
      for (int s = 0; s < S; ++s) nxt[s] = load(s, sa_.at(k + 1));
      P.tap(k);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        xa[s] = P.step_a(xa[s], cur[s], k);
        xb[s] = P.step_b(xb[s], nxt[s], k);
        cur[s] = nxt[s];
      }
    }
  } else {
    const ParStream<CAP> sb_(jb0);             // only here: most waves take `same`
#pragma unroll
    for (int k = 0; k < N; ++k) {
      P.tap(k);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        xa[s] = P.step_a(xa[s], load(s, sa_.at(k)), k);
        xb[s] = P.step_b(xb[s], load(s, sb_.at(k)), k);
      }
    }
  }
}

// S series from parity-split LDS rows w[s] (measured links, possibly of
// several templates).
template <int N, int CAP, int S>
__device__ __forceinline__ void stream_multi(double ea, double eb, bool same,
                                             const double* const (&w)[S],
                                             const ParStream<CAP>& sa_, int jb0,
                                             double (&xa)[S], double (&xb)[S]) {
  stream_series<N, CAP, S>(ea, eb, same, [&w](int s, int i) { return w[s][i]; }, sa_, jb0, xa,
                           xb);
}

// Global-memory version for one sample (clamped indices).
template <int N>
__device__ __forceinline__ double stream_global(double eps, const double* ys, int64_t j0,
                                                int64_t n) {
  LagrangeStream<N> A(eps);
  double x = 0.0;
#pragma unroll 1
  for (int k = 0; k < N; ++k) {
    int64_t j = j0 + k;
    j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
    A.tap(k);
    x = A.step(x, ys[j], k);
  }
  return x;                         // unscaled, like stream_pair
}

__device__ __forceinline__ void light_times(const OrbitView& o, double tau, double (&L)[6]) {
  orbit_series<9, 6>(o, tau, L);
}

template <int N, int GEN>
__global__ __launch_bounds__(kBlock, LR_TDI_MIN_WAVES) void tdi_kernel(TdiArgs a) {
  constexpr int H = N / 2;
  constexpr int CAP = kFwdTile + N + kSlack;
  constexpr int ND = TdiTab<GEN>::v.ndirect;
  const GroupTable<GEN>& GT = group_table<GEN>();
  __shared__ double win[6 * CAP];
  __shared__ int red[2][kBlock / 64];

  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kFwdTile;
  const int last = (int)min((int64_t)(kFwdTile - 1), a.n_out - 1 - i0);
  const bool act_a = kPerLane * tid <= last, act_b = kPerLane * tid + 1 <= last;
  const int ra = act_a ? kPerLane * tid : last;
  const int64_t pa = a.out_start + i0 + ra;          // y-index of sample a; b is pa + 1

  double La[6], Lb[6];
  light_times(a.orb, a.t_off + (double)pa * a.dt, La);
  light_times(a.orb, a.t_off + (double)(pa + 1) * a.dt, Lb);

  double dlo_a, dhi_a, dlo_b, dhi_b;
  group_delay_bounds(La, GT.chain, dlo_a, dhi_a);
  group_delay_bounds(Lb, GT.chain, dlo_b, dhi_b);
  double e_unused;
  const int lo = min(0, min(split_delay(dhi_a, a.inv_dt, e_unused),
                            split_delay(dhi_b, a.inv_dt, e_unused) + 1) - (H - 1));
  const int hi = max(1, max(split_delay(dlo_a, a.inv_dt, e_unused),
                            split_delay(dlo_b, a.inv_dt, e_unused) + 1) + H);
  int wlo, whi;
  block_range<kBlock>(ra + lo, ra + hi, red, wlo, whi);
  const int count = whi - wlo + 1;
  const int64_t base = a.out_start + i0 + wlo;
  const int64_t ymax = a.n_y - 1;
  const int c0 = ra - wlo;

  // delayed terms accumulate unscaled streams; the undelayed ones are added
  // after the scale, at the end
  double acc_a[3] = {0.0, 0.0, 0.0}, acc_b[3] = {0.0, 0.0, 0.0};
  double dir_a[3] = {0.0, 0.0, 0.0}, dir_b[3] = {0.0, 0.0, 0.0};
  const bool lds = count > 0 && count <= CAP;
  if (lds) {
    for (int k = tid; k < count; k += kBlock) {
      int64_t j = base + k;
      j = j < 0 ? 0 : (j > ymax ? ymax : j);
#pragma unroll
      for (int l = 0; l < 6; ++l) win[l * CAP + par<CAP>(k)] = a.y[(int64_t)l * a.n_y + j];
    }
    __syncthreads();
    // rows that feed one channel c: a one-link group adds one stream to
    // acc[c]; a two-link group of one channel interpolates the signed sum of
    // its two link series (the same delay, so the same weights)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll 1
      for (int g = GT.first[c]; g < GT.comb[c]; ++g) {
        const GroupRow& G = GT.row[g];
        double ea, eb;
        const int sa = split_delay(row_delay(G, La), a.inv_dt, ea);
        const int sb = split_delay(row_delay(G, Lb), a.inv_dt, eb);
        const bool same = __all(sa == sb);
        const ParStream<CAP> pa_(c0 + sa - (H - 1));
        const double* const w0 = win + G.link[0] * CAP;
        double xa[1], xb[1];
        stream_series<N, CAP, 1>(ea, eb, same, [w0](int, int i) { return w0[i]; }, pa_,
                                 c0 + 1 + sb - (H - 1), xa, xb);
        acc_a[c] = fma(G.sign, xa[0], acc_a[c]);
        acc_b[c] = fma(G.sign, xb[0], acc_b[c]);
      }
#pragma unroll 1
      for (int g = GT.comb[c]; g < GT.first[c + 1]; ++g) {
        const GroupRow& G = GT.row[g];
        double ea, eb;
        const int sa = split_delay(row_delay(G, La), a.inv_dt, ea);
        const int sb = split_delay(row_delay(G, Lb), a.inv_dt, eb);
        const bool same = __all(sa == sb);
        const ParStream<CAP> pa_(c0 + sa - (H - 1));
        const double* const w0 = win + G.link[0] * CAP;
        const double* const w1 = win + G.link[1] * CAP;
        const double q = G.ratio;
        double xa[1], xb[1];
        stream_series<N, CAP, 1>(ea, eb, same,
                                 [w0, w1, q](int, int i) { return fma(q, w1[i], w0[i]); }, pa_,
                                 c0 + 1 + sb - (H - 1), xa, xb);
        acc_a[c] = fma(G.sign, xa[0], acc_a[c]);
        acc_b[c] = fma(G.sign, xb[0], acc_b[c]);
      }
    }
    // two-link groups whose uses feed different channels
#pragma unroll 1
    for (int g = GT.first[3]; g < GT.n; ++g) {
      const GroupRow& G = GT.row[g];
      double ea, eb;
      const int sa = split_delay(row_delay(G, La), a.inv_dt, ea);
      const int sb = split_delay(row_delay(G, Lb), a.inv_dt, eb);
      const bool same = __all(sa == sb);
      const ParStream<CAP> pa_(c0 + sa - (H - 1));
      const int jb0 = c0 + 1 + sb - (H - 1);
      const double* const w[2] = {win + G.link[0] * CAP, win + G.link[1] * CAP};
      double xa[2], xb[2];
      stream_multi<N, CAP, 2>(ea, eb, same, w, pa_, jb0, xa, xb);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc_a[c] = fma(G.sgn[0][c], xa[0], fma(G.sgn[1][c], xa[1], acc_a[c]));
        acc_b[c] = fma(G.sgn[0][c], xb[0], fma(G.sgn[1][c], xb[1], acc_b[c]));
      }
    }
  } else {
#pragma unroll 1
    for (int g = 0; g < GT.n; ++g) {
      const GroupRow& G = GT.row[g];
      double ea, eb;
      const int sa = split_delay(row_delay(G, La), a.inv_dt, ea);
      const int sb = split_delay(row_delay(G, Lb), a.inv_dt, eb);
#pragma unroll 1
      for (int k = 0; k < G.nuse; ++k) {
        const double* ys = a.y + (int64_t)G.link[k] * a.n_y;
        const double xa = stream_global<N>(ea, ys, pa + sa - (H - 1), a.n_y);
        const double xb = stream_global<N>(eb, ys, pa + 1 + sb - (H - 1), a.n_y);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc_a[c] = fma(G.sgn[k][c], xa, acc_a[c]);
          acc_b[c] = fma(G.sgn[k][c], xb, acc_b[c]);
        }
      }
    }
  }

  // the sample indices again from the lane's tile row: an opaque copy keeps
  // the compiler from holding the 64-bit indices in registers through the
  // group loops (they spilled at the four-wave budget)
  int rl = ra;
  asm volatile("" : "+v"(rl));
  const int64_t pl = a.out_start + i0 + rl;
#pragma unroll
  for (int t = 0; t < ND; ++t) {
    const Direct dr = TdiTab<GEN>::v.direct[t];
    if (lds) {
      dir_a[dr.chan] += (double)dr.sign * win[dr.link * CAP + par<CAP>(c0)];
      dir_b[dr.chan] += (double)dr.sign * win[dr.link * CAP + par<CAP>(c0 + 1)];
    } else {
      const double* ys = a.y + (int64_t)dr.link * a.n_y;
      dir_a[dr.chan] += (double)dr.sign * ys[pl];
      dir_b[dr.chan] += (double)dr.sign * ys[min(pl + 1, ymax)];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc_a[c] = fma(LagrangeStream<N>::kScale, acc_a[c], dir_a[c]);
    acc_b[c] = fma(LagrangeStream<N>::kScale, acc_b[c], dir_b[c]);
  }
  if (!act_a) return;
  const int64_t i = i0 + rl;
  store_channels(acc_a, a.channels, a.out, a.n_out, i);
  if (act_b) store_channels(acc_b, a.channels, a.out, a.n_out, i + 1);
}

// ---------------------------------------------------------------------------
// Launchers (explicitly instantiated per tap count in forward_*.hip)
// ---------------------------------------------------------------------------
template <int N>
hipError_t launch_project(const ProjArgs& a, hipStream_t s) {
  const int64_t blocks = (a.n_y + kFwdTile - 1) / kFwdTile;
  hipLaunchKernelGGL(project_links_kernel<N>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_tdi(const TdiArgs& a, int gen, hipStream_t s) {
  const int64_t blocks = (a.n_out + kFwdTile - 1) / kFwdTile;
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
