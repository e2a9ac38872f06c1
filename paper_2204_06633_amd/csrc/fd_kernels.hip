// Frequency-domain noise-weighted likelihood (Sec. II.A: the inner product
// weighted by the one-sided noise PSD, log L = -<d-h|d-h>/2, the optimal
// and extraction SNRs) for batches of A/E/T channel series.
//
// Each template contributes complex signals of N = 2^p points: A + iE, and
// T + i0 when T is used (A and E share one noise curve, so the weighted sum
// of |A~ + iE~|^2 over the full spectrum splits into the two channels' sums:
// the cross terms cancel between bins k and N - k).  The FFT of a signal is
// one to three passes over HBM; every pass transforms 4096-point tiles in
// LDS: one line of R = 2^q points along axis s of the [A][R][B] view of the
// signal, C = 4096 / R lines per tile (C adjacent columns when B > 1, so
// every global access is a run of C consecutive elements; C rows when B = 1).
// The DFT along a line is a Stockham sequence of radix-4/8/16 stages with
// the butterflies in registers.  Between passes the elements are multiplied
// by exp(-2 pi i k_s b / (R B)) (the four-step decomposition); the spectrum
// stays in the resulting digit-permuted order, which the data spectrum and
// the weights share.  The last forward pass applies the weights and sums
// rr, hh, dh per tile, and for the gradient multiplies by the weights and
// starts the inverse transform at once; the inverse passes run the forward
// passes' transposes in reverse order back to the time series.
#include "internal.hpp"
#include "fd_types.hpp"

namespace lr {
namespace fd {

constexpr int kThreads = 256;
constexpr int kTile = 4096;                 // complex points per workgroup
constexpr int kPer = kTile / kThreads;      // points per thread

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}

// exp(-2 pi i idx / N) from the two-level table (idx < N <= 2^24).
__device__ __forceinline__ double2 twiddle(const double2* lo, const double2* hi, int idx) {
  return cmul(hi[idx >> 12], lo[idx & 4095]);
}

constexpr int bit_reverse(int k, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r = (r << 1) | ((k >> i) & 1);
  return r;
}

// t *= exp(-+2 pi i e / 16) (forward: minus), e compile-time after unrolling.
template <bool INV>
__device__ __forceinline__ void rotate16(double2& t, int e) {
  constexpr double c8 = 0.9238795325112867, s8 = 0.3826834323650898, r2 = 0.7071067811865476;
  if (e == 0) return;
  if (e == 4) {  // -i (forward) or +i (inverse)
    t = INV ? make_double2(-t.y, t.x) : make_double2(t.y, -t.x);
    return;
  }
  double c, s;
  switch (e) {
    case 1: c = c8; s = s8; break;
    case 2: c = r2; s = r2; break;
    case 3: c = s8; s = c8; break;
    case 5: c = -s8; s = c8; break;
    case 6: c = -r2; s = r2; break;
    default: c = -c8; s = s8; break;   // 7
  }
  t = cmul(t, make_double2(c, INV ? s : -s));
}

// In-register DFT of RHO <= 16 points by radix-2 decimation in frequency:
// natural order in, bit-reversed order out.
template <int RHO, bool INV>
__device__ __forceinline__ void dft(double2 (&v)[RHO]) {
#pragma unroll
  for (int half = RHO / 2; half >= 1; half >>= 1) {
#pragma unroll
    for (int s = 0; s < RHO; s += 2 * half) {
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const double2 a = v[s + i], b = v[s + i + half];
        v[s + i] = cadd(a, b);
        double2 t = csub(a, b);
        rotate16<INV>(t, i * (RHO / (2 * half)) * (16 / RHO));
        v[s + i + half] = t;
      }
    }
  }
}

// Stages of a line of 2^Q points: ceil(Q / 4) radix-2^b stages, larger
// radices first (Q = 5: 8, 4; 6: 8, 8; 7: 16, 8; 8: 16, 16; 12: 16, 16, 16).
constexpr int num_stages(int q) { return (q + 3) >> 2; }
constexpr int stage_bits(int q, int s) {
  int nst = num_stages(q), rem = q;
  for (int i = 0; i < s; ++i) rem -= (rem + (nst - i) - 1) / (nst - i);
  return (rem + (nst - s) - 1) / (nst - s);
}

// LDS layout: line c at c * line_stride, element x at x + x / 16 (one pad
// per 16 elements, and an odd line stride in 16-byte units, LR_FD_LS_EXTRA
// in fd_types.hpp), so that the strided stage writes and the column-wise
// accesses hit distinct banks.
constexpr int line_stride(int q) { return (1 << q) + (1 << q) / 16 + LR_FD_LS_EXTRA; }
__device__ __forceinline__ int lpad(int x) { return x + (x >> 4); }

// Where a tile's elements live: element (line c, index r) of the tile is at
// base + c * cstep + r * rstep of its signal; b0 + c is the inner index b of
// a column line (column mode: C adjacent columns of the [A][R][B] view;
// row mode, B = 1: C consecutive rows).
struct Tile {
  bool col;
  int logA;
  int64_t base, b0, cstep, rstep;
};

// Butterfly u of this thread in a radix-2^LR stage: line c and index j.
// Column mode puts consecutive lines on consecutive lanes (global accesses
// are runs of C elements), row mode consecutive j (runs of R / 2^LR).
template <int Q, int LR>
__device__ __forceinline__ void coords(bool col, int u, int& c, int& j) {
  constexpr int logC = 12 - Q, PL = Q - LR;
  const int beta = (int)threadIdx.x + kThreads * u;
  if (col) {
    c = beta & ((1 << logC) - 1);
    j = beta >> logC;
  } else {
    j = beta & ((1 << PL) - 1);
    c = beta >> PL;
  }
}

template <bool IN_REAL>
__device__ __forceinline__ double2 load_elem(const PassArgs& a, const double2* x, int64_t pos,
                                             int64_t tpl, int kind) {
  if (!IN_REAL) return x[pos];
  double2 v = make_double2(0.0, 0.0);
  if (pos < a.n) {
    const double* h = a.h + tpl * a.t_stride + pos;
    if (kind == 0) v = make_double2(h[0], h[a.c_stride]);
    else v.x = h[2 * a.c_stride];
  }
  return v;
}

// First stage (sub-transforms of one point, no twiddle) straight from
// global memory, output to LDS.  PRETW: the transpose of the forward
// inter-pass twiddle, applied before an inverse line transform.
template <int Q, int LR, bool IN_REAL, bool INV>
__device__ __forceinline__ void first_stage(const PassArgs& a, const Tile& T, const double2* x,
                                            int64_t tpl, int kind, bool pretw, double2* lds) {
  constexpr int RHO = 1 << LR, BPT = kPer / RHO, PL = Q - LR, LS = line_stride(Q);
  double2 v[BPT][RHO];
  int cc[BPT], jj[BPT];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    coords<Q, LR>(T.col, u, cc[u], jj[u]);
#pragma unroll
    for (int k = 0; k < RHO; ++k) {
      const int r = jj[u] + (k << PL);
      v[u][k] = load_elem<IN_REAL>(a, x, T.base + cc[u] * T.cstep + r * T.rstep, tpl, kind);
    }
  }
  if (pretw) {
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      // conj(exp(-2 pi i r b / (R B))) for r = j + k R / RHO: w0 * step^k
      const int64_t b = T.b0 + cc[u];
      double2 w = twiddle(a.tlo, a.thi, (int)(((int64_t)jj[u] * b) << T.logA));
      double2 st = twiddle(a.tlo, a.thi, (int)((b << PL) << T.logA));
      w.y = -w.y;
      st.y = -st.y;
#pragma unroll
      for (int k = 0; k < RHO; ++k) {
        v[u][k] = cmul(v[u][k], w);
        if (k + 1 < RHO) w = cmul(w, st);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    dft<RHO, INV>(v[u]);
#pragma unroll
    for (int k = 0; k < RHO; ++k)
      lds[cc[u] * LS + lpad((jj[u] << LR) + k)] = v[u][bit_reverse(k, LR)];
  }
}

// A middle Stockham stage, LDS to LDS (sub-transforms of 2^ns_log points
// done); lanes take consecutive butterflies of a line.
template <int Q, int LR, bool INV>
__device__ __forceinline__ void mid_stage(double2* lds, int ns_log, int logN, const double2* tlo,
                                          const double2* thi) {
  constexpr int RHO = 1 << LR, BPT = kPer / RHO, PL = Q - LR, LS = line_stride(Q);
  const int ns_mask = (1 << ns_log) - 1;
  double2 v[BPT][RHO];
  int cd[BPT], xd[BPT];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    int c, j;
    coords<Q, LR>(false, u, c, j);
#pragma unroll
    for (int k = 0; k < RHO; ++k) v[u][k] = lds[c * LS + lpad(j + (k << PL))];
    const int m = j & ns_mask;
    if (m != 0) {
      double2 w = twiddle(tlo, thi, m << (logN - ns_log - LR));
      if (INV) w.y = -w.y;
      double2 wk = w;
#pragma unroll
      for (int k = 1; k < RHO; ++k) {
        v[u][k] = cmul(v[u][k], wk);
        if (k + 1 < RHO) wk = cmul(wk, w);
      }
    }
    dft<RHO, INV>(v[u]);
    cd[u] = c * LS;
    xd[u] = ((j >> ns_log) << (ns_log + LR)) | m;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
#pragma unroll
    for (int k = 0; k < RHO; ++k) lds[cd[u] + lpad(xd[u] + (k << ns_log))] = v[u][bit_reverse(k, LR)];
  }
  __syncthreads();
}

// Last stage, LDS to registers: sub-transforms of R / 2^LR points done, so
// butterfly j's twiddles are exp(-+2 pi i j k / R) and its outputs are the
// line's elements j + k R / 2^LR in natural order: o[u * RHO + k].
template <int Q, int LR, bool INV>
__device__ __forceinline__ void last_stage(bool col, const double2* lds, int logN,
                                           const double2* tlo, const double2* thi,
                                           double2 (&o)[kPer]) {
  constexpr int RHO = 1 << LR, BPT = kPer / RHO, PL = Q - LR, LS = line_stride(Q);
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    int c, j;
    coords<Q, LR>(col, u, c, j);
    double2 v[RHO];
#pragma unroll
    for (int k = 0; k < RHO; ++k) v[k] = lds[c * LS + lpad(j + (k << PL))];
    if (j != 0) {
      double2 w = twiddle(tlo, thi, j << (logN - Q));
      if (INV) w.y = -w.y;
      double2 wk = w;
#pragma unroll
      for (int k = 1; k < RHO; ++k) {
        v[k] = cmul(v[k], wk);
        if (k + 1 < RHO) wk = cmul(wk, w);
      }
    }
    dft<RHO, INV>(v);
#pragma unroll
    for (int k = 0; k < RHO; ++k) o[u * RHO + k] = v[bit_reverse(k, LR)];
  }
}

// Store the last stage's outputs (POSTTW: the forward inter-pass twiddle).
template <int Q, int LR, bool OUT_REAL>
__device__ __forceinline__ void store_out(const PassArgs& a, const Tile& T, double2* x,
                                          int64_t tpl, int kind, bool posttw,
                                          const double2 (&o)[kPer]) {
  constexpr int RHO = 1 << LR, BPT = kPer / RHO, PL = Q - LR;
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    int c, j;
    coords<Q, LR>(T.col, u, c, j);
    // exp(-2 pi i r b / (R B)) for r = j + k R / RHO: w0 * step^k
    double2 w = make_double2(1.0, 0.0), st = w;
    if (posttw) {
      const int64_t b = T.b0 + c;
      w = twiddle(a.tlo, a.thi, (int)(((int64_t)j * b) << T.logA));
      st = twiddle(a.tlo, a.thi, (int)((b << PL) << T.logA));
    }
#pragma unroll
    for (int k = 0; k < RHO; ++k) {
      const int r = j + (k << PL);
      const int64_t pos = T.base + c * T.cstep + r * T.rstep;
      double2 val = o[u * RHO + k];
      if (posttw) {
        val = cmul(val, w);
        if (k + 1 < RHO) w = cmul(w, st);
      }
      if (OUT_REAL) {
        if (pos < a.n) {
          double* g = a.g + tpl * a.t_stride + pos;
          if (kind == 0) { g[0] = val.x; g[a.c_stride] = val.y; }
          else g[2 * a.c_stride] = val.x;
        }
      } else {
        x[pos] = val;
      }
    }
  }
}

// One pass over lines of 2^Q points.  IN_REAL: the signals are read from
// the channel series (first forward pass); OUT_REAL: written to channel
// series (last inverse pass); SPEC: 0 a plain pass in direction INV; 1 the
// forward line transform and the weighted sums; 2 also the weighted
// residual and its inverse line transform (stage order reversed, so that
// its first stage runs on the registers the forward transform ended with).
template <int Q, bool IN_REAL, bool OUT_REAL, int SPEC, bool INV>
__global__ __launch_bounds__(kThreads) void fft_pass_kernel(PassArgs a) {
  constexpr int NST = num_stages(Q);
  constexpr int LS = line_stride(Q);
  constexpr int logC = 12 - Q;
  constexpr int R = 1 << Q;
  constexpr bool DIR = INV && SPEC == 0;      // direction of the first line transform
  constexpr int LR0 = stage_bits(Q, 0), LRL = stage_bits(Q, NST - 1);
  __shared__ double2 lds[(kTile >> Q) * LS];
  const int tid = threadIdx.x;
  const int64_t N = (int64_t)1 << a.logN;
  // Tile tau = signal * tiles per signal + tile position.  The last forward
  // pass reads the data spectrum and weights at the tile's positions, the
  // same for every template: work-groups go to the 8 XCDs (separate L2s) in
  // turn, so each XCD takes a contiguous run of work indices ordered
  // (position, kind, template), and consecutive groups on one XCD share the
  // spectrum and weights through its L2.
  int64_t tau = blockIdx.x;
  if (SPEC > 0 && a.n_tpl > 1 && (gridDim.x & 7) == 0) {
    const int64_t per = gridDim.x >> 3;
    const int64_t w = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int64_t t = w % a.n_tpl, rest = w / a.n_tpl;
    const int64_t kd = rest % a.sig_per_tpl, pos = rest / a.sig_per_tpl;
    tau = ((t * a.sig_per_tpl + kd) << a.tiles_log) + pos;
  }
  const int64_t sig = tau >> a.tiles_log;
  const int64_t tp = tau & (((int64_t)1 << a.tiles_log) - 1);

  Tile T;
  T.col = a.logB > 0;
  T.logA = a.logN - Q - a.logB;
  if (T.col) {
    const int logTa = a.logB - logC;          // tiles per index a
    const int64_t aa = tp >> logTa;
    T.b0 = (tp & (((int64_t)1 << logTa) - 1)) << logC;
    T.base = (aa << (Q + a.logB)) + T.b0;
    T.cstep = 1;
    T.rstep = (int64_t)1 << a.logB;
  } else {
    T.b0 = 0;
    T.base = tp << 12;
    T.cstep = R;
    T.rstep = 1;
  }
  const int64_t tpl = sig / a.sig_per_tpl;
  const int kind = (int)(sig - tpl * a.sig_per_tpl);   // 0: A + iE, 1: T
  double2* x = a.x + sig * N;

  first_stage<Q, LR0, IN_REAL, DIR>(a, T, x, tpl, kind, DIR && a.twiddle, lds);
  __syncthreads();
  if (NST == 3) mid_stage<Q, stage_bits(Q, 1), DIR>(lds, LR0, a.logN, a.tlo, a.thi);
  double2 o[kPer];
  last_stage<Q, LRL, DIR>(T.col, lds, a.logN, a.tlo, a.thi, o);
  if (SPEC == 0) {
    store_out<Q, LRL, OUT_REAL>(a, T, x, tpl, kind, !INV && a.twiddle, o);
    return;
  }

  // ---- weighted sums over this tile's bins (row mode)
  constexpr int RHO = 1 << LRL, BPT = kPer / RHO, PL = Q - LRL;
  double acc[3] = {0.0, 0.0, 0.0};
  const double2* D = a.dspec + kind * N;
  const double* W = a.wpos + kind * N;
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    int c, j;
    coords<Q, LRL>(false, u, c, j);
#pragma unroll
    for (int k = 0; k < RHO; ++k) {
      const int64_t pos = T.base + c * R + j + (k << PL);
      const double2 H = o[u * RHO + k];
      const double2 Dv = D[pos];
      const double w = W[pos];
      const double2 Z = csub(Dv, H);
      acc[0] = fma(w, fma(Z.x, Z.x, Z.y * Z.y), acc[0]);
      acc[1] = fma(w, fma(H.x, H.x, H.y * H.y), acc[1]);
      acc[2] = fma(w, fma(Dv.x, H.x, Dv.y * H.y), acc[2]);
      if (SPEC == 2) o[u * RHO + k] = make_double2(w * Z.x, w * Z.y);
    }
  }
  // fixed-order sums: a shuffle tree within each wave, then the waves in
  // order (the now free LDS holds the wave partials)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_down(acc[i], off);
  }
  double* red = reinterpret_cast<double*>(lds);
  __syncthreads();
  if ((tid & 63) == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) red[(tid >> 6) * 3 + i] = acc[i];
  }
  __syncthreads();
  if (tid == 0) {
    double* p = a.part + 3 * tau;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double t = red[i];
#pragma unroll
      for (int w = 1; w < kThreads / 64; ++w) t += red[w * 3 + i];
      p[i] = t;
    }
  }
  if (SPEC == 1) return;
  __syncthreads();

  // ---- inverse line transform of the weighted residual: stages reversed
  {
    constexpr int LS_ = LS;
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      int c, j;
      coords<Q, LRL>(false, u, c, j);
      double2 v[RHO];
#pragma unroll
      for (int k = 0; k < RHO; ++k) v[k] = o[u * RHO + k];
      dft<RHO, true>(v);
#pragma unroll
      for (int k = 0; k < RHO; ++k) lds[c * LS_ + lpad((j << LRL) + k)] = v[bit_reverse(k, LRL)];
    }
  }
  __syncthreads();
  if (NST == 3) mid_stage<Q, stage_bits(Q, 1), true>(lds, LRL, a.logN, a.tlo, a.thi);
  last_stage<Q, LR0, true>(false, lds, a.logN, a.tlo, a.thi, o);
  store_out<Q, LR0, OUT_REAL>(a, T, x, tpl, kind, false, o);
}

// Fixed-order sum of three per-thread values over the workgroup.
__device__ __forceinline__ void block_sum3(double (&v)[3], double (&red)[3][kThreads]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 3; ++j) red[j][tid] = v[j];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int j = 0; j < 3; ++j) red[j][tid] += red[j][tid + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) v[j] = red[j][0];
}

// stats[t] = (rr, hh, dh): the partial sums of template t's signals and
// tiles in a fixed order (one workgroup per template).
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double* part, int64_t per_tpl,
                                                            double* stats) {
  __shared__ double red[3][kThreads];
  const int64_t t = blockIdx.x;
  const double* p = part + 3 * t * per_tpl;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t k = threadIdx.x; k < per_tpl; k += kThreads) {
    acc[0] += p[3 * k];
    acc[1] += p[3 * k + 1];
    acc[2] += p[3 * k + 2];
  }
  block_sum3(acc, red);
  if (threadIdx.x == 0) {
    stats[3 * t] = acc[0];
    stats[3 * t + 1] = acc[1];
    stats[3 * t + 2] = acc[2];
  }
}

// lo[j] = exp(-2 pi i j / N) for j < min(N, 4096); hi[i] = exp(-2 pi i 4096 i / N).
__global__ void twiddle_kernel(double2* lo, double2* hi, int logN) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)1 << logN;
  const int64_t nlo = N < 4096 ? N : 4096, nhi = N > 4096 ? N / 4096 : 1;
  double s, c;
  if (k < nlo) {
    sincospi(2.0 * (double)k / (double)N, &s, &c);   // exact argument: N is a power of two
    lo[k] = make_double2(c, -s);
  } else if (k < nlo + nhi) {
    const int64_t i = k - nlo;
    sincospi(2.0 * (double)(i * 4096) / (double)N, &s, &c);
    hi[i] = make_double2(c, -s);
  }
}

// Weights in the transform's output order: position -> bin k (mixed-radix
// digit reversal of the pass sizes), two-sided weight W_k = w_|k| / 2 off
// DC and Nyquist, times dt^2 (the spectra are plain DFTs).
__global__ void weights_kernel(double* wpos, const double* w_ae, const double* w_t, int logN,
                               int passes, int q0, int q1, int q2, double dt2) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)1 << logN;
  if (pos >= N) return;
  const int qs[3] = {q0, q1, q2};
  int64_t bin = 0;
  int shift = logN, low = 0;
  for (int s = 0; s < passes; ++s) {
    shift -= qs[s];
    const int64_t ks = (pos >> shift) & ((1 << qs[s]) - 1);
    bin |= ks << low;
    low += qs[s];
  }
  const int64_t kk = bin <= N / 2 ? bin : N - bin;
  const double f = (kk == 0 || 2 * kk == N) ? dt2 : 0.5 * dt2;
  wpos[pos] = f * w_ae[kk];
  wpos[N + pos] = w_t ? f * w_t[kk] : 0.0;
}

}  // namespace fd

using fd::PassArgs;

template <int Q>
static void launch_q(const PassArgs& a, dim3 grid, bool in_real, bool out_real, int spec,
                     bool inv, hipStream_t s) {
  const dim3 block(fd::kThreads);
#define LR_FD_LAUNCH(IR, OR, SP, IV) \
  hipLaunchKernelGGL((fd::fft_pass_kernel<Q, IR, OR, SP, IV>), grid, block, 0, s, a)
  if (spec == 0 && !inv) {
    if (in_real) LR_FD_LAUNCH(true, false, 0, false);
    else LR_FD_LAUNCH(false, false, 0, false);
  } else if (spec == 0) {
    if (out_real) LR_FD_LAUNCH(false, true, 0, true);
    else LR_FD_LAUNCH(false, false, 0, true);
  } else if (spec == 1) {
    if (in_real) LR_FD_LAUNCH(true, false, 1, false);
    else LR_FD_LAUNCH(false, false, 1, false);
  } else {
    if (in_real) LR_FD_LAUNCH(true, true, 2, false);
    else LR_FD_LAUNCH(false, false, 2, false);
  }
#undef LR_FD_LAUNCH
}

static hipError_t launch_pass(const PassArgs& a, int64_t tiles, bool in_real, bool out_real,
                              int spec, bool inv, hipStream_t s) {
  const dim3 grid((unsigned)tiles);
  switch (a.q) {
    case 5: launch_q<5>(a, grid, in_real, out_real, spec, inv, s); break;
    case 6: launch_q<6>(a, grid, in_real, out_real, spec, inv, s); break;
    case 7: launch_q<7>(a, grid, in_real, out_real, spec, inv, s); break;
    case 8: launch_q<8>(a, grid, in_real, out_real, spec, inv, s); break;
    case 12: launch_q<12>(a, grid, in_real, out_real, spec, inv, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Geometry of pass s (0-based) of the plan.
static void pass_geometry(const FdGeometry& g, int s, PassArgs& a) {
  a.logN = g.logN;
  a.q = g.q[s];
  int inner = 0;
  for (int i = s + 1; i < g.passes; ++i) inner += g.q[i];
  a.logB = inner;
  a.tiles_log = g.logN - 12;
}

hipError_t run_fd_prepare(const FdGeometry& g, const FdBuffers& b, const double* data,
                          int64_t data_cstride, const double* w_ae, const double* w_t, double dt,
                          hipStream_t s) {
  const int64_t N = (int64_t)1 << g.logN;
  {
    const int64_t n = 8192;
    hipLaunchKernelGGL(fd::twiddle_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       b.tlo, b.thi, g.logN);
  }
  hipLaunchKernelGGL(fd::weights_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                     b.wpos, w_ae, w_t, g.logN, g.passes, g.q[0], g.q[1], g.q[2], dt * dt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // data spectrum: the forward passes without the spectral step
  PassArgs a{};
  a.x = b.dspec;
  a.tlo = b.tlo;
  a.thi = b.thi;
  a.h = data;
  a.t_stride = 0;
  a.c_stride = data_cstride;
  a.n = g.n;
  a.sig_per_tpl = g.sig_per_tpl;
  const int64_t tiles = g.sig_per_tpl * (N >> 12);
  for (int p = 0; p < g.passes; ++p) {
    pass_geometry(g, p, a);
    a.twiddle = p + 1 < g.passes;
    e = launch_pass(a, tiles, p == 0, false, 0, false, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_fd_loglike(const FdGeometry& g, const FdBuffers& b, int64_t n_tpl, const double* h,
                          int64_t t_stride, int64_t c_stride, double* stats, double* g_h,
                          hipStream_t s) {
  const int64_t N = (int64_t)1 << g.logN;
  const int64_t tiles = n_tpl * g.sig_per_tpl * (N >> 12);
  PassArgs a{};
  a.x = b.work;
  a.tlo = b.tlo;
  a.thi = b.thi;
  a.h = h;
  a.g = g_h;
  a.t_stride = t_stride;
  a.c_stride = c_stride;
  a.n = g.n;
  a.sig_per_tpl = g.sig_per_tpl;
  a.dspec = b.dspec;
  a.wpos = b.wpos;
  a.part = b.part;
  a.n_tpl = n_tpl;
  const int P = g.passes;
  const int spec = g_h ? 2 : 1;
  hipError_t e;
  for (int p = 0; p + 1 < P; ++p) {              // forward passes before the last
    pass_geometry(g, p, a);
    a.twiddle = 1;
    e = launch_pass(a, tiles, p == 0, false, 0, false, s);
    if (e != hipSuccess) return e;
  }
  pass_geometry(g, P - 1, a);                      // last forward pass + spectrum
  a.twiddle = 0;
  e = launch_pass(a, tiles, P == 1, P == 1, spec, false, s);
  if (e != hipSuccess) return e;
  if (g_h) {
    for (int p = P - 2; p >= 0; --p) {             // inverse passes
      pass_geometry(g, p, a);
      a.twiddle = 1;
      e = launch_pass(a, tiles, false, p == 0, 0, true, s);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(fd::finalize_kernel, dim3((unsigned)n_tpl), dim3(fd::kThreads), 0, s, b.part,
                     g.sig_per_tpl * (N >> 12), stats);
  return hipGetLastError();
}

}  // namespace lr
