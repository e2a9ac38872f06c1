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
constexpr int kMaxLines = 128;              // lines per tile at R = 32

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

// One Stockham stage of radix 2^LR over all C lines of the tile (line c at
// lds + c * ls, R = 2^q points, sub-transforms of 2^ns_log points done).
template <int LR, bool INV>
__device__ __forceinline__ void stage(double2* lds, int q, int ls, int ns_log, int logN,
                                      const double2* tlo, const double2* thi) {
  constexpr int RHO = 1 << LR;
  constexpr int BPT = kPer / RHO;
  const int tid = threadIdx.x;
  const int pl_log = q - LR;                 // butterflies per line = R / RHO
  const int pl_mask = (1 << pl_log) - 1;
  const int ns_mask = (1 << ns_log) - 1;
  double2 v[BPT][RHO];
  int dst[BPT];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int beta = tid + kThreads * u;
    const int c = beta >> pl_log, j = beta & pl_mask;
    const double2* src = lds + c * ls + j;
#pragma unroll
    for (int k = 0; k < RHO; ++k) v[u][k] = src[k << pl_log];
    const int m = j & ns_mask;
    if (m != 0) {
      // exp(-2 pi i m k / (Ns RHO)), k = 1 .. RHO-1, by successive powers
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
    dst[u] = c * ls + (((j >> ns_log) << (ns_log + LR)) | m);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
#pragma unroll
    for (int k = 0; k < RHO; ++k) lds[dst[u] + (k << ns_log)] = v[u][bit_reverse(k, LR)];
  }
  __syncthreads();
}

// DFT of every line of the tile (natural order in and out), R = 2^q with
// 5 <= q <= 12: ceil(q / 4) stages, larger radices first.
template <bool INV>
__device__ __forceinline__ void line_fft(double2* lds, int q, int ls, int logN,
                                         const double2* tlo, const double2* thi) {
  const int nst = (q + 3) >> 2;
  int ns_log = 0, rem = q;
  for (int s = 0; s < nst; ++s) {
    const int bits = (rem + (nst - s) - 1) / (nst - s);   // ceil(rem / stages left)
    if (bits == 4) stage<4, INV>(lds, q, ls, ns_log, logN, tlo, thi);
    else if (bits == 3) stage<3, INV>(lds, q, ls, ns_log, logN, tlo, thi);
    else stage<2, INV>(lds, q, ls, ns_log, logN, tlo, thi);
    ns_log += bits;
    rem -= bits;
  }
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

// One pass.  IN_REAL: the signals are read from the channel series (first
// forward pass); OUT_REAL: written back to channel series (last inverse
// pass); SPEC: 0 plain pass in direction INV, 1 forward DFT + weighted sums,
// 2 forward DFT + weighted sums + weighted residual + inverse DFT.
template <bool IN_REAL, bool OUT_REAL, int SPEC, bool INV>
__global__ __launch_bounds__(kThreads) void fft_pass_kernel(PassArgs a) {
  __shared__ double2 lds[kTile + kMaxLines];
  __shared__ double red[3][kThreads];
  const int tid = threadIdx.x;
  const int q = a.q, logC = 12 - q, C = 1 << logC, R = 1 << q;
  const int ls = R + 1;                       // one pad per line
  const int64_t N = (int64_t)1 << a.logN;
  const int64_t tau = blockIdx.x;
  const int64_t sig = tau >> a.tiles_log;
  const int64_t tp = tau & (((int64_t)1 << a.tiles_log) - 1);
  const bool col = a.logB > 0;
  const int logA = a.logN - q - a.logB;

  int64_t base;        // element (c, r) at base + c * cstep + r * rstep
  int64_t b0 = 0;
  int64_t cstep, rstep;
  if (col) {
    const int logTa = a.logB - logC;          // tiles per index a
    const int64_t aa = tp >> logTa;
    b0 = (tp & (((int64_t)1 << logTa) - 1)) << logC;
    base = (aa << (q + a.logB)) + b0;
    cstep = 1;
    rstep = (int64_t)1 << a.logB;
  } else {
    base = tp << 12;
    cstep = R;
    rstep = 1;
  }
  const int64_t tpl = sig / a.sig_per_tpl;
  const int kind = (int)(sig - tpl * a.sig_per_tpl);   // 0: A + iE, 1: T
  double2* x = a.x + sig * N;

  // ---- load (coalesced: C consecutive elements per run)
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int e = tid + kThreads * i;
    int c, r;
    if (col) { r = e >> logC; c = e & (C - 1); }
    else { c = e >> q; r = e & (R - 1); }
    const int64_t pos = base + c * cstep + r * rstep;
    double2 val;
    if (IN_REAL) {
      val = make_double2(0.0, 0.0);
      if (pos < a.n) {
        const double* h = a.h + tpl * a.t_stride + pos;
        if (kind == 0) val = make_double2(h[0], h[a.c_stride]);
        else val.x = h[2 * a.c_stride];
      }
    } else {
      val = x[pos];
    }
    if (INV && SPEC == 0 && a.twiddle) {
      // transpose of the forward twiddle, before the inverse DFT
      double2 w = twiddle(a.tlo, a.thi, (int)((r * (b0 + c)) << logA));
      w.y = -w.y;
      val = cmul(val, w);
    }
    lds[c * ls + r] = val;
  }
  __syncthreads();

  line_fft<INV && SPEC == 0>(lds, q, ls, a.logN, a.tlo, a.thi);

  if (SPEC > 0) {
    // weighted sums over this tile's bins (row mode: positions tp*4096 + e)
    double acc[3] = {0.0, 0.0, 0.0};
    const double2* D = a.dspec + kind * N + base;
    const double* W = a.wpos + kind * N + base;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + kThreads * i;
      const int c = e >> q, r = e & (R - 1);
      const double2 H = lds[c * ls + r];
      const double2 Dv = D[e];
      const double w = W[e];
      const double2 Z = csub(Dv, H);
      acc[0] = fma(w, fma(Z.x, Z.x, Z.y * Z.y), acc[0]);
      acc[1] = fma(w, fma(H.x, H.x, H.y * H.y), acc[1]);
      acc[2] = fma(w, fma(Dv.x, H.x, Dv.y * H.y), acc[2]);
      if (SPEC == 2) lds[c * ls + r] = make_double2(w * Z.x, w * Z.y);
    }
    block_sum3(acc, red);
    if (tid == 0) {
      double* p = a.part + 3 * tau;
      p[0] = acc[0];
      p[1] = acc[1];
      p[2] = acc[2];
    }
    if (SPEC == 1) return;
    // block_sum3 ends with a barrier: the weighted residual is in LDS
    line_fft<true>(lds, q, ls, a.logN, a.tlo, a.thi);
  }

  // ---- store
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int e = tid + kThreads * i;
    int c, r;
    if (col) { r = e >> logC; c = e & (C - 1); }
    else { c = e >> q; r = e & (R - 1); }
    const int64_t pos = base + c * cstep + r * rstep;
    double2 val = lds[c * ls + r];
    if (!INV && SPEC == 0 && a.twiddle)
      val = cmul(val, twiddle(a.tlo, a.thi, (int)((r * (b0 + c)) << logA)));
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

static hipError_t launch_pass(const PassArgs& a, int64_t tiles, bool in_real, bool out_real,
                              int spec, bool inv, hipStream_t s) {
  const dim3 grid((unsigned)tiles), block(fd::kThreads);
#define LR_FD_LAUNCH(IR, OR, SP, IV) \
  hipLaunchKernelGGL((fd::fft_pass_kernel<IR, OR, SP, IV>), grid, block, 0, s, a)
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
