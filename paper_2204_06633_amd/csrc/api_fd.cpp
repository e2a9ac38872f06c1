// C-ABI host layer of the frequency-domain likelihood: plan geometry,
// workspace layout, validation and launches.  See include/lisaresp.h for the
// contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/lisaresp.h"
#include "fd_types.hpp"
#include "internal.hpp"
#include "trace.hpp"

namespace {

using lr::set_error;

constexpr int kMinLog = 12;   // one 4096-point tile
constexpr int kMaxLog = 24;

enum Region { R_TLO, R_THI, R_DSPEC, R_WPOS, R_WORK, R_PART, R_COUNT };
static_assert(R_COUNT <= (int)(sizeof(((lr_fd_plan*)nullptr)->off) / sizeof(size_t)),
              "lr_fd_plan.off has a slot per workspace region");

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int log2_length(int64_t n) {
  int p = kMinLog;
  while (p <= kMaxLog && ((int64_t)1 << p) < n) ++p;
  return p;
}

// Pass sizes: one pass of 4096 points, or two or three passes of 2^5..2^8
// in ascending order (so every pass but the last has B >= C, and every
// global access is a run of at least 128 bytes).
int split_passes(int logN, int q[3]) {
  q[0] = q[1] = q[2] = 0;
  if (logN == kMinLog) {
    q[0] = logN;
    return 1;
  }
  const int P = logN <= 16 ? 2 : 3;
  for (int s = 0; s < P; ++s) q[s] = logN / P;
  for (int i = 0; i < logN - (logN / P) * P; ++i) q[P - 1 - i] += 1;
  return P;
}

struct Layout {
  size_t off[R_COUNT];
  size_t total;
};

Layout layout(int logN, int sig, int64_t max_batch) {
  const size_t N = (size_t)1 << logN;
  size_t bytes[R_COUNT];
  bytes[R_TLO] = 4096 * sizeof(double2);
  bytes[R_THI] = 4096 * sizeof(double2);
  bytes[R_DSPEC] = 2 * N * sizeof(double2);
  bytes[R_WPOS] = 2 * N * sizeof(double);
  bytes[R_WORK] = (size_t)max_batch * sig * N * sizeof(double2);
  bytes[R_PART] = (size_t)max_batch * sig * (N >> 12) * 3 * sizeof(double);
  Layout L;
  size_t o = 0;
  for (int r = 0; r < R_COUNT; ++r) {
    L.off[r] = o;
    o += align256(bytes[r]);
  }
  L.total = o;
  return L;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

template <class T>
T* at(const lr_fd_plan* p, int r) {
  return reinterpret_cast<T*>(static_cast<char*>(p->ws) + p->off[r]);
}

lr::FdGeometry geometry(const lr_fd_plan* p) {
  lr::FdGeometry g;
  g.n = p->n;
  g.logN = p->log2n;
  g.passes = p->passes;
  for (int s = 0; s < 3; ++s) g.q[s] = p->q[s];
  g.sig_per_tpl = p->channels == 3 ? 2 : 1;
  return g;
}

lr::FdBuffers buffers(const lr_fd_plan* p) {
  lr::FdBuffers b;
  b.tlo = at<double2>(p, R_TLO);
  b.thi = at<double2>(p, R_THI);
  b.dspec = at<double2>(p, R_DSPEC);
  b.wpos = at<double>(p, R_WPOS);
  b.work = at<double2>(p, R_WORK);
  b.part = at<double>(p, R_PART);
  return b;
}

}  // namespace

extern "C" {

int64_t lr_fd_length(int64_t n) {
  if (n < 1 || n > ((int64_t)1 << kMaxLog)) return -1;
  return (int64_t)1 << log2_length(n);
}

size_t lr_fd_workspace(int64_t n, int channels, int64_t max_batch) {
  if (lr_fd_length(n) < 0 || (channels != 2 && channels != 3) || max_batch < 1) return 0;
  return layout(log2_length(n), channels == 3 ? 2 : 1, max_batch).total;
}

int lr_fd_prepare(int64_t n, int channels, double dt, const double* data, int64_t data_cstride,
                  const double* w_ae, const double* w_t, int64_t max_batch, void* ws,
                  size_t ws_bytes, lr_fd_plan* out, void* stream) {
  LR_CALL_RANGE();
  if (!out) return set_error(LR_E_ARG, "null plan");
  *out = lr_fd_plan{};
  if (n < 1) return set_error(LR_E_ARG, "n = %lld samples", (long long)n);
  if (n > ((int64_t)1 << kMaxLog))
    return set_error(LR_E_UNSUPPORTED, "n = %lld > 2^24 samples", (long long)n);
  if (channels != 2 && channels != 3) return set_error(LR_E_ARG, "channels %d (2 or 3)", channels);
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(LR_E_ARG, "dt must be positive");
  if (max_batch < 1) return set_error(LR_E_ARG, "max_batch %lld", (long long)max_batch);
  if (data_cstride < n) return set_error(LR_E_ARG, "data channel stride < n");
  if (!data || !w_ae || (channels == 3 && !w_t) || !ws) return set_error(LR_E_ARG, "null pointer");
  const int logN = log2_length(n);
  const int sig = channels == 3 ? 2 : 1;
  const Layout L = layout(logN, sig, max_batch);
  if (ws_bytes < L.total)
    return set_error(LR_E_WORKSPACE, "workspace %zu bytes < %zu", ws_bytes, L.total);
  const size_t N = (size_t)1 << logN;
  const size_t wbytes = (N / 2 + 1) * sizeof(double);
  const size_t dbytes = ((size_t)(channels - 1) * data_cstride + n) * sizeof(double);
  if (overlap(ws, ws_bytes, data, dbytes) || overlap(ws, ws_bytes, w_ae, wbytes) ||
      (channels == 3 && overlap(ws, ws_bytes, w_t, wbytes)))
    return set_error(LR_E_ARG, "an input overlaps the workspace");
  lr_fd_plan p{};
  p.n = n;
  p.n_fft = (int64_t)N;
  p.max_batch = max_batch;
  p.channels = channels;
  p.log2n = logN;
  p.passes = split_passes(logN, p.q);
  p.dt = dt;
  p.ws = ws;
  p.ws_bytes = ws_bytes;
  for (int r = 0; r < R_COUNT; ++r) p.off[r] = L.off[r];
  hipError_t e = lr::run_fd_prepare(geometry(&p), buffers(&p), data, data_cstride, w_ae,
                                    channels == 3 ? w_t : nullptr, dt,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_error(LR_E_HIP, "lr_fd_prepare launch: %s", hipGetErrorString(e));
  *out = p;
  return LR_OK;
}

int lr_fd_loglike(const lr_fd_plan* p, int64_t n_templates, const double* h, int64_t t_stride,
                  int64_t c_stride, double* stats, double* g_h, void* stream) {
  LR_CALL_RANGE();
  if (!p || !p->ws || p->n < 1 || p->log2n < kMinLog || p->log2n > kMaxLog)
    return set_error(LR_E_ARG, "plan not prepared");
  if (n_templates < 0) return set_error(LR_E_ARG, "negative template count");
  if (n_templates == 0) return LR_OK;
  if (!h || !stats) return set_error(LR_E_ARG, "null pointer");
  const int C = p->channels;
  if (c_stride < p->n || t_stride < (int64_t)(C - 1) * c_stride + p->n)
    return set_error(LR_E_ARG, "strides: channel %lld, template %lld for %lld samples",
                     (long long)c_stride, (long long)t_stride, (long long)p->n);
  const size_t hbytes =
      ((size_t)(n_templates - 1) * t_stride + (size_t)(C - 1) * c_stride + p->n) * sizeof(double);
  const size_t sbytes = (size_t)n_templates * 3 * sizeof(double);
  if (overlap(stats, sbytes, p->ws, p->ws_bytes) || overlap(stats, sbytes, h, hbytes) ||
      overlap(stats, sbytes, g_h, hbytes))
    return set_error(LR_E_ARG, "stats overlaps an input, g_h or the workspace");
  if (g_h && (overlap(g_h, hbytes, h, hbytes) || overlap(g_h, hbytes, p->ws, p->ws_bytes)))
    return set_error(LR_E_ARG, "g_h overlaps h or the workspace");
  if (overlap(h, hbytes, p->ws, p->ws_bytes)) return set_error(LR_E_ARG, "h overlaps the workspace");
  const lr::FdGeometry g = geometry(p);
  const lr::FdBuffers b = buffers(p);
  for (int64_t t0 = 0; t0 < n_templates; t0 += p->max_batch) {
    const int64_t m = n_templates - t0 < p->max_batch ? n_templates - t0 : p->max_batch;
    hipError_t e = lr::run_fd_loglike(g, b, m, h + t0 * t_stride, t_stride, c_stride,
                                      stats + 3 * t0, g_h ? g_h + t0 * t_stride : nullptr,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
      return set_error(LR_E_HIP, "lr_fd_loglike launch: %s", hipGetErrorString(e));
  }
  return LR_OK;
}

}  // extern "C"
