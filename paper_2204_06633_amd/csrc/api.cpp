// C-ABI host layer: argument validation, orbit spline fit, padding rules and
// kernel dispatch.  See include/lisaresp.h for the contract of every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lisaresp.h"
#include "internal.hpp"
#include "trace.hpp"

namespace {
thread_local std::string g_err;
}  // namespace

namespace lr {
int set_error(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return status;
}

// Wave row capacity of the carry adjoint kernels (even), or 0 when the
// rows would not fit LDS (the atomic kernels then run).  `spread` bounds, in
// seconds, how far apart the delays of one wave's stencils can lie; each row
// holds the wave's 128 sources plus that spread plus one stencil.  `extra`:
// further doubles of LDS per wave.
int carry_row_capacity(int order, double spread, double dt, int rows, int ncarry, int extra) {
  const int N = order + 1;
  const double s = std::ceil(spread / dt);
  if (!(s >= 0.0) || s > 1e6) return 0;
  int cap = N + 128 + (int)s + 4;
  cap += cap & 1;
  const size_t bytes =
      (size_t)4 * ((size_t)rows * cap + (size_t)ncarry * (N - 1) + (size_t)extra) * sizeof(double);
  return bytes <= (size_t)150 * 1024 ? cap : 0;
}

}  // namespace lr

namespace {

#define fail lr::set_error

int hip_fail(hipError_t e, const char* where) {
  return fail(LR_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool is_finite(double v) { return std::isfinite(v); }

bool valid_order(int order) { return order >= 1 && order <= 31 && (order % 2) == 1; }

// Byte ranges [a, a+na) and [b, b+nb) overlap.
bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

// Not-a-knot cubic spline through y[0..n-1] on a uniform grid of spacing h.
// Second derivatives M solve M[i-1] + 4 M[i] + M[i+1] = 6 (y[i+1] - 2 y[i] +
// y[i-1]) / h^2 (i = 1..n-2) with third-derivative continuity at the second
// and second-to-last knots, M[0] - 2 M[1] + M[2] = 0 (and mirror).  On a
// uniform grid those conditions turn rows 1 and n-2 into 6 M = rhs, which
// leaves a tridiagonal system for M[2..n-3] (Thomas algorithm).
void fit_not_a_knot(const double* y, ptrdiff_t stride, int64_t n, double h, double* coef,
                    ptrdiff_t cstride) {
  std::vector<double> M(n), r(n);
  for (int64_t i = 1; i + 1 < n; ++i)
    r[i] = 6.0 * (y[(i + 1) * stride] - 2.0 * y[i * stride] + y[(i - 1) * stride]) / (h * h);
  M[1] = r[1] / 6.0;
  M[n - 2] = r[n - 2] / 6.0;
  const int64_t m = n - 4;   // unknowns M[2..n-3]
  if (m > 0) {
    std::vector<double> cp(m), dp(m);
    for (int64_t k = 0; k < m; ++k) {
      const int64_t i = k + 2;
      double rhs = r[i];
      if (k == 0) rhs -= M[1];
      if (k == m - 1) rhs -= M[n - 2];
      const double sub = (k == 0) ? 0.0 : 1.0;
      const double den = 4.0 - sub * (k == 0 ? 0.0 : cp[k - 1]);
      cp[k] = 1.0 / den;
      dp[k] = (rhs - sub * (k == 0 ? 0.0 : dp[k - 1])) / den;
    }
    M[m + 1] = dp[m - 1];
    for (int64_t k = m - 2; k >= 0; --k) M[k + 2] = dp[k] - cp[k] * M[k + 3];
  }
  M[0] = 2.0 * M[1] - M[2];
  M[n - 1] = 2.0 * M[n - 2] - M[n - 3];
  for (int64_t i = 0; i + 1 < n; ++i) {
    const double y0 = y[i * stride], y1 = y[(i + 1) * stride];
    double* c = coef + i * cstride;
    c[0] = y0;
    c[1] = (y1 - y0) / h - h * (2.0 * M[i] + M[i + 1]) / 6.0;
    c[2] = 0.5 * M[i];
    c[3] = (M[i + 1] - M[i]) / (6.0 * h);
  }
}

// Largest |p(u)| for u in [0, h] of a cubic, bounded by sum |c_k| h^k.
double seg_abs_bound(const double* c, double h) {
  return std::fabs(c[0]) + h * (std::fabs(c[1]) + h * (std::fabs(c[2]) + h * std::fabs(c[3])));
}

lr::OrbitView view_of(const lr_orbits* o) {
  lr::OrbitView v;
  v.coef = static_cast<const double*>(o->coef);
  v.dt = o->dt;
  v.inv_dt = 1.0 / o->dt;
  v.nseg = o->n - 1;
  return v;
}

int check_orbits(const lr_orbits* o) {
  if (!o || !o->coef || o->n < 4 || !(o->dt > 0.0) || !is_finite(o->t0) || !is_finite(o->dt))
    return fail(LR_E_ARG, "orbits not initialised");
  return LR_OK;
}

// The padding rules need the bounds only (a handle from lr_orbits_bounds,
// without device storage, will do).
int check_orbit_bounds(const lr_orbits* o) {
  if (!o || o->n < 4 || !(o->dt > 0.0) || !is_finite(o->L_min) || !is_finite(o->L_max) ||
      !is_finite(o->R_max))
    return fail(LR_E_ARG, "orbits not initialised");
  return LR_OK;
}

// Every time t0 + j*dt, j in [j0, j1], lies on the orbit grid.
int check_orbit_span(const lr_orbits* o, double t_off, double dt, int64_t j0, int64_t j1) {
  const double span = (double)(o->n - 1) * o->dt;
  const double a = t_off + (double)j0 * dt, b = t_off + (double)j1 * dt;
  if (!(a >= 0.0) || !(b <= span))
    return fail(LR_E_RANGE, "sample times [%.17g, %.17g] s leave the orbit grid [0, %.17g] s "
                            "(relative to its first sample)", a, b, span);
  return LR_OK;
}

}  // namespace

extern "C" int lr_projection_padding(const lr_orbits*, int, double, int64_t*, int64_t*);
extern "C" int lr_tdi_padding(const lr_orbits*, int, int, double, int64_t*, int64_t*);

namespace {

// Shared checks of the projection calls: sizes, padding and orbit coverage.
int check_projection(const lr_orbits* orb, double t0_h, double dt, int64_t n_h, int order,
                     int64_t y_start, int64_t n_y) {
  if (int st = check_orbits(orb)) return st;
  if (!valid_order(order)) return fail(LR_E_UNSUPPORTED, "order %d (odd 1..31)", order);
  if (n_y < 0 || n_h < 0 || y_start < 0) return fail(LR_E_ARG, "negative size or start");
  if (!(dt > 0.0) || !is_finite(dt) || !is_finite(t0_h)) return fail(LR_E_ARG, "non-finite t0 or dt");
  if (n_y == 0) return LR_OK;
  if (n_y > ((int64_t)1 << 40) || n_h > ((int64_t)1 << 40)) return fail(LR_E_ARG, "size too large");
  int64_t front, back;
  if (int st = lr_projection_padding(orb, order, dt, &front, &back)) return st;
  if (y_start - front < 0 || y_start + n_y - 1 + back > n_h - 1)
    return fail(LR_E_RANGE, "h covers [0, %lld) but the link samples [%lld, %lld) need "
                            "%lld before and %lld after", (long long)n_h, (long long)y_start,
                (long long)(y_start + n_y), (long long)front, (long long)back);
  return check_orbit_span(orb, t0_h - orb->t0, dt, y_start, y_start + n_y - 1);
}

// Shared checks of the TDI calls.
int check_tdi(const lr_orbits* orb, double t0_y, double dt, int64_t n_y, int generation,
              int order, int channels, int64_t out_start, int64_t n_out) {
  if (int st = check_orbits(orb)) return st;
  if (!valid_order(order)) return fail(LR_E_UNSUPPORTED, "order %d (odd 1..31)", order);
  if (generation != 1 && generation != 2)
    return fail(LR_E_UNSUPPORTED, "generation %d (1 or 2)", generation);
  if (channels != LR_XYZ && channels != LR_AET && channels != LR_XYZ_AET)
    return fail(LR_E_UNSUPPORTED, "channels %d (LR_XYZ, LR_AET or LR_XYZ_AET)", channels);
  if (n_out < 0 || n_y < 0 || out_start < 0) return fail(LR_E_ARG, "negative size or start");
  if (!(dt > 0.0) || !is_finite(dt) || !is_finite(t0_y)) return fail(LR_E_ARG, "non-finite t0 or dt");
  if (n_out == 0) return LR_OK;
  if (n_out > ((int64_t)1 << 40) || n_y > ((int64_t)1 << 40)) return fail(LR_E_ARG, "size too large");
  int64_t front, back;
  if (int st = lr_tdi_padding(orb, order, generation, dt, &front, &back)) return st;
  if (out_start - front < 0 || out_start + n_out - 1 + back > n_y - 1)
    return fail(LR_E_RANGE, "y covers [0, %lld) but the outputs [%lld, %lld) need %lld "
                            "before and %lld after", (long long)n_y, (long long)out_start,
                (long long)(out_start + n_out), (long long)front, (long long)back);
  return check_orbit_span(orb, t0_y - orb->t0, dt, out_start, out_start + n_out - 1);
}

}  // namespace

namespace {

// Spline fit of the coarse samples (Sec. IV.A: positions and light times are
// interpolated with not-a-knot cubic splines) and the rigorous bounds of the
// fitted light times and distances; host only.
int fit_orbits(double t0, double dt, int64_t n, const double* x_sc, const double* ltt,
               std::vector<double>& coef, lr_orbits& bounds) {
  if (!x_sc || !ltt) return fail(LR_E_ARG, "null pointer");
  if (n < 4) return fail(LR_E_ARG, "need at least 4 coarse orbit samples (got %lld)", (long long)n);
  if (!(dt > 0.0) || !is_finite(dt) || !is_finite(t0)) return fail(LR_E_ARG, "bad orbit grid t0/dt");
  for (int64_t i = 0; i < n * 9; ++i)
    if (!is_finite(x_sc[i])) return fail(LR_E_ARG, "non-finite spacecraft position");
  for (int64_t i = 0; i < n * 6; ++i)
    if (!is_finite(ltt[i])) return fail(LR_E_ARG, "non-finite light travel time");

  const int64_t nseg = n - 1;
  coef.assign((size_t)nseg * lr::kSegStride, 0.0);
  for (int s = 0; s < 9; ++s)
    fit_not_a_knot(x_sc + s, 9, n, dt, coef.data() + 4 * s, lr::kSegStride);
  for (int l = 0; l < 6; ++l)
    fit_not_a_knot(ltt + l, 6, n, dt, coef.data() + 4 * (9 + l), lr::kSegStride);

  double rmax = 0.0, lmax = -INFINITY, lmin = INFINITY;
  for (int64_t k = 0; k < nseg; ++k) {
    const double* seg = coef.data() + k * lr::kSegStride;
    for (int sc = 0; sc < 3; ++sc) {
      double r2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        double b = seg_abs_bound(seg + 4 * (3 * sc + c), dt);
        r2 += b * b;
      }
      rmax = std::max(rmax, std::sqrt(r2));
    }
    for (int l = 0; l < 6; ++l) {
      const double* c = seg + 4 * (9 + l);
      double var = dt * (std::fabs(c[1]) + dt * (std::fabs(c[2]) + dt * std::fabs(c[3])));
      lmax = std::max(lmax, c[0] + var);
      lmin = std::min(lmin, c[0] - var);
    }
  }
  bounds = lr_orbits{};
  bounds.t0 = t0;
  bounds.dt = dt;
  bounds.n = n;
  bounds.coef = nullptr;
  bounds.L_min = lmin;
  bounds.L_max = lmax;
  bounds.R_max = rmax;
  return LR_OK;
}

}  // namespace

extern "C" {

const char* lr_status_str(int s) {
  switch (s) {
    case LR_OK: return "LR_OK";
    case LR_E_ARG: return "LR_E_ARG: invalid argument";
    case LR_E_RANGE: return "LR_E_RANGE: stencil or orbit evaluation outside the data";
    case LR_E_UNSUPPORTED: return "LR_E_UNSUPPORTED: unsupported order, generation or mode";
    case LR_E_WORKSPACE: return "LR_E_WORKSPACE: storage or workspace too small";
    case LR_E_HIP: return "LR_E_HIP: HIP runtime error";
    default: return "unknown lr_status";
  }
}

const char* lr_last_error(void) { return g_err.c_str(); }

int lr_abi_version(void) { return LR_ABI_VERSION; }

size_t lr_orbits_bytes(int64_t n) {
  if (n < 4) return 0;
  return (size_t)(n - 1) * lr::kSegStride * sizeof(double);
}


int lr_orbits_bounds(double t0, double dt, int64_t n, const double* x_sc, const double* ltt,
                     lr_orbits* out) {
  if (!out) return fail(LR_E_ARG, "null pointer");
  std::vector<double> coef;
  lr_orbits b;
  if (int st = fit_orbits(t0, dt, n, x_sc, ltt, coef, b)) return st;
  *out = b;
  return LR_OK;
}

int lr_orbits_init(double t0, double dt, int64_t n, const double* x_sc, const double* ltt,
                   void* d_storage, size_t bytes, lr_orbits* out, void* stream) {
  LR_CALL_RANGE();
  if (!out || !x_sc || !ltt || !d_storage) return fail(LR_E_ARG, "null pointer");
  if (n < 4) return fail(LR_E_ARG, "need at least 4 coarse orbit samples (got %lld)", (long long)n);
  if (!(dt > 0.0) || !is_finite(dt) || !is_finite(t0)) return fail(LR_E_ARG, "bad orbit grid t0/dt");
  if (bytes < lr_orbits_bytes(n))
    return fail(LR_E_WORKSPACE, "orbit storage %zu bytes < %zu", bytes, lr_orbits_bytes(n));
  std::vector<double> coef;
  lr_orbits b;
  if (int st = fit_orbits(t0, dt, n, x_sc, ltt, coef, b)) return st;

  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(d_storage, coef.data(), coef.size() * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "lr_orbits_init copy");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "lr_orbits_init sync");

  *out = b;
  out->coef = d_storage;
  return LR_OK;
}

int lr_projection_padding(const lr_orbits* orb, int order, double dt, int64_t* front,
                          int64_t* back) {
  if (int st = check_orbit_bounds(orb)) return st;
  if (!front || !back) return fail(LR_E_ARG, "null pointer");
  if (!valid_order(order)) return fail(LR_E_UNSUPPORTED, "order %d (odd 1..31)", order);
  if (!(dt > 0.0) || !is_finite(dt)) return fail(LR_E_ARG, "bad dt");
  const int half = (order + 1) / 2;
  const double rc = orb->R_max / lr::kC;
  const double dmax = std::max(orb->L_max, 0.0) + rc;   // largest retarded delay
  const double dmin = std::min(orb->L_min, 0.0) - rc;   // most negative one
  *front = (int64_t)std::ceil(dmax / dt) + half + 1;
  *back = (int64_t)std::ceil(-dmin / dt) + half + 1;
  return LR_OK;
}

int lr_tdi_padding(const lr_orbits* orb, int order, int generation, double dt, int64_t* front,
                   int64_t* back) {
  if (int st = check_orbit_bounds(orb)) return st;
  if (!front || !back) return fail(LR_E_ARG, "null pointer");
  if (!valid_order(order)) return fail(LR_E_UNSUPPORTED, "order %d (odd 1..31)", order);
  if (generation != 1 && generation != 2)
    return fail(LR_E_UNSUPPORTED, "generation %d (1 or 2)", generation);
  if (!(dt > 0.0) || !is_finite(dt)) return fail(LR_E_ARG, "bad dt");
  const int half = (order + 1) / 2;
  const int chain = generation == 1 ? 3 : 7;             // longest chain of link delays
  const double dmax = chain * std::max(orb->L_max, 0.0);
  const double dmin = chain * std::min(orb->L_min, 0.0);
  *front = (int64_t)std::ceil(dmax / dt) + half + 1;
  *back = (int64_t)std::ceil(-dmin / dt) + half + 1;
  return LR_OK;
}

int lr_project_links(const lr_orbits* orb, double t0_h, double dt, int64_t n_h, const double* hp,
                     const double* hc, const double* sky, int order, int64_t y_start,
                     int64_t n_y, double* y, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_projection(orb, t0_h, dt, n_h, order, y_start, n_y)) return st;
  if (n_y == 0) return LR_OK;
  if (!hp || !hc || !y || !sky) return fail(LR_E_ARG, "null pointer");
  const size_t ybytes = 6 * (size_t)n_y * sizeof(double), hbytes = (size_t)n_h * sizeof(double);
  if (overlap(y, ybytes, hp, hbytes) || overlap(y, ybytes, hc, hbytes) ||
      overlap(y, ybytes, sky, 2 * sizeof(double)))
    return fail(LR_E_ARG, "y overlaps an input");
  const double t_off = t0_h - orb->t0;

  lr::ProjArgs a;
  a.orb = view_of(orb);
  a.hp = hp;
  a.hc = hc;
  a.n_h = n_h;
  a.t_off = t_off;
  a.dt = dt;
  a.inv_dt = 1.0 / dt;
  a.sky = sky;
  a.y_start = y_start;
  a.n_y = n_y;
  a.y = y;
  hipError_t e = lr::run_project_links(order, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lr_project_links launch");
  return LR_OK;
}

int lr_tdi_combine(const lr_orbits* orb, double t0_y, double dt, int64_t n_y, const double* y,
                   int generation, int order, int channels, int64_t out_start, int64_t n_out,
                   double* out, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_tdi(orb, t0_y, dt, n_y, generation, order, channels, out_start, n_out))
    return st;
  if (n_out == 0) return LR_OK;
  if (!y || !out) return fail(LR_E_ARG, "null pointer");
  const int64_t rows = channels == LR_XYZ_AET ? 6 : 3;
  if (overlap(out, rows * n_out * sizeof(double), y, 6 * n_y * sizeof(double)))
    return fail(LR_E_ARG, "out overlaps y");
  const double t_off = t0_y - orb->t0;

  lr::TdiArgs a;
  a.orb = view_of(orb);
  a.y = y;
  a.n_y = n_y;
  a.t_off = t_off;
  a.dt = dt;
  a.inv_dt = 1.0 / dt;
  a.out_start = out_start;
  a.n_out = n_out;
  a.channels = channels;
  a.out = out;
  hipError_t e = lr::run_tdi(order, generation, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lr_tdi_combine launch");
  return LR_OK;
}

int lr_tdi_adjoint(const lr_orbits* orb, double t0_y, double dt, int64_t n_y, int generation,
                   int order, int channels, int64_t out_start, int64_t n_out,
                   const double* g_out, double* g_y, void* stream) {
  LR_CALL_RANGE();
  if (int st = check_tdi(orb, t0_y, dt, n_y, generation, order, channels, out_start, n_out))
    return st;
  if (n_y == 0) return LR_OK;
  if (!g_y || (n_out > 0 && !g_out)) return fail(LR_E_ARG, "null pointer");
  const int64_t rows = channels == LR_XYZ_AET ? 6 : 3;
  if (overlap(g_y, 6 * n_y * sizeof(double), g_out, rows * n_out * sizeof(double)))
    return fail(LR_E_ARG, "g_y overlaps g_out");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = lr::run_fill_zero(g_y, 6 * n_y, s);
  if (e != hipSuccess) return hip_fail(e, "lr_tdi_adjoint fill");
  if (n_out == 0) return LR_OK;
  lr::TdiAdjArgs a;
  a.orb = view_of(orb);
  a.g_out = g_out;
  a.channels = channels;
  a.n_y = n_y;
  a.t_off = t0_y - orb->t0;
  a.dt = dt;
  a.inv_dt = 1.0 / dt;
  a.out_start = out_start;
  a.n_out = n_out;
  a.g_y = g_y;
  a.rl_cap = lr::carry_row_capacity(order, (generation == 1 ? 3 : 7) * orb->L_max, dt, 6, 2, 0);
  e = lr::run_tdi_adjoint(order, generation, a, s);
  if (e != hipSuccess) return hip_fail(e, "lr_tdi_adjoint launch");
  return LR_OK;
}

size_t lr_project_adjoint_workspace(int64_t n_y) {
  if (n_y <= 0) return 0;
  return (size_t)((n_y + lr::kTile - 1) / lr::kTile) * 2 * sizeof(double);
}

int lr_project_adjoint(const lr_orbits* orb, double t0_h, double dt, int64_t n_h,
                       const double* hp, const double* hc, const double* sky, int order,
                       int64_t y_start, int64_t n_y, const double* g_y, double* g_hp,
                       double* g_hc, double* g_sky, void* work, size_t work_bytes,
                       void* stream) {
  LR_CALL_RANGE();
  if (int st = check_projection(orb, t0_h, dt, n_h, order, y_start, n_y)) return st;
  if (!g_hp || !g_hc || !sky || (n_y > 0 && !g_y)) return fail(LR_E_ARG, "null pointer");
  if (g_sky && (!hp || !hc)) return fail(LR_E_ARG, "the sky gradient needs h+ and hx");
  const size_t hbytes = (size_t)n_h * sizeof(double), ybytes = 6 * (size_t)n_y * sizeof(double);
  if (overlap(g_hp, hbytes, g_hc, hbytes) || overlap(g_hp, hbytes, g_y, ybytes) ||
      overlap(g_hc, hbytes, g_y, ybytes) || overlap(g_hp, hbytes, hp, hbytes) ||
      overlap(g_hp, hbytes, hc, hbytes) || overlap(g_hc, hbytes, hp, hbytes) ||
      overlap(g_hc, hbytes, hc, hbytes))
    return fail(LR_E_ARG, "an output overlaps an input or the other output");
  if (g_sky) {
    if (work_bytes < lr_project_adjoint_workspace(n_y) || (n_y > 0 && !work))
      return fail(LR_E_WORKSPACE, "workspace %zu bytes < %zu", work_bytes,
                  lr_project_adjoint_workspace(n_y));
    if (overlap(g_sky, 2 * sizeof(double), work, work_bytes) ||
        overlap(g_sky, 2 * sizeof(double), g_hp, hbytes) ||
        overlap(g_sky, 2 * sizeof(double), g_hc, hbytes))
      return fail(LR_E_ARG, "g_sky overlaps the workspace or g_h");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = lr::run_fill_zero(g_hp, n_h, s);
  if (e == hipSuccess) e = lr::run_fill_zero(g_hc, n_h, s);
  if (e == hipSuccess && g_sky && n_y == 0) e = lr::run_fill_zero(g_sky, 2, s);
  if (e != hipSuccess) return hip_fail(e, "lr_project_adjoint fill");
  if (n_y == 0) return LR_OK;
  lr::ProjAdjArgs a;
  a.orb = view_of(orb);
  a.hp = hp;
  a.hc = hc;
  a.n_h = n_h;
  a.t_off = t0_h - orb->t0;
  a.dt = dt;
  a.inv_dt = 1.0 / dt;
  a.sky = sky;
  a.y_start = y_start;
  a.n_y = n_y;
  a.g_y = g_y;
  a.g_hp = g_hp;
  a.g_hc = g_hc;
  a.sky_part = g_sky ? static_cast<double*>(work) : nullptr;
  a.rl_cap = lr::carry_row_capacity(order, 2.01 * orb->L_max, dt, 2, 2, 21 * 64);
  a.params = nullptr;
  a.k0 = 0;
  a.gb_part = nullptr;
  e = lr::run_project_adjoint(order, a, s);
  if (e == hipSuccess && g_sky)
    e = lr::run_sky_finalize(a.sky_part, (n_y + lr::kTile - 1) / lr::kTile, g_sky, s);
  if (e != hipSuccess) return hip_fail(e, "lr_project_adjoint launch");
  return LR_OK;
}

size_t lr_loglike_workspace(void) { return lr::loglike_workspace_bytes(); }

int lr_loglike(const double* h, const double* data, int64_t n, double sigma, double* loglike,
               double* g_h, void* work, size_t work_bytes, void* stream) {
  LR_CALL_RANGE();
  if (n < 0) return fail(LR_E_ARG, "negative size");
  if (!(sigma > 0.0) || !is_finite(sigma)) return fail(LR_E_ARG, "sigma must be positive");
  if (!loglike || !work || (n > 0 && (!h || !data))) return fail(LR_E_ARG, "null pointer");
  if (work_bytes < lr::loglike_workspace_bytes())
    return fail(LR_E_WORKSPACE, "workspace %zu bytes < %zu", work_bytes,
                lr::loglike_workspace_bytes());
  const size_t nb = (size_t)n * sizeof(double);
  if (g_h && (overlap(g_h, nb, h, nb) || overlap(g_h, nb, data, nb) ||
              overlap(g_h, nb, work, work_bytes) || overlap(g_h, nb, loglike, sizeof(double))))
    return fail(LR_E_ARG, "g_h overlaps an input, the workspace or loglike");
  if (overlap(loglike, sizeof(double), work, work_bytes))
    return fail(LR_E_ARG, "loglike overlaps the workspace");
  hipError_t e = lr::run_loglike(h, data, n, 1.0 / (sigma * sigma), g_h,
                                 static_cast<double*>(work), loglike,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lr_loglike launch");
  return LR_OK;
}

}  // extern "C"
