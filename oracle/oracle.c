/*
 * oracle.c -- plain, slow, FP64 CPU reference of the generic LISA
 * time-domain response: projection of h+ / hx onto the six links, then the
 * first- and second-generation Michelson TDI combinations.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * table or constant with the HIP library.
 *
 * Every function below follows the paper (arXiv:2204.06633) step by step:
 *   - sky basis and polarisation vectors ........ Sec. IV.A
 *   - antenna patterns, link projection ......... Sec. IV.B, eq. (projected strain)
 *   - link response y_ij at reception time ...... Sec. IV.B, eq. (instrument response)
 *   - delay operator, chained delays as sums .... Sec. IV.C
 *   - X1 / X2 term lists .......................... Sec. IV.C, eqs. (tdi1), (tdi2)
 *   - centred Lagrange fractional-delay interpolation of user order ... Sec. IV.E
 *
 * Readings of points the paper leaves open (also listed in the design notes):
 *   - "order" is the polynomial degree; order + 1 taps; odd orders only; the
 *     stencil for position p is floor(p) - (order-1)/2 ... floor(p) + (order+1)/2;
 *   - a position is an integer sample index minus a small delay in seconds,
 *     split into integer part and fraction before any rounding at the scale
 *     of the index;
 *   - orbit quantities are cubic splines (coefficients supplied by the caller)
 *     evaluated at reception time; n_ij = (x_i - x_j)/|x_i - x_j|;
 *   - a stencil that leaves the supplied series is an error (no extrapolation).
 *
 * Plain loops, textbook O(n^2) Lagrange weights, OpenMP only over independent
 * output samples of the forward maps; the adjoint scatters run serially.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORC_C 299792458.0
#define ORC_MAX_TAPS 64

/* Coarse-grid orbit splines: series s (0..8: x1,y1,z1,x2,..,z3; 9..14: the
 * six light travel times in link order 12,23,31,13,32,21) on segment k is
 * coef[(s*nseg + k)*4 + p] * u^p, u = tau - k*dt, tau = time since the first
 * coarse sample. */
typedef struct {
    double dt;
    int64_t nseg;
    const double *coef;
} orc_orbits;

static const int LINK_RECV[6] = {1, 2, 3, 1, 3, 2};
static const int LINK_EMIT[6] = {2, 3, 1, 3, 2, 1};

static double spline_value(const orc_orbits *o, int series, double tau)
{
    int64_t k = (int64_t)floor(tau / o->dt);
    if (k < 0) k = 0;
    if (k > o->nseg - 1) k = o->nseg - 1;
    double u = tau - (double)k * o->dt;
    const double *c = o->coef + ((int64_t)series * o->nseg + k) * 4;
    return c[0] + c[1] * u + c[2] * u * u + c[3] * u * u * u;
}

/* positions x[sc][xyz] (sc = 0..2 for spacecraft 1..3) and light times L[6] */
static void orbit_state(const orc_orbits *o, double tau, double x[3][3], double L[6])
{
    for (int s = 0; s < 3; ++s)
        for (int c = 0; c < 3; ++c)
            x[s][c] = spline_value(o, 3 * s + c, tau);
    for (int l = 0; l < 6; ++l)
        L[l] = spline_value(o, 9 + l, tau);
}

/* Sec. IV.A: e_r, e_theta, e_phi from ecliptic (lambda, beta);
 * k = -e_r, u = -e_phi, v = -e_theta. */
static void sky_basis(double lam, double beta, double k[3], double u[3], double v[3])
{
    double cb = cos(beta), sb = sin(beta), cl = cos(lam), sl = sin(lam);
    double er[3] = {cb * cl, cb * sl, sb};
    double et[3] = {sb * cl, sb * sl, -cb};
    double ep[3] = {-sl, cl, 0.0};
    for (int i = 0; i < 3; ++i) {
        k[i] = -er[i];
        u[i] = -ep[i];
        v[i] = -et[i];
    }
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Textbook Lagrange weights on the nodes x_m = m - (h-1), m = 0..order,
 * h = (order+1)/2:  w_m(eps) = prod_{m' != m} (eps - x_m') / (x_m - x_m'). */
void orc_lagrange_weights(int order, double eps, double *w)
{
    int n = order + 1, h = n / 2;
    for (int m = 0; m < n; ++m) {
        double xm = (double)(m - (h - 1));
        double p = 1.0;
        for (int mm = 0; mm < n; ++mm) {
            if (mm == m) continue;
            double xmm = (double)(mm - (h - 1));
            p *= (eps - xmm) / (xm - xmm);
        }
        w[m] = p;
    }
}

/* Split the position q - d/dt into j0 = floor(position) and eps in [0,1)
 * without ever forming q - d/dt as one floating-point number. */
static void split_position(int64_t q, double d, double dt, int64_t *j0, double *eps)
{
    double a = -d / dt;
    double fl = floor(a);
    *j0 = q + (int64_t)fl;
    *eps = a - fl;
}

/* Value of the centred Lagrange interpolant of f at j0 + eps.  Returns -1 if
 * the stencil leaves [0, n). */
static int interp(const double *f, int64_t n, int order, int64_t j0, double eps, double *out)
{
    int taps = order + 1, h = taps / 2;
    int64_t lo = j0 - (h - 1);
    if (lo < 0 || lo + taps - 1 >= n) return -1;
    double w[ORC_MAX_TAPS];
    orc_lagrange_weights(order, eps, w);
    double s = 0.0;
    for (int m = 0; m < taps; ++m) s += w[m] * f[lo + m];
    *out = s;
    return 0;
}

int orc_interp(const double *f, int64_t n, int order, int64_t j0, double eps, double *out)
{
    if (order < 1 || order % 2 == 0 || order + 1 > ORC_MAX_TAPS) return -2;
    return interp(f, n, order, j0, eps, out);
}

void orc_orbit_state(double dt_o, int64_t nseg, const double *coef, double tau,
                     double *x9, double *L6)
{
    orc_orbits o = {dt_o, nseg, coef};
    double x[3][3];
    orbit_state(&o, tau, x, L6);
    memcpy(x9, x, sizeof(x));
}

/*
 * Link response y_l at the h-indices q[i] (Sec. IV.B):
 *   y_ij(t) = [H_ij(t - L_ij - k.x_j/c) - H_ij(t - k.x_i/c)] / (2 (1 - k.n_ij)),
 *   H_ij(s) = h+(s) xi+(n_ij) + hx(s) xix(n_ij),
 *   xi+ = (u.n)^2 - (v.n)^2, xix = 2 (u.n)(v.n),
 * every orbit quantity taken at the reception time t = t_off + q*dt (time
 * measured from the first coarse orbit sample).  h[j] sits at t_off + j*dt.
 * Output y[l*nq + i].  Returns 0, or -1 if a stencil leaves h.
 */
int orc_project(double dt_o, int64_t nseg, const double *coef, double t_off, double dt,
                const double *hp, const double *hc, int64_t n_h, double lam, double beta,
                int order, const int64_t *q, int64_t nq, double *y)
{
    if (order < 1 || order % 2 == 0 || order + 1 > ORC_MAX_TAPS) return -2;
    orc_orbits o = {dt_o, nseg, coef};
    double k[3], u[3], v[3];
    sky_basis(lam, beta, k, u, v);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < nq; ++i) {
        double x[3][3], L[6];
        orbit_state(&o, t_off + (double)q[i] * dt, x, L);
        for (int l = 0; l < 6; ++l) {
            const double *xr = x[LINK_RECV[l] - 1], *xe = x[LINK_EMIT[l] - 1];
            double n[3] = {xr[0] - xe[0], xr[1] - xe[1], xr[2] - xe[2]};
            double nn = sqrt(dot3(n, n));
            for (int c = 0; c < 3; ++c) n[c] /= nn;
            double un = dot3(u, n), vn = dot3(v, n);
            double xip = un * un - vn * vn, xic = 2.0 * un * vn;
            double d_emit = L[l] + dot3(k, xe) / ORC_C;
            double d_recv = dot3(k, xr) / ORC_C;
            int64_t je, jr;
            double ee, er;
            split_position(q[i], d_emit, dt, &je, &ee);
            split_position(q[i], d_recv, dt, &jr, &er);
            double hpe, hce, hpr, hcr;
            int st = interp(hp, n_h, order, je, ee, &hpe) | interp(hc, n_h, order, je, ee, &hce) |
                     interp(hp, n_h, order, jr, er, &hpr) | interp(hc, n_h, order, jr, er, &hcr);
            if (st) { bad = 1; continue; }
            double H_e = hpe * xip + hce * xic;
            double H_r = hpr * xip + hcr * xic;
            y[(int64_t)l * nq + i] = (H_e - H_r) / (2.0 * (1.0 - dot3(k, n)));
        }
    }
    return bad ? -1 : 0;
}

/* Delay of a chained operator D_{i1 i2 ... in}: sum of L_{ik ik+1} at time t
 * (Sec. IV.C; the chain is summed, not nested). path holds spacecraft 1..3. */
static int link_index(int recv, int emit)
{
    for (int l = 0; l < 6; ++l)
        if (LINK_RECV[l] == recv && LINK_EMIT[l] == emit) return l;
    return -1;
}

static double chain_delay(const int *path, int len, const double L[6])
{
    double d = 0.0;
    for (int s = 0; s + 1 < len; ++s) d += L[link_index(path[s], path[s + 1])];
    return d;
}

/*
 * TDI channels at the y-indices p[i].  Term t contributes
 *   sign[t] * D_{path[t]} y_{link[t]}
 * to channel chan[t]; a path of length 1 means no delay (the sample itself).
 * y[l*n_y + j] sits at time t_off_y + j*dt; orbit light times are taken at
 * the output time t_off_y + p*dt.  Output out[c*np + i], c = 0,1,2 (X,Y,Z).
 */
int orc_tdi(double dt_o, int64_t nseg, const double *coef, double t_off_y, double dt,
            const double *y, int64_t n_y, int order, int nterms, const int *chan,
            const int *sign, const int *link, const int *pathlen, const int *path /*[nterms][8]*/,
            const int64_t *p, int64_t np, double *out)
{
    if (order < 1 || order % 2 == 0 || order + 1 > ORC_MAX_TAPS) return -2;
    orc_orbits o = {dt_o, nseg, coef};
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < np; ++i) {
        double x[3][3], L[6];
        orbit_state(&o, t_off_y + (double)p[i] * dt, x, L);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int t = 0; t < nterms; ++t) {
            const double *yl = y + (int64_t)link[t] * n_y;
            double val;
            if (pathlen[t] <= 1) {
                if (p[i] < 0 || p[i] >= n_y) { bad = 1; continue; }
                val = yl[p[i]];
            } else {
                double D = chain_delay(path + 8 * t, pathlen[t], L);
                int64_t j0;
                double eps;
                split_position(p[i], D, dt, &j0, &eps);
                if (interp(yl, n_y, order, j0, eps, &val)) { bad = 1; continue; }
            }
            acc[chan[t]] += (double)sign[t] * val;
        }
        for (int c = 0; c < 3; ++c) out[(int64_t)c * np + i] = acc[c];
    }
    return bad ? -1 : 0;
}

/*
 * Adjoint (transpose) of orc_tdi with respect to y: for every output sample,
 * term and tap, g_y[link][tap] += sign * w_tap * g_out[chan][i].  g_y is
 * accumulated (the caller zeroes it).  Serial loops.
 */
int orc_tdi_adjoint(double dt_o, int64_t nseg, const double *coef, double t_off_y, double dt,
                    int64_t n_y, int order, int nterms, const int *chan, const int *sign,
                    const int *link, const int *pathlen, const int *path, const int64_t *p,
                    int64_t np, const double *g_out, double *g_y)
{
    if (order < 1 || order % 2 == 0 || order + 1 > ORC_MAX_TAPS) return -2;
    orc_orbits o = {dt_o, nseg, coef};
    int taps = order + 1, h = taps / 2;
    double w[ORC_MAX_TAPS];
    for (int64_t i = 0; i < np; ++i) {
        double x[3][3], L[6];
        orbit_state(&o, t_off_y + (double)p[i] * dt, x, L);
        for (int t = 0; t < nterms; ++t) {
            double g = (double)sign[t] * g_out[(int64_t)chan[t] * np + i];
            double *gl = g_y + (int64_t)link[t] * n_y;
            if (pathlen[t] <= 1) {
                if (p[i] < 0 || p[i] >= n_y) return -1;
                gl[p[i]] += g;
                continue;
            }
            double D = chain_delay(path + 8 * t, pathlen[t], L);
            int64_t j0;
            double eps;
            split_position(p[i], D, dt, &j0, &eps);
            int64_t lo = j0 - (h - 1);
            if (lo < 0 || lo + taps - 1 >= n_y) return -1;
            orc_lagrange_weights(order, eps, w);
            for (int m = 0; m < taps; ++m) gl[lo + m] += w[m] * g;
        }
    }
    return 0;
}

/*
 * Adjoint of orc_project with respect to (h+, hx): for every link sample and
 * tap, g_h[tap] += (+/-) xi * w_tap * g_y / (2 (1 - k.n)), + at the emission
 * position and - at the reception position.  Accumulates into g_hp, g_hc.
 */
int orc_project_adjoint(double dt_o, int64_t nseg, const double *coef, double t_off, double dt,
                        int64_t n_h, double lam, double beta, int order, const int64_t *q,
                        int64_t nq, const double *g_y, double *g_hp, double *g_hc)
{
    if (order < 1 || order % 2 == 0 || order + 1 > ORC_MAX_TAPS) return -2;
    orc_orbits o = {dt_o, nseg, coef};
    double k[3], u[3], v[3];
    sky_basis(lam, beta, k, u, v);
    int taps = order + 1, h = taps / 2;
    double w[ORC_MAX_TAPS];
    for (int64_t i = 0; i < nq; ++i) {
        double x[3][3], L[6];
        orbit_state(&o, t_off + (double)q[i] * dt, x, L);
        for (int l = 0; l < 6; ++l) {
            const double *xr = x[LINK_RECV[l] - 1], *xe = x[LINK_EMIT[l] - 1];
            double n[3] = {xr[0] - xe[0], xr[1] - xe[1], xr[2] - xe[2]};
            double nn = sqrt(dot3(n, n));
            for (int c = 0; c < 3; ++c) n[c] /= nn;
            double un = dot3(u, n), vn = dot3(v, n);
            double xip = un * un - vn * vn, xic = 2.0 * un * vn;
            double scale = g_y[(int64_t)l * nq + i] / (2.0 * (1.0 - dot3(k, n)));
            double delays[2] = {L[l] + dot3(k, xe) / ORC_C, dot3(k, xr) / ORC_C};
            double sgn[2] = {1.0, -1.0};
            for (int e = 0; e < 2; ++e) {
                int64_t j0;
                double eps;
                split_position(q[i], delays[e], dt, &j0, &eps);
                int64_t lo = j0 - (h - 1);
                if (lo < 0 || lo + taps - 1 >= n_h) return -1;
                orc_lagrange_weights(order, eps, w);
                for (int m = 0; m < taps; ++m) {
                    g_hp[lo + m] += sgn[e] * scale * xip * w[m];
                    g_hc[lo + m] += sgn[e] * scale * xic * w[m];
                }
            }
        }
    }
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops (timing runs at one thread and at all
   cores). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* Sky basis (k, u, v) of Sec. IV.A, exposed for the pin tests. */
void orc_sky_basis(double lam, double beta, double *k, double *u, double *v)
{
    sky_basis(lam, beta, k, u, v);
}
