/* Drives every entry point of oracle/oracle.c on small inputs, in range and
 * at the edges where a stencil leaves its series (which must be reported,
 * not read), for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer.  Exit status 0 and "ok" when every call behaved. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_lagrange_weights(int order, double eps, double *w);
int orc_interp(const double *f, int64_t n, int order, int64_t j0, double eps, double *out);
void orc_orbit_state(double dt_o, int64_t nseg, const double *coef, double tau, double *x9,
                     double *L6);
int orc_project(double dt_o, int64_t nseg, const double *coef, double t_off, double dt,
                const double *hp, const double *hc, int64_t n_h, double lam, double beta,
                int order, const int64_t *q, int64_t nq, double *y);
int orc_tdi(double dt_o, int64_t nseg, const double *coef, double t_off_y, double dt,
            const double *y, int64_t n_y, int order, int nterms, const int *chan,
            const int *sign, const int *link, const int *pathlen, const int *path,
            const int64_t *p, int64_t np, double *out);
int orc_tdi_adjoint(double dt_o, int64_t nseg, const double *coef, double t_off_y, double dt,
                    int64_t n_y, int order, int nterms, const int *chan, const int *sign,
                    const int *link, const int *pathlen, const int *path, const int64_t *p,
                    int64_t np, const double *g_out, double *g_y);
int orc_project_adjoint(double dt_o, int64_t nseg, const double *coef, double t_off, double dt,
                        int64_t n_h, double lam, double beta, int order, const int64_t *q,
                        int64_t nq, const double *g_y, double *g_hp, double *g_hc);
void orc_sky_basis(double lam, double beta, double *k, double *u, double *v);
int orc_max_threads(void);
void orc_set_threads(int n);

static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

static uint64_t rng = 12345;
static double uniform(void) {
  rng = rng * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(rng >> 11) / 9007199254740992.0 - 0.5;
}

int main(void) {
  /* static equilateral triangle of 3 light-seconds in the ecliptic plane,
   * constant light times: splines with the constant coefficient only */
  const int64_t nseg = 4;
  const double dt_o = 100.0, Ls = 3.0 * 299792458.0;
  double *coef = calloc(15 * nseg * 4, sizeof(double));
  const double pos[3][3] = {{0, 0, 0}, {Ls, 0, 0}, {0.5 * Ls, 0.8660254037844386 * Ls, 0}};
  for (int s = 0; s < 15; ++s)
    for (int64_t k = 0; k < nseg; ++k)
      coef[(s * nseg + k) * 4] = s < 9 ? pos[s / 3][s % 3] : 3.0;
  const int64_t n_h = 400;
  double *hp = malloc(n_h * sizeof(double)), *hc = malloc(n_h * sizeof(double));
  for (int64_t j = 0; j < n_h; ++j) { hp[j] = uniform(); hc[j] = uniform(); }

  double w[64], v;
  for (int order = 1; order <= 31; order += 2) {
    orc_lagrange_weights(order, 0.37, w);
    double s = 0;
    for (int m = 0; m <= order; ++m) s += w[m];
    CHECK(fabs(s - 1.0) < 1e-9);
    CHECK(orc_interp(hp, n_h, order, 100, 0.25, &v) == 0);
    CHECK(orc_interp(hp, n_h, order, 0, 0.25, &v) != 0 || order == 1);
    CHECK(orc_interp(hp, n_h, order, n_h - 1, 0.25, &v) != 0);
  }
  double x9[9], L6[6], k3[3], u3[3], v3[3];
  orc_orbit_state(dt_o, nseg, coef, 150.0, x9, L6);
  CHECK(L6[0] == 3.0);
  orc_sky_basis(0.3, -1.1, k3, u3, v3);

  const int order = 9, dt = 1;
  int64_t q[200];
  for (int i = 0; i < 200; ++i) q[i] = 100 + i;
  double *y = malloc(6 * 200 * sizeof(double));
  CHECK(orc_project(dt_o, nseg, coef, 0.0, dt, hp, hc, n_h, 0.3, -1.1, order, q, 200, y) == 0);
  int64_t qbad[2] = {2, 100};
  double ybad[12];
  CHECK(orc_project(dt_o, nseg, coef, 0.0, dt, hp, hc, n_h, 0.3, -1.1, order, qbad, 2, ybad) != 0);
  CHECK(orc_project(dt_o, nseg, coef, 0.0, dt, hp, hc, n_h, 0.3, -1.1, 4, q, 200, y) != 0);

  /* X1 terms of eq. (tdi1) for the X channel */
  const int nt = 8;
  const int chan[8] = {0, 0, 0, 0, 0, 0, 0, 0}, sign[8] = {1, 1, 1, 1, -1, -1, -1, -1};
  const int link[8] = {3, 2, 0, 5, 0, 5, 3, 2}, plen[8] = {1, 2, 3, 4, 1, 2, 3, 4};
  const int path[8][8] = {{1}, {1, 3}, {1, 3, 1}, {1, 3, 1, 2}, {1}, {1, 2}, {1, 2, 1},
                          {1, 2, 1, 3}};
  int64_t p[100];
  for (int i = 0; i < 100; ++i) p[i] = 40 + i;
  double out[300], gx[300], *g_y = calloc(6 * 200, sizeof(double));
  for (int i = 0; i < 300; ++i) gx[i] = uniform();
  CHECK(orc_tdi(dt_o, nseg, coef, 100.0, dt, y, 200, order, nt, chan, sign, link, plen,
                &path[0][0], p, 100, out) == 0);
  CHECK(orc_tdi_adjoint(dt_o, nseg, coef, 100.0, dt, 200, order, nt, chan, sign, link, plen,
                        &path[0][0], p, 100, gx, g_y) == 0);
  int64_t pbad[1] = {3};
  CHECK(orc_tdi(dt_o, nseg, coef, 100.0, dt, y, 200, order, nt, chan, sign, link, plen,
                &path[0][0], pbad, 1, out) != 0);
  CHECK(orc_tdi_adjoint(dt_o, nseg, coef, 100.0, dt, 200, order, nt, chan, sign, link, plen,
                        &path[0][0], pbad, 1, gx, g_y) != 0);
  double *g_hp = calloc(n_h, sizeof(double)), *g_hc = calloc(n_h, sizeof(double));
  CHECK(orc_project_adjoint(dt_o, nseg, coef, 0.0, dt, n_h, 0.3, -1.1, order, q, 200, g_y,
                            g_hp, g_hc) == 0);
  CHECK(orc_project_adjoint(dt_o, nseg, coef, 0.0, dt, n_h, 0.3, -1.1, order, qbad, 2, g_y,
                            g_hp, g_hc) != 0);
  orc_set_threads(1);
  CHECK(orc_max_threads() == 1);
  free(coef); free(hp); free(hc); free(y); free(g_y); free(g_hp); free(g_hc);
  if (fails) return 1;
  printf("ok\n");
  return 0;
}
