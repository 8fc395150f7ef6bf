/* Drives the C oracle through every entry point on small grids (linear and
 * quadratic shapes, with and without the moving window), for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * compiled and run by tests/test_sanitizers.py).  Exit status 0 when every
 * call succeeds; the sanitizers abort on any memory or UB error. */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc orc;
orc *orc_create(int Nz, int Nr, int M, double dz, double dr, double dt, int N, const double *CE, const double *CB);
void orc_destroy(orc *o);
void orc_set_flags(orc *o, int freeze_fields, int deposit_rho);
long orc_num_particles(const orc *o);
int orc_get_field(orc *o, int comp, int m, double *out);
int orc_set_field(orc *o, int comp, int m, const double *in);
int orc_gauss_residual(orc *o, int m, double *out);
double orc_field_energy(orc *o, int m);
void orc_gather(orc *o, double zc, double xc, double yc, double *EB);
void orc_deposit_rho(orc *o);
void orc_step(orc *o, int nsteps);
void orc_field_step(orc *o, int nsteps);
void orc_start_fields(orc *o);
int orc_load_plasma(orc *o, int ppc, double n0, double ramp_start, double ramp_len, uint64_t seed, int n_tracked,
                    double down_start, double down_len);
int orc_tracked(orc *o, int64_t *ids, double *W, double *gamma, double *gamma_acc);
int orc_cartesian_work(orc *o, double *wz, double *wperp);
double orc_kinetic(orc *o);
int orc_add_laser(orc *o, double a0, double w0, double tau, double zc, double taper);
void orc_cell_order(orc *o, int Tz, int Tr, int64_t *ord);
int orc_set_shape(orc *o, int order);
void orc_set_exact_jz(orc *o, int on);
void orc_set_window(orc *o, int K, double speed, int guard);
long orc_window_cells(const orc *o);
int orc_set_particles(orc *o, long np, const double *z, const double *x, const double *y, const double *ux,
                      const double *uy, const double *uz, const double *w, int track_all);

/* shape: particle shape order; window: a move every `window` steps (0: none);
 * exact: the exact J_z switch */
static int run(int M, int N, const double *C, int shape, int window, int exact) {
  const int Nz = 24, Nr = 8;
  orc *o = orc_create(Nz, Nr, M, 0.4, 1.6, 0.15, N, C, C);
  if (!o) return 1;
  if (orc_set_shape(o, shape)) return 9;
  orc_set_exact_jz(o, exact);
  if (orc_load_plasma(o, 2, 0.02, 2.0, 4.0, 7u, 12, 8.0, 3.0)) return 2;
  if (M >= 1 && orc_add_laser(o, 1.5, 4.0, 3.0, 4.8, 1.0)) return 3;
  orc_start_fields(o);
  orc_set_flags(o, 0, 1);
  orc_deposit_rho(o);
  if (window) orc_set_window(o, window, 1.0, 2);
  orc_step(o, 6);
  if (window && orc_window_cells(o) <= 0) return 10;
  orc_field_step(o, 1);
  const size_t plane = (size_t)(Nr + 1) * Nz;
  double *buf = (double *)calloc(2 * plane, sizeof(double));
  for (int m = 0; m <= M; ++m) {
    if (orc_gauss_residual(o, m, buf)) return 4;
    if (orc_get_field(o, 0, m, buf) || orc_set_field(o, 0, m, buf)) return 5;
    if (!(orc_field_energy(o, m) >= 0.0)) return 6;
  }
  const long np = orc_num_particles(o);
  int64_t *ord = (int64_t *)calloc((size_t)np, sizeof(int64_t));
  orc_cell_order(o, 8, 4, ord);
  int64_t ids[12];
  double W[12 * 4], g[12], ga[12], wz[12], wp[12], EB[6];
  if (orc_tracked(o, ids, W, g, ga) != 12 || orc_cartesian_work(o, wz, wp) != 12) return 7;
  orc_gather(o, 3.3, 0.2, -0.1, EB);  /* within half a cell of the axis */
  orc_gather(o, 3.3, 6.9, 0.0, EB);   /* next to the wall row */
  /* electrons whose stencils reach the first columns, the axis and the row
   * past the wall (an access beyond the last array shows there) */
  const double pz[3] = {0.3, 0.2, 23.8}, px[3] = {6.8, 0.2, 6.7}, py[3] = {0.0, 0.1, -0.3};
  const double pu[3] = {0.1, -0.2, 0.05}, pw[3] = {1e-3, 1e-3, 1e-3};
  if (orc_set_particles(o, 3, pz, px, py, pu, pu, pu, pw, 1)) return 11;
  orc_step(o, 2);
  orc_gather(o, 3.3, 1.2, -2.1, EB);
  if (!(orc_kinetic(o) >= 0.0)) return 8;
  free(ord);
  free(buf);
  orc_destroy(o);
  return 0;
}

int main(void) {
  const double yee[1] = {1.0};
  const double two[2] = {1.1, -1.0 / 30.0};  /* sum (2l - 1) C_l = 1 */
  for (int M = 0; M <= 3; ++M) {
    int rc = run(M, 1, yee, 1, 0, 0);
    if (!rc) rc = run(M, 2, two, 1, 0, 0);
    if (!rc) rc = run(M, 2, two, 2, 0, 0);  /* quadratic shapes */
    if (!rc) rc = run(M, 2, two, 2, 2, 1);  /* quadratic, moving window, exact J_z */
    if (rc) {
      fprintf(stderr, "oracle run M=%d failed: %d\n", M, rc);
      return rc;
    }
  }
  puts("oracle ok");
  return 0;
}
