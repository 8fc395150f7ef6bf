/* Drives the C oracle through every entry point on small grids, for a build
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

static int run(int M, int N, const double *C) {
  const int Nz = 24, Nr = 8;
  orc *o = orc_create(Nz, Nr, M, 0.4, 1.6, 0.15, N, C, C);
  if (!o) return 1;
  if (orc_load_plasma(o, 2, 0.02, 2.0, 4.0, 7u, 12, 8.0, 3.0)) return 2;
  if (M >= 1 && orc_add_laser(o, 1.5, 4.0, 3.0, 4.8, 1.0)) return 3;
  orc_start_fields(o);
  orc_set_flags(o, 0, 1);
  orc_deposit_rho(o);
  orc_step(o, 6);
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
    int rc = run(M, 1, yee);
    if (!rc) rc = run(M, 2, two);
    if (rc) {
      fprintf(stderr, "oracle run M=%d failed: %d\n", M, rc);
      return rc;
    }
  }
  puts("oracle ok");
  return 0;
}
