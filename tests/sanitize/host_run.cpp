// Drives the library's host set-up code (coefficient fit, Courant limit,
// electron loading, laser fields) on small runs, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
// compiled and run by tests/test_sanitizers.py with the host sources only).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../paper_2303_12874_amd/csrc/pic_internal.h"

using namespace pic;

int main() {
  for (int M = 0; M <= 3; ++M) {
    pic_run_desc d;
    std::memset(&d, 0, sizeof d);
    d.Nz = 48;
    d.Nr = 10;
    d.M = M;
    d.ppc = 3;
    d.dz = 0.39;
    d.dr = 1.57;
    d.n0 = 0.01;
    d.ramp_start = 2.0;
    d.ramp_len = 6.0;
    d.down_start = 10.0;
    d.down_len = 4.0;
    d.n_pulses = M >= 1 ? 1 : 0;
    d.pulse[0].a0 = 1.0;
    d.pulse[0].w0 = 6.0;
    d.pulse[0].tau = 4.0;
    d.pulse[0].zc = 9.0;
    d.taper = 2.0;
    d.seed = 99;
    d.n_tracked = 20;
    const double lim = courant_limit_fitted(PIC_SOLVER_DUAL, 16, M, d.dz, d.dr, 2.0943951023931953);
    std::vector<double> CE(16), CB(16);
    fit_dual(16, 0.95 * lim, 2.0943951023931953, CE.data(), CB.data());
    const double yee = courant_limit_fitted(PIC_SOLVER_YEE, 1, M, d.dz, d.dr, 0.0);
    if (!(lim > 0 && lim <= 1 && yee > 0 && yee <= 1)) {
      std::fprintf(stderr, "Courant limits M=%d: dual %g, Yee %g\n", M, lim, yee);
      return 1;
    }
    const int64_t np = run_particle_count(d);
    std::vector<double> z(np), x(np), y(np), w(np);
    std::vector<int64_t> id(np), tr(d.n_tracked);
    load_electrons(d, z.data(), x.data(), y.data(), w.data(), id.data(), tr.data());
    const size_t nvec = (size_t)3 * (2 * M + 1) * (size_t)(d.Nr + 1) * d.Nz;
    std::vector<double> E(nvec, 0.0), B(nvec, 0.0);
    laser_fields(d, E.data(), B.data());
  }
  std::puts("host ok");
  return 0;
}
