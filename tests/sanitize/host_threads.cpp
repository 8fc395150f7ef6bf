// Drives the library's host set-up code from several threads at once (the
// memo of fitted Courant limits, the once-initialised radial eigenvalues, the
// coefficient fit, the inverse-filter taps and the multithreaded loader), for
// a build with ThreadSanitizer: each thread's results must equal the serial
// ones.  Test infrastructure, compiled and run by tests/test_sanitizers.py
// with the host sources only.
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "../../paper_2303_12874_amd/csrc/pic_internal.h"

using namespace pic;

namespace {

struct Result {
  double lim[4], yee[4];
  std::vector<double> CB, h, w;
  int nh = 0;
};

pic_run_desc small_run(int M) {
  pic_run_desc d;
  std::memset(&d, 0, sizeof d);
  d.Nz = 40;
  d.Nr = 8;
  d.M = M;
  d.ppc = 2;
  d.dz = 0.39;
  d.dr = 1.57;
  d.n0 = 0.01;
  d.ramp_len = 4.0;
  d.seed = 7;
  d.n_tracked = 5;
  return d;
}

Result work(int salt) {
  Result r;
  const double band = 2.0943951023931953;
  for (int M = 0; M <= 3; ++M) {
    r.lim[M] = courant_limit_fitted(PIC_SOLVER_DUAL, 16, M, 0.39, 1.57, band);
    r.yee[M] = courant_limit_fitted(PIC_SOLVER_YEE, 1, M, 0.39 + 0.01 * (salt % 2), 1.57, 0.0);
  }
  std::vector<double> CE(16);
  r.CB.resize(16);
  fit_dual(16, 0.7, band, CE.data(), r.CB.data());
  r.h.resize(128);
  jz_inverse_taps(r.CB.data(), 16, 0x1p-53, 128, r.h.data(), &r.nh);
  const pic_run_desc d = small_run(2);
  const int64_t np = run_particle_count(d);
  std::vector<double> z(np), x(np), y(np);
  std::vector<int64_t> id(np), tr(d.n_tracked);
  r.w.resize(np);
  load_electrons(d, z.data(), x.data(), y.data(), r.w.data(), id.data(), tr.data());
  return r;
}

bool same(const Result &a, const Result &b) {
  for (int M = 0; M <= 3; ++M)
    if (a.lim[M] != b.lim[M]) return false;
  return a.CB == b.CB && a.nh == b.nh && a.h == b.h && a.w == b.w;
}

}  // namespace

int main() {
  const int nt = 6;
  std::vector<Result> res(nt);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back([&res, t] { res[(size_t)t] = work(t); });
  for (auto &x : th) x.join();
  const Result serial = work(0);
  for (int t = 0; t < nt; ++t)
    if (!same(res[(size_t)t], serial)) {
      std::fprintf(stderr, "thread %d differs from the serial result\n", t);
      return 1;
    }
  std::puts("threads ok");
  return 0;
}
