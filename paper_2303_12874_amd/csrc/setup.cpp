// setup.cpp -- host-side (FP64) setup of a run: dual-solver coefficients,
// Courant limit, electron loading and laser initialisation.  Runs once per
// run inside pic_init; nothing here is on the per-step path.
#include "pic_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

namespace pic {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Least squares min |A x - b| for a column-major m x n matrix (m >= n) by
// Householder QR.  A and b are overwritten.
void householder_lstsq(std::vector<double> &A, int m, int n, std::vector<double> &b,
                       std::vector<double> &x) {
  for (int k = 0; k < n; ++k) {
    double *col = &A[(size_t)k * m];
    double norm = 0.0;
    for (int i = k; i < m; ++i) norm += col[i] * col[i];
    norm = std::sqrt(norm);
    if (norm == 0.0) continue;
    double alpha = col[k] > 0 ? -norm : norm;
    // v = col[k:] - alpha e1, stored in place
    col[k] -= alpha;
    double vnorm2 = 0.0;
    for (int i = k; i < m; ++i) vnorm2 += col[i] * col[i];
    for (int j = k + 1; j < n; ++j) {
      double *cj = &A[(size_t)j * m];
      double s = 0.0;
      for (int i = k; i < m; ++i) s += col[i] * cj[i];
      s = 2.0 * s / vnorm2;
      for (int i = k; i < m; ++i) cj[i] -= s * col[i];
    }
    double s = 0.0;
    for (int i = k; i < m; ++i) s += col[i] * b[i];
    s = 2.0 * s / vnorm2;
    for (int i = k; i < m; ++i) b[i] -= s * col[i];
    // R(k,k) = alpha; keep it on the diagonal slot (the reflector is no longer needed)
    col[k] = alpha;
  }
  x.assign(n, 0.0);
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[(size_t)j * m + k] * x[j];
    x[k] = s / A[(size_t)k * m + k];
  }
}

// dz * symbol of a staggered difference: sum_l C_l 2 sin((2l-1) kappa/2)
double symbol_dz(const double *C, int N, double kappa) {
  double s = 0.0;
  for (int l = 1; l <= N; ++l) s += C[l - 1] * 2.0 * std::sin((2 * l - 1) * kappa * 0.5);
  return s;
}

}  // namespace

// Fit of the dual operators (Sec. III.A).  Eqs. (11) and (15) fix the two
// symbols separately (their product and ratio): dz[k]_E = tan(nu kappa/2)/(nu/2),
// dz[k]_B = sin(nu kappa)/nu with kappa = k dz and nu = c dt/dz.  Each operator is
// a least-squares fit on kappa in (0, band] (midpoint samples) under
// sum_l (2l-1) C_l = 1 (the operator is a consistent first derivative); the
// constraint is removed by writing C = g/|g|^2 + Z y with Z an orthonormal
// basis of the complement of g = (1, 3, 5, ...) (a Householder reflector).
void fit_dual(int N, double nu, double band, double *CE, double *CB) {
  if (N == 1) {
    CE[0] = CB[0] = 1.0;
    return;
  }
  const int ns = kFitSamples;
  std::vector<double> g(N), cp(N);
  double gg = 0.0;
  for (int l = 0; l < N; ++l) { g[l] = 2.0 * l + 1.0; gg += g[l] * g[l]; }
  for (int l = 0; l < N; ++l) cp[l] = g[l] / gg;
  // Householder H = I - 2 v v^T / v.v with H g = -sign(g0)|g| e1; columns 1..N-1 of H span g-perp.
  std::vector<double> v(g);
  double gn = std::sqrt(gg);
  v[0] += gn;  // g0 > 0
  double vv = 0.0;
  for (int l = 0; l < N; ++l) vv += v[l] * v[l];
  std::vector<double> Z((size_t)N * (N - 1));  // column-major N x (N-1)
  for (int c = 1; c < N; ++c)
    for (int r = 0; r < N; ++r) Z[(size_t)(c - 1) * N + r] = (r == c ? 1.0 : 0.0) - 2.0 * v[r] * v[c] / vv;
  // A (ns x N) and AZ (ns x (N-1)), A cp (ns)
  std::vector<double> A((size_t)ns * N), Acp(ns);
  for (int s = 0; s < ns; ++s) {
    double kap = (s + 0.5) * band / ns;
    double acc = 0.0;
    for (int l = 0; l < N; ++l) {
      double a = 2.0 * std::sin((2 * l + 1) * kap * 0.5);
      A[(size_t)s * N + l] = a;
      acc += a * cp[l];
    }
    Acp[s] = acc;
  }
  for (int which = 0; which < 2; ++which) {
    std::vector<double> AZ((size_t)ns * (N - 1)), rhs(ns), y;
    for (int c = 0; c < N - 1; ++c)
      for (int s = 0; s < ns; ++s) {
        double acc = 0.0;
        for (int l = 0; l < N; ++l) acc += A[(size_t)s * N + l] * Z[(size_t)c * N + l];
        AZ[(size_t)c * ns + s] = acc;
      }
    for (int s = 0; s < ns; ++s) {
      double kap = (s + 0.5) * band / ns;
      double t = which == 0 ? std::tan(0.5 * nu * kap) / (0.5 * nu) : std::sin(nu * kap) / nu;
      rhs[s] = t - Acp[s];
    }
    householder_lstsq(AZ, ns, N - 1, rhs, y);
    double *C = which == 0 ? CE : CB;
    for (int l = 0; l < N; ++l) {
      double acc = cp[l];
      for (int c = 0; c < N - 1; ++c) acc += Z[(size_t)c * N + l] * y[c];
      C[l] = acc;
    }
  }
}

// max and min over kappa in (0, pi] of dz^2 [k]_B [k]_E.
void z_product_range(const double *CE, const double *CB, int N, double *pmax, double *pmin) {
  double hi = -1e300, lo = 1e300;
  for (int s = 1; s < kKappaSamples; ++s) {
    double kap = kPi * s / (kKappaSamples - 1);
    double p = symbol_dz(CE, N, kap) * symbol_dz(CB, N, kap);
    hi = std::max(hi, p);
    lo = std::min(lo, p);
  }
  *pmax = hi;
  *pmin = lo;
}

// Largest eigenvalue (times dr^2) of curl_B curl_E of mode m with no z
// variation, with the axis and wall rules of the field update, by power
// iteration (the operator is similar to a symmetric one with a clear gap).
double radial_lambda(int m, int nr) {
  typedef std::complex<double> cd;
  const double dr = 1.0;
  const cd im(0.0, (double)m);
  const int n = nr + 1;
  std::vector<cd> Er(n), Ep(n), Ez(n), Br(n), Bp(n), Bz(n), Lr(n), Lp(n), Lz(n);
  for (int j = 0; j < n; ++j) {  // deterministic start vector
    Er[j] = cd(1.0 + 0.1 * j, 0.3);
    Ep[j] = cd(0.5, -0.2 * j);
    Ez[j] = cd(0.7 - 0.01 * j, 0.1);
  }
  auto clean = [&](std::vector<cd> &r, std::vector<cd> &p, std::vector<cd> &z) {
    r[nr] = 0.0;
    p[nr] = 0.0;
    z[nr] = 0.0;
    if (m != 1) p[0] = 0.0;
    if (m != 0) z[0] = 0.0;
  };
  clean(Er, Ep, Ez);
  double mu = 0.0;
  for (int it = 0; it < 4000; ++it) {
    for (int j = 0; j < n; ++j) {
      if (j == 0) Br[j] = (m == 1) ? cd(0.0, 1.0) * Ez[1] / dr : cd(0.0);
      else Br[j] = im / (j * dr) * Ez[j];
      if (j < nr) {
        double rh = (j + 0.5) * dr;
        Bp[j] = -(Ez[j + 1] - Ez[j]) / dr;
        Bz[j] = ((j + 1) * dr * Ep[j + 1] - j * dr * Ep[j]) / (rh * dr) - im / rh * Er[j];
      } else {
        Bp[j] = 0.0;
        Bz[j] = 0.0;
      }
    }
    for (int j = 0; j < n; ++j) {
      Lr[j] = j < nr ? im / ((j + 0.5) * dr) * Bz[j] : cd(0.0);
      if (j == nr || (j == 0 && m != 1)) Lp[j] = 0.0;
      else if (j == 0) Lp[j] = -2.0 * Bz[0] / dr;
      else Lp[j] = -(Bz[j] - Bz[j - 1]) / dr;
      if (j == nr || (j == 0 && m != 0)) Lz[j] = 0.0;
      else if (j == 0) Lz[j] = 4.0 * Bp[0] / dr;
      else Lz[j] = ((j + 0.5) * Bp[j] - (j - 0.5) * Bp[j - 1]) / (j * dr) - im / (j * dr) * Br[j];
    }
    double nrm = 0.0, nv = 0.0;
    for (int j = 0; j < n; ++j) {
      nrm += std::norm(Lr[j]) + std::norm(Lp[j]) + std::norm(Lz[j]);
      nv += std::norm(Er[j]) + std::norm(Ep[j]) + std::norm(Ez[j]);
    }
    mu = std::sqrt(nrm / nv);
    double s = 1.0 / std::sqrt(nrm);
    for (int j = 0; j < n; ++j) { Er[j] = Lr[j] * s; Ep[j] = Lp[j] * s; Ez[j] = Lz[j] * s; }
  }
  return mu * dr * dr;
}

double radial_lambda_max(int M) {
  // every mode's eigenvalue, computed once (thread-safe static initialisation)
  static const std::array<double, PIC_MAX_MODES + 1> lam = [] {
    std::array<double, PIC_MAX_MODES + 1> v{};
    for (int m = 0; m <= PIC_MAX_MODES; ++m) v[(size_t)m] = radial_lambda(m, 32);
    return v;
  }();
  double out = 0.0;
  for (int m = 0; m <= M; ++m) out = std::max(out, lam[(size_t)m]);
  return out;
}

// (nu/2)^2 (max dz^2 [k]_B[k]_E + Lambda_M (dz/dr)^2): stable iff <= 1 and the
// product is nowhere negative.
bool stable_at(const double *CE, const double *CB, int N, int M, double dz, double dr, double nu) {
  double pmax, pmin;
  z_product_range(CE, CB, N, &pmax, &pmin);
  double s = 0.25 * nu * nu * (pmax + radial_lambda_max(M) * (dz / dr) * (dz / dr));
  return s <= 1.0 && pmin >= 0.0;
}

double courant_limit_of(const double *CE, const double *CB, int N, int M, double dz, double dr) {
  double pmax, pmin;
  z_product_range(CE, CB, N, &pmax, &pmin);
  if (pmin < 0.0) return 0.0;
  return 2.0 / std::sqrt(pmax + radial_lambda_max(M) * (dz / dr) * (dz / dr));
}

// Bisection on c dt/dz with a refit at every trial (the targets depend on dt).
// The fitted limit depends on dz and dr only through dz/dr; runs that share
// (solver, N, M, dz/dr, band) -- the cells of a resolution scan -- share it.
static double courant_limit_search(int solver, int N, int M, double dz, double dr, double band);

double courant_limit_fitted(int solver, int N, int M, double dz, double dr, double band) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, double, double>, double> memo;
  const auto key = std::make_tuple(solver, N, M, dz / dr, band);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  const double lim = courant_limit_search(solver, N, M, dz, dr, band);
  std::lock_guard<std::mutex> lk(mu);
  memo[key] = lim;
  return lim;
}

static double courant_limit_search(int solver, int N, int M, double dz, double dr, double band) {
  std::vector<double> CE(N), CB(N);
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    double mid = 0.5 * (lo + hi);
    if (solver == PIC_SOLVER_YEE) { CE[0] = CB[0] = 1.0; }
    else fit_dual(N, mid, band, CE.data(), CB.data());
    if (stable_at(CE.data(), CB.data(), solver == PIC_SOLVER_YEE ? 1 : N, M, dz, dr, mid)) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Inverse of the z filter P (taps p_l = sum_{l' > |l|} C^B_{l'}).  P is a
// convolution with symbol P(k) = p_0 + 2 sum_{l >= 1} p_l cos(l k dz), a
// positive trigonometric polynomial for the usual fits, so 1/P(k) is smooth
// and its Fourier coefficients h_l decay geometrically: h is P^{-1} on the
// infinite line, and a cut where the taps fall below eps h_0 leaves an error
// of that order.  h_l = (1/K) sum_q cos(2 pi q l / K) / P(2 pi q / K) with
// K = 8192 samples (the aliasing of the K-periodic series is h_{K-l}, nil),
// summed in the host's extended precision so that the rounding of the sums
// stays far below the FP64 cut.
int jz_inverse_taps(const double *CB, int N, double eps, int max_taps, double *h, int *nh) {
  using X = long double;
  constexpr int K = 8192;
  std::vector<X> p((size_t)N, 0.0L);  // p_0 .. p_{N-1}
  for (int l = 0; l < N; ++l)
    for (int lp = l + 1; lp <= N; ++lp) p[(size_t)l] += CB[lp - 1];
  std::vector<X> cs(K), inv(K);
  const X two_pi = 2.0L * 3.141592653589793238462643383279502884L;
  for (int k = 0; k < K; ++k) cs[(size_t)k] = std::cos(two_pi * k / K);
  for (int q = 0; q < K; ++q) {
    X P = p[0];
    for (int l = 1; l < N; ++l) P += 2.0L * p[(size_t)l] * cs[(size_t)((long long)l * q % K)];
    if (!(P > 0.0L)) return 1;
    inv[(size_t)q] = 1.0L / P;
  }
  const int scan = 2 * max_taps;  // taps examined beyond the cut
  std::vector<double> hh((size_t)scan);
  for (int l = 0; l < scan; ++l) {
    X acc = 0.0L;
    for (int q = 0; q < K; ++q) acc += cs[(size_t)((long long)l * q % K)] * inv[(size_t)q];
    hh[(size_t)l] = (double)(acc / K);
  }
  int n = 1;
  for (int l = 1; l < scan; ++l)
    if (std::fabs(hh[(size_t)l]) > eps * std::fabs(hh[0])) n = l + 1;
  if (n > max_taps) return 2;
  for (int l = 0; l < n; ++l) h[l] = hh[(size_t)l];
  *nh = n;
  return 0;
}

// ---------------------------------------------------------------------------
// loading: counter-based SplitMix64; draw d of electron pid is output number
// 4 pid + d + 1 of the stream seeded with `seed`.

static inline uint64_t splitmix_out(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline double draw(uint64_t seed, int64_t pid, int d) {
  return (double)(splitmix_out(seed, 4ULL * (uint64_t)pid + (uint64_t)d + 1ULL) >> 11) *
         (1.0 / 9007199254740992.0);
}

int64_t run_particle_count(const pic_run_desc &r) { return (int64_t)r.Nz * (r.Nr - 1) * r.ppc; }

// Electron pid of the plasma, in absolute column a and radial cell ir:
// absolute z (cells), x, y (cells) and weight.
static inline void plasma_electron(const pic_run_desc &r, int64_t pid, int64_t a, int ir, double *zc, double *x,
                                   double *y, double *w) {
#pragma clang fp contract(off)  // each operation rounded on its own, so that every loader gets these bits
  const double z = (double)a + draw(r.seed, pid, 0);
  const double rc = ir + draw(r.seed, pid, 1);
  const double phi = 2.0 * kPi * draw(r.seed, pid, 2);
  double n = r.n0;
  if (r.ramp_len > 0.0) {
    double f = (z * r.dz - r.ramp_start) / r.ramp_len;
    f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    n = r.n0 * f;
  }
  if (r.down_len > 0.0) {
    double g = 1.0 - (z * r.dz - r.down_start) / r.down_len;
    g = g < 0.0 ? 0.0 : (g > 1.0 ? 1.0 : g);
    n *= g;
  }
  *zc = z;
  *x = rc * std::cos(phi);
  *y = rc * std::sin(phi);
  *w = n * (2.0 * kPi) * (rc * r.dr) * r.dr * r.dz / r.ppc;
}

// The plasma of absolute columns [a0, a1) (all radial cells, ppc each, pid
// order), z in the cells of a box whose column 0 is absolute column S.
void load_columns(const pic_run_desc &r, int64_t a0, int64_t a1, int64_t S, double *z, double *x, double *y,
                  double *w, int64_t *id) {
  const int nrc = r.Nr - 1;
  int64_t p = 0;
  for (int64_t a = a0; a < a1; ++a)
    for (int ir = 0; ir < nrc; ++ir)
      for (int k = 0; k < r.ppc; ++k, ++p) {
        const int64_t pid = (a * nrc + ir) * r.ppc + k;
        double zc;
        plasma_electron(r, pid, a, ir, &zc, x + p, y + p, w + p);
        z[p] = zc - (double)S;
        id[p] = pid;
      }
}

// Cold electrons: ppc per cell for r < (Nr-1) dr at uniform-random (z, r, phi)
// in the cell; the density n(z) (with its linear up- and down-ramps) and the annulus
// volume enter the weight w = n 2 pi r dr dr dz / ppc, so the density is
// uniform in r.  The n_tracked electrons with the smallest (draw 3, pid) are
// tracked; tracked ids are returned ascending.
void load_electrons(const pic_run_desc &r, double *z, double *x, double *y, double *w, int64_t *id,
                    int64_t *tracked) {
  const int nrc = r.Nr - 1;
  const int64_t np = run_particle_count(r);
  const int nt_want = r.n_tracked > 0 && tracked ? r.n_tracked : 0;
  // Every draw is a pure function of (seed, pid, d), so z-columns load in
  // parallel with bit-identical results.  Each thread also keeps the
  // n_tracked smallest (U3, pid) of its columns; the union holds the global
  // n_tracked smallest.
  using Key = std::pair<double, int64_t>;
  unsigned nth = std::thread::hardware_concurrency();
  nth = nth < 1 ? 1 : (nth > 16 ? 16 : nth);
  if ((int64_t)nth > r.Nz) nth = (unsigned)r.Nz;
  std::vector<std::vector<Key>> best(nth);
  auto work = [&](unsigned t) {
    const int z0 = (int)((int64_t)r.Nz * t / nth), z1 = (int)((int64_t)r.Nz * (t + 1) / nth);
    std::vector<Key> &cand = best[t];
    for (int iz = z0; iz < z1; ++iz)
      for (int ir = 0; ir < nrc; ++ir)
        for (int s = 0; s < r.ppc; ++s) {
          int64_t pid = ((int64_t)iz * nrc + ir) * r.ppc + s;
          double zc, xc, yc, wc;
          plasma_electron(r, pid, iz, ir, &zc, &xc, &yc, &wc);
          if (z) z[pid] = zc;
          if (x) x[pid] = xc;
          if (y) y[pid] = yc;
          if (w) w[pid] = wc;
          if (id) id[pid] = pid;
          if (nt_want) {
            cand.push_back({draw(r.seed, pid, 3), pid});
            if (cand.size() >= 2 * (size_t)nt_want + 1024) {  // keep the n_tracked smallest
              std::nth_element(cand.begin(), cand.begin() + (nt_want - 1), cand.end());
              cand.resize((size_t)nt_want);
            }
          }
        }
  };
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nth; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto &th : pool) th.join();
  if (nt_want && np > 0) {
    std::vector<Key> keys;
    for (auto &c : best) keys.insert(keys.end(), c.begin(), c.end());
    std::nth_element(keys.begin(), keys.begin() + (nt_want - 1), keys.end());
    std::sort(keys.begin(), keys.begin() + nt_want);
    std::vector<int64_t> sel((size_t)nt_want);
    for (int k = 0; k < nt_want; ++k) sel[(size_t)k] = keys[(size_t)k].second;
    std::sort(sel.begin(), sel.end());
    for (int k = 0; k < nt_want; ++k) tracked[k] = sel[(size_t)k];
  }
}

// ---------------------------------------------------------------------------
// Laser of Eq. (18) near focus, x-polarised, in the m = 1 arrays at t = 0
// (k = omega = 1):  E_r^1 = E, E_phi^1 = i E, E_z^1 = (2 r/w0^2) A cos,
// B_r^1 = -i B, B_phi^1 = B, B_z^1 = -i (2 r/w0^2) A cos, with
// E = B = A sin(theta), theta = -(z - zc), A = a0 g(z) exp(-r^2/w0^2).
// Values are added into host arrays in device layout: plane (comp, q) of
// (Nr+1) x Nz reals, q = 1 (Re m=1), 2 (Im m=1).

static double pulse_envelope(double zp, const pic_pulse &p, double L, double taper) {
  double g = std::exp(-2.0 * std::log(2.0) * (zp - p.zc) * (zp - p.zc) / (p.tau * p.tau));
  if (taper > 0.0) {
    if (zp < taper) { double s = std::sin(0.5 * kPi * zp / taper); g *= s * s; }
    if (zp > L - taper) { double s = std::sin(0.5 * kPi * (L - zp) / taper); g *= s * s; }
  }
  return g;
}

void laser_fields(const pic_run_desc &r, double *E, double *B) {
  if (r.M < 1) return;
  const int Nz = r.Nz, Nr = r.Nr, NM = 2 * r.M + 1;
  const size_t plane = (size_t)(Nr + 1) * Nz;
  const double L = Nz * r.dz;
  auto at = [&](double *F, int comp, int q, int j, int i) -> double & {
    return F[((size_t)comp * NM + q) * plane + (size_t)j * Nz + i];
  };
  for (int pidx = 0; pidx < r.n_pulses; ++pidx) {
    const pic_pulse &p = r.pulse[pidx];
    const double w2 = p.w0 * p.w0;
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= Nr; ++j)
      for (int i = 0; i < Nz; ++i) {
        double zi = i * r.dz, zh = (i + 0.5) * r.dz, rj = j * r.dr, rh = (j + 0.5) * r.dr;
        double gi = pulse_envelope(zi, p, L, r.taper), gh = pulse_envelope(zh, p, L, r.taper);
        double thi = -(zi - p.zc), thh = -(zh - p.zc);
        if (j < Nr) {
          double A = p.a0 * gi * std::exp(-rh * rh / w2);  // (z_i, r_{j+1/2})
          at(E, 0, 1, j, i) += A * std::sin(thi);                       // E_r  (Re)
          at(B, 2, 2, j, i) += -(2.0 * rh / w2) * A * std::cos(thi);    // B_z  (Im)
          A = p.a0 * gi * std::exp(-rj * rj / w2);                     // (z_i, r_j)
          at(E, 1, 2, j, i) += A * std::sin(thi);                       // E_phi (Im)
          A = p.a0 * gh * std::exp(-rj * rj / w2);                     // (z_{i+1/2}, r_j)
          at(E, 2, 1, j, i) += (2.0 * rj / w2) * A * std::cos(thh);     // E_z  (Re)
          at(B, 0, 2, j, i) += -A * std::sin(thh);                      // B_r  (Im)
          A = p.a0 * gh * std::exp(-rh * rh / w2);                     // (z_{i+1/2}, r_{j+1/2})
          at(B, 1, 1, j, i) += A * std::sin(thh);                       // B_phi (Re)
        } else {
          double A = p.a0 * gh * std::exp(-rj * rj / w2);
          at(B, 0, 2, j, i) += -A * std::sin(thh);  // B_r on the wall row
        }
      }
  }
}

uint32_t sort_flags_text(uint32_t flags, int run, char *buf, size_t n) {
  if (!buf || n == 0) return flags;
  buf[0] = 0;
  if (!flags) return 0;
  int w = std::snprintf(buf, n, "run %d: the cell sort met inconsistent data and skipped it (electrons lost or "
                        "duplicated):", run);
  const struct {
    uint32_t bit;
    const char *what;
  } names[] = {{kSortBadCount, " cell counts do not sum to the electrons;"},
               {kSortBadTile, " a tile's electron range out of bounds;"},
               {kSortBadSlot, " a sorted slot out of bounds;"},
               {kSortBadSource, " a source electron out of bounds;"}};
  for (const auto &nm : names)
    if ((flags & nm.bit) && w >= 0 && (size_t)w < n) w += std::snprintf(buf + w, n - (size_t)w, "%s", nm.what);
  return flags;
}

}  // namespace pic
