// dla.hip -- ensemble integration of the reduced model of an electron in a
// bubble with a laser pulse (Sec. II, Eq. (8); integration as in App. A).
//
// Units c = omega_p = 1, charge -1, motion in the x-z plane.  State per
// electron: x, zeta = z - t, xd, zetad (zd = zetad + 1).  The right-hand side
// is Eq. (8) written explicitly: with G the laser force terms minus the bubble
// terms (the force over gamma), gamma-dot / gamma = G . v, and the
// accelerations are G - (G . v) v.  One thread integrates one electron from
// its injection time t0 to t_end in n = ceil((t_end - t0) / h) equal steps of
// the fifth-order Dormand-Prince solution (six stages).  Everything is FP64;
// the electrons are independent, so the kernel is bound by FP64 arithmetic
// (Bessel functions, sincos and the stage algebra), not by memory.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pic_internal.h"

namespace pic {
namespace {

constexpr double kDlaMaxSteps = 16777216.0;  // steps per electron, 2^24

struct Model {
  double a0, kz, vphi, w0, kperp, kk, kpz, cB, wake;  // kk = (kperp/kz)^2, kpz = kperp/kz
};

// J0(s) and J1(s)/s from their power series in q = s^2/4,
//   J0 = sum_k (-q)^k / (k!)^2,   J1/s = (1/2) sum_k (-q)^k / (k! (k+1)!),
// 15 terms: absolute error below 1e-15 for |s| <= 3, which covers electrons
// inside the bubble (k_perp x <= 3); beyond it the library's j0, j1 are used.
constexpr int kBesselTerms = 15;
constexpr double kBesselSeriesMax = 3.0;
struct BesselSeries {
  double j0[kBesselTerms], j1s[kBesselTerms];
};
constexpr BesselSeries make_bessel_series() {
  BesselSeries c{};
  double f = 1.0;  // k!
  for (int k = 0; k < kBesselTerms; ++k) {
    if (k > 0) f *= k;
    const double sg = (k % 2 == 0) ? 1.0 : -1.0;
    c.j0[k] = sg / (f * f);
    c.j1s[k] = 0.5 * sg / (f * f * (k + 1));
  }
  return c;
}

// J0 and J1 beyond the series' range (electrons outside the bubble), out of
// line so that the main path is not allocated around the library's code
__device__ __noinline__ void bessel_far(double s, double *a, double *b) {
  *a = j0(s);
  *b = j1(s);
}

// d/dt (x, zeta, xd, zetad) at time t
__device__ __forceinline__ void dla_rhs(const Model &m, double t, const double y[4], double d[4]) {
  const double x = y[0], zeta = y[1], u = y[2], w = y[3];
  const double zd = w + 1.0;
  const double ig = sqrt(-w * (2.0 + w) - u * u);  // 1 / gamma = (1 - v^2)^(1/2), free of the cancellation of 1 - zd^2
  const double wb2 = 0.5 * ig;                       // omega_beta^2 = 1 / (2 gamma), Eq. (1)
  const double xi = zeta + (1.0 - m.vphi) * t;
  double sn, cs;
  sincos(m.kz * xi, &sn, &cs);
  const double s = m.kperp * x;
  double j0v, j1v, j1p;  // J0(s), J1(s), J1'(s) = J0 - J1/s
  if (fabs(s) <= kBesselSeriesMax) {
    constexpr BesselSeries C = make_bessel_series();
    const double q = 0.25 * s * s;
    double a = C.j0[kBesselTerms - 1], b = C.j1s[kBesselTerms - 1];
#pragma unroll
    for (int k = kBesselTerms - 2; k >= 0; --k) {
      a = fma(a, q, C.j0[k]);
      b = fma(b, q, C.j1s[k]);
    }
    j0v = a;
    j1v = b * s;
    j1p = a - b;
  } else {
    bessel_far(s, &j0v, &j1v);
    j1p = j0v - j1v / s;
  }
  const double amp = m.a0 * ig;
  const double mag = m.cB * m.kz * (j0v + m.kk * j1p) * sn;  // magnetic terms, per unit velocity
  const double gx = amp * (m.w0 * j0v * sn - zd * mag) - m.wake * 0.5 * wb2 * (1.0 + zd) * x;
  const double gz = -amp * (m.kpz * m.w0 * j1v * cs - u * mag) - m.wake * wb2 * (zeta - 0.5 * x * u);
  const double gv = gx * u + gz * zd;  // gamma-dot / gamma
  d[0] = u;
  d[1] = w;
  d[2] = gx - gv * u;
  d[3] = gz - gv * zd;
}

__global__ __launch_bounds__(256) void dla_kernel(const Model m, long long n, const double *__restrict__ t0,
                                                  double *__restrict__ X, double *__restrict__ Z,
                                                  double *__restrict__ U, double *__restrict__ W, double t_end,
                                                  double h) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // Dormand & Prince (1980): nodes, stage coefficients and fifth-order weights
  constexpr double c2 = 1.0 / 5.0, c3 = 3.0 / 10.0, c4 = 4.0 / 5.0, c5 = 8.0 / 9.0;
  constexpr double a21 = 1.0 / 5.0;
  constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
  constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
  constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0, a54 = -212.0 / 729.0;
  constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0, a64 = 49.0 / 176.0,
                   a65 = -5103.0 / 18656.0;
  constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0, b5 = -2187.0 / 6784.0,
                   b6 = 11.0 / 84.0;
  const double ts = t0[i];
  const double span = t_end - ts;
  const double nsd = span > 0.0 ? ceil(span / h) : 0.0;
  if (!(nsd <= kDlaMaxSteps)) {  // too many steps (or NaN times): the electron is not integrated
    X[i] = Z[i] = U[i] = W[i] = NAN;
    return;
  }
  const long long ns = (long long)nsd;
  const double hs = ns > 0 ? span / (double)ns : 0.0;
  double y[4] = {X[i], Z[i], U[i], W[i]};
  for (long long k = 0; k < ns; ++k) {
    const double t = ts + (double)k * hs;
    double k1[4], k2[4], k3[4], k4[4], k5[4], k6[4], yt[4];
    dla_rhs(m, t, y, k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) yt[q] = y[q] + hs * (a21 * k1[q]);
    dla_rhs(m, t + c2 * hs, yt, k2);
#pragma unroll
    for (int q = 0; q < 4; ++q) yt[q] = y[q] + hs * (a31 * k1[q] + a32 * k2[q]);
    dla_rhs(m, t + c3 * hs, yt, k3);
#pragma unroll
    for (int q = 0; q < 4; ++q) yt[q] = y[q] + hs * (a41 * k1[q] + a42 * k2[q] + a43 * k3[q]);
    dla_rhs(m, t + c4 * hs, yt, k4);
#pragma unroll
    for (int q = 0; q < 4; ++q) yt[q] = y[q] + hs * (a51 * k1[q] + a52 * k2[q] + a53 * k3[q] + a54 * k4[q]);
    dla_rhs(m, t + c5 * hs, yt, k5);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      yt[q] = y[q] + hs * (a61 * k1[q] + a62 * k2[q] + a63 * k3[q] + a64 * k4[q] + a65 * k5[q]);
    dla_rhs(m, t + hs, yt, k6);
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] += hs * (b1 * k1[q] + b3 * k3[q] + b4 * k4[q] + b5 * k5[q] + b6 * k6[q]);
  }
  X[i] = y[0];
  Z[i] = y[1];
  U[i] = y[2];
  W[i] = y[3];
}

}  // namespace

int launch_dla(const pic_dla_model &d, long long n, const double *t0, double *x, double *zeta, double *xd, double *zetad,
               double t_end, double h, void *stream) {
  if (n == 0) return PIC_OK;
  Model m;
  m.a0 = d.a0;
  m.kz = d.kz;
  m.vphi = d.vphi;
  m.w0 = d.kz * d.vphi;
  m.kperp = sqrt(m.w0 * m.w0 - d.kz * d.kz);
  m.kpz = m.kperp / d.kz;
  m.kk = m.kpz * m.kpz;
  m.cB = d.cB;
  m.wake = d.wake;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  dla_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>(m, n, t0, x, zeta, xd, zetad, t_end, h);
  return record_device_error((int)hipGetLastError(), "dla_kernel");
}

}  // namespace pic
