// kernels.hip -- gfx950 kernels of the quasi-3D r-z PIC step with the dual
// Maxwell solver (arXiv 2303.12874, Sec. III).  One step of a run is
//   push:   gather E^n and (B^{n-1/2} + B^{n+1/2})/2 (Eq. (12)) at each
//           electron, Boris push (Eq. (6)), per-mode work of tracked
//           electrons (Eq. (16)), move, charge-conserving deposit of the
//           current J^{n+1/2} into the mode arrays (global atomics);
//   efield: E^{n+1} = E^n + dt (curl_B B^{n+1/2} - J'), J' = (P J_r, P J_phi, J_z)
//           with the z filter P that makes the two-point continuity of the
//           deposit hold for D_B (Gauss's law with [k]_B, Eq. (10));
//           also clears the other current buffer;
//   bfield: B^{n+3/2} = B^{n+1/2} - dt curl_E E^{n+1}, into the buffer that
//           held B^{n-1/2}.
// Every global index is clamped or wrapped into its array, whatever the
// particle data hold, so corrupted particles give NaN fields, not faults.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "pic_internal.h"

namespace pic {
namespace {

constexpr double kPi = 3.14159265358979323846;

template <typename R>
struct C2 {
  R re, im;
};

__device__ __forceinline__ int wrap_once(int c, int n) {
  c += (c < 0) ? n : 0;
  c -= (c >= n) ? n : 0;
  return c;
}
__device__ __forceinline__ int wrap_any(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// largest integer j with j^2 <= r2 (r = sqrt(r2) rounded)
template <typename R>
__device__ __forceinline__ int radial_index(R r2, R r) {
  int j = (int)floor(r);
  if ((R)j * (R)j > r2) j -= 1;
  if ((R)(j + 1) * (R)(j + 1) <= r2) j += 1;
  return j;
}

template <typename R>
__device__ __forceinline__ void atomic_add(R *a, R v) {
  unsafeAtomicAdd(a, v);
}

// mirror sign of plane q at r_{-1/2}: (-1)^{m+1} for r/phi components,
// (-1)^m for z components, m = (q+1)/2.
__host__ __device__ constexpr int mode_of(int q) { return (q + 1) / 2; }
__host__ __device__ constexpr int mirror_sign(int q, bool zcomp) {
  return ((mode_of(q) % 2 == 0) == zcomp) ? 1 : -1;
}

// Bilinear interpolation of the NM planes of one component.
template <typename R, int NM, bool HALF_R, bool ZCOMP>
__device__ __forceinline__ void interp(const R *__restrict__ F, long long plane, int Nz, int ca, int cb,
                                       int row0, bool mirror, R fz, R fr, R out[NM]) {
  const R w00 = (R(1) - fz) * (R(1) - fr), w10 = fz * (R(1) - fr);
  const R w01 = (R(1) - fz) * fr, w11 = fz * fr;
  const long long o0 = (long long)(mirror ? 0 : row0) * Nz;
  const long long o1 = (long long)(row0 + 1) * Nz;
#pragma unroll
  for (int q = 0; q < NM; ++q) {
    const R *P = F + q * plane;
    R v00 = P[o0 + ca], v10 = P[o0 + cb];
    if (HALF_R && mirror) {
      const R s = (R)mirror_sign(q, ZCOMP);
      v00 *= s;
      v10 *= s;
    }
    out[q] = w00 * v00 + w10 * v10 + w01 * P[o1 + ca] + w11 * P[o1 + cb];
  }
}

// One workgroup per sort tile of Tz x Tr cells.  The tile's electrons (the
// range the last cell sort assigned to it) are processed in contiguous
// per-thread chunks, so that at any instant the 64 lanes of a wavefront sit
// in different cells: their field reads fall on neighbouring nodes and their
// LDS atomics rarely collide.  The current of the whole tile is accumulated
// in LDS over the node window [z0-1, z0+Tz+2) x [r0-1, r0+Tr+2) (every move
// of less than one cell from a cell of the tile stays inside it) and added to
// the global arrays once; an electron that drifted out of the window since
// the last sort deposits straight to global memory.
template <typename R, int M>
__global__ __launch_bounds__(256) void push_kernel(KRun k, int par) {
  constexpr int NM = 2 * M + 1;
  constexpr bool F64 = std::is_same<R, double>::value;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  R *lds = (R *)lds_raw;
  const int tile = blockIdx.x;
  const int TZ = k.Tz, TR = k.Tr;
  const int WZ = TZ + 3, WR = TR + 3;
  const int tz = tile % k.ntz, tr = tile / k.ntz;
  const int zlo = tz * TZ - 1, rlo = tr * TR - 1;
  const long long TT = (long long)TZ * TR;
  const int beg = k.cell_start[tile * TT], end = k.cell_start[(tile + 1) * TT];
  if (beg >= end) return;
  const int nlds = 3 * NM * WZ * WR;
  for (int e = threadIdx.x; e < nlds; e += blockDim.x) lds[e] = R(0);
  __syncthreads();

  const int Nz = k.Nz, Nr = k.Nr;
  const long long plane = k.plane;
  const R dt = (R)k.dt, dz = (R)k.dz, dr = (R)k.dr;
  const R *E = (const R *)k.E;
  const R *Bb = (const R *)k.Bbar;
  R *J = (R *)k.J[par];
  R *X = (R *)k.px, *Y = (R *)k.py, *UX = (R *)k.pux, *UY = (R *)k.puy, *UZ = (R *)k.puz;

  // add v to component c (0 r, 1 phi, 2 z), plane q, node (row, unwrapped column)
  auto dep = [&](int c, int q, int row, int colu, R v) {
    const int lc = colu - zlo, lr = row - rlo;
    if ((unsigned)lc < (unsigned)WZ && (unsigned)lr < (unsigned)WR)
      atomic_add(&lds[((c * NM + q) * WR + lr) * WZ + lc], v);
    else
      atomic_add(J + (long long)(c * NM + q) * plane + (long long)row * Nz + wrap_once(colu, Nz), v);
  };

  const int n = end - beg;
  const int chunk = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  const int my0 = beg + (int)threadIdx.x * chunk;
  const int my1 = min(my0 + chunk, end);
  for (int p = my0; p < my1; ++p) {
    const R q = -((const R *)k.pw)[p];
    const uint32_t pidw = k.pid[p];

    // ---- old position ----
    int i0;
    R f0, z0 = 0;
    if constexpr (F64) {
      z0 = ((const double *)k.pz)[p];
      const R fl = floor(z0);
      i0 = (int)fl;
      f0 = z0 - fl;
    } else {
      i0 = ((const int *)k.pz)[p];
      f0 = ((const float *)k.pfz)[p];
    }
    i0 = wrap_any(i0, Nz);
    const R x0 = X[p], y0 = Y[p];
    const R r20 = fma(x0, x0, y0 * y0), r0 = sqrt(r20);
    const int j0 = clampi(radial_index(r20, r0), 0, Nr - 2);
    R c0 = 1, s0 = 0;
    if (r0 > R(0)) {
      c0 = x0 / r0;
      s0 = y0 / r0;
    }

    // ---- gather E^n and Bbar^n = (B^{n-1/2} + B^{n+1/2})/2 (Eq. (12)) ----
    int ih;
    R fh;
    if constexpr (F64) {
      const R zz = z0 - R(0.5);
      const R fl = floor(zz);
      ih = (int)fl;
      fh = zz - fl;
    } else {
      if (f0 >= R(0.5)) {
        ih = i0;
        fh = f0 - R(0.5);
      } else {
        ih = i0 - 1;
        fh = f0 + R(0.5);
      }
    }
    const int ci0 = i0, ci1 = wrap_once(i0 + 1, Nz);
    const int ch0 = wrap_any(ih, Nz), ch1 = wrap_once(ch0 + 1, Nz);
    const R fr = r0 - (R)j0;
    const R rr = r0 - R(0.5);
    const R flr = floor(rr);
    int jh = (int)flr;
    const R frh = rr - flr;
    jh = clampi(jh, -1, Nr - 2);
    const bool mir = jh < 0;

    R er[NM], ep[NM], ez[NM], br[NM], bp[NM], bz[NM];
    interp<R, NM, true, false>(E + 0 * NM * plane, plane, Nz, ci0, ci1, jh, mir, f0, frh, er);
    interp<R, NM, false, false>(E + 1 * NM * plane, plane, Nz, ci0, ci1, j0, false, f0, fr, ep);
    interp<R, NM, false, true>(E + 2 * NM * plane, plane, Nz, ch0, ch1, j0, false, fh, fr, ez);
    interp<R, NM, false, false>(Bb + 0 * NM * plane, plane, Nz, ch0, ch1, j0, false, fh, fr, br);
    interp<R, NM, true, false>(Bb + 1 * NM * plane, plane, Nz, ch0, ch1, jh, mir, fh, frh, bp);
    interp<R, NM, true, true>(Bb + 2 * NM * plane, plane, Nz, ci0, ci1, jh, mir, f0, frh, bz);

    // ---- reconstruct Re sum_m F^m e^{i m phi}, rotate to Cartesian ----
    R Em[M + 1][3];
    R Ec[3], Bc[3];
    {
      Em[0][0] = er[0] * c0 - ep[0] * s0;
      Em[0][1] = er[0] * s0 + ep[0] * c0;
      Em[0][2] = ez[0];
      Bc[0] = br[0] * c0 - bp[0] * s0;
      Bc[1] = br[0] * s0 + bp[0] * c0;
      Bc[2] = bz[0];
      R ere = 1, eim = 0;
#pragma unroll
      for (int m = 1; m <= M; ++m) {
        const R nre = ere * c0 - eim * s0;
        const R nim = ere * s0 + eim * c0;
        ere = nre;
        eim = nim;
        const int a = 2 * m - 1, b = 2 * m;
        const R Fr = er[a] * ere - er[b] * eim, Fp = ep[a] * ere - ep[b] * eim;
        Em[m][0] = Fr * c0 - Fp * s0;
        Em[m][1] = Fr * s0 + Fp * c0;
        Em[m][2] = ez[a] * ere - ez[b] * eim;
        const R Gr = br[a] * ere - br[b] * eim, Gp = bp[a] * ere - bp[b] * eim;
        Bc[0] += Gr * c0 - Gp * s0;
        Bc[1] += Gr * s0 + Gp * c0;
        Bc[2] += bz[a] * ere - bz[b] * eim;
      }
      Ec[0] = Em[0][0];
      Ec[1] = Em[0][1];
      Ec[2] = Em[0][2];
#pragma unroll
      for (int m = 1; m <= M; ++m) {
        Ec[0] += Em[m][0];
        Ec[1] += Em[m][1];
        Ec[2] += Em[m][2];
      }
    }

    // ---- Boris, q/m = -1 (Eq. (6)) ----
    const R u[3] = {UX[p], UY[p], UZ[p]};
    R um[3], up[3], un[3], tt[3], ss[3], u1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) um[a] = u[a] - R(0.5) * dt * Ec[a];
    const R gm = sqrt(R(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) tt[a] = -R(0.5) * dt * Bc[a] / gm;
    const R t2 = tt[0] * tt[0] + tt[1] * tt[1] + tt[2] * tt[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) ss[a] = R(2) * tt[a] / (R(1) + t2);
    u1[0] = um[0] + (um[1] * tt[2] - um[2] * tt[1]);
    u1[1] = um[1] + (um[2] * tt[0] - um[0] * tt[2]);
    u1[2] = um[2] + (um[0] * tt[1] - um[1] * tt[0]);
    up[0] = um[0] + (u1[1] * ss[2] - u1[2] * ss[1]);
    up[1] = um[1] + (u1[2] * ss[0] - u1[0] * ss[2]);
    up[2] = um[2] + (u1[0] * ss[1] - u1[1] * ss[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) un[a] = up[a] - R(0.5) * dt * Ec[a];
    const R g_new = sqrt(R(1) + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);

    // ---- per-mode work of tracked electrons (FP64), Eq. (16) ----
    if (pidw & kTrackedBit) {
      const int32_t idv = (int32_t)(pidw & kIdMask);
      int lo = 0, hi = k.n_tracked;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (k.tracked[mid] < idv) lo = mid + 1;
        else hi = mid;
      }
      if (lo < k.n_tracked && k.tracked[lo] == idv) {
        const double g_old = sqrt(1.0 + (double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]);
        const double inv = 1.0 / (g_old + (double)g_new);
        const double v0 = ((double)um[0] + (double)up[0]) * inv;
        const double v1 = ((double)um[1] + (double)up[1]) * inv;
        const double v2 = ((double)um[2] + (double)up[2]) * inv;
        double *W = k.W + (long long)lo * (M + 1);
#pragma unroll
        for (int m = 0; m <= M; ++m)
          W[m] += -k.dt * ((double)Em[m][0] * v0 + (double)Em[m][1] * v1 + (double)Em[m][2] * v2);
      }
    }

    // ---- move ----
    int i1;
    R f1;
    R z1 = 0;
    if constexpr (F64) {
      z1 = z0 + dt * un[2] / g_new / dz;
      const R fl = floor(z1);
      i1 = (int)fl;
      f1 = z1 - fl;
    } else {
      f1 = f0 + dt * un[2] / g_new / dz;
      i1 = i0;
      if (f1 >= R(1)) {
        f1 -= R(1);
        i1 += 1;
      } else if (f1 < R(0)) {
        f1 += R(1);
        i1 -= 1;
        if (f1 == R(1)) {
          f1 = R(0);
          i1 += 1;
        }
      }
    }
    R x1 = x0 + dt * un[0] / g_new / dr;
    R y1 = y0 + dt * un[1] / g_new / dr;
    const R Rw = (R)(Nr - 1);
    R r21 = fma(x1, x1, y1 * y1), r1 = sqrt(r21);
    if (r1 >= Rw) {  // specular reflection at r = (Nr - 1) dr
      const R nx = x1 / r1, ny = y1 / r1;
      const R sc = (R(2) * Rw - r1) / r1;
      x1 *= sc;
      y1 *= sc;
      const R ur = un[0] * nx + un[1] * ny;
      un[0] -= R(2) * ur * nx;
      un[1] -= R(2) * ur * ny;
      r21 = fma(x1, x1, y1 * y1);
      r1 = sqrt(r21);
      if (r1 >= Rw) {  // rounding left it on the wall: pull it just inside
        const R sc2 = (Rw * (R(1) - R(F64 ? 1e-12 : 1e-6))) / r1;
        x1 *= sc2;
        y1 *= sc2;
        r21 = fma(x1, x1, y1 * y1);
        r1 = sqrt(r21);
      }
    }
    int j1 = clampi(radial_index(r21, r1), j0 - 1, j0 + 1);
    j1 = clampi(j1, 0, Nr - 2);
    R c1 = 1, s1 = 0;
    if (r1 > R(0)) {
      c1 = x1 / r1;
      s1 = y1 / r1;
    }
    const R g1 = r1 - (R)j1;

    // ---- charge-conserving deposit of J^{n+1/2} ----
    {
      const R xm = R(0.5) * (x0 + x1), ym = R(0.5) * (y0 + y1);
      const R rm = sqrt(xm * xm + ym * ym);
      R cmid = 1, smid = 0, vphi = 0;
      if (rm > R(0)) {
        cmid = xm / rm;
        smid = ym / rm;
        vphi = (cmid * un[1] - smid * un[0]) / g_new;
      }
      const int di = clampi(i1 - i0, -1, 1);
      const int oz0 = di < 0 ? 1 : 0, oz1 = oz0 + di;  // cells of the two positions in the 3-node window
      const int ib = i0 - oz0;
      const int dj = j1 - j0;
      const int or0 = dj < 0 ? 1 : 0, or1 = or0 + dj;
      const int jb = j0 - or0;
      R Sz0[3], Sz1[3], Sr0[3], Sr1[3];
      const R g0 = fr;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Sz0[a] = (a == oz0) ? R(1) - f0 : ((a == oz0 + 1) ? f0 : R(0));
        Sz1[a] = (a == oz1) ? R(1) - f1 : ((a == oz1 + 1) ? f1 : R(0));
        Sr0[a] = (a == or0) ? R(1) - g0 : ((a == or0 + 1) ? g0 : R(0));
        Sr1[a] = (a == or1) ? R(1) - g1 : ((a == or1 + 1) ? g1 : R(0));
      }
      R Wz[3][3], Wr[3][3], Ss[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          Wz[a][b] = (Sz1[a] - Sz0[a]) * (Sr0[b] + Sr1[b]) * R(0.5);
          Wr[a][b] = (Sr1[b] - Sr0[b]) * (Sz0[a] + Sz1[a]) * R(0.5);
          Ss[a][b] = Sz0[a] * Sr0[b] + Sz1[a] * Sr1[b];
        }
      // e^{-i m phi} at the old, new and mid positions, by recurrence
      R e0r = 1, e0i = 0, e1r = 1, e1i = 0, emr = 1, emi = 0;
#pragma unroll
      for (int m = 0; m <= M; ++m) {
        if (m > 0) {
          R tr_ = e0r * c0 + e0i * s0, ti = e0i * c0 - e0r * s0;
          e0r = tr_;
          e0i = ti;
          tr_ = e1r * c1 + e1i * s1;
          ti = e1i * c1 - e1r * s1;
          e1r = tr_;
          e1i = ti;
          tr_ = emr * cmid + emi * smid;
          ti = emi * cmid - emr * smid;
          emr = tr_;
          emi = ti;
        }
        const R cq = (m == 0 ? R(1) : R(2)) * q;
        const R xr = R(0.5) * (e0r + e1r), xi = R(0.5) * (e0i + e1i);
        const int qa = m == 0 ? 0 : 2 * m - 1, qb = 2 * m;
        // J_z at (ib+a+1/2, jb+b): minus the running sum of Wz behind the face
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          R run = 0;
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            run += Wz[a][b];
            const R v = -cq * run;
            dep(2, qa, jb + b, ib + a, v * xr);
            if (m > 0) dep(2, qb, jb + b, ib + a, v * xi);
          }
        }
        // J_r at (ib+a, jb+b+1/2)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          R run = 0;
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            run += Wr[a][b];
            const R v = -cq * run;
            dep(0, qa, jb + b, ib + a, v * xr);
            if (m > 0) dep(0, qb, jb + b, ib + a, v * xi);
          }
        }
        // J_phi at (ib+a, jb+b)
        const R dre = e1r - e0r, dim_ = e1i - e0i;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const int j = jb + b;
            const R h = R(0.5) * cq * Ss[a][b];
            if (m == 0) {
              dep(1, 0, j, ib + a, h * vphi);
            } else if (m == 1 && j == 0) {
              dep(1, qa, j, ib + a, h * vphi * emr);
              dep(1, qb, j, ib + a, h * vphi * emi);
            } else if (j > 0) {  // the closure carries r_j: nothing on the axis
              // (i/m)(e1 - e0) = (-(e1-e0).im, (e1-e0).re) / m
              dep(1, qa, j, ib + a, -h * dim_ / (R)m);
              dep(1, qb, j, ib + a, h * dre / (R)m);
            }
          }
      }
    }

    // ---- store (periodic in z) ----
    if constexpr (F64) {
      if (z1 < R(0)) z1 += (R)Nz;
      if (z1 >= (R)Nz) z1 -= (R)Nz;
      ((double *)k.pz)[p] = z1;
    } else {
      ((int *)k.pz)[p] = wrap_any(i1, Nz);
      ((float *)k.pfz)[p] = f1;
    }
    X[p] = x1;
    Y[p] = y1;
    UX[p] = un[0];
    UY[p] = un[1];
    UZ[p] = un[2];
  }

  // ---- flush the tile's current ----
  __syncthreads();
  for (int e = threadIdx.x; e < nlds; e += blockDim.x) {
    const R v = lds[e];
    if (v == R(0)) continue;
    const int lc = e % WZ;
    const int rest = e / WZ;
    const int lr = rest % WR;
    const int cq = rest / WR;  // c * NM + q
    const int row = rlo + lr;
    if (row < 0 || row > Nr) continue;
    atomic_add(J + (long long)cq * plane + (long long)row * Nz + wrap_once(zlo + lc, Nz), v);
  }
}

// ---------------------------------------------------------------------------
// field update

template <typename R>
__device__ __forceinline__ R DB(const R *__restrict__ g, const R *__restrict__ CB, int N, int Nz, int i) {
  // sum_l C^B_l (g_{i+l-1/2} - g_{i-l+1/2}), g_{k+1/2} stored at column k
  R s = 0;
  for (int l = 1; l <= N; ++l) s += CB[l - 1] * (g[wrap_once(i + l - 1, Nz)] - g[wrap_once(i - l, Nz)]);
  return s;
}
template <typename R>
__device__ __forceinline__ R DE(const R *__restrict__ f, const R *__restrict__ CE, int N, int Nz, int i) {
  // sum_l C^E_l (f_{i+l} - f_{i-l+1}), evaluated at z_{i+1/2}
  R s = 0;
  for (int l = 1; l <= N; ++l) s += CE[l - 1] * (f[wrap_once(i + l, Nz)] - f[wrap_once(i - l + 1, Nz)]);
  return s;
}
template <typename R>
__device__ __forceinline__ R Pf(const R *__restrict__ f, const R *__restrict__ P, int N, int Nz, int i) {
  R s = 0;
  for (int l = -(N - 1); l <= N - 1; ++l) s += P[l + N - 1] * f[wrap_once(i + l, Nz)];
  return s;
}

template <typename R, int M>
__global__ __launch_bounds__(256) void efield_kernel(KRun k, int par) {
  constexpr int NM = 2 * M + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= k.Nz) return;
  const int Nz = k.Nz, Nr = k.Nr, N = k.N;
  const long long plane = k.plane;
  const R dt = (R)k.dt, dr = (R)k.dr;
  const R *CB = (const R *)k.CB, *P = (const R *)k.P;
  R *E = (R *)k.E;
  const R *B = (const R *)k.B[par ^ 1];
  const R *Jc = (const R *)k.J[par];
  R *Jn = (R *)k.J[par ^ 1];
  const long long row = (long long)j * Nz, rowm = (long long)(j - 1) * Nz;
  // physical current = raw deposit * factor of the row
  const double dzd = k.dz, drd = k.dr, dtd = k.dt;
  const double Vj = j == 0 ? kPi * drd * drd * dzd / 4.0 : 2.0 * kPi * (j * drd) * drd * dzd;
  const R fz = (R)(1.0 / (dtd * (Vj / dzd)));
  const R frr = (R)(1.0 / (dtd * (2.0 * kPi * ((j + 0.5) * drd) * dzd)));
  const R fp_direct = (R)(1.0 / Vj);
  const R fp_closure = (R)(1.0 / (dtd * 2.0 * kPi * drd * dzd));
  const R rh = ((R)j + R(0.5)) * dr;

#pragma unroll
  for (int m = 0; m <= M; ++m) {
    const int qa = m == 0 ? 0 : 2 * m - 1, qb = 2 * m;
    const int nq = m == 0 ? 1 : 2;
    const R mm = (R)m;
    // (re, im) of the quantities needed, for both planes of the mode
    R Er_new[2], Ep_new[2], Ez_new[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) { Er_new[h] = 0; Ep_new[h] = 0; Ez_new[h] = 0; }
    // E_r at (i, j+1/2)
    if (j < Nr) {
      R bzr = B[(2 * NM + qa) * plane + row + i], bzi = (m > 0) ? B[(2 * NM + qb) * plane + row + i] : R(0);
      // (i m / r) B_z = (-m Bz_im, m Bz_re) / r
      R cr[2] = {-mm * bzi / rh, mm * bzr / rh};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nq) break;
        const int qq = h == 0 ? qa : qb;
        cr[h] -= DB(B + (1 * NM + qq) * plane + row, CB, N, Nz, i) / (R)k.dz;
        const R jr = Pf(Jc + (0 * NM + qq) * plane + row, P, N, Nz, i) * frr;
        Er_new[h] = E[(0 * NM + qq) * plane + row + i] + dt * (cr[h] - jr);
      }
    }
    // E_phi at (i, j)
    const bool phi_zero = (j == Nr) || (j == 0 && m != 1);
    if (!phi_zero) {
      const R fpf = (m == 0 || j == 0) ? fp_direct : fp_closure;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nq) break;
        const int qq = h == 0 ? qa : qb;
        R cp = DB(B + (0 * NM + qq) * plane + row, CB, N, Nz, i) / (R)k.dz;
        if (j == 0) cp -= R(2) * B[(2 * NM + qq) * plane + row + i] / dr;
        else cp -= (B[(2 * NM + qq) * plane + row + i] - B[(2 * NM + qq) * plane + rowm + i]) / dr;
        const R jp = Pf(Jc + (1 * NM + qq) * plane + row, P, N, Nz, i) * fpf;
        Ep_new[h] = E[(1 * NM + qq) * plane + row + i] + dt * (cp - jp);
      }
    }
    // E_z at (i+1/2, j)
    const bool z_zero = (j == Nr) || (j == 0 && m != 0);
    if (!z_zero) {
      if (j == 0) {
        const R cz = R(4) * B[(1 * NM + qa) * plane + row + i] / dr;
        Ez_new[0] = E[(2 * NM + qa) * plane + row + i] + dt * (cz - Jc[(2 * NM + qa) * plane + row + i] * fz);
      } else {
        const R rj = (R)j * dr;
        R brr = B[(0 * NM + qa) * plane + row + i], bri = (m > 0) ? B[(0 * NM + qb) * plane + row + i] : R(0);
        R imb[2] = {-mm * bri / rj, mm * brr / rj};  // (i m / r) B_r
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h >= nq) break;
          const int qq = h == 0 ? qa : qb;
          const R cz = (((R)j + R(0.5)) * B[(1 * NM + qq) * plane + row + i] -
                        ((R)j - R(0.5)) * B[(1 * NM + qq) * plane + rowm + i]) / rj - imb[h];
          Ez_new[h] = E[(2 * NM + qq) * plane + row + i] + dt * (cz - Jc[(2 * NM + qq) * plane + row + i] * fz);
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h >= nq) break;
      const int qq = h == 0 ? qa : qb;
      E[(0 * NM + qq) * plane + row + i] = Er_new[h];
      E[(1 * NM + qq) * plane + row + i] = Ep_new[h];
      E[(2 * NM + qq) * plane + row + i] = Ez_new[h];
    }
  }
  // clear the other current buffer for the next deposit
#pragma unroll
  for (int c = 0; c < 3 * NM; ++c) Jn[c * plane + row + i] = R(0);
}

// Bout = Bin - tau curl_E E; with avg != nullptr also avg = (Bin + Bout)/2,
// the time-centred B that the next gather uses (Eq. (12)).
template <typename R, int M>
__global__ __launch_bounds__(256) void bfield_kernel(KRun k, R *Bout, const R *Bin, R tau, R *avg) {
  constexpr int NM = 2 * M + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= k.Nz) return;
  const int Nz = k.Nz, Nr = k.Nr, N = k.N;
  const long long plane = k.plane;
  const R dr = (R)k.dr, dz = (R)k.dz;
  const R *CE = (const R *)k.CE;
  const R *E = (const R *)k.E;
  const long long row = (long long)j * Nz, rowp = (long long)(j + 1) * Nz;
  const int ip = wrap_once(i + 1, Nz);
  (void)ip;
#pragma unroll
  for (int m = 0; m <= M; ++m) {
    const int qa = m == 0 ? 0 : 2 * m - 1, qb = 2 * m;
    const int nq = m == 0 ? 1 : 2;
    const R mm = (R)m;
    R nbr[2] = {0, 0}, nbp[2] = {0, 0}, nbz[2] = {0, 0};
    // B_r at (i+1/2, j)
    const bool br_zero = (j == 0 && m != 1);
    if (!br_zero) {
      R curl[2];
      if (j == 0) {  // m = 1: (i m/r) E_z -> i E_z(r_1)/dr
        const R ezr = E[(2 * NM + qa) * plane + rowp + i], ezi = E[(2 * NM + qb) * plane + rowp + i];
        curl[0] = -ezi / dr;
        curl[1] = ezr / dr;
      } else {
        const R rj = (R)j * dr;
        const R ezr = E[(2 * NM + qa) * plane + row + i], ezi = (m > 0) ? E[(2 * NM + qb) * plane + row + i] : R(0);
        curl[0] = -mm * ezi / rj;
        curl[1] = mm * ezr / rj;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nq) break;
        const int qq = h == 0 ? qa : qb;
        const R c = curl[h] - DE(E + (1 * NM + qq) * plane + row, CE, N, Nz, i) / dz;
        nbr[h] = Bin[(0 * NM + qq) * plane + row + i] - tau * c;
      }
    }
    if (j < Nr) {
      const R rh = ((R)j + R(0.5)) * dr;
      // B_phi at (i+1/2, j+1/2)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nq) break;
        const int qq = h == 0 ? qa : qb;
        const R c = DE(E + (0 * NM + qq) * plane + row, CE, N, Nz, i) / dz -
                    (E[(2 * NM + qq) * plane + rowp + i] - E[(2 * NM + qq) * plane + row + i]) / dr;
        nbp[h] = Bin[(1 * NM + qq) * plane + row + i] - tau * c;
      }
      // B_z at (i, j+1/2)
      const R err = E[(0 * NM + qa) * plane + row + i], eri = (m > 0) ? E[(0 * NM + qb) * plane + row + i] : R(0);
      const R ime[2] = {-mm * eri / rh, mm * err / rh};  // (i m / r) E_r
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nq) break;
        const int qq = h == 0 ? qa : qb;
        const R c = (((R)(j + 1) * dr) * E[(1 * NM + qq) * plane + rowp + i] -
                     ((R)j * dr) * E[(1 * NM + qq) * plane + row + i]) / (rh * dr) - ime[h];
        nbz[h] = Bin[(2 * NM + qq) * plane + row + i] - tau * c;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h >= nq) break;
      const int qq = h == 0 ? qa : qb;
      const long long o0 = (0 * NM + qq) * plane + row + i, o1 = (1 * NM + qq) * plane + row + i,
                      o2 = (2 * NM + qq) * plane + row + i;
      if (avg) {
        avg[o0] = R(0.5) * (Bin[o0] + nbr[h]);
        avg[o1] = R(0.5) * (Bin[o1] + nbp[h]);
        avg[o2] = R(0.5) * (Bin[o2] + nbz[h]);
      }
      Bout[o0] = nbr[h];
      Bout[o1] = nbp[h];
      Bout[o2] = nbz[h];
    }
  }
}

// ---------------------------------------------------------------------------
// small utility kernels

__global__ void zero_kernel(uint4 *p, size_t n16, unsigned char *tail, size_t ntail) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t a = t; a < n16; a += stride) p[a] = make_uint4(0, 0, 0, 0);
  if (t < ntail) tail[t] = 0;
}

// charge density of the electrons (diagnostic), physical units
template <typename R, int M>
__global__ __launch_bounds__(256) void rho_kernel(KRun k) {
  constexpr int NM = 2 * M + 1;
  constexpr bool F64 = std::is_same<R, double>::value;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= k.np) return;
  const int Nz = k.Nz, Nr = k.Nr;
  int i0;
  R f0;
  if constexpr (F64) {
    const R z0 = ((const double *)k.pz)[p];
    const R fl = floor(z0);
    i0 = (int)fl;
    f0 = z0 - fl;
  } else {
    i0 = ((const int *)k.pz)[p];
    f0 = ((const float *)k.pfz)[p];
  }
  i0 = wrap_any(i0, Nz);
  const R x = ((const R *)k.px)[p], y = ((const R *)k.py)[p];
  const R r2 = fma(x, x, y * y), r = sqrt(r2);
  const int j0 = clampi(radial_index(r2, r), 0, Nr - 1);
  const R fr = r - (R)j0;
  R c = 1, s = 0;
  if (r > R(0)) { c = x / r; s = y / r; }
  const double q = -(double)((const R *)k.pw)[p];
  double *rho = (double *)k.rho;
  const double dzd = k.dz, drd = k.dr;
  double er = 1, ei = 0;
  for (int m = 0; m <= M; ++m) {
    if (m > 0) {
      const double tr = er * c + ei * s, ti = ei * c - er * s;
      er = tr;
      ei = ti;
    }
    const double cm = m == 0 ? 1.0 : 2.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const int j = j0 + b;
        if (m > 0 && j == 0) continue;  // the m >= 1 density vanishes on the axis
        const double V = j == 0 ? kPi * drd * drd * dzd / 4.0 : 2.0 * kPi * (j * drd) * drd * dzd;
        const double S = (a ? (double)f0 : 1.0 - (double)f0) * (b ? (double)fr : 1.0 - (double)fr);
        const long long o = (long long)j * Nz + wrap_once(i0 + a, Nz);
        const int qa = m == 0 ? 0 : 2 * m - 1;
        atomic_add(rho + qa * k.plane + o, cm * q * er * S / V);
        if (m > 0) atomic_add(rho + (2 * m) * k.plane + o, cm * q * ei * S / V);
      }
  }
  (void)NM;
}

// field energy per mode: per-block partial sums red[block * (M+1) + m]
template <typename R, int M>
__global__ __launch_bounds__(256) void energy_kernel(KRun k, int par) {
  constexpr int NM = 2 * M + 1;
  __shared__ double sh[256 * (M + 1)];
  const long long n = k.plane;
  const int tid = threadIdx.x;
  double acc[M + 1];
  for (int m = 0; m <= M; ++m) acc[m] = 0.0;
  const R *E = (const R *)k.E, *B0 = (const R *)k.B[par], *B1 = (const R *)k.B[par ^ 1];
  const double dzd = k.dz, drd = k.dr;
  for (long long idx = (long long)blockIdx.x * blockDim.x + tid; idx < n; idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / k.Nz);
    const double vn = j == 0 ? kPi * drd * drd * dzd / 4.0 : 2.0 * kPi * (j * drd) * drd * dzd;
    const double vh = j < k.Nr ? 2.0 * kPi * ((j + 0.5) * drd) * drd * dzd : 0.0;
    for (int q = 0; q < NM; ++q) {
      const int m = (q + 1) / 2;
      auto bb = [&](int c) {
        const double v = 0.5 * ((double)B0[(c * NM + q) * n + idx] + (double)B1[(c * NM + q) * n + idx]);
        return v * v;
      };
      const double er = E[(0 * NM + q) * n + idx], ep = E[(1 * NM + q) * n + idx], ez = E[(2 * NM + q) * n + idx];
      acc[m] += vh * (er * er + bb(1) + bb(2)) + vn * (ep * ep + ez * ez + bb(0));
    }
  }
  for (int m = 0; m <= M; ++m) sh[m * 256 + tid] = acc[m];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
      for (int m = 0; m <= M; ++m) sh[m * 256 + tid] += sh[m * 256 + tid + s];
    __syncthreads();
  }
  if (tid == 0)
    for (int m = 0; m <= M; ++m) k.red[blockIdx.x * (M + 1) + m] = 0.5 * sh[m * 256] * (m == 0 ? 1.0 : 0.5);
}

template <typename R>
__global__ __launch_bounds__(256) void kinetic_kernel(KRun k) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  const R *UX = (const R *)k.pux, *UY = (const R *)k.puy, *UZ = (const R *)k.puz, *W = (const R *)k.pw;
  for (long long p = (long long)blockIdx.x * blockDim.x + tid; p < k.np; p += (long long)gridDim.x * blockDim.x) {
    const double ux = UX[p], uy = UY[p], uz = UZ[p];
    acc += (double)W[p] * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
  }
  sh[tid] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  if (tid == 0) k.red[blockIdx.x] = sh[0];
}

template <typename R>
__global__ __launch_bounds__(256) void tracked_gamma_kernel(KRun k, double *gamma, int64_t *ids) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= k.np) return;
  const uint32_t w = k.pid[p];
  if (!(w & kTrackedBit)) return;
  const int32_t idv = (int32_t)(w & kIdMask);
  int lo = 0, hi = k.n_tracked;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (k.tracked[mid] < idv) lo = mid + 1;
    else hi = mid;
  }
  if (lo >= k.n_tracked || k.tracked[lo] != idv) return;
  const double ux = ((const R *)k.pux)[p], uy = ((const R *)k.puy)[p], uz = ((const R *)k.puz)[p];
  gamma[lo] = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
  ids[lo] = idv;
}


// ---------------------------------------------------------------------------
// cell sort: electrons ordered by (tile, cell in tile, id); tiles of Tz x Tr
// cells numbered z-fastest, cells inside a tile z-fastest.  Counting sort on
// the cell order, then the ids of each cell in ascending order, so that the
// permutation is unique whatever order the atomics ran in.

template <typename R>
__device__ __forceinline__ int cell_order(const KRun &k, long long p) {
  int iz;
  if constexpr (std::is_same<R, double>::value) {
    iz = (int)floor(((const double *)k.pz)[p]);
  } else {
    iz = ((const int *)k.pz)[p];
  }
  iz = wrap_any(iz, k.Nz);
  const R x = ((const R *)k.px)[p], y = ((const R *)k.py)[p];
  const R r2 = fma(x, x, y * y);
  const int ir = clampi(radial_index(r2, sqrt(r2)), 0, k.Nr - 1);
  const int tile = (ir / k.Tr) * k.ntz + iz / k.Tz;
  const int local = (ir % k.Tr) * k.Tz + iz % k.Tz;
  return tile * (k.Tz * k.Tr) + local;
}

template <typename R>
__global__ __launch_bounds__(256) void sort_key_kernel(KRun k, int32_t *keys) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= k.np) return;
  const int key = cell_order<R>(k, p);
  keys[p] = key;
  atomicAdd(&k.cell_count[key], 1);
}

// exclusive scan of 1024-element blocks; block totals to bsum
__global__ __launch_bounds__(256) void scan_block_kernel(const int32_t *in, int32_t *out, int32_t *bsum,
                                                          long long n) {
  __shared__ int32_t sh[256];
  const long long base = (long long)blockIdx.x * 1024 + threadIdx.x * 4;
  int32_t v[4];
  int32_t tot = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    v[a] = (base + a < n) ? in[base + a] : 0;
    tot += v[a];
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan of the thread totals
    const int32_t t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = sh[threadIdx.x] - tot;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (base + a < n) out[base + a] = run;
    run += v[a];
  }
  if (threadIdx.x == 255 && bsum) bsum[blockIdx.x] = sh[255];
}

__global__ __launch_bounds__(256) void scan_add_kernel(int32_t *out, const int32_t *boff, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += boff[i / 1024];
}

__global__ __launch_bounds__(256) void copy_i32_kernel(int32_t *dst, const int32_t *src, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void sort_scatter_kernel(KRun k, const int32_t *keys, int32_t *cursor) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= k.np) return;
  const int key = keys[p];
  const int pos = atomicAdd(&cursor[key], 1);
  k.perm[pos] = (int32_t)p;
}

// within each cell, order the electrons by id (insertion sort; cells are short)
__global__ __launch_bounds__(256) void sort_cells_kernel(KRun k) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k.n_keys) return;
  const int b = k.cell_start[c], e = k.cell_start[c + 1];
  for (int a = b + 1; a < e; ++a) {
    const int32_t v = k.perm[a];
    const uint32_t key = k.pid[v] & kIdMask;
    int t = a - 1;
    while (t >= b && (k.pid[k.perm[t]] & kIdMask) > key) {
      k.perm[t + 1] = k.perm[t];
      --t;
    }
    k.perm[t + 1] = v;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void sort_permute_kernel(KRun k) {
  const long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= k.np) return;
  const int s = k.perm[d];
  if constexpr (std::is_same<R, double>::value) {
    ((double *)k.sz)[d] = ((const double *)k.pz)[s];
  } else {
    ((int *)k.sz)[d] = ((const int *)k.pz)[s];
    ((float *)k.sfz)[d] = ((const float *)k.pfz)[s];
  }
  ((R *)k.sx)[d] = ((const R *)k.px)[s];
  ((R *)k.sy)[d] = ((const R *)k.py)[s];
  ((R *)k.sux)[d] = ((const R *)k.pux)[s];
  ((R *)k.suy)[d] = ((const R *)k.puy)[s];
  ((R *)k.suz)[d] = ((const R *)k.puz)[s];
  ((R *)k.sw)[d] = ((const R *)k.pw)[s];
  k.spid[d] = k.pid[s];
}

// ---------------------------------------------------------------------------
// launch helpers

thread_local char g_err[256] = "";

size_t push_lds_bytes(const KRun &k, size_t word) {
  return (size_t)3 * (2 * k.M + 1) * (k.Tz + 3) * (k.Tr + 3) * word;
}



int check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
    return PIC_E_DEVICE;
  }
  return PIC_OK;
}

int scan_exclusive(int32_t *data_in, int32_t *out, long long n, int32_t *tmp, hipStream_t s) {
  const long long nb = (n + 1023) / 1024;
  int32_t *bsum = nb > 1 ? tmp : nullptr;
  scan_block_kernel<<<(unsigned)nb, 256, 0, s>>>(data_in, out, bsum, n);
  int rc = check(hipGetLastError(), "scan_block_kernel");
  if (rc || nb <= 1) return rc;
  rc = scan_exclusive(bsum, bsum, nb, tmp + nb, s);
  if (rc) return rc;
  scan_add_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, bsum, n);
  return check(hipGetLastError(), "scan_add_kernel");
}

template <template <typename, int> class F, typename... A>
int dispatch_M(int prec, int M, A &&...a) {
  if (prec == PIC_PREC_FP64) {
    switch (M) {
      case 0: return F<double, 0>::run(a...);
      case 1: return F<double, 1>::run(a...);
      case 2: return F<double, 2>::run(a...);
      case 3: return F<double, 3>::run(a...);
    }
  } else {
    switch (M) {
      case 0: return F<float, 0>::run(a...);
      case 1: return F<float, 1>::run(a...);
      case 2: return F<float, 2>::run(a...);
      case 3: return F<float, 3>::run(a...);
    }
  }
  return PIC_E_INVALID;
}

template <typename R, int M>
struct PushL {
  static int run(const KRun &k, int par, hipStream_t s) {
    if (k.np == 0) return PIC_OK;
    const unsigned blocks = (unsigned)((long long)k.ntz * k.ntr);
    const size_t lds = push_lds_bytes(k, sizeof(R));
    push_kernel<R, M><<<blocks, 256, lds, s>>>(k, par);
    return check(hipGetLastError(), "push_kernel");
  }
};
template <typename R, int M>
struct EL {
  static int run(const KRun &k, int par, hipStream_t s) {
    dim3 g((k.Nz + 255) / 256, k.Nr + 1);
    efield_kernel<R, M><<<g, 256, 0, s>>>(k, par);
    return check(hipGetLastError(), "efield_kernel");
  }
};
template <typename R, int M>
struct BL {
  static int run(const KRun &k, void *out, const void *in, double tau, void *avg, hipStream_t s) {
    dim3 g((k.Nz + 255) / 256, k.Nr + 1);
    bfield_kernel<R, M><<<g, 256, 0, s>>>(k, (R *)out, (const R *)in, (R)tau, (R *)avg);
    return check(hipGetLastError(), "bfield_kernel");
  }
};
template <typename R, int M>
struct RhoL {
  static int run(const KRun &k, hipStream_t s) {
    if (k.np == 0) return PIC_OK;
    rho_kernel<R, M><<<(unsigned)((k.np + 255) / 256), 256, 0, s>>>(k);
    return check(hipGetLastError(), "rho_kernel");
  }
};
template <typename R, int M>
struct EnL {
  static int run(const KRun &k, int par, int nb, hipStream_t s) {
    energy_kernel<R, M><<<nb, 256, 0, s>>>(k, par);
    return check(hipGetLastError(), "energy_kernel");
  }
};

}  // namespace

const char *last_device_error() { return g_err; }

int launch_push(const KRun &k, int prec, int par, void *stream) {
  return dispatch_M<PushL>(prec, k.M, k, par, (hipStream_t)stream);
}
int launch_efield(const KRun &k, int prec, int par, void *stream) {
  return dispatch_M<EL>(prec, k.M, k, par, (hipStream_t)stream);
}
int launch_bfield(const KRun &k, int prec, void *Bout, const void *Bin, double tau, void *avg, void *stream) {
  return dispatch_M<BL>(prec, k.M, k, Bout, Bin, tau, avg, (hipStream_t)stream);
}
int launch_rho(const KRun &k, int prec, void *stream) {
  return dispatch_M<RhoL>(prec, k.M, k, (hipStream_t)stream);
}
int launch_zero(void *ptr, size_t bytes, void *stream) {
  if (bytes == 0) return PIC_OK;
  const size_t n16 = bytes / 16, tail = bytes % 16;
  unsigned blocks = (unsigned)((n16 + 255) / 256);
  if (blocks > 65535u * 4u) blocks = 65535u * 4u;
  if (blocks == 0) blocks = 1;
  zero_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>((uint4 *)ptr, n16, (unsigned char *)ptr + n16 * 16, tail);
  return check(hipGetLastError(), "zero_kernel");
}
int launch_energy(const KRun &k, int prec, int par, int nblocks_max, int *nblocks, void *stream) {
  long long want = (k.plane + 255) / 256;
  int nb = (int)(want < nblocks_max ? want : nblocks_max);
  if (nb < 1) nb = 1;
  *nblocks = nb;
  return dispatch_M<EnL>(prec, k.M, k, par, nb, (hipStream_t)stream);
}
int launch_kinetic(const KRun &k, int prec, int *nblocks, void *stream) {
  long long want = (k.np + 255) / 256;
  int nb = (int)(want < 1024 ? want : 1024);
  if (nb < 1) nb = 1;
  *nblocks = nb;
  if (prec == PIC_PREC_FP64) kinetic_kernel<double><<<nb, 256, 0, (hipStream_t)stream>>>(k);
  else kinetic_kernel<float><<<nb, 256, 0, (hipStream_t)stream>>>(k);
  return check(hipGetLastError(), "kinetic_kernel");
}
int launch_tracked_gamma(const KRun &k, int prec, double *gamma, int64_t *ids, void *stream) {
  if (k.np == 0 || k.n_tracked == 0) return PIC_OK;
  const unsigned blocks = (unsigned)((k.np + 255) / 256);
  if (prec == PIC_PREC_FP64) tracked_gamma_kernel<double><<<blocks, 256, 0, (hipStream_t)stream>>>(k, gamma, ids);
  else tracked_gamma_kernel<float><<<blocks, 256, 0, (hipStream_t)stream>>>(k, gamma, ids);
  return check(hipGetLastError(), "tracked_gamma_kernel");
}
size_t lds_bytes_of(const KRun &k, int prec) { return push_lds_bytes(k, prec == PIC_PREC_FP64 ? 8 : 4); }

int launch_sort(KRun &k, int prec, void *stream) {
  const hipStream_t s = (hipStream_t)stream;
  const long long nk = k.n_keys + 1;
  int rc = launch_zero(k.cell_count, (size_t)nk * 4, stream);
  if (rc) return rc;
  if (k.np > 0) {
    const unsigned pb = (unsigned)((k.np + 255) / 256);
    int32_t *keys = (int32_t *)k.spid;  // free until the permutation writes it
    if (prec == PIC_PREC_FP64) sort_key_kernel<double><<<pb, 256, 0, s>>>(k, keys);
    else sort_key_kernel<float><<<pb, 256, 0, s>>>(k, keys);
    if ((rc = check(hipGetLastError(), "sort_key_kernel"))) return rc;
    if ((rc = scan_exclusive(k.cell_count, k.cell_start, nk, k.scan_tmp, s))) return rc;
    copy_i32_kernel<<<(unsigned)((nk + 255) / 256), 256, 0, s>>>(k.cell_count, k.cell_start, nk);
    if ((rc = check(hipGetLastError(), "copy_i32_kernel"))) return rc;
    sort_scatter_kernel<<<pb, 256, 0, s>>>(k, keys, k.cell_count);
    if ((rc = check(hipGetLastError(), "sort_scatter_kernel"))) return rc;
    sort_cells_kernel<<<(unsigned)((k.n_keys + 255) / 256), 256, 0, s>>>(k);
    if ((rc = check(hipGetLastError(), "sort_cells_kernel"))) return rc;
    if (prec == PIC_PREC_FP64) sort_permute_kernel<double><<<pb, 256, 0, s>>>(k);
    else sort_permute_kernel<float><<<pb, 256, 0, s>>>(k);
    if ((rc = check(hipGetLastError(), "sort_permute_kernel"))) return rc;
    std::swap(k.pz, k.sz);
    std::swap(k.pfz, k.sfz);
    std::swap(k.px, k.sx);
    std::swap(k.py, k.sy);
    std::swap(k.pux, k.sux);
    std::swap(k.puy, k.suy);
    std::swap(k.puz, k.suz);
    std::swap(k.pw, k.sw);
    std::swap(k.pid, k.spid);
  } else {
    if ((rc = scan_exclusive(k.cell_count, k.cell_start, nk, k.scan_tmp, s))) return rc;
  }
  return PIC_OK;
}

}  // namespace pic
