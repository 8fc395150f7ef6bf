/*
 * q3d_oracle.c -- plain FP64 CPU oracle of the quasi-3D (azimuthal-mode) r-z
 * particle-in-cell time step with the "dual" finite-difference Maxwell solver
 * of Miller et al., "Accurate simulation of direct laser acceleration in a
 * laser wakefield accelerator" (arXiv 2303.12874).
 *
 * TEST INFRASTRUCTURE ONLY.  It is compiled into liborc.so and loaded by the
 * tests, by the smoke check and by the CPU-baseline leg of the benchmark; the
 * product library never links, loads or calls it, and the two share no code.
 * It is written to be slow, serial and readable against the paper:
 *
 *   Sec. III.A, Eq. (9)   Faraday and Ampere with distinct z-difference
 *                         operators: D_E acts on E, D_B acts on B.
 *   Sec. III.A, Eq. (10)  Gauss's law uses D_B; the dispersion relation is
 *                         [w]_t^2 = [k]_B [k]_E.  The deposited current is
 *                         made to conserve charge with D_B either by the z
 *                         filter P on J_r, J_phi or, as a switch, by P^{-1}
 *                         on J_z (a DFT on each periodic z line).
 *   Sec. III.A, Eq. (12)  the force uses E^n and the time average
 *                         (B^{n-1/2} + B^{n+1/2})/2; B is kept at half steps.
 *   Sec. II,   Eq. (6)    relativistic Lorentz force, integrated with Boris.
 *   Sec. III.B            fields are Re sum_m F^m(r,z) e^{i m phi}.
 *   Sec. III.B, Eq. (16)  per-mode work  W_m = -sum dt E^m . v.
 *   Sec. III.B, Eq. (18)  near-focus linearly polarised Gaussian laser.
 *
 * Normalised units: c = w0 = 1 (laser frequency), lengths in c/w0, time in
 * 1/w0, fields in m c w0/e, densities in n_c, electron q/m = -1,
 * dB/dt = -curl E, dE/dt = curl B - J, div E = rho.
 *
 * Readings of points the paper leaves open (grid staggering, axis rules,
 * deposit, filter, boundaries) are stated where they are used.
 *
 * Grid.  Nodes z_i = i dz (i = 0..Nz-1, periodic in z), r_j = j dr
 * (j = 0..Nr; j = 0 is the axis, j = Nr a perfectly conducting wall).
 * Staggering (cylindrical Yee cell):
 *   E_r (i, j+1/2)   E_phi (i, j)       E_z (i+1/2, j)
 *   B_r (i+1/2, j)   B_phi (i+1/2, j+1/2)  B_z (i, j+1/2)
 *   J like E;  rho (i, j).
 * A quantity at z_{i+1/2} is stored at z-index i, one at r_{j+1/2} at row j.
 * Every array is complex [M+1][Nr+1][Nz] (m = 0 has zero imaginary part).
 *
 * Particles carry z in units of dz and x, y in units of dr.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

#define ORC_PI 3.14159265358979323846

enum { CR = 0, CP = 1, CZ = 2 };

typedef struct orc {
  int Nz, Nr, M, N;
  double dz, dr, dt;
  double *CE, *CB;    /* C^E_l, C^B_l for l = 1..N, stored at [l-1] */
  double *P;          /* filter taps p_l, l = -(N-1)..N-1, stored at [l+N-1] */
  size_t nf;          /* complex entries per component array */
  cplx *E[3];         /* E^n */
  cplx *Bo[3];        /* B^{n-1/2} */
  cplx *Bn[3];        /* B^{n+1/2} */
  cplx *J[3];         /* J^{n+1/2} of the last step, as deposited (before P) */
  cplx *rho;          /* charge density of the particles (diagnostic) */
  long np;
  double *z, *x, *y, *ux, *uy, *uz, *w;
  int64_t *id;
  int32_t *slot;      /* tracked slot, -1 if not tracked */
  int ntr;
  double *W;          /* [ntr][M+1] per-mode work */
  double *Wc;         /* [ntr][2] work of E_z and of E_perp, Eq. (17) */
  double *gam0;       /* [ntr] gamma when tracking started */
  int64_t *tr_id;     /* [ntr] id of each tracked slot */
  long nstep;
  int freeze_fields;  /* 1: Maxwell update skipped (prescribed fields) */
  int deposit_rho;    /* 1: deposit rho after every step */
  int exact_jz;       /* 1: J_z <- P^{-1} J_z, J_r and J_phi unfiltered */
  int shape;          /* particle shape order: 1 linear (default), 2 quadratic */
  /* plasma of the last orc_load_plasma, for the fresh columns of the window */
  int ppc;
  uint64_t seed;
  double n0, ramp_start, ramp_len, down_start, down_len;
  /* moving window: every win_K steps the box advances by the whole cells
   * the light front has crossed since the start (speed win_speed c)       */
  int win_K, win_guard;
  double win_speed;
  long win_S;         /* cells moved so far: box column i is absolute column i + win_S */
} orc;

/* ------------------------------------------------------------------------ */
/* indexing                                                                 */

static inline int wrapz(const orc *o, int i) {
  int n = o->Nz;
  i %= n;
  return i < 0 ? i + n : i;
}
static inline size_t ix(const orc *o, int m, int j, int i) {
  return ((size_t)m * (size_t)(o->Nr + 1) + (size_t)j) * (size_t)o->Nz + (size_t)wrapz(o, i);
}

/* cell volume belonging to integer radial node j (the axis node owns the disc
 * of radius dr/2), and the face areas used by the fluxes.                   */
static double vol_node(const orc *o, int j) {
  if (j == 0) return ORC_PI * o->dr * o->dr * o->dz / 4.0;
  return 2.0 * ORC_PI * (j * o->dr) * o->dr * o->dz;
}
static double area_z(const orc *o, int j) { return vol_node(o, j) / o->dz; }
static double area_r(const orc *o, int j) { /* face at r_{j+1/2} */
  return 2.0 * ORC_PI * ((j + 0.5) * o->dr) * o->dz;
}
static double vol_half(const orc *o, int j) { /* volume around r_{j+1/2} */
  return 2.0 * ORC_PI * ((j + 0.5) * o->dr) * o->dr * o->dz;
}

static cplx ipow(cplx e, int m) {
  cplx r = 1.0;
  for (int k = 0; k < m; ++k) r *= e;
  return r;
}

/* ------------------------------------------------------------------------ */
/* life cycle                                                               */

orc *orc_create(int Nz, int Nr, int M, double dz, double dr, double dt, int N,
                const double *CE, const double *CB) {
  if (Nz < 1 || Nr < 2 || M < 0 || N < 1) return NULL;
  orc *o = (orc *)calloc(1, sizeof(orc));
  o->Nz = Nz; o->Nr = Nr; o->M = M; o->N = N;
  o->dz = dz; o->dr = dr; o->dt = dt;
  o->shape = 1;
  o->CE = (double *)malloc(sizeof(double) * N);
  o->CB = (double *)malloc(sizeof(double) * N);
  memcpy(o->CE, CE, sizeof(double) * N);
  memcpy(o->CB, CB, sizeof(double) * N);
  /* The extended D_B factors as the two-point difference applied after a
   * symmetric z filter P with taps p_l = sum_{l' > |l|} C^B_{l'}: matching the
   * Fourier symbols sum_l C_l 2 sin((2l-1)k dz/2) = 2 sin(k dz/2) P(k) term
   * by term gives C_l = p_{l-1} - p_l.  Used to make the deposited current
   * satisfy the D_B continuity equation (Sec. III.A: the solver conserves
   * charge with Gauss's law written with [k]_B, Eq. (10)).                  */
  o->P = (double *)calloc((size_t)(2 * N - 1), sizeof(double));
  for (int l = 0; l < N; ++l) {
    double p = 0.0;
    for (int lp = l + 1; lp <= N; ++lp) p += CB[lp - 1];
    o->P[N - 1 + l] = p;
    o->P[N - 1 - l] = p;
  }
  o->nf = (size_t)(M + 1) * (size_t)(Nr + 1) * (size_t)Nz;
  for (int c = 0; c < 3; ++c) {
    o->E[c] = (cplx *)calloc(o->nf, sizeof(cplx));
    o->Bo[c] = (cplx *)calloc(o->nf, sizeof(cplx));
    o->Bn[c] = (cplx *)calloc(o->nf, sizeof(cplx));
    o->J[c] = (cplx *)calloc(o->nf, sizeof(cplx));
  }
  o->rho = (cplx *)calloc(o->nf, sizeof(cplx));
  return o;
}

static void free_particles(orc *o) {
  free(o->z); free(o->x); free(o->y); free(o->ux); free(o->uy); free(o->uz);
  free(o->w); free(o->id); free(o->slot); free(o->W); free(o->Wc); free(o->gam0); free(o->tr_id);
  o->z = o->x = o->y = o->ux = o->uy = o->uz = o->w = NULL;
  o->id = NULL; o->slot = NULL; o->W = o->Wc = o->gam0 = NULL; o->tr_id = NULL;
  o->np = 0; o->ntr = 0;
}

void orc_destroy(orc *o) {
  if (!o) return;
  free_particles(o);
  for (int c = 0; c < 3; ++c) { free(o->E[c]); free(o->Bo[c]); free(o->Bn[c]); free(o->J[c]); }
  free(o->rho); free(o->CE); free(o->CB); free(o->P);
  free(o);
}

void orc_set_flags(orc *o, int freeze_fields, int deposit_rho) {
  o->freeze_fields = freeze_fields;
  o->deposit_rho = deposit_rho;
}

void orc_set_exact_jz(orc *o, int on) { o->exact_jz = on; }
int orc_set_shape(orc *o, int order) {
  if (order != 1 && order != 2) return -1;
  o->shape = order;
  return 0;
}

long orc_num_particles(const orc *o) { return o->np; }
long orc_num_steps(const orc *o) { return o->nstep; }
const double *orc_filter_taps(const orc *o) { return o->P; }

/* ------------------------------------------------------------------------ */
/* field access.  comp: 0..2 = E_r,E_phi,E_z (E^n); 3..5 = B^{n-1/2};       */
/* 6..8 = B^{n+1/2}; 9..11 = J of the last step; 12 = rho.  Buffers are     */
/* interleaved complex [Nr+1][Nz] for one mode m.                           */

static cplx *field_ptr(orc *o, int comp) {
  if (comp < 3) return o->E[comp];
  if (comp < 6) return o->Bo[comp - 3];
  if (comp < 9) return o->Bn[comp - 6];
  if (comp < 12) return o->J[comp - 9];
  if (comp == 12) return o->rho;
  return NULL;
}

int orc_get_field(orc *o, int comp, int m, double *out) {
  cplx *f = field_ptr(o, comp);
  if (!f || m < 0 || m > o->M) return -1;
  size_t n = (size_t)(o->Nr + 1) * o->Nz;
  memcpy(out, f + (size_t)m * n, n * sizeof(cplx));
  return 0;
}

int orc_set_field(orc *o, int comp, int m, const double *in) {
  cplx *f = field_ptr(o, comp);
  if (!f || m < 0 || m > o->M) return -1;
  size_t n = (size_t)(o->Nr + 1) * o->Nz;
  memcpy(f + (size_t)m * n, in, n * sizeof(cplx));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* z-difference operators of Eq. (9)                                         */

/* D_E of integer-z data f, evaluated at z_{i+1/2}:
 *   sum_{l=1..N} C^E_l (f_{i+l} - f_{i-l+1}) / dz                          */
static cplx D_E(const orc *o, const cplx *f, int m, int j, int i) {
  cplx s = 0.0;
  for (int l = 1; l <= o->N; ++l)
    s += o->CE[l - 1] * (f[ix(o, m, j, i + l)] - f[ix(o, m, j, i - l + 1)]);
  return s / o->dz;
}

/* D_B of half-z data g (g at z_{k+1/2} stored at index k), evaluated at z_i:
 *   sum_{l=1..N} C^B_l (g_{i+l-1/2} - g_{i-l+1/2}) / dz                    */
static cplx D_B(const orc *o, const cplx *g, int m, int j, int i) {
  cplx s = 0.0;
  for (int l = 1; l <= o->N; ++l)
    s += o->CB[l - 1] * (g[ix(o, m, j, i + l - 1)] - g[ix(o, m, j, i - l)]);
  return s / o->dz;
}

/* The z filter P (same taps for integer or half-integer data).             */
static cplx filterP(const orc *o, const cplx *f, int m, int j, int i) {
  cplx s = 0.0;
  for (int l = -(o->N - 1); l <= o->N - 1; ++l) s += o->P[l + o->N - 1] * f[ix(o, m, j, i + l)];
  return s;
}

/* The inverse of P on one periodic z line of Nz values, by the discrete
 * Fourier transform: P is a circulant convolution whose symbol at
 * k_q dz = 2 pi q / Nz is P_q = sum_l p_l cos(2 pi q l / Nz) (real, as
 * p_{-l} = p_l), so the line is transformed, divided by P_q and transformed
 * back.  A plain O(Nz^2) DFT.  Returns -1 if some P_q <= 0 (not invertible
 * as a positive filter).                                                   */
static int inverse_filter_line(const orc *o, const cplx *in, cplx *out) {
  const int Nz = o->Nz;
  cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)Nz);  /* e^{-2 pi i k / Nz} */
  cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)Nz);
  int rc = 0;
  for (int k = 0; k < Nz; ++k) tw[k] = cexp(-2.0 * ORC_PI * I * (double)k / (double)Nz);
  for (int q = 0; q < Nz; ++q) {
    cplx sum = 0.0;
    for (int i = 0; i < Nz; ++i) sum += in[i] * tw[(long)q * i % Nz];
    double Pq = 0.0;
    for (int l = -(o->N - 1); l <= o->N - 1; ++l) Pq += o->P[l + o->N - 1] * creal(tw[wrapz(o, q * l)]);
    if (!(Pq > 0.0)) rc = -1;
    X[q] = sum / Pq;
  }
  for (int i = 0; i < Nz; ++i) {
    cplx sum = 0.0;
    for (int q = 0; q < Nz; ++q) sum += X[q] * conj(tw[(long)q * i % Nz]);
    out[i] = sum / (double)Nz;
  }
  free(tw);
  free(X);
  return rc;
}

/* P^{-1} applied to one interleaved complex line of Nz values.              */
int orc_inverse_filter(orc *o, const double *in, double *out) {
  return inverse_filter_line(o, (const cplx *)in, (cplx *)out);
}

/* ------------------------------------------------------------------------ */
/* Faraday: Bout = Bin - tau * curl_E(E), mode by mode (d/dphi -> i m).      */
/* Axis rules (reading; the paper defers to the quasi-3D algorithm paper):  */
/*   m = 0: B_r(axis) = 0;  m = 1: (i m / r) E_z -> i E_z(r_1) / dr since   */
/*   E_z^1 vanishes linearly on the axis;  m >= 2: B_r(axis) = 0.           */
/* Bout may alias Bin (the update is pointwise in B).                       */

static void faraday(orc *o, cplx *Bout[3], cplx *Bin[3], cplx *E[3], double tau) {
  const int Nz = o->Nz, Nr = o->Nr;
  const double dr = o->dr;
  for (int m = 0; m <= o->M; ++m) {
    const cplx im = I * (double)m;
    for (int j = 0; j <= Nr; ++j) {
      for (int i = 0; i < Nz; ++i) {
        /* B_r at (i+1/2, j) */
        cplx curl_r;
        int zero_r = 0;
        if (j == 0) {
          if (m == 1) curl_r = I * E[CZ][ix(o, m, 1, i)] / dr - D_E(o, E[CP], m, 0, i);
          else { curl_r = 0.0; zero_r = 1; }
        } else {
          curl_r = im / (j * dr) * E[CZ][ix(o, m, j, i)] - D_E(o, E[CP], m, j, i);
        }
        size_t k = ix(o, m, j, i);
        Bout[CR][k] = zero_r ? 0.0 : Bin[CR][k] - tau * curl_r;

        if (j < Nr) {
          /* B_phi at (i+1/2, j+1/2) */
          cplx curl_p = D_E(o, E[CR], m, j, i) - (E[CZ][ix(o, m, j + 1, i)] - E[CZ][ix(o, m, j, i)]) / dr;
          Bout[CP][k] = Bin[CP][k] - tau * curl_p;
          /* B_z at (i, j+1/2) */
          double rh = (j + 0.5) * dr;
          cplx curl_z = ((j + 1) * dr * E[CP][ix(o, m, j + 1, i)] - (j * dr) * E[CP][ix(o, m, j, i)]) / (rh * dr)
                        - im / rh * E[CR][ix(o, m, j, i)];
          Bout[CZ][k] = Bin[CZ][k] - tau * curl_z;
        } else {
          Bout[CP][k] = 0.0;
          Bout[CZ][k] = 0.0;
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Ampere: E += dt * (curl_B(B) - J'), with J' = (P J_r, P J_phi, J_z), or  */
/* with exact_jz set J' = (J_r, J_phi, P^{-1} J_z): both satisfy the D_B     */
/* continuity equation, since D_B = D_Yee o P and the deposit satisfies the  */
/* two-point one.                                                            */
/* Axis rules: m = 0: E_phi(axis) = 0 and E_z(axis) uses the flux of B_phi  */
/* through the disc of radius dr/2, i.e. 4 B_phi(1/2)/dr;  m = 1: E_z = 0,  */
/* E_phi uses -dB_z/dr = -2 B_z(1/2)/dr (B_z^1 vanishes linearly);          */
/* m >= 2: E_phi = E_z = 0 on the axis.  Wall r = Nr dr: E_phi = E_z = 0.   */

static void ampere(orc *o, cplx *B[3]) {
  const int Nz = o->Nz, Nr = o->Nr;
  const double dr = o->dr, dt = o->dt;
  cplx *jz = o->J[CZ];
  if (o->exact_jz) {
    jz = (cplx *)malloc(o->nf * sizeof(cplx));
    for (int m = 0; m <= o->M; ++m)
      for (int j = 0; j <= Nr; ++j) inverse_filter_line(o, o->J[CZ] + ix(o, m, j, 0), jz + ix(o, m, j, 0));
  }
  for (int m = 0; m <= o->M; ++m) {
    const cplx im = I * (double)m;
    for (int j = 0; j <= Nr; ++j) {
      for (int i = 0; i < Nz; ++i) {
        size_t k = ix(o, m, j, i);
        /* E_r at (i, j+1/2) */
        if (j < Nr) {
          double rh = (j + 0.5) * dr;
          cplx cr = im / rh * B[CZ][k] - D_B(o, B[CP], m, j, i);
          cplx jr = o->exact_jz ? o->J[CR][k] : filterP(o, o->J[CR], m, j, i);
          o->E[CR][k] += dt * (cr - jr);
        } else {
          o->E[CR][k] = 0.0;
        }
        /* E_phi at (i, j) */
        if (j == Nr || (j == 0 && m != 1)) {
          o->E[CP][k] = 0.0;
        } else {
          cplx cp;
          if (j == 0) cp = D_B(o, B[CR], m, 0, i) - 2.0 * B[CZ][ix(o, m, 0, i)] / dr;
          else cp = D_B(o, B[CR], m, j, i) - (B[CZ][ix(o, m, j, i)] - B[CZ][ix(o, m, j - 1, i)]) / dr;
          cplx jp = o->exact_jz ? o->J[CP][k] : filterP(o, o->J[CP], m, j, i);
          o->E[CP][k] += dt * (cp - jp);
        }
        /* E_z at (i+1/2, j) */
        if (j == Nr || (j == 0 && m != 0)) {
          o->E[CZ][k] = 0.0;
        } else {
          cplx cz;
          if (j == 0) cz = 4.0 * B[CP][ix(o, m, 0, i)] / dr;
          else cz = ((j + 0.5) * B[CP][ix(o, m, j, i)] - (j - 0.5) * B[CP][ix(o, m, j - 1, i)]) / (j * dr)
                    - im / (j * dr) * B[CR][k];
          o->E[CZ][k] += dt * (cz - jz[k]);
        }
      }
    }
  }
  if (jz != o->J[CZ]) free(jz);
}

/* ------------------------------------------------------------------------ */
/* Gauss residual of Eq. (10): G = D_B E_z + (1/r) d(r E_r)/dr + (i m/r) E_phi
 * - P rho (- rho with exact_jz), on nodes where Gauss's law is evolved
 * (interior rows; axis row for m = 0 only).  Written into out as
 * interleaved complex [Nr+1][Nz].                                          */
int orc_gauss_residual(orc *o, int m, double *out) {
  if (m < 0 || m > o->M) return -1;
  const int Nz = o->Nz, Nr = o->Nr;
  const double dr = o->dr;
  const cplx im = I * (double)m;
  cplx *g = (cplx *)out;
  for (int j = 0; j <= Nr; ++j)
    for (int i = 0; i < Nz; ++i) {
      cplx v = 0.0;
      const cplx q = o->exact_jz ? o->rho[ix(o, m, j, i)] : filterP(o, o->rho, m, j, i);
      if (j == 0 && m == 0) {
        v = D_B(o, o->E[CZ], m, 0, i) + 4.0 * o->E[CR][ix(o, m, 0, i)] / dr - q;
      } else if (j >= 1 && j < Nr) {
        v = D_B(o, o->E[CZ], m, j, i)
            + ((j + 0.5) * o->E[CR][ix(o, m, j, i)] - (j - 0.5) * o->E[CR][ix(o, m, j - 1, i)]) / (j * dr)
            + im / (j * dr) * o->E[CP][ix(o, m, j, i)] - q;
      }
      g[(size_t)j * Nz + i] = v;
    }
  return 0;
}

/* Field energy of mode m: (1/2) sum V (|E^m|^2 + |Bbar^m|^2), with weight 1
 * for m = 0 and 1/2 for m >= 1 (the phi-average of Re(F e^{i m phi})^2).   */
double orc_field_energy(orc *o, int m) {
  const int Nz = o->Nz, Nr = o->Nr;
  double s = 0.0;
  for (int j = 0; j <= Nr; ++j)
    for (int i = 0; i < Nz; ++i) {
      size_t k = ix(o, m, j, i);
      double vn = vol_node(o, j), vh = j < Nr ? vol_half(o, j) : 0.0;
      cplx br = 0.5 * (o->Bo[CR][k] + o->Bn[CR][k]);
      cplx bp = 0.5 * (o->Bo[CP][k] + o->Bn[CP][k]);
      cplx bz = 0.5 * (o->Bo[CZ][k] + o->Bn[CZ][k]);
      s += vh * (creal(o->E[CR][k] * conj(o->E[CR][k])) + creal(bp * conj(bp)) + creal(bz * conj(bz)));
      s += vn * (creal(o->E[CP][k] * conj(o->E[CP][k])) + creal(o->E[CZ][k] * conj(o->E[CZ][k]))
                 + creal(br * conj(br)));
    }
  return 0.5 * s * (m == 0 ? 1.0 : 0.5);
}

/* ------------------------------------------------------------------------ */
/* radial cell index of a particle at (x, y) (units of dr): the largest      */
/* integer j with j^2 <= x^2 + y^2, with x^2 + y^2 formed as fma(x,x,y*y).   */
static int radial_index(double r2, double r) {
  int j = (int)floor(r);
  if ((double)j * (double)j > r2) j -= 1;
  if ((double)(j + 1) * (double)(j + 1) <= r2) j += 1;
  return j;
}

/* Linear interpolation of one component of mode m at (zc, rc).  zhalf/rhalf
 * select the staggered location; on the half-r grid the value at r_{-1/2}
 * is the mirror image sign * F(r_{1/2}) (sign (-1)^{m+1} for r and phi
 * components, (-1)^m for z components: the point (-r, phi) is (r, phi+pi)). */
static cplx interp(const orc *o, const cplx *f, int m, double zc, double rc, int jint,
                   int zhalf, int rhalf, double mirror) {
  double zz = zhalf ? zc - 0.5 : zc;
  int i0 = (int)floor(zz);
  double fz = zz - i0;
  int j0;
  double fr;
  if (rhalf) {
    double rr = rc - 0.5;
    j0 = (int)floor(rr);
    fr = rr - j0;
  } else {
    j0 = jint;
    fr = rc - jint;
  }
  cplx v00, v10, v01, v11;
  if (j0 < 0) {
    v00 = mirror * f[ix(o, m, 0, i0)];
    v10 = mirror * f[ix(o, m, 0, i0 + 1)];
  } else {
    v00 = f[ix(o, m, j0, i0)];
    v10 = f[ix(o, m, j0, i0 + 1)];
  }
  v01 = f[ix(o, m, j0 + 1, i0)];
  v11 = f[ix(o, m, j0 + 1, i0 + 1)];
  return (1.0 - fz) * (1.0 - fr) * v00 + fz * (1.0 - fr) * v10 + (1.0 - fz) * fr * v01 + fz * fr * v11;
}

/* Quadratic shapes: the weights of the quadratic B-spline centred on x (cell
 * units) at the three nodes nearest x, i-1, i, i+1 with i the nearest node:
 * with d = x - i in [-1/2, 1/2), (1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2. */
static int qweights(double x, double w[3]) {
  int i = (int)floor(x + 0.5);
  double d = x - i;
  w[0] = 0.5 * (0.5 - d) * (0.5 - d);
  w[1] = 0.75 - d * d;
  w[2] = 0.5 * (0.5 + d) * (0.5 + d);
  return i;
}

/* Quadratic interpolation of one component of mode m at (zc, rc): 3 x 3
 * nodes of its staggered grid.  A row below the axis is the mirror image of
 * the row above it (integer grid: r_{-1} of r_1; half grid: r_{-1/2} of
 * r_{1/2}) times the component's mirror sign.                               */
static cplx interp2(const orc *o, const cplx *f, int m, double zc, double rc, int zhalf, int rhalf,
                    double mirror) {
  double wz[3], wr[3];
  int i = qweights(zhalf ? zc - 0.5 : zc, wz);
  int j = qweights(rhalf ? rc - 0.5 : rc, wr);
  cplx acc = 0.0;
  for (int b = 0; b < 3; ++b) {
    int row = j - 1 + b;
    double sg = 1.0;
    if (row < 0) {
      row = rhalf ? -row - 1 : -row;
      sg = mirror;
    }
    for (int a = 0; a < 3; ++a) acc += wz[a] * wr[b] * sg * f[ix(o, m, row, i - 1 + a)];
  }
  return acc;
}

/* All six components of every mode at one position.  out[c][m], c = E_r,
 * E_phi, E_z, B_r, B_phi, B_z; B is the time average of Eq. (12).          */
static void gather_modes(const orc *o, double zc, double rc, int jr, cplx out[6][8]) {
  for (int m = 0; m <= o->M; ++m) {
    double s_rp = (m % 2 == 0) ? -1.0 : 1.0; /* (-1)^{m+1} */
    double s_z = -s_rp;                        /* (-1)^m */
    if (o->shape == 2) {
      out[0][m] = interp2(o, o->E[CR], m, zc, rc, 0, 1, s_rp);
      out[1][m] = interp2(o, o->E[CP], m, zc, rc, 0, 0, s_rp);
      out[2][m] = interp2(o, o->E[CZ], m, zc, rc, 1, 0, s_z);
      out[3][m] = 0.5 * (interp2(o, o->Bo[CR], m, zc, rc, 1, 0, s_rp) + interp2(o, o->Bn[CR], m, zc, rc, 1, 0, s_rp));
      out[4][m] = 0.5 * (interp2(o, o->Bo[CP], m, zc, rc, 1, 1, s_rp) + interp2(o, o->Bn[CP], m, zc, rc, 1, 1, s_rp));
      out[5][m] = 0.5 * (interp2(o, o->Bo[CZ], m, zc, rc, 0, 1, s_z) + interp2(o, o->Bn[CZ], m, zc, rc, 0, 1, s_z));
      continue;
    }
    out[0][m] = interp(o, o->E[CR], m, zc, rc, jr, 0, 1, s_rp);
    out[1][m] = interp(o, o->E[CP], m, zc, rc, jr, 0, 0, 0.0);
    out[2][m] = interp(o, o->E[CZ], m, zc, rc, jr, 1, 0, 0.0);
    cplx bo_r = interp(o, o->Bo[CR], m, zc, rc, jr, 1, 0, 0.0);
    cplx bn_r = interp(o, o->Bn[CR], m, zc, rc, jr, 1, 0, 0.0);
    cplx bo_p = interp(o, o->Bo[CP], m, zc, rc, jr, 1, 1, s_rp);
    cplx bn_p = interp(o, o->Bn[CP], m, zc, rc, jr, 1, 1, s_rp);
    cplx bo_z = interp(o, o->Bo[CZ], m, zc, rc, jr, 0, 1, s_z);
    cplx bn_z = interp(o, o->Bn[CZ], m, zc, rc, jr, 0, 1, s_z);
    out[3][m] = 0.5 * (bo_r + bn_r);
    out[4][m] = 0.5 * (bo_p + bn_p);
    out[5][m] = 0.5 * (bo_z + bn_z);
  }
}

/* Cartesian field of mode m at azimuth (c, s) = (cos phi, sin phi):
 * F_r = Re(F_r^m e^{i m phi}), F_phi likewise, rotated to (x, y).           */
static void mode_to_cartesian(const cplx fr, const cplx fp, const cplx fz, cplx eimphi,
                              double c, double s, double v[3]) {
  double Fr = creal(fr * eimphi), Fp = creal(fp * eimphi);
  v[0] = Fr * c - Fp * s;
  v[1] = Fr * s + Fp * c;
  v[2] = creal(fz * eimphi);
}

/* Public helper for the gather pins: Cartesian E and B (Eq. (12) average) at
 * a point given in cell units.                                               */
void orc_gather(orc *o, double zc, double xc, double yc, double *EB) {
  double r2 = fma(xc, xc, yc * yc), rc = sqrt(r2);
  int jr = radial_index(r2, rc);
  double c = 1.0, s = 0.0;
  if (rc > 0.0) { c = xc / rc; s = yc / rc; }
  cplx g[6][8];
  gather_modes(o, zc, rc, jr, g);
  for (int k = 0; k < 6; ++k) EB[k] = 0.0;
  for (int m = 0; m <= o->M; ++m) {
    cplx e = ipow(c + I * s, m);
    double ve[3], vb[3];
    mode_to_cartesian(g[0][m], g[1][m], g[2][m], e, c, s, ve);
    mode_to_cartesian(g[3][m], g[4][m], g[5][m], e, c, s, vb);
    for (int k = 0; k < 3; ++k) { EB[k] += ve[k]; EB[3 + k] += vb[k]; }
  }
}

/* ------------------------------------------------------------------------ */
/* Boris rotation for q/m = -1 (Eq. (6)):                                    */
/*   u- = u - (dt/2) E;  t = -(dt/2) B / gamma-;  s = 2 t / (1 + t.t)        */
/*   u' = u- + u- x t;   u+ = u- + u' x s;        u_new = u+ - (dt/2) E     */
/* Returns u-, u+ (for the work of Eq. (16)) and the new u.                  */
static void boris(const double u[3], const double Ec[3], const double Bc[3], double dt,
                  double um[3], double up[3], double unew[3]) {
  for (int k = 0; k < 3; ++k) um[k] = u[k] - 0.5 * dt * Ec[k];
  double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  double t[3], s[3], up1[3];
  for (int k = 0; k < 3; ++k) t[k] = -0.5 * dt * Bc[k] / gm;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int k = 0; k < 3; ++k) s[k] = 2.0 * t[k] / (1.0 + t2);
  up1[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up1[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up1[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  up[0] = um[0] + (up1[1] * s[2] - up1[2] * s[1]);
  up[1] = um[1] + (up1[2] * s[0] - up1[0] * s[2]);
  up[2] = um[2] + (up1[0] * s[1] - up1[1] * s[0]);
  for (int k = 0; k < 3; ++k) unew[k] = up[k] - 0.5 * dt * Ec[k];
}

/* Pusher alone, for the orbit pins: one Boris step with given fields.       */
void orc_boris(double *u, const double *Ec, const double *Bc, double dt) {
  double um[3], up[3], un[3];
  boris(u, Ec, Bc, dt, um, up, un);
  u[0] = un[0]; u[1] = un[1]; u[2] = un[2];
}

/* ------------------------------------------------------------------------ */
/* Charge-conserving deposit of one particle moving from (z0, r0, phi0) to   */
/* (z1, r1, phi1) (cell units) during one step, charge q, for every mode.    */
/*                                                                           */
/* Reading (the paper only states that the solver conserves charge):         */
/*  * linear shapes S = S_z S_r on the nodes; node charge Q^m = c_m q        */
/*    e^{-i m phi} S (c_0 = 1, c_m = 2), rho^m = Q^m / V_j;                  */
/*  * Q1 - Q0 = xi (S1 - S0) + (e1 - e0)(S0 + S1)/2 with xi = (e0 + e1)/2;   */
/*    the first part is split in z and r fluxes by the 2D Esirkepov identity */
/*    S1 - S0 = Wz + Wr, Wz = dSz (Sr0 + Sr1)/2, Wr = dSr (Sz0 + Sz1)/2, and  */
/*    the flux through a face is minus the running sum of W behind it; the   */
/*    second part is carried by J_phi through the (i m / r) term of the      */
/*    divergence, which gives J_phi^m = c_m q (i r_j / m)(e1 - e0)(S0 + S1)  */
/*    / (2 dt V_j).  The result satisfies the two-point (Yee) continuity     */
/*    equation exactly; the filter P applied later makes it satisfy the D_B  */
/*    one.                                                                   */
/*  * m = 0 (no phi term in the divergence) and m = 1 on the axis node       */
/*    (where r_j = 0 and Gauss's law is not evolved): J_phi is deposited     */
/*    directly as c_m q v_phi e^{-i m phi_mid} (S0 + S1) / (2 V_j).          */
static void deposit_particle(orc *o, double q, double z0, double r0, int j0, double c0, double s0,
                             double z1, double r1, int j1, double c1, double s1,
                             double vphi, double cmid, double smid) {
  const double dt = o->dt, dr = o->dr;
  int i0 = (int)floor(z0), i1 = (int)floor(z1);
  double f0 = z0 - i0, f1 = z1 - i1;
  double g0 = r0 - j0, g1 = r1 - j1;
  int ib = i0 < i1 ? i0 : i1;
  int jb = j0 < j1 ? j0 : j1;
  double Sz0[3] = {0, 0, 0}, Sz1[3] = {0, 0, 0}, Sr0[3] = {0, 0, 0}, Sr1[3] = {0, 0, 0};
  Sz0[i0 - ib] += 1.0 - f0; Sz0[i0 - ib + 1] += f0;
  Sz1[i1 - ib] += 1.0 - f1; Sz1[i1 - ib + 1] += f1;
  Sr0[j0 - jb] += 1.0 - g0; Sr0[j0 - jb + 1] += g0;
  Sr1[j1 - jb] += 1.0 - g1; Sr1[j1 - jb + 1] += g1;
  double Wz[3][3], Wr[3][3], Ssum[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      Wz[a][b] = (Sz1[a] - Sz0[a]) * (Sr0[b] + Sr1[b]) * 0.5;
      Wr[a][b] = (Sr1[b] - Sr0[b]) * (Sz0[a] + Sz1[a]) * 0.5;
      Ssum[a][b] = Sz0[a] * Sr0[b] + Sz1[a] * Sr1[b];
    }
  for (int m = 0; m <= o->M; ++m) {
    double cm = m == 0 ? 1.0 : 2.0;
    cplx e0 = ipow(c0 - I * s0, m), e1 = ipow(c1 - I * s1, m);
    cplx xi = 0.5 * (e0 + e1);
    /* J_z at (ib+a+1/2, jb+b), a = 0, 1 */
    for (int b = 0; b < 3; ++b) {
      double run = 0.0;
      for (int a = 0; a < 2; ++a) {
        run += Wz[a][b];
        int j = jb + b;
        o->J[CZ][ix(o, m, j, ib + a)] += -cm * q * xi * run / (dt * area_z(o, j));
      }
    }
    /* J_r at (ib+a, jb+b+1/2), b = 0, 1 */
    for (int a = 0; a < 3; ++a) {
      double run = 0.0;
      for (int b = 0; b < 2; ++b) {
        run += Wr[a][b];
        int j = jb + b;
        o->J[CR][ix(o, m, j, ib + a)] += -cm * q * xi * run / (dt * area_r(o, j));
      }
    }
    /* J_phi at (ib+a, jb+b) */
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        int j = jb + b;
        cplx v;
        if (m == 0 || (m == 1 && j == 0)) {
          cplx emid = ipow(cmid - I * smid, m);
          v = cm * q * vphi * emid * Ssum[a][b] / (2.0 * vol_node(o, j));
        } else {
          v = cm * q * (I * (j * dr) / m) * (e1 - e0) * Ssum[a][b] / (2.0 * dt * vol_node(o, j));
        }
        o->J[CP][ix(o, m, j, ib + a)] += v;
      }
  }
}

/* Quadratic shapes: the same charge-conserving deposit on the 4 x 4 nodes
 * that hold both positions' 3 x 3 supports (a move of less than a cell),
 * S = Sz Sr with quadratic B-splines.  A particle within half a cell of the
 * axis has shape on row r_{-1}; the point (-r, phi) is (r, phi + pi), so
 * that charge belongs to row r_1 with the mode's sign (-1)^m, and the
 * z-flux of row r_{-1}, the r-flux through r_{-1/2} and the phi-current of
 * row r_{-1} belong to row r_1, face r_{1/2} and row r_1 with the signs of a
 * z, an r and a phi component ((-1)^m, (-1)^{m+1}, (-1)^{m+1}).  Folded so,
 * the node charges of rows r >= dr (every m) and of the axis row (m = 0)
 * change by exactly minus the divergence of the folded fluxes.  The phi
 * closure of a folded row is (-1)^m times its value at r_1, the m = 0 direct
 * term (-1) times it.                                                        */
static void deposit_particle2(orc *o, double q, double z0, double r0, double c0, double s0,
                              double z1, double r1, double c1, double s1,
                              double vphi, double cmid, double smid) {
  const double dt = o->dt, dr = o->dr;
  double wz0[3], wz1[3], wr0[3], wr1[3];
  int i0 = qweights(z0, wz0), i1 = qweights(z1, wz1);
  int j0 = qweights(r0, wr0), j1 = qweights(r1, wr1);
  int ib = (i0 < i1 ? i0 : i1) - 1, jb = (j0 < j1 ? j0 : j1) - 1;
  double Sz0[4] = {0, 0, 0, 0}, Sz1[4] = {0, 0, 0, 0}, Sr0[4] = {0, 0, 0, 0}, Sr1[4] = {0, 0, 0, 0};
  for (int k = 0; k < 3; ++k) {
    Sz0[i0 - 1 - ib + k] += wz0[k];
    Sz1[i1 - 1 - ib + k] += wz1[k];
    Sr0[j0 - 1 - jb + k] += wr0[k];
    Sr1[j1 - 1 - jb + k] += wr1[k];
  }
  double Wz[4][4], Wr[4][4], Ssum[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      Wz[a][b] = (Sz1[a] - Sz0[a]) * (Sr0[b] + Sr1[b]) * 0.5;
      Wr[a][b] = (Sr1[b] - Sr0[b]) * (Sz0[a] + Sz1[a]) * 0.5;
      Ssum[a][b] = Sz0[a] * Sr0[b] + Sz1[a] * Sr1[b];
    }
  for (int m = 0; m <= o->M; ++m) {
    double cm = m == 0 ? 1.0 : 2.0;
    double s_z = (m % 2 == 0) ? 1.0 : -1.0, s_rp = -s_z;
    cplx e0 = ipow(c0 - I * s0, m), e1 = ipow(c1 - I * s1, m);
    cplx xi = 0.5 * (e0 + e1);
    /* J_z at (ib+a+1/2, jb+b), a = 0..2; a row past r_Nr has zero weight
     * (both positions nearest r_{Nr-1}) and is skipped */
    for (int b = 0; b < 4; ++b) {
      int j = jb + b;
      double sg = 1.0;
      if (j > o->Nr) continue;
      if (j < 0) { j = -j; sg = s_z; }
      double run = 0.0;
      for (int a = 0; a < 3; ++a) {
        run += Wz[a][b];
        o->J[CZ][ix(o, m, j, ib + a)] += sg * (-cm * q * xi * run) / (dt * area_z(o, j));
      }
    }
    /* J_r at (ib+a, jb+b+1/2), b = 0..2 (face index jb+b) */
    for (int a = 0; a < 4; ++a) {
      double run = 0.0;
      for (int b = 0; b < 3; ++b) {
        run += Wr[a][b];
        int j = jb + b;
        double sg = 1.0;
        if (j < 0) { j = -j - 1; sg = s_rp; }
        o->J[CR][ix(o, m, j, ib + a)] += sg * (-cm * q * xi * run) / (dt * area_r(o, j));
      }
    }
    /* J_phi at (ib+a, jb+b) */
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int j = jb + b;
        double sg = 1.0;
        if (j > o->Nr) continue;
        if (j < 0) { j = -j; sg = -1.0; }
        cplx v;
        if (m == 0 || (m == 1 && j == 0 && sg > 0)) {
          cplx emid = ipow(cmid - I * smid, m);
          v = sg * cm * q * vphi * emid * Ssum[a][b] / (2.0 * vol_node(o, j));
        } else {
          v = (sg < 0 ? s_z : 1.0) * cm * q * (I * (j * dr) / m) * (e1 - e0) * Ssum[a][b] / (2.0 * dt * vol_node(o, j));
        }
        o->J[CP][ix(o, m, j, ib + a)] += v;
      }
  }
}

/* rho^m = c_m q e^{-i m phi} S / V_j of every particle at its position.    */
static void deposit_rho_all(orc *o) {
  memset(o->rho, 0, o->nf * sizeof(cplx));
  for (long p = 0; p < o->np; ++p) {
    double zc = o->z[p], xc = o->x[p], yc = o->y[p];
    double r2 = fma(xc, xc, yc * yc), rc = sqrt(r2);
    int jr = radial_index(r2, rc);
    double c = 1.0, s = 0.0;
    if (rc > 0.0) { c = xc / rc; s = yc / rc; }
    int i0 = (int)floor(zc);
    double fz = zc - i0, fr = rc - jr;
    double q = -o->w[p];
    for (int m = 0; m <= o->M; ++m) {
      double cm = m == 0 ? 1.0 : 2.0;
      cplx e = ipow(c - I * s, m);
      if (o->shape == 2) { /* rows below the axis folded with (-1)^m, as in the deposit */
        double wz[3], wr[3];
        int i = qweights(zc, wz), j = qweights(rc, wr);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            int row = j - 1 + b;
            double sg = 1.0;
            if (row < 0) { row = -row; sg = (m % 2 == 0) ? 1.0 : -1.0; }
            o->rho[ix(o, m, row, i - 1 + a)] += sg * cm * q * e * wz[a] * wr[b] / vol_node(o, row);
          }
        continue;
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          double S = (a ? fz : 1.0 - fz) * (b ? fr : 1.0 - fr);
          o->rho[ix(o, m, jr + b, i0 + a)] += cm * q * e * S / vol_node(o, jr + b);
        }
    }
  }
  /* the m >= 1 density vanishes on the axis */
  for (int m = 1; m <= o->M; ++m)
    for (int i = 0; i < o->Nz; ++i) o->rho[ix(o, m, 0, i)] = 0.0;
}

void orc_deposit_rho(orc *o) { deposit_rho_all(o); }

/* Charge-conserving current of one particle alone (for brute-force pins):
 * clears J, deposits the move (z0,x0,y0) -> (z1,x1,y1) with charge q and
 * azimuthal velocity vphi (used only where J_phi is deposited directly).    */
/* Adds the current of one particle's move to o->J (orc_deposit_one clears
 * the current first).                                                       */
void orc_deposit_add(orc *o, double q, double z0, double x0, double y0, double z1, double x1,
                     double y1, double vphi) {
  double r20 = fma(x0, x0, y0 * y0), r0 = sqrt(r20);
  double r21 = fma(x1, x1, y1 * y1), r1 = sqrt(r21);
  int j0 = radial_index(r20, r0), j1 = radial_index(r21, r1);
  double c0 = 1, s0 = 0, c1 = 1, s1 = 0;
  if (r0 > 0) { c0 = x0 / r0; s0 = y0 / r0; }
  if (r1 > 0) { c1 = x1 / r1; s1 = y1 / r1; }
  double xm = 0.5 * (x0 + x1), ym = 0.5 * (y0 + y1), rm = sqrt(xm * xm + ym * ym);
  double cm = 1, sm = 0;
  if (rm > 0) { cm = xm / rm; sm = ym / rm; }
  if (o->shape == 2) deposit_particle2(o, q, z0, r0, c0, s0, z1, r1, c1, s1, vphi, cm, sm);
  else deposit_particle(o, q, z0, r0, j0, c0, s0, z1, r1, j1, c1, s1, vphi, cm, sm);
}

void orc_deposit_one(orc *o, double q, double z0, double x0, double y0, double z1, double x1,
                     double y1, double vphi) {
  for (int c = 0; c < 3; ++c) memset(o->J[c], 0, o->nf * sizeof(cplx));
  orc_deposit_add(o, q, z0, x0, y0, z1, x1, y1, vphi);
}

/* ------------------------------------------------------------------------ */
/* one PIC step n -> n+1                                                     */

static void push_and_deposit(orc *o) {
  const double dt = o->dt, dz = o->dz, dr = o->dr;
  const int M = o->M;
  const double Rwall = (double)(o->Nr - 1); /* particles stay below r = (Nr-1) dr */
  for (int c = 0; c < 3; ++c) memset(o->J[c], 0, o->nf * sizeof(cplx));
  for (long p = 0; p < o->np; ++p) {
    double z0 = o->z[p], x0 = o->x[p], y0 = o->y[p];
    double r20 = fma(x0, x0, y0 * y0), r0 = sqrt(r20);
    int j0 = radial_index(r20, r0);
    double c0 = 1.0, s0 = 0.0;
    if (r0 > 0.0) { c0 = x0 / r0; s0 = y0 / r0; }

    /* gather E^n and Bbar^n (Eq. (12)), per mode and in total */
    cplx g[6][8];
    gather_modes(o, z0, r0, j0, g);
    double Ec[3] = {0, 0, 0}, Bc[3] = {0, 0, 0}, Em[8][3];
    for (int m = 0; m <= M; ++m) {
      cplx e = ipow(c0 + I * s0, m);
      double vb[3];
      mode_to_cartesian(g[0][m], g[1][m], g[2][m], e, c0, s0, Em[m]);
      mode_to_cartesian(g[3][m], g[4][m], g[5][m], e, c0, s0, vb);
      for (int k = 0; k < 3; ++k) { Ec[k] += Em[m][k]; Bc[k] += vb[k]; }
    }

    /* push (Eq. (6)) */
    double u[3] = {o->ux[p], o->uy[p], o->uz[p]}, um[3], up[3], un[3];
    double g_old = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    boris(u, Ec, Bc, dt, um, up, un);
    double g_new = sqrt(1.0 + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);

    /* per-mode work of Eq. (16) for tracked particles, with the velocity
     * v_eff = (u- + u+)/(gamma^{n-1/2} + gamma^{n+1/2}), for which the modes
     * sum exactly to gamma^{n+1/2} - gamma^{n-1/2}.                         */
    if (o->slot[p] >= 0) {
      double inv = 1.0 / (g_old + g_new);
      double v[3] = {(um[0] + up[0]) * inv, (um[1] + up[1]) * inv, (um[2] + up[2]) * inv};
      double *W = o->W + (size_t)o->slot[p] * (M + 1);
      for (int m = 0; m <= M; ++m)
        W[m] += -dt * (Em[m][0] * v[0] + Em[m][1] * v[1] + Em[m][2] * v[2]);
      /* the same work split by field direction instead of mode, Eq. (17):
       * W_z = -e int E_z v_z dt, W_perp = -e int E_perp . v_perp dt */
      double ez = 0.0, ep = 0.0;
      for (int m = 0; m <= M; ++m) {
        ez += Em[m][2];
        ep += Em[m][0] * v[0] + Em[m][1] * v[1];
      }
      double *Wc = o->Wc + (size_t)o->slot[p] * 2;
      Wc[0] += -dt * ez * v[2];
      Wc[1] += -dt * ep;
    }

    /* move: x^{n+1} = x^n + dt u^{n+1/2} / gamma^{n+1/2}, in cell units */
    double z1 = z0 + dt * un[2] / g_new / dz;
    double x1 = x0 + dt * un[0] / g_new / dr;
    double y1 = y0 + dt * un[1] / g_new / dr;
    double r21 = fma(x1, x1, y1 * y1), r1 = sqrt(r21);
    if (r1 >= Rwall) { /* specular reflection at r = (Nr-1) dr */
      double nx = x1 / r1, ny = y1 / r1;
      double sc = (2.0 * Rwall - r1) / r1;
      x1 *= sc; y1 *= sc;
      double ur = un[0] * nx + un[1] * ny;
      un[0] -= 2.0 * ur * nx;
      un[1] -= 2.0 * ur * ny;
      r21 = fma(x1, x1, y1 * y1);
      r1 = sqrt(r21);
    }
    int j1 = radial_index(r21, r1);
    double c1 = 1.0, s1 = 0.0;
    if (r1 > 0.0) { c1 = x1 / r1; s1 = y1 / r1; }

    /* deposit J^{n+1/2} */
    double xm = 0.5 * (x0 + x1), ym = 0.5 * (y0 + y1);
    double rm = sqrt(xm * xm + ym * ym), cmid = 1.0, smid = 0.0, vphi = 0.0;
    if (rm > 0.0) {
      cmid = xm / rm; smid = ym / rm;
      vphi = (cmid * un[1] - smid * un[0]) / g_new;
    }
    if (o->shape == 2)
      deposit_particle2(o, -o->w[p], z0, r0, c0, s0, z1, r1, c1, s1, vphi, cmid, smid);
    else
      deposit_particle(o, -o->w[p], z0, r0, j0, c0, s0, z1, r1, j1, c1, s1, vphi, cmid, smid);

    if (o->win_K > 0) {
      /* moving window: an electron that left the box through either end
       * carries no charge from the next step on and is dropped at the next
       * window move (its position is kept as it is, outside [0, Nz))       */
      if (z1 < 0.0 || z1 >= o->Nz) o->w[p] = 0.0;
    } else { /* periodic in z */
      if (z1 < 0.0) z1 += o->Nz;
      if (z1 >= o->Nz) z1 -= o->Nz;
    }
    o->z[p] = z1; o->x[p] = x1; o->y[p] = y1;
    o->ux[p] = un[0]; o->uy[p] = un[1]; o->uz[p] = un[2];
  }
  /* the m >= 1 J_z vanishes on the axis (E_z^m is held at zero there) */
  for (int m = 1; m <= M; ++m)
    for (int i = 0; i < o->Nz; ++i) o->J[CZ][ix(o, m, 0, i)] = 0.0;
}

static void swap_b(orc *o) {
  for (int c = 0; c < 3; ++c) { cplx *t = o->Bo[c]; o->Bo[c] = o->Bn[c]; o->Bn[c] = t; }
}

/* Field update of one step with the current already in o->J:
 *   E^{n+1}   = E^n + dt (curl_B B^{n+1/2} - J')       (Ampere, Eq. (9))
 *   B^{n+3/2} = B^{n+1/2} - dt curl_E E^{n+1}         (Faraday, Eq. (9))   */
static void field_update(orc *o) {
  ampere(o, o->Bn);
  faraday(o, o->Bo, o->Bn, o->E, o->dt);
  swap_b(o);
}

static void load_electron(orc *o, long p, int64_t pid, long S);

/* Moving window (App. A: the box follows the pulse through the plasma).
 * Done before a step when the steps taken are a positive multiple of win_K:
 * the box advances by the s = floor(v n dt / dz) - S whole cells the front,
 * moving at v = win_speed c, crossed since the last move.  E^n, B^{n-1/2}
 * and B^{n+1/2} move back by s columns with zeros entering at the front and
 * the win_guard columns at the back are cleared (what the z-periodic
 * stencils carry round from the back would otherwise reach the front); the
 * electrons move back by s cells, those outside [0, Nz) are dropped (left
 * through the back, or earlier through either end), and the plasma of the
 * s new absolute columns is loaded as orc_load_plasma loads it.            */
static void window_move(orc *o) {
  const long target = (long)floor(o->win_speed * (double)o->nstep * o->dt / o->dz);
  long s = target - o->win_S;
  if (s <= 0) return;
  const int Nz = o->Nz;
  for (int c = 0; c < 3; ++c) {
    cplx *arr[3] = {o->E[c], o->Bo[c], o->Bn[c]};
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m <= o->M; ++m)
        for (int j = 0; j <= o->Nr; ++j) {
          cplx *row = arr[a] + ((size_t)m * (size_t)(o->Nr + 1) + (size_t)j) * (size_t)Nz;
          for (int i = 0; i < Nz; ++i) row[i] = (i + s < Nz) ? row[i + s] : 0.0;
          for (int i = 0; i < o->win_guard && i < Nz; ++i) row[i] = 0.0;
        }
  }
  long keep = 0;
  for (long p = 0; p < o->np; ++p) {
    const double z = o->z[p] - (double)s;
    if (z < 0.0 || z >= Nz) continue;
    o->z[keep] = z; o->x[keep] = o->x[p]; o->y[keep] = o->y[p];
    o->ux[keep] = o->ux[p]; o->uy[keep] = o->uy[p]; o->uz[keep] = o->uz[p];
    o->w[keep] = o->w[p]; o->id[keep] = o->id[p]; o->slot[keep] = o->slot[p];
    ++keep;
  }
  const int nrc = o->Nr - 1;
  const long fresh = (s < Nz ? s : Nz) * (long)nrc * o->ppc;
  const long np = keep + fresh;
  o->z = (double *)realloc(o->z, sizeof(double) * (np > 0 ? np : 1));
  o->x = (double *)realloc(o->x, sizeof(double) * (np > 0 ? np : 1));
  o->y = (double *)realloc(o->y, sizeof(double) * (np > 0 ? np : 1));
  o->ux = (double *)realloc(o->ux, sizeof(double) * (np > 0 ? np : 1));
  o->uy = (double *)realloc(o->uy, sizeof(double) * (np > 0 ? np : 1));
  o->uz = (double *)realloc(o->uz, sizeof(double) * (np > 0 ? np : 1));
  o->w = (double *)realloc(o->w, sizeof(double) * (np > 0 ? np : 1));
  o->id = (int64_t *)realloc(o->id, sizeof(int64_t) * (np > 0 ? np : 1));
  o->slot = (int32_t *)realloc(o->slot, sizeof(int32_t) * (np > 0 ? np : 1));
  /* the new columns are absolute columns [target + Nz - s', target + Nz) */
  const long a0 = target + Nz - (s < Nz ? s : Nz);
  long p = keep;
  for (long a = a0; a < target + Nz; ++a)
    for (int ir = 0; ir < nrc; ++ir)
      for (int k = 0; k < o->ppc; ++k, ++p) {
        const int64_t pid = ((int64_t)a * nrc + ir) * o->ppc + k;
        load_electron(o, p, pid, target);
        o->slot[p] = -1;
      }
  o->np = np;
  o->win_S = target;
}

void orc_set_window(orc *o, int K, double speed, int guard) {
  o->win_K = K > 0 ? K : 0;
  o->win_speed = speed;
  o->win_guard = guard > 0 ? guard : 0;
}
long orc_window_cells(const orc *o) { return o->win_S; }

void orc_step(orc *o, int nsteps) {
  for (int s = 0; s < nsteps; ++s) {
    if (o->win_K > 0 && o->nstep > 0 && o->nstep % o->win_K == 0) window_move(o);
    push_and_deposit(o);
    if (!o->freeze_fields) field_update(o);
    if (o->deposit_rho) deposit_rho_all(o);
    o->nstep++;
  }
}

/* Field-only steps with zero current (vacuum).                              */
void orc_field_step(orc *o, int nsteps) {
  for (int c = 0; c < 3; ++c) memset(o->J[c], 0, o->nf * sizeof(cplx));
  for (int s = 0; s < nsteps; ++s) field_update(o);
}

/* Given E^0 in o->E and B^0 in o->Bn, form B^{-1/2} = B^0 + (dt/2) curl_E E^0
 * and B^{+1/2} = B^0 - (dt/2) curl_E E^0, so that their average is B^0.     */
void orc_start_fields(orc *o) {
  faraday(o, o->Bo, o->Bn, o->E, -0.5 * o->dt);
  faraday(o, o->Bn, o->Bn, o->E, 0.5 * o->dt);
}

/* ------------------------------------------------------------------------ */
/* Loading (synthetic plasma; the paper's runs use ionisation injection).    */
/* Counter-based SplitMix64: the k-th output of the stream seeded with s is  */
/* mix(s + k * 0x9E3779B97F4A7C15), mix = the published SplitMix64 finaliser.*/

static uint64_t splitmix64_out(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
uint64_t orc_splitmix64(uint64_t seed, uint64_t k) { return splitmix64_out(seed, k); }

/* uniform in [0, 1) with 53 random bits: draw d of particle pid */
static double uniform_draw(uint64_t seed, int64_t pid, int d) {
  uint64_t k = 4ULL * (uint64_t)pid + (uint64_t)d + 1ULL;
  return (double)(splitmix64_out(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

static int cmp_track(const void *a, const void *b) {
  const double *x = (const double *)a, *y = (const double *)b;
  if (x[0] < y[0]) return -1;
  if (x[0] > y[0]) return 1;
  return (x[1] < y[1]) ? -1 : (x[1] > y[1]);
}

/* Electron pid of the plasma (pid = (a (Nr-1) + ir) ppc + s for absolute
 * column a, radial cell ir, sample s) into particle slot p, in the
 * coordinates of a box whose column 0 is absolute column S.                 */
static void load_electron(orc *o, long p, int64_t pid, long S) {
  const int nrc = o->Nr - 1, ppc = o->ppc;
  const int64_t a = pid / ((int64_t)nrc * ppc), ir = (pid / ppc) % nrc;
  double U0 = uniform_draw(o->seed, pid, 0), U1 = uniform_draw(o->seed, pid, 1);
  double U2 = uniform_draw(o->seed, pid, 2);
  double zc = (double)a + U0, rc = (double)ir + U1, phi = 2.0 * ORC_PI * U2;
  double n = o->n0;
  if (o->ramp_len > 0.0) {
    double f = (zc * o->dz - o->ramp_start) / o->ramp_len;
    if (f < 0.0) f = 0.0;
    if (f > 1.0) f = 1.0;
    n = o->n0 * f;
  }
  if (o->down_len > 0.0) {
    double g = 1.0 - (zc * o->dz - o->down_start) / o->down_len;
    if (g < 0.0) g = 0.0;
    if (g > 1.0) g = 1.0;
    n *= g;
  }
  o->z[p] = zc - (double)S;
  o->x[p] = rc * cos(phi);
  o->y[p] = rc * sin(phi);
  o->ux[p] = o->uy[p] = o->uz[p] = 0.0;
  o->w[p] = n * (2.0 * ORC_PI) * (rc * o->dr) * o->dr * o->dz / ppc;
  o->id[p] = pid;
}

/* Cold electrons, ppc per cell in cells iz = 0..Nz-1, ir = 0..Nr-2, at
 * uniform-random (z, r, phi) in the cell; density n(z) = n0 times a linear
 * up-ramp over [ramp_start, ramp_start + ramp_len] and a linear down-ramp
 * over [down_start, down_start + down_len] (physical z; App. A's profile is
 * up-ramp, plateau, down-ramp; a zero length means no ramp) enters the
 * weight w = n(z) 2 pi r dr dr dz / ppc (r physical), so that the density is
 * uniform in r.  Particle pid = (iz (Nr-1) + ir) ppc + s.  The n_tracked
 * particles with the smallest (draw 3, pid) are tracked.                    */
int orc_load_plasma(orc *o, int ppc, double n0, double ramp_start, double ramp_len, uint64_t seed,
                    int n_tracked, double down_start, double down_len) {
  free_particles(o);
  const int Nz = o->Nz, nrc = o->Nr - 1;
  long np = (long)Nz * nrc * ppc;
  if (n_tracked > np) return -1;
  o->np = np;
  o->z = (double *)malloc(sizeof(double) * np);
  o->x = (double *)malloc(sizeof(double) * np);
  o->y = (double *)malloc(sizeof(double) * np);
  o->ux = (double *)calloc(np, sizeof(double));
  o->uy = (double *)calloc(np, sizeof(double));
  o->uz = (double *)calloc(np, sizeof(double));
  o->w = (double *)malloc(sizeof(double) * np);
  o->id = (int64_t *)malloc(sizeof(int64_t) * np);
  o->slot = (int32_t *)malloc(sizeof(int32_t) * np);
  o->ppc = ppc; o->seed = seed; o->n0 = n0;
  o->ramp_start = ramp_start; o->ramp_len = ramp_len;
  o->down_start = down_start; o->down_len = down_len;
  o->win_S = 0;
  for (int iz = 0; iz < Nz; ++iz)
    for (int ir = 0; ir < nrc; ++ir)
      for (int s = 0; s < ppc; ++s) {
        int64_t pid = ((int64_t)iz * nrc + ir) * ppc + s;
        load_electron(o, pid, pid, 0);
        o->slot[pid] = -1;
      }
  o->ntr = n_tracked;
  o->W = (double *)calloc((size_t)(n_tracked > 0 ? n_tracked : 1) * (o->M + 1), sizeof(double));
  o->Wc = (double *)calloc((size_t)(n_tracked > 0 ? n_tracked : 1) * 2, sizeof(double));
  o->gam0 = (double *)calloc((size_t)(n_tracked > 0 ? n_tracked : 1), sizeof(double));
  o->tr_id = (int64_t *)calloc((size_t)(n_tracked > 0 ? n_tracked : 1), sizeof(int64_t));
  if (n_tracked > 0) {
    double *key = (double *)malloc(sizeof(double) * 2 * np);
    for (long p = 0; p < np; ++p) { key[2 * p] = uniform_draw(seed, p, 3); key[2 * p + 1] = (double)p; }
    qsort(key, np, 2 * sizeof(double), cmp_track);
    /* slots are numbered in ascending particle id */
    int64_t *sel = (int64_t *)malloc(sizeof(int64_t) * n_tracked);
    for (int k = 0; k < n_tracked; ++k) sel[k] = (int64_t)key[2 * k + 1];
    for (int a = 1; a < n_tracked; ++a) { /* insertion sort of the chosen ids */
      int64_t v = sel[a];
      int b = a - 1;
      while (b >= 0 && sel[b] > v) { sel[b + 1] = sel[b]; --b; }
      sel[b + 1] = v;
    }
    for (int k = 0; k < n_tracked; ++k) { o->slot[sel[k]] = k; o->gam0[k] = 1.0; o->tr_id[k] = sel[k]; }
    free(sel);
    free(key);
  }
  return 0;
}

/* Replace the particle set (tests with hand-placed particles).  All tracked. */
int orc_set_particles(orc *o, long np, const double *z, const double *x, const double *y,
                      const double *ux, const double *uy, const double *uz, const double *w,
                      int track_all) {
  free_particles(o);
  o->np = np;
  o->z = (double *)malloc(sizeof(double) * (np ? np : 1));
  o->x = (double *)malloc(sizeof(double) * (np ? np : 1));
  o->y = (double *)malloc(sizeof(double) * (np ? np : 1));
  o->ux = (double *)malloc(sizeof(double) * (np ? np : 1));
  o->uy = (double *)malloc(sizeof(double) * (np ? np : 1));
  o->uz = (double *)malloc(sizeof(double) * (np ? np : 1));
  o->w = (double *)malloc(sizeof(double) * (np ? np : 1));
  o->id = (int64_t *)malloc(sizeof(int64_t) * (np ? np : 1));
  o->slot = (int32_t *)malloc(sizeof(int32_t) * (np ? np : 1));
  for (long p = 0; p < np; ++p) {
    o->z[p] = z[p]; o->x[p] = x[p]; o->y[p] = y[p];
    o->ux[p] = ux[p]; o->uy[p] = uy[p]; o->uz[p] = uz[p]; o->w[p] = w[p];
    o->id[p] = p;
    o->slot[p] = track_all ? (int32_t)p : -1;
  }
  o->ntr = track_all ? (int)np : 0;
  o->W = (double *)calloc((size_t)(o->ntr > 0 ? o->ntr : 1) * (o->M + 1), sizeof(double));
  o->Wc = (double *)calloc((size_t)(o->ntr > 0 ? o->ntr : 1) * 2, sizeof(double));
  o->gam0 = (double *)calloc((size_t)(o->ntr > 0 ? o->ntr : 1), sizeof(double));
  o->tr_id = (int64_t *)malloc(sizeof(int64_t) * (o->ntr > 0 ? o->ntr : 1));
  for (int k = 0; k < o->ntr; ++k) {
    o->gam0[k] = sqrt(1.0 + ux[k] * ux[k] + uy[k] * uy[k] + uz[k] * uz[k]);
    o->tr_id[k] = k;
  }
  return 0;
}

/* Copy the particle state out: arrays of length np (any may be NULL).       */
void orc_get_particles(orc *o, double *z, double *x, double *y, double *ux, double *uy, double *uz,
                       double *w, int64_t *id) {
  for (long p = 0; p < o->np; ++p) {
    if (z) z[p] = o->z[p];
    if (x) x[p] = o->x[p];
    if (y) y[p] = o->y[p];
    if (ux) ux[p] = o->ux[p];
    if (uy) uy[p] = o->uy[p];
    if (uz) uz[p] = o->uz[p];
    if (w) w[p] = o->w[p];
    if (id) id[p] = o->id[p];
  }
}

/* Overwrite positions/momenta of the existing particles (same count).       */
void orc_put_particles(orc *o, const double *z, const double *x, const double *y, const double *ux,
                       const double *uy, const double *uz, const double *w) {
  for (long p = 0; p < o->np; ++p) {
    o->z[p] = z[p]; o->x[p] = x[p]; o->y[p] = y[p];
    o->ux[p] = ux[p]; o->uy[p] = uy[p]; o->uz[p] = uz[p]; o->w[p] = w[p];
  }
}

/* Tracked output, slot order: ids, W [ntr][M+1], gamma from u, and the FP64
 * accumulated gamma0 + sum_m W_m.                                           */
int orc_tracked(orc *o, int64_t *ids, double *W, double *gamma, double *gamma_acc) {
  /* every slot reports its id, work and gamma_acc; gamma is NaN for a
   * tracked electron no longer in the box (dropped by the moving window)   */
  for (int k = 0; k < o->ntr; ++k) {
    if (ids) ids[k] = o->tr_id[k];
    double s = o->gam0[k];
    for (int m = 0; m <= o->M; ++m) {
      if (W) W[(size_t)k * (o->M + 1) + m] = o->W[(size_t)k * (o->M + 1) + m];
      s += o->W[(size_t)k * (o->M + 1) + m];
    }
    if (gamma) gamma[k] = NAN;
    if (gamma_acc) gamma_acc[k] = s;
  }
  if (gamma)
    for (long p = 0; p < o->np; ++p) {
      int k = o->slot[p];
      if (k >= 0) gamma[k] = sqrt(1.0 + o->ux[p] * o->ux[p] + o->uy[p] * o->uy[p] + o->uz[p] * o->uz[p]);
    }
  return o->ntr;
}

/* Work of E_z and of E_perp on the tracked particles (Eq. (17)), slot order. */
int orc_cartesian_work(orc *o, double *wz, double *wperp) {
  for (int k = 0; k < o->ntr; ++k) {
    if (wz) wz[k] = o->Wc[2 * (size_t)k];
    if (wperp) wperp[k] = o->Wc[2 * (size_t)k + 1];
  }
  return o->ntr;
}

/* Kinetic energy sum w (gamma - 1).                                         */
double orc_kinetic(orc *o) {
  double s = 0.0;
  for (long p = 0; p < o->np; ++p) {
    double g = sqrt(1.0 + o->ux[p] * o->ux[p] + o->uy[p] * o->uy[p] + o->uz[p] * o->uz[p]);
    s += o->w[p] * (g - 1.0);
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Laser of Eq. (18) near focus, linearly polarised along x, placed in the   */
/* m = 1 arrays at t = 0 (reading: initial condition, not an antenna):       */
/*   E_x = A sin(theta),  E_z = (2 x / (k w0^2)) A cos(theta),  B_y = E_x,   */
/*   B_z = (2 y / (k w0^2)) A cos(theta)  (from div B = 0),                  */
/*   A = a0 g(z) exp(-r^2/w0^2),  theta = -k (z - zc)  (k = w0 = 1 here),     */
/* g = exp(-2 ln2 (z - zc)^2 / tau^2) (intensity FWHM tau) times a sin^2     */
/* taper over the outer `taper` length of the periodic box.  Mode form:      */
/* E_r^1 = E, E_phi^1 = iE, E_z^1 = (2r/(k w0^2)) A cos, B_r^1 = -iB,        */
/* B_phi^1 = B, B_z^1 = -i (2r/(k w0^2)) A cos.  Adds into E^n and B^{n+1/2}  */
/* (which holds B^0 until orc_start_fields is called).                       */

static double envelope(double zp, double zc, double tau, double L, double taper) {
  double g = exp(-2.0 * log(2.0) * (zp - zc) * (zp - zc) / (tau * tau));
  if (taper > 0.0) {
    if (zp < taper) { double s = sin(0.5 * ORC_PI * zp / taper); g *= s * s; }
    if (zp > L - taper) { double s = sin(0.5 * ORC_PI * (L - zp) / taper); g *= s * s; }
  }
  return g;
}

int orc_add_laser(orc *o, double a0, double w0, double tau, double zc, double taper) {
  if (o->M < 1) return -1;
  const int Nz = o->Nz, Nr = o->Nr;
  const double dz = o->dz, dr = o->dr, L = Nz * dz, k = 1.0;
  for (int j = 0; j <= Nr; ++j)
    for (int i = 0; i < Nz; ++i) {
      size_t q = ix(o, 1, j, i);
      double zi = i * dz, zh = (i + 0.5) * dz, rj = j * dr, rh = (j + 0.5) * dr;
      /* (z_i, r_{j+1/2}): E_r, B_z */
      double A = a0 * envelope(zi, zc, tau, L, taper) * exp(-rh * rh / (w0 * w0));
      double th = -k * (zi - zc);
      if (j < Nr) {
        o->E[CR][q] += A * sin(th);
        o->Bn[CZ][q] += -I * (2.0 * rh / (k * w0 * w0)) * A * cos(th);
      }
      /* (z_i, r_j): E_phi */
      A = a0 * envelope(zi, zc, tau, L, taper) * exp(-rj * rj / (w0 * w0));
      if (j < Nr) o->E[CP][q] += I * A * sin(th);
      /* (z_{i+1/2}, r_j): E_z, B_r */
      A = a0 * envelope(zh, zc, tau, L, taper) * exp(-rj * rj / (w0 * w0));
      th = -k * (zh - zc);
      if (j < Nr) o->E[CZ][q] += (2.0 * rj / (k * w0 * w0)) * A * cos(th);
      o->Bn[CR][q] += -I * A * sin(th);
      /* (z_{i+1/2}, r_{j+1/2}): B_phi */
      A = a0 * envelope(zh, zc, tau, L, taper) * exp(-rh * rh / (w0 * w0));
      if (j < Nr) o->Bn[CP][q] += A * sin(th);
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Round the state to what an FP32 run starts from: positions as int32 cell  */
/* plus FP32 offset in z, FP32 x, y (cells), FP32 momenta and weights, FP32  */
/* fields.  An offset that rounds to 1.0f carries into the cell index.       */
void orc_round_to_fp32(orc *o) {
  for (long p = 0; p < o->np; ++p) {
    double iz = floor(o->z[p]);
    float fz = (float)(o->z[p] - iz);
    if (fz >= 1.0f) { fz = 0.0f; iz += 1.0; if (iz >= o->Nz) iz -= o->Nz; }
    o->z[p] = iz + (double)fz;
    o->x[p] = (double)(float)o->x[p];
    o->y[p] = (double)(float)o->y[p];
    o->ux[p] = (double)(float)o->ux[p];
    o->uy[p] = (double)(float)o->uy[p];
    o->uz[p] = (double)(float)o->uz[p];
    o->w[p] = (double)(float)o->w[p];
  }
  cplx *arrs[6] = {o->E[0], o->E[1], o->E[2], o->Bn[0], o->Bn[1], o->Bn[2]};
  for (int a = 0; a < 6; ++a)
    for (size_t k = 0; k < o->nf; ++k)
      arrs[a][k] = (double)(float)creal(arrs[a][k]) + I * (double)(float)cimag(arrs[a][k]);
}

/* ------------------------------------------------------------------------ */
/* Sort key of the particle order used by the GPU path's cell sort: tiles of
 * Tz x Tr cells, tiles ordered z-fastest, cells inside a tile z-fastest, and
 * equal cells ordered by particle id.  Writes, for each particle, the cell
 * order number ord and returns nothing; the test sorts (ord, id).           */
void orc_cell_order(orc *o, int Tz, int Tr, int64_t *ord) {
  int ntz = (o->Nz + Tz - 1) / Tz;
  for (long p = 0; p < o->np; ++p) {
    int iz = (int)floor(o->z[p]);
    double r2 = fma(o->x[p], o->x[p], o->y[p] * o->y[p]);
    int ir = radial_index(r2, sqrt(r2));
    int64_t tile = (int64_t)(ir / Tr) * ntz + iz / Tz;
    int64_t local = (int64_t)(ir % Tr) * Tz + iz % Tz;
    ord[p] = tile * (int64_t)(Tz * Tr) + local;
  }
}
