/*
 * pic.h -- C ABI of the MI355X (gfx950) quasi-3D r-z particle-in-cell step
 * with the "dual" finite-difference Maxwell solver (Miller et al., arXiv
 * 2303.12874).
 *
 * The library advances a laser-plasma simulation in the azimuthal-mode
 * ("quasi-3D") geometry of Sec. III.B: every field is Re sum_{m=0..M}
 * F^m(r,z) e^{i m phi}.  One step is
 *   cell sort (every K steps) -> gather of E^n and of the time-averaged
 *   B^n = (B^{n-1/2} + B^{n+1/2})/2 (Eq. (12)) -> relativistic Boris push
 *   (Eq. (6)) with per-mode work on tracked electrons (Eq. (16)) ->
 *   charge-conserving deposit into the mode arrays -> dual-solver update of
 *   E and B with distinct z-difference operators D_E, D_B (Eq. (9)) whose
 *   coefficients satisfy the dispersion condition Eq. (11) and the
 *   Lorentz-force condition Eq. (15).
 * Around the step: FP64 diagnostics (per-mode work Eq. (16), work by field
 * direction and the Pukhov-corrected estimate Eqs. (17), (20)-(21), field
 * and kinetic energy, beam divergence), checkpoint and restore, a measuring
 * autotuner of the sort tile and interval, and, independent of any
 * context, the ensemble integrator of the reduced model of Sec. II (Eq. (8)).
 *
 * Units: c = omega_0 = 1 (omega_0 the laser frequency), lengths in c/omega_0
 * (the laser wavelength is 2 pi), time in 1/omega_0, fields in
 * m c omega_0 / e, densities in units of the critical density.  Electrons
 * (q/m = -1) move over immobile ions.  The box is periodic in z, has the axis
 * at r = 0 and a perfectly conducting wall at r = Nr dr; electrons are
 * reflected at r = (Nr - 1) dr.
 *
 * Memory and streams belong to the caller: device memory is one workspace
 * buffer the caller allocates, the stream is the caller's hipStream_t.  The
 * library never frees caller memory.  No C++ exception crosses this ABI;
 * every call returns PIC_OK (0) or a negative PIC_E_* code, and
 * pic_last_error() (thread local) describes the last failure.
 *
 * Threads: calls on different contexts may run on different threads at once
 * (the state the library shares between contexts -- the registry of live
 * contexts and the memo of fitted Courant limits -- is locked, and its
 * per-launch caches are thread local); calls on one context must not overlap.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define PIC_OK 0
#define PIC_E_INVALID (-1) /* a descriptor or argument is out of range          */
#define PIC_E_CFL (-2)     /* requested dt above the solver's Courant limit      */
#define PIC_E_NOMEM (-3)   /* workspace or caller buffer too small               */
#define PIC_E_STATE (-4)   /* NULL or destroyed context, wrong call order        */
#define PIC_E_DEVICE (-5)  /* a HIP call failed (message in pic_last_error)      */
#define PIC_E_NUMERIC (-6) /* a reduction met NaN or Inf                         */

/* ---- options ------------------------------------------------------------ */
#define PIC_PREC_FP64 64 /* fields, particles, currents in FP64                   */
#define PIC_PREC_FP32 32 /* FP32 fields/particles, z as int32 cell + FP32 offset;
                            FP64 only in setup, reductions and tracked work   */
#define PIC_SOLVER_DUAL 0 /* N-coefficient operators fitted to Eqs. (11), (15)  */
#define PIC_SOLVER_YEE 1  /* the two-point (one-coefficient) Yee operator      */
/* How the deposited current is made to conserve charge with D_B (Sec. III.A:
 * the solver conserves charge, with Gauss's law written with [k]_B,
 * Eq. (10)).  D_B is the two-point difference after a symmetric z filter P
 * with taps p_l = sum_{l' > |l|} C^B_{l'}.                                   */
#define PIC_CURRENT_FILTER 0   /* P on J_r and J_phi, J_z as deposited: keeps
                                  div_B E - P rho constant (default)          */
#define PIC_CURRENT_EXACT_JZ 1 /* P^{-1} on J_z, J_r and J_phi as deposited:
                                  keeps div_B E - rho constant; P^{-1} is
                                  applied as the symmetric stencil of
                                  pic_jz_inverse_taps                          */
#define PIC_MAX_JZ_TAPS 128    /* one-sided taps of that stencil, at most     */

/* ---- field components for pic_fields ------------------------------------ */
#define PIC_ER 0   /* E_r   at (z_i,       r_{j+1/2}), time n                  */
#define PIC_EPHI 1 /* E_phi at (z_i,       r_j)                                */
#define PIC_EZ 2   /* E_z   at (z_{i+1/2}, r_j)                                */
#define PIC_BR 3   /* B_r   at (z_{i+1/2}, r_j),       time average at n       */
#define PIC_BPHI 4 /* B_phi at (z_{i+1/2}, r_{j+1/2})                          */
#define PIC_BZ 5   /* B_z   at (z_i,       r_{j+1/2})                          */
#define PIC_JR 6   /* J_r   of the last step, as deposited (before the z filter) */
#define PIC_JPHI 7 /* J_phi                                                   */
#define PIC_JZ 8   /* J_z                                                     */
#define PIC_RHO 9  /* charge density of the electrons at their positions      */
#define PIC_BR_OLD 10  /* B_r   at time n - 1/2 (staggered storage)           */
#define PIC_BPHI_OLD 11
#define PIC_BZ_OLD 12
#define PIC_BR_NEW 13  /* B_r   at time n + 1/2                               */
#define PIC_BPHI_NEW 14
#define PIC_BZ_NEW 15

#define PIC_MAX_PULSES 2
#define PIC_MAX_MODES 3  /* M <= 3 */
#define PIC_MAX_COEF 32

/* One laser pulse of Eq. (18), linearly polarised along x, placed in the
 * m = 1 arrays at t = 0: E_x = A sin(theta), E_z = (2x/w0^2) A cos(theta),
 * B_y = E_x, B_z = (2y/w0^2) A cos(theta), theta = -(z - zc),
 * A = a0 exp(-2 ln2 (z - zc)^2 / tau^2) exp(-r^2/w0^2) times a sin^2 taper
 * over the outer `taper` length at both ends of the periodic box.          */
typedef struct pic_pulse {
  double a0;  /* peak normalised amplitude                                   */
  double w0;  /* spot size (1/e field radius)                                */
  double tau; /* intensity FWHM, as a length (c = 1)                         */
  double zc;  /* centroid z                                                  */
} pic_pulse;

/* One simulation ("run").  Several runs may be passed to one pic_init; they
 * advance together in one launch per phase (all must share M and precision). */
typedef struct pic_run_desc {
  int32_t Nz;       /* cells along z (periodic), >= 8                         */
  int32_t Nr;       /* cells along r, >= 4; wall at r = Nr dr                 */
  int32_t M;        /* highest azimuthal mode, 0..PIC_MAX_MODES               */
  int32_t ppc;      /* electrons per cell, >= 1 (loaded for r < (Nr-1) dr)    */
  double dz, dr;    /* cell sizes                                             */
  double n0;        /* electron density (units of n_c)                        */
  double ramp_start, ramp_len; /* linear up-ramp of the density along z,
                                  0 at ramp_start to n0 at ramp_start +
                                  ramp_len (ramp_len = 0: none)               */
  double down_start, down_len; /* linear down-ramp, n0 at down_start to 0 at
                                  down_start + down_len (down_len = 0: none);
                                  the profile of App. A is up-ramp, plateau,
                                  down-ramp                                   */
  int32_t n_pulses; /* 0..PIC_MAX_PULSES                                      */
  pic_pulse pulse[PIC_MAX_PULSES];
  double taper;     /* laser taper length at the box ends (0: none)           */
  uint64_t seed;    /* counter-based SplitMix64 seed of the loading           */
  int32_t n_tracked;/* electrons whose work is accumulated (FP64), per mode
                       and by field direction                                 */
  int64_t n_steps;  /* steps this run takes in total (0: no limit); pic_step
                       leaves a run alone once it has taken them, so runs of
                       one context can end at different times                 */
} pic_run_desc;

typedef struct pic_opts {
  int32_t precision;    /* PIC_PREC_FP64 or PIC_PREC_FP32                     */
  int32_t solver;       /* PIC_SOLVER_DUAL or PIC_SOLVER_YEE                  */
  int32_t n_coef;       /* coefficients per dual operator (1..PIC_MAX_COEF); 16 */
  double fit_band;      /* k dz fit band upper edge; 0 means 2 pi / 3         */
  double cfl_fraction;  /* dt = fraction * Courant limit when dt == 0; 0 -> 0.95 */
  double dt;            /* > 0: use this dt (PIC_E_CFL if above the limit)    */
  const double *coef_E; /* optional n_coef values of C^E (else fitted)        */
  const double *coef_B; /* optional n_coef values of C^B (else fitted)        */
  int32_t sort_interval;/* steps between cell sorts; 0 -> default              */
  int32_t tile_z, tile_r; /* sort tile in cells; 0 -> default                 */
  int32_t use_graph;    /* 1: capture each distinct step (the launches of all
                           runs) once as a hipGraph and replay it             */
  int32_t current;      /* PIC_CURRENT_FILTER (0) or PIC_CURRENT_EXACT_JZ    */
  /* Per-run set-up, for a context of runs on different cells (a resolution
   * scan): arrays over the runs in their order, caller owned, read during
   * pic_init only; NULL leaves each run to the shared dt / coef_E / coef_B
   * above.  run_dt[i] > 0 is run i's dt (PIC_E_CFL above its limit);
   * run_coef_E, run_coef_B (both or neither) hold n_coef values per run,
   * run i's at [i * n_coef].                                                 */
  const double *run_dt;
  const double *run_coef_E;
  const double *run_coef_B;
  /* 1 (PIC_PREC_FP64 only): bitwise reproducible steps.  The deposit's sums,
   * whose order the atomics choose, are taken exactly in integers: each
   * contribution v (|v| <= 4 |q|, q the largest electron charge of the run)
   * is scaled by a power of two 2^K with 4 |q| 2^K <= 2^30 and split into
   * a = rint(v 2^K) and b = rint((v 2^K - a) 2^31), both summed with 64-bit
   * integer atomics, and each node's current is a 2^-K + b 2^-(K+31) in
   * FP64 (quantisation below 2^-62 of the largest contribution).  Results
   * are then the same whatever the order of the atomics, the sort tile and
   * interval, and with or without captured graphs; the deposit costs more
   * (about twice the LDS and more arithmetic).  PIC_E_INVALID in FP32.      */
  int32_t deterministic;
  /* Moving window (App. A: the box follows the pulse through a plasma longer
   * than the box).  window_interval K > 0: before a step whose count of
   * steps taken n is a positive multiple of K, every run's box advances by
   * s = floor(v n dt / dz) - S whole cells (v = window_speed c, 0 -> c; S
   * the cells moved so far, box column i is absolute column i + S): E^n,
   * B^{n-1/2}, B^{n+1/2} move back s columns with zeros entering at the
   * front, the window_guard columns at the back are cleared, electrons move
   * back s cells and those outside the box are dropped, and the plasma of
   * the s new absolute columns is loaded as pic_init loads the run's plasma
   * (same draws, ids pid = (a (Nr-1) + ir) ppc + k, density profile at the
   * absolute position; none tracked).  An electron leaving the box through
   * either end keeps its position outside the box and zero weight until the
   * next move drops it.  The electron count then varies
   * (pic_run_info.n_particles); the arrays hold the initial count plus four
   * moves' worth of fresh columns and 1 %, and a move beyond that fails with
   * PIC_E_NOMEM.  Not with use_graph, deterministic or pic_checkpoint
   * (PIC_E_INVALID).  0: the static z-periodic box.                         */
  int32_t window_interval;
  int32_t window_guard;
  double window_speed;
  /* Particle shape order of the gather and the deposit (the order the paper
   * leaves open, Sec. III): 0 or 1 linear (cloud in cell: 2 x 2 nodes), 2
   * quadratic B-splines (3 x 3 nodes round the nearest node; the
   * charge-conserving deposit on the 4 x 4 nodes holding both positions'
   * supports, with the continuity of the dual D_B kept exact).  A stencil
   * row below the axis, r_{-1} (or r_{-1/2}), is the row r_1 (or r_{1/2})
   * seen from the other side: the gather reads it as that row times the
   * component's mirror sign per mode ((-1)^m for z components and the
   * charge, (-1)^(m+1) for r and phi components) and the deposit folds onto
   * it with the same signs (the phi closure current, whose factor r changes
   * sign with the row, with (-1)^m; the m = 0 phi current with -1).         */
  int32_t shape;
} pic_opts;

typedef struct pic_ctx pic_ctx;

/* Per-run facts after pic_init.                                             */
typedef struct pic_run_info {
  double dt;             /* time step in use                                 */
  double courant_limit;  /* largest stable c dt / dz for these coefficients  */
  int64_t n_particles;   /* electrons in the run (varies with a moving window) */
  int64_t steps_done;    /* steps taken (those of a restored checkpoint
                            included)                                        */
  int32_t n_coef;        /* coefficients per operator                        */
  int32_t n_tracked;
  int32_t tile_z;        /* sort tile in use (cells along z and r)           */
  int32_t tile_r;
  int64_t window_cells;  /* moving window: cells moved (box column i is
                            absolute column i + window_cells); else 0        */
} pic_run_info;

/* ---- host-only setup (no GPU needed) ----------------------------------- */

/* Solver coefficients and time step (Sec. III.A).  The dual operators are
 * fitted by constrained least squares on k dz in (0, fit_band] to
 * [k]_E = tan(k dt/2)/(dt/2) and [k]_B = sin(k dt)/dt, which together are
 * Eqs. (11) and (15); the Courant limit combines max_k [k]_B[k]_E with the
 * largest radial eigenvalue of modes 0..M, and dt = cfl_fraction * limit
 * (coefficients refitted at that dt).  coef_E, coef_B: n_coef doubles each
 * (caller owned).  Returns PIC_E_INVALID on bad sizes.                      */
int pic_solver_setup(int32_t solver, int32_t n_coef, int32_t M, double dz, double dr,
                     double cfl_fraction, double fit_band, double *dt, double *courant_limit,
                     double *coef_E, double *coef_B);

/* Courant limit (largest stable c dt / dz) of given coefficients.           */
int pic_courant_limit(int32_t n_coef, const double *coef_E, const double *coef_B, int32_t M,
                      double dz, double dr, double *courant_limit);

/* The inverse of the z filter P of coef_B (n_coef values) as a symmetric
 * stencil: taps[l] = h_l = h_{-l}, l = 0..*n_taps-1, with
 * sum_l h_l p_{k-l} = delta_k on the infinite line.  h is the Fourier
 * series of 1/P(k), P(k) = sum_l p_l cos(l k dz), summed in the host's
 * extended precision over 8192 samples of P and rounded to FP64, and cut
 * after the last tap above 2^-53 (precision
 * PIC_PREC_FP64) or 2^-24 (PIC_PREC_FP32) times h_0: the taps decay
 * geometrically, so the cut changes P^{-1} by about that fraction, and on a
 * periodic line of any length the stencil (wrapped) is P^{-1} to that
 * accuracy.  taps: PIC_MAX_JZ_TAPS doubles, caller owned.  PIC_E_INVALID if
 * P(k) <= 0 for some k (P has no inverse; some fits with many coefficients
 * do this near k dz = pi) or if more than PIC_MAX_JZ_TAPS taps are needed.  */
int pic_jz_inverse_taps(int32_t n_coef, const double *coef_B, int32_t precision, double *taps,
                        int32_t *n_taps);

/* The electrons pic_init loads for `run`, on the host, in FP64: positions in
 * cell units (z in dz, x and y in dr), weights w (charge -w), ids.  Arrays of
 * length n = Nz (Nr - 1) ppc, caller owned; *n_out receives n (call with
 * NULL arrays to query).  tracked_ids (n_tracked, ascending) may be NULL.   */
int pic_load_host(const pic_run_desc *run, double *z, double *x, double *y, double *w,
                  int64_t *id, int64_t *tracked_ids, int64_t *n_out);

/* ---- device life cycle --------------------------------------------------- */

/* Set up and upload n_runs runs: the problem of Sec. II and App. A (a laser
 * driving a wake in an under-dense plasma) in the quasi-3D representation of
 * Sec. III.B.  Per run:
 *   - the dual operators' coefficients C^E, C^B fitted to Eqs. (11) and (15)
 *     (Sec. III.A), and dt at cfl_fraction of the Courant limit they and the
 *     modes 0..M allow (or the caller's dt / coefficients);
 *   - cold electrons over immobile ions with the density profile of App. A
 *     (up-ramp, plateau, down-ramp), loaded on the host;
 *   - E^0 and B^0 of the pulses of Eq. (18) in the m = 1 arrays, and the
 *     half-step B^{-1/2}, B^{+1/2} of the staggering of Eq. (12);
 *   - the first cell sort.
 * Validate, set up and upload n_runs runs into device_workspace on
 * hip_stream.  With device_workspace == NULL only
 * *workspace_bytes is written (size query, no device call).  Otherwise
 * *workspace_bytes must be at least the queried size; the buffer must stay
 * allocated until pic_destroy.  *out receives the context.  Errors:
 * PIC_E_INVALID for a bad descriptor or option (with PIC_CURRENT_EXACT_JZ
 * also when a run's filter has no inverse stencil, see pic_jz_inverse_taps),
 * PIC_E_CFL for a dt above the Courant limit of the coefficients,
 * PIC_E_NOMEM for a short workspace, PIC_E_DEVICE for a failed HIP call.    */
int pic_init(const pic_run_desc *runs, int32_t n_runs, const pic_opts *opts,
             void *device_workspace, size_t *workspace_bytes, void *hip_stream, pic_ctx **out);

/* Enqueue n_steps time steps of every run on the context's stream
 * (asynchronous).  One step is the loop of Sec. III: gather of E^n and of
 * the time average (B^{n-1/2} + B^{n+1/2})/2 of Eq. (12) at each electron
 * from the modes F = Re sum_m F^m e^{i m phi} (Sec. III.B); the relativistic
 * push of Eq. (6) (Boris), with the per-mode work of Eq. (16) accumulated on
 * tracked electrons; the charge-conserving deposit of J^{n+1/2} into the
 * mode arrays; and the dual-solver update of Eq. (9), Ampere's law with D_B
 * and the current made to conserve charge with it (Gauss's law with [k]_B,
 * Eq. (10)), then Faraday's law with D_E.  A cell sort precedes every
 * sort_interval-th step.  Runs that have taken their n_steps are left
 * alone.  Errors found on the device (a cell sort that met inconsistent
 * data) are reported by the next synchronising call.                       */
int pic_step(pic_ctx *ctx, int64_t n_steps);

/* Synchronise the stream and copy out FP64 diagnostics of one run (any
 * pointer may be NULL): work[n_tracked][M+1] per-mode work -sum dt E^m . v
 * (Eq. (16)); gamma[n_tracked] from the momentum; gamma_acc[n_tracked] the
 * initial gamma plus the work summed over modes (FP64 accumulation);
 * ids[n_tracked] (ascending); field_energy[M+1]; kinetic[1] = sum w (gamma-1).
 * PIC_E_NUMERIC if a reduction is not finite.                               */
int pic_mode_work(pic_ctx *ctx, int32_t run, double *work, double *gamma, double *gamma_acc,
                  int64_t *ids, double *field_energy, double *kinetic);

/* Synchronise and copy out the work on the tracked electrons of one run split
 * by field direction (Sec. III.B), arrays of n_tracked FP64 values in the
 * order of pic_mode_work's ids, caller owned, any may be NULL:
 *   wz     = -sum dt E_z v_z,  wperp = -sum dt E_perp . v_perp, each field
 *            summed over modes (Eq. (17)), accumulated with the per-mode work;
 *   f      = -2 sqrt(2 gamma) / (omega_p w0^2), Eq. (20) with c = omega_0 = 1,
 *            omega_p = sqrt(n0), w0 of pulse 0 and gamma the electron's
 *            Lorentz factor now;
 *   w_lwfa = wz - f wperp,  w_dla = (1 + f) wperp (Eq. (21)).
 * PIC_E_INVALID if f, w_lwfa or w_dla is asked for and the run has no pulse
 * or n0 <= 0; PIC_E_NUMERIC if a value is not finite.                       */
int pic_cartesian_work(pic_ctx *ctx, int32_t run, double *wz, double *wperp, double *f, double *w_lwfa,
                       double *w_dla);

/* Synchronise and reduce the divergence of the energetic electrons of one
 * run, the quantity Secs. IV.A-IV.B compare between solvers: over electrons
 * with Lorentz factor >= gamma_min and u_z > 0, with theta_x = atan(u_x/u_z)
 * and theta_y = atan(u_y/u_z), out[6] (caller owned) receives
 *   out[0] = sum w,  out[1] = sum w theta_x^2,  out[2] = sum w theta_y^2,
 *   out[3] = number of electrons counted,
 *   out[4] = sqrt(out[1] / out[0]), out[5] = sqrt(out[2] / out[0]): the
 *            charge-weighted RMS angles (0 when no electron is counted),
 * FP64 sums.  The selection compares |u|^2 with gamma_min^2 - 1.
 * PIC_E_INVALID if gamma_min < 1 or out is NULL; PIC_E_NUMERIC if a sum is
 * not finite.                                                              */
int pic_divergence(pic_ctx *ctx, int32_t run, double gamma_min, double *out);

/* ---- checkpoint and restore ------------------------------------------------ */

/* Synchronise and copy the whole state of the context (every run: fields,
 * currents, electrons in their current order, the tile ranges of the last
 * sort, tracked work, step counts) into host_buf, caller owned.  With
 * host_buf NULL only *bytes is written (size query).  PIC_E_NOMEM if *bytes
 * is short.                                                                 */
int pic_checkpoint(pic_ctx *ctx, void *host_buf, size_t *bytes);

/* Load a checkpoint into a context created by pic_init with the same runs and
 * options (checked: format version, run descriptors, precision, sort tile
 * and interval, current correction, deterministic mode, solver
 * coefficients); stepping then
 * continues where the checkpointed
 * context was.  PIC_E_INVALID if the checkpoint does not belong to such a
 * context; nothing is changed then.                                         */
int pic_restore(pic_ctx *ctx, const void *host_buf, size_t bytes);

/* ---- reduced model of Sec. II (independent of any context) -------------- */

/* Parameters of Eq. (8), units c = omega_p = 1 (time 1/omega_p, length
 * c/omega_p).  The laser mode has wavenumber kz and phase velocity vphi >= 1
 * (frequency kz vphi, transverse wavenumber kz (vphi^2 - 1)^(1/2)); the
 * bubble is spherical and moves at c.                                       */
typedef struct pic_dla_model {
  double a0;   /* normalised vector potential of the laser                   */
  double kz;   /* longitudinal wavenumber, > 0                               */
  double vphi; /* phase velocity, >= 1                                       */
  double cB;   /* factor on the laser's magnetic terms: 1 for the exact
                  fields, cos(omega_0 dt / 2) for the time-staggering error of
                  a Yee-type PIC step (Sec. IV.A)                             */
  double wake; /* factor on the bubble terms: 1 for the model, 0 laser only  */
} pic_dla_model;

/* Integrate n electrons of the model (Sec. II, Eq. (8)) with the fifth-order
 * Dormand-Prince solution at a fixed step (App. A names only an explicit
 * fifth-order Runge-Kutta method): electron i goes from its injection time
 * t0[i] to t_end in ceil((t_end - t0[i]) / h) equal steps (none if t0[i] >=
 * t_end).  Device arrays of n FP64 values, caller owned, updated in place:
 * x, zeta = z - t, xd = dx/dt, zetad = dzeta/dt (so v_z = zetad + 1; the
 * state must have speed < 1).  Asynchronous on hip_stream; an electron driven
 * to a non-physical state, or asked for more than 2^24 steps, ends as NaN.
 * PIC_E_INVALID on NULL arrays with n > 0, n < 0, h <= 0, a non-finite
 * t_end or an out-of-range model.                                          */
int pic_dla_integrate(const pic_dla_model *model, int64_t n, const double *t0, double *x, double *zeta, double *xd,
                      double *zetad, double t_end, double h, void *hip_stream);

/* Synchronise and copy one component of mode m of one run into out: the
 * amplitude F^m(r, z) of F = Re sum_m F^m e^{i m phi} (Sec. III.B), the
 * per-mode fields whose work Eq. (16) separates (m = 0 the wake, m = 1 the
 * laser), at the staggered places listed with PIC_ER..PIC_BZ_NEW.  FP64 interleaved complex
 * [(Nr+1)][Nz] (2 (Nr+1) Nz doubles; m = 0 has zero imaginary part),
 * physical units, FP64 also for FP32 runs.  PIC_E_NOMEM if out_len (in
 * doubles) is short; PIC_E_STATE if a cell sort met inconsistent data.      */
int pic_fields(pic_ctx *ctx, int32_t run, int32_t comp, int32_t m, double *out, size_t out_len);

/* Synchronise and copy the electrons of one run in device order (FP64, cell
 * units: z = cell + offset for FP32 runs).  Any pointer may be NULL; arrays
 * hold n_particles values (out_len checked).                                */
int pic_particles(pic_ctx *ctx, int32_t run, double *z, double *x, double *y, double *ux,
                  double *uy, double *uz, double *w, int64_t *id, size_t out_len);

/* Coefficients in use: coef_E, coef_B (n_coef each) and the z-filter taps
 * (2 n_coef - 1) applied to J_r and J_phi; any may be NULL.                 */
int pic_coefficients(pic_ctx *ctx, int32_t run, double *coef_E, double *coef_B, double *taps);

int pic_run_info_get(pic_ctx *ctx, int32_t run, pic_run_info *info);

/* ---- per-phase timing -------------------------------------------------- */
#define PIC_PHASE_SORT 0   /* cell sort of the electrons                       */
#define PIC_PHASE_PUSH 1   /* gather + push + deposit                          */
#define PIC_PHASE_EFIELD 2 /* E update (with the z filter of J)                */
#define PIC_PHASE_BFIELD 3 /* B update                                         */
#define PIC_PHASE_STEP 4   /* a whole step replayed from a captured graph      */
#define PIC_NPHASES 5

/* enable != 0: from now on pic_step brackets every phase launch with HIP
 * events on the context's stream (the counters restart at zero); 0: stop.   */
int pic_profile(pic_ctx *ctx, int32_t enable);

/* Synchronise and return, per phase, the summed event time in ms and the
 * number of launches timed since pic_profile(ctx, 1).                       */
int pic_profile_read(pic_ctx *ctx, double *ms, int64_t *launches);

/* ---- autotuner ---------------------------------------------------------- */
#define PIC_MAX_TUNE 16

typedef struct pic_tune_report {
  int32_t n;                          /* tiles tried                          */
  int32_t tile_z[PIC_MAX_TUNE], tile_r[PIC_MAX_TUNE];
  int32_t interval[PIC_MAX_TUNE];     /* best sort interval for that tile     */
  double ms_per_step[PIC_MAX_TUNE];   /* measured cost per step at it         */
  int32_t best;                       /* index of the choice written to opts  */
} pic_tune_report;

/* Pick the sort tile and the sort interval K for these runs and options by
 * measurement (neither changes the physics, only the summation order of the
 * deposit).  For every candidate tile whose push workgroup fits the LDS
 * (the tile in opts, if set, is the only candidate) a trial context is built
 * in device_workspace on hip_stream; after trial_steps untimed steps and a
 * timed sort, trial_steps steps (4..64) are timed one by one with HIP
 * events, t_k at k steps after the sort, and K = argmin (t_sort +
 * sum_{k<K} t_k) / K.  The fastest (tile, K) is written to opts->tile_z,
 * tile_r, sort_interval; the trial contexts are destroyed.  With
 * device_workspace NULL only the bytes needed (the largest trial context)
 * are written to *workspace_bytes.  report may be NULL.  Times are those of
 * the early plasma of the trial, which the caller should keep in mind for
 * long runs.                                                                */
int pic_autotune(const pic_run_desc *runs, int32_t n_runs, pic_opts *opts, void *device_workspace,
                 size_t *workspace_bytes, void *hip_stream, int32_t trial_steps, pic_tune_report *report);

/* ---- allocation-free variant ---------------------------------------------- */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the reduction of
 * pic_divergence over n electrons in caller-owned device arrays, with no
 * context and no workspace.  ux, uy, uz (momentum per mass, units of c) and w
 * (macro-particle charge weight) hold n values each, FP64 (precision
 * PIC_PREC_FP64) or FP32 (PIC_PREC_FP32); out[6] (host, caller owned)
 * receives what pic_divergence's out does, over the electrons with Lorentz
 * factor >= gamma_min and u_z > 0.  The per-block partial sums live in a
 * fixed device array of 2048 x 4 doubles (64 KiB) that the library holds on
 * each GPU it runs on until the process ends: the call allocates nothing,
 * enqueues one kernel and one copy on hip_stream and synchronises it.  One
 * call takes at most 2048 x 256 x 64 = 33554432 electrons (PIC_E_NOMEM above
 * that, before any device work).  Calls that overlap on one GPU share that
 * array and race.  PIC_E_INVALID on a bad precision, NULL arrays with n > 0,
 * n < 0 or gamma_min < 1; PIC_E_NUMERIC if a sum is not finite.            */
int pic_divergence_arrays(int32_t precision, int64_t n, const void *ux, const void *uy, const void *uz,
                          const void *w, double gamma_min, double *out, void *hip_stream);

/* Free host objects of the context (not the workspace).                     */
int pic_destroy(pic_ctx *ctx);

/* Description of the last failure on this thread ("" if none).             */
const char *pic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
