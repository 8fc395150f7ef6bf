// pic_internal.h -- declarations shared by the host runtime (capi.cpp,
// setup.cpp) and the HIP kernels (kernels.hip).  Not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/pic.h"

namespace pic {

constexpr int kFitSamples = 4000;     // midpoint samples of the coefficient fit
constexpr int kKappaSamples = 20001;  // samples of k dz in [0, pi] for the Courant limit
constexpr uint32_t kTrackedBit = 0x80000000u;  // particle id flag: work is accumulated
constexpr uint32_t kIdMask = 0x7fffffffu;

// ---- host setup (setup.cpp) -------------------------------------------------
void fit_dual(int N, double nu, double band, double *CE, double *CB);
void z_product_range(const double *CE, const double *CB, int N, double *pmax, double *pmin);
double radial_lambda(int m, int nr);
double radial_lambda_max(int M);
bool stable_at(const double *CE, const double *CB, int N, int M, double dz, double dr, double nu);
double courant_limit_of(const double *CE, const double *CB, int N, int M, double dz, double dr);
// taps h_0..h_{nh-1} of the inverse of the z filter of CB, cut below eps h_0;
// 0, or 1 if P(k) <= 0 somewhere, or 2 if more than max_taps are needed
int jz_inverse_taps(const double *CB, int N, double eps, int max_taps, double *h, int *nh);
double courant_limit_fitted(int solver, int N, int M, double dz, double dr, double band);
int64_t run_particle_count(const pic_run_desc &r);
// moving window: the plasma of absolute columns [a0, a1), z in a box whose
// column 0 is absolute column S, (a1 - a0) (Nr-1) ppc electrons in pid order
void load_columns(const pic_run_desc &r, int64_t a0, int64_t a1, int64_t S, double *z, double *x, double *y,
                  double *w, int64_t *id);
void load_electrons(const pic_run_desc &r, double *z, double *x, double *y, double *w, int64_t *id,
                    int64_t *tracked);
void laser_fields(const pic_run_desc &r, double *E, double *B);

// ---- integrity of the cell sort ----------------------------------------------
// The sort kernels raise these bits in the run's flag word (device memory,
// zeroed by pic_init) where data would otherwise send them out of range, and
// skip that access; the calls that synchronise report a raised bit as
// PIC_E_STATE.  A raised bit means electrons were lost or duplicated.
constexpr uint32_t kSortBadCount = 1u;   // the cell counts do not sum to the electrons
constexpr uint32_t kSortBadTile = 2u;    // a tile's electron range is not inside [0, np]
constexpr uint32_t kSortBadSlot = 4u;    // a ranked entry's slot is outside [0, np)
constexpr uint32_t kSortBadSource = 8u;  // an entry names an electron outside [0, np)
// (constexpr functions are host and device functions alike)
// (a sort that drops electrons, a window move, keeps at most np)
constexpr uint32_t sort_count_flags(long long total, long long np, bool drops = false) {
  return (drops ? total > np || total < 0 : total != np) ? kSortBadCount : 0u;
}
constexpr uint32_t sort_tile_flags(long long beg, long long end, long long np) {
  return (beg < 0 || end < beg || end > np) ? kSortBadTile : 0u;
}
constexpr uint32_t sort_index_flags(long long i, long long np, uint32_t bit) { return (i < 0 || i >= np) ? bit : 0u; }
// message for raised bits (host): writes at most n bytes, returns the bits
uint32_t sort_flags_text(uint32_t flags, int run, char *buf, size_t n);

// ---- device view of one run ---------------------------------------------------
// Field storage: component-major planes of (Nr+1) x Nz reals, z fastest; a
// component holds NM = 2M+1 planes: q = 0 is Re(m=0), q = 2m-1 / 2m are Re / Im
// of mode m >= 1.  A quantity at z_{i+1/2} is stored at column i, one at
// r_{j+1/2} at row j.  J planes hold the raw deposit (charge moved per step);
// the physical current is raw times a per-row factor (see kernels.hip).
struct KRun {
  int Nz, Nr, M, N;       // grid, modes, coefficients per operator
  double dz, dr, dt;
  long long np;           // electrons
  long long plane;        // (Nr+1) * Nz
  void *E;                // 3 * NM planes
  void *B[2];             // B at alternate half steps: B[n%2] = B^{n-1/2}, B[1-n%2] = B^{n+1/2}
  void *Bbar;             // (B^{n-1/2} + B^{n+1/2})/2, written by the B update
  void *J[2];             // deposit target of step n is J[n%2]; the other is kept zeroed
  void *rho;              // NM planes (diagnostic)
  void *pz;               // FP64: double z (cells);  FP32: int iz
  void *pfz;              // FP32: float fz in [0, 1)
  void *px, *py, *pux, *puy, *puz, *pw;
  uint32_t *pid;          // particle id | kTrackedBit
  double *W;              // [n_tracked][M+1] per-mode work (FP64)
  double *Wc;             // [n_tracked][2] work of E_z and of E_perp (FP64)
  const int32_t *tracked; // tracked ids, ascending
  int n_tracked;
  const void *CE, *CB, *P;  // coefficient arrays (real type of the run), P has 2N-1 taps
  const void *H;            // taps h_0..h_{NH-1} of P^{-1} (exact J_z correction)
  int NH;                   // 0: the current is filtered by P instead
  // sort scratch
  void *sz, *sfz, *sx, *sy, *sux, *suy, *suz, *sw;  // second particle buffer
  uint32_t *spid;
  int32_t *cell_count;    // n_keys + 1
  int32_t *cell_start;    // n_keys + 1
  uint64_t *perm;         // np sort entries: id << 32 | source index
  int32_t *scan_tmp;      // scan block sums
  int Tz, Tr;             // sort tile (cells)
  int ntz, ntr;           // tiles along z and r
  long long n_keys;       // tiles * Tz * Tr
  double *red;            // reduction partials
  int32_t *work;          // the persistent push's 8 tile ticket counters, one per XCD (run 0's serve a batch)
  uint32_t *flags;        // cell-sort integrity bits (kSort*), sticky
  // deterministic mode: the deposit's integer sums, pairs (a, b) per value
  // of the J layout (interleaved), zero between steps, and the scale 2^K
  unsigned long long *Jfix;
  double qscale;
  // moving window: positions are kept unwrapped in z and an electron that
  // leaves the box gets zero weight (window); at a window move the sort
  // shifts every electron back `shift` cells and drops those outside the box
  int window, shift;
  int shape;              // particle shape order: 1 linear, 2 quadratic (every run of a batch alike)
};

// ---- push workgroup LDS ---------------------------------------------------------
// One push workgroup per sort tile of Tz x Tr cells.  Its LDS holds
//  * the tile's current window, FP64 for both precisions, 3 components x NM
//    planes x (Tz+1+2 sh) x (Tr+1+2 sh) nodes from node (z0-sh, r0-sh), sh
//    the shape order (1 linear, 2 quadratic): every move of less than a cell
//    from a cell of the tile deposits inside it (linear: the 3 x 3 nodes
//    round both cells; quadratic: the 4 x 4 nodes round both nearest nodes);
//  * the field window of E and Bbar, one record per node for
//    (Tz+2+2 kFieldMarginZ+sh-1) x (Tr+2+2 kFieldMarginR+sh-1) nodes from
//    column z0-1-kFieldMarginZ and row r0-1-kFieldMarginR (the gather stencil
//    of every electron within the margins of the tile: linear 2 x 2 nodes,
//    quadratic 3 x 3 round the nearest node), 6 components of 2 (M+1) reals
//    each (Re and Im of every mode, Im of m = 0 held as zero), padded so that
//    a component is read with 16-byte (or 8-byte) vector loads.  For the
//    quadratic shape a row below the axis holds the mirror image of the row
//    above (each mode times its mirror sign), so that the gather needs no
//    axis rule.
constexpr int kFieldMarginZ = 1;  // columns for electrons that drifted since the sort
constexpr int kFieldMarginR = 0;
constexpr size_t kPushLdsDefault = 81920;  // default tile choice: two workgroups per CU
constexpr size_t kPushLdsMax = 163840;     // gfx950 LDS per workgroup

// LDS banks as measured on gfx950: an access of 4 bytes per lane costs the
// largest number of lanes that fall on one of 32 four-byte banks, one of 8
// bytes the same with 32 eight-byte banks; lanes on one address share it.
// The current window is row-padded: the wavefront's lanes work on
// consecutive cells of the tile (z fastest, then the next row), and a row
// stride congruent to Tz nodes modulo 256 bytes keeps those lanes on distinct
// banks when a wavefront spans two rows.
constexpr int kBankBytes = 256;
constexpr int field_window_z(int Tz, int sh = 1) { return Tz + 2 + 2 * kFieldMarginZ + sh - 1; }
constexpr int field_window_r(int Tr, int sh = 1) { return Tr + 2 + 2 * kFieldMarginR + sh - 1; }
constexpr int current_window_z(int Tz, int sh = 1) { return Tz + 1 + 2 * sh; }
constexpr int current_window_r(int Tr, int sh = 1) { return Tr + 1 + 2 * sh; }
constexpr int pos_mod(int a, int m) { return ((a % m) + m) % m; }
// 8-byte words per current-window row: current_window_z nodes of 3 NM sums,
// plus the pad; a sum is one word (FP64), or two (the integer pair of the
// deterministic mode, det).  The tile current is summed in FP64 for both
// precisions: on gfx950 the LDS FP32 atomic add (ds_add_f32) costs about 20
// times the FP64 one (measured: 193 against 8.8 cycles per wavefront
// instruction without bank conflicts), and an FP32 tile current made the
// FP32 push of the 8192 x 512 run 6.8x slower.
constexpr int current_window_row(int M, int Tz, bool det = false, int sh = 1) {
  return (det ? 2 : 1) * 3 * (2 * M + 1) * current_window_z(Tz, sh) +
         pos_mod(-(1 + 2 * sh) * (det ? 2 : 1) * 3 * (2 * M + 1), kBankBytes / 8);
}
// Field-window records.  FP32 with 2 (M+1) a multiple of 4 (M odd): a
// component holds its 2 (M+1) reals (Re and Im of every mode, Im of m = 0 as
// zero) and is read with 16-byte vector loads; the record stride is an odd
// number of 16-byte vectors, so that lanes reading the same component of
// different nodes fall on distinct banks, also when the half-cell stencils
// of neighbouring lanes start one node apart (measured on the gather pattern
// of a 16 x 4 tile: 4.1 cycles per 8 bytes, against 6.0 for records of
// 4-byte planes).  Otherwise (FP64, or M even): a component holds its NM
// planes (no Im of m = 0), read one real at a time, and the record is
// 6 NM + 1 reals, odd (16-byte vectors measured slower there, and the larger
// records shrink the default tiles).
constexpr int field_vec_bytes(int M, int precision) {
  return (precision == PIC_PREC_FP32 && (2 * (M + 1)) % 4 == 0) ? 16 : 0;
}
constexpr int field_comp_reals(int M, int precision) {
  return field_vec_bytes(M, precision) ? 2 * (M + 1) : 2 * M + 1;
}
constexpr int field_node_reals(int M, int precision) {
  return field_vec_bytes(M, precision) ? (6 * (2 * (M + 1)) / 4 % 2 ? 6 * (2 * (M + 1)) : 6 * (2 * (M + 1)) + 4)
                                       : 6 * (2 * M + 1) + 1;
}
// reals per field-window row (record layout: a whole number of vectors;
// plane layout: padded so that the row stride is congruent to Tz records
// modulo 256 bytes, like the current window)
constexpr int field_window_row(int M, int Tz, int precision, int sh = 1) {
  return field_vec_bytes(M, precision)
             ? field_node_reals(M, precision) * field_window_z(Tz, sh)
             : field_node_reals(M, precision) * field_window_z(Tz, sh) +
                   pos_mod(-(field_window_z(Tz, sh) - Tz) * field_node_reals(M, precision),
                           kBankBytes / (precision == PIC_PREC_FP64 ? 8 : 4));
}
constexpr size_t current_window_words(int M, int Tz, int Tr, bool det = false, int sh = 1) {
  return (size_t)current_window_row(M, Tz, det, sh) * current_window_r(Tr, sh);
}
// 8-byte words before the field window (the current window, rounded up to 16 bytes)
constexpr size_t field_window_offset_words(int M, int Tz, int Tr, bool det = false, int sh = 1) {
  return (current_window_words(M, Tz, Tr, det, sh) + 1) / 2 * 2;
}
inline size_t push_lds_bytes(int M, int Tz, int Tr, int precision, bool det = false, int sh = 1) {
  const size_t w = precision == PIC_PREC_FP64 ? 8 : 4;
  return field_window_offset_words(M, Tz, Tr, det, sh) * 8 +
         (size_t)field_window_row(M, Tz, precision, sh) * field_window_r(Tr, sh) * w;
}

// ---- batched launches ---------------------------------------------------------
// The hot kernels take up to kMaxBatch runs at once (one launch per phase for
// all of them): a workgroup finds its run from its block index and the
// per-run first blocks in `off`, which the launcher fills.  Runs of one batch
// share precision, M, N and the sort tile, and step together (same parity).
constexpr int kMaxBatch = 8;
struct Batch {
  int n;                            // runs in the batch
  int par;                          // step parity: deposit into J[par], B^{n+1/2} in B[par ^ 1]
  int det;                          // deterministic mode (integer deposit sums, FP64 only)
  int deal_xcd;                     // push: tiles dealt per XCD (set by the launcher), else in one order
  long long off[kMaxBatch + 1];     // first block of each run in the launch (set by the launcher)
  KRun run[kMaxBatch];
  // B update operands per run: Bout = Bin - tau curl_E E, and avg = (Bin + Bout)/2 when not NULL
  void *bout[kMaxBatch];
  const void *bin[kMaxBatch];
  void *avg[kMaxBatch];
  double tau[kMaxBatch];
};

// kernel arguments are at most 4 KB
static_assert(sizeof(Batch) <= 4096, "a Batch is passed by value as the kernel argument");

// the message pic_last_error returns (capi.cpp); returns code ("" clears it)
int set_error(int code, const char *fmt, ...);

// ---- kernel launchers (kernels.hip); all enqueue on `stream` -----------------
int launch_push(Batch &b, int prec, void *stream);
int launch_efield(Batch &b, int prec, void *stream);
int launch_bfield(Batch &b, int prec, void *stream);
int launch_sort(Batch &b, int prec, void *stream);  // swaps the runs' particle buffers in b
// moving window: E, B[0], B[1], Bbar of run k back by k.shift columns (zeros
// entering at the front), then the first `guard` columns cleared
int launch_window_shift(const KRun &k, int prec, int guard, void *stream);
int prepare_kernels(int prec, int M, int Tz, int Tr, bool det, int sh);  // per-kernel attributes, before any capture
int launch_fix_convert(Batch &b, void *stream);  // deterministic mode: integer sums -> J[par], sums cleared
int launch_zero(void *ptr, size_t bytes, void *stream);
int launch_rho(const KRun &k, int prec, void *stream);
int launch_energy(const KRun &k, int prec, int par, int nblocks_max, int *nblocks, void *stream);
int launch_kinetic(const KRun &k, int prec, int *nblocks, void *stream);
// 4 sums per block into k.red (nblocks <= nblocks_max, red holds 4 per block)
int launch_divergence(const KRun &k, int prec, double u2min, int nblocks_max, int *nblocks, void *stream);
int launch_tracked_gamma(const KRun &k, int prec, double *gamma, int64_t *ids, void *stream);
const char *last_device_error();
// record a failed HIP status (as int) with a label for pic_last_error; returns PIC_OK or PIC_E_DEVICE
int record_device_error(int hip_status, const char *what);
// reduced-model ensemble (dla.hip): n electrons in place on `stream`
int launch_dla(const pic_dla_model &m, long long n, const double *t0, double *x, double *zeta, double *xd,
               double *zetad, double t_end, double h, void *stream);

}  // namespace pic
