// capi.cpp -- the C ABI of include/pic.h: validation, workspace layout,
// set-up and upload of runs, the step loop and FP64 read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "pic_internal.h"

using namespace pic;

namespace {

thread_local char g_msg[512] = "";

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace

// the message of pic_last_error, for entry points outside this file
int pic::set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return code;
}

namespace {

int hip_ok(hipError_t e, const char *what) {
  if (e != hipSuccess) return fail(PIC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return PIC_OK;
}

#define TRY(expr)                 \
  do {                            \
    int _rc = (expr);             \
    if (_rc != PIC_OK) {          \
      if (_rc == PIC_E_DEVICE && g_msg[0] == 0) fail(_rc, "%s", last_device_error()); \
      return _rc;                 \
    }                             \
  } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr uint32_t kMagic = 0x51D3A1C7u;
constexpr size_t kAlign = 256;
constexpr int kRedBlocks = 1024;
constexpr int kDefaultSortInterval = 8;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct RunHost {
  pic_run_desc d;
  KRun k;
  int N = 1;
  double dt = 0, nu_lim = 0;
  std::vector<double> CE, CB, P;
  std::vector<double> H;  // taps of P^{-1} (exact J_z correction), else empty
  std::vector<double> gam0;
  int64_t steps = 0;
  int64_t win_S = 0;    // moving window: cells moved (box column i is absolute column i + win_S)
  int64_t cap = 0;      // particle slots of the run's arrays
  std::vector<int64_t> tr_ids;  // tracked ids, ascending
  size_t offset = 0, bytes = 0;
  double *dev_gamma = nullptr;  // scratch for pic_mode_work
  int64_t *dev_ids = nullptr;
};

// Layout of one run in the workspace (offsets from the run's base).
struct Layout {
  size_t E, B0, B1, Bbar, J0, J1, rho, pz, pfz, px, py, pux, puy, puz, pw, pid;
  size_t sz, sfz, sx, sy, sux, suy, suz, sw, spid, perm, ccount, cstart, scan;
  size_t W, Wc, tracked, CE, CB, P, H, red, gam, ids, work, Jfix, total;
};

// Particle slots of a run: its electrons, and with a moving window of
// interval K four moves' worth of fresh columns (a move crosses at most
// ceil(K v) + 1 columns, c dt < dz) and 1 %.
int64_t particle_capacity(const pic_run_desc &d, const pic_opts &o) {
  const int64_t np = run_particle_count(d);
  if (o.window_interval <= 0) return np;
  const double v = o.window_speed > 0 ? o.window_speed : 1.0;
  const int64_t cols = (int64_t)std::ceil(o.window_interval * v) + 1;
  return np + 4 * cols * (int64_t)(d.Nr - 1) * d.ppc + np / 100 + 1024;
}

Layout layout_of(const pic_run_desc &d, int prec, int N, int Tz, int Tr, long long n_keys, bool det, int64_t cap) {
  const size_t rs = prec == PIC_PREC_FP64 ? 8 : 4;
  const int NM = 2 * d.M + 1;  // mode planes per component
  const size_t plane = (size_t)(d.Nr + 1) * d.Nz;
  const size_t np = (size_t)cap;
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t vec = 3 * NM * plane * rs;
  L.E = take(vec);
  L.B0 = take(vec);
  L.B1 = take(vec);
  L.Bbar = take(vec);
  L.J0 = take(vec);
  L.J1 = take(vec);
  L.rho = take(NM * plane * 8);
  L.pz = take(np * (prec == PIC_PREC_FP64 ? 8 : 4));
  L.pfz = take(prec == PIC_PREC_FP64 ? 0 : np * 4);
  L.px = take(np * rs);
  L.py = take(np * rs);
  L.pux = take(np * rs);
  L.puy = take(np * rs);
  L.puz = take(np * rs);
  L.pw = take(np * rs);
  L.pid = take(np * 4);
  L.sz = take(np * (prec == PIC_PREC_FP64 ? 8 : 4));
  L.sfz = take(prec == PIC_PREC_FP64 ? 0 : np * 4);
  L.sx = take(np * rs);
  L.sy = take(np * rs);
  L.sux = take(np * rs);
  L.suy = take(np * rs);
  L.suz = take(np * rs);
  L.sw = take(np * rs);
  L.spid = take(np * 4);
  L.perm = take(np * 8);
  L.ccount = take((size_t)(n_keys + 1) * 4);
  L.cstart = take((size_t)(n_keys + 1) * 4);
  L.scan = take(((size_t)(n_keys + 1) / 256 + 2) * 4 * 2);
  L.W = take((size_t)(d.n_tracked > 0 ? d.n_tracked : 1) * (d.M + 1) * 8);
  L.Wc = take((size_t)(d.n_tracked > 0 ? d.n_tracked : 1) * 2 * 8);
  L.tracked = take((size_t)(d.n_tracked > 0 ? d.n_tracked : 1) * 4);
  L.CE = take((size_t)N * rs);
  L.CB = take((size_t)N * rs);
  L.P = take((size_t)(2 * N - 1) * rs);
  L.H = take((size_t)PIC_MAX_JZ_TAPS * rs);
  L.red = take((size_t)kRedBlocks * (PIC_MAX_MODES + 1) * 8);
  L.work = take(64);  // the push's 8 tile ticket counters (32 bytes), then the sort's flag word
  L.gam = take((size_t)(d.n_tracked > 0 ? d.n_tracked : 1) * 8);
  L.ids = take((size_t)(d.n_tracked > 0 ? d.n_tracked : 1) * 8);
  // deterministic mode: an integer pair (2 x 8 bytes) per value of J
  L.Jfix = det ? take((size_t)2 * 3 * NM * plane * 8) : 0;
  L.total = o;
  (void)Tz;
  (void)Tr;
  return L;
}

}  // namespace

struct pic_ctx {
  uint32_t magic = kMagic;
  int prec = PIC_PREC_FP64;
  hipStream_t stream = nullptr;
  unsigned char *ws = nullptr;
  int sort_interval = 0;
  int current = PIC_CURRENT_FILTER;
  bool det = false;  // deterministic mode: integer deposit sums
  int win_K = 0, win_guard = 0;  // moving window: steps between moves (0: static box), guard columns
  double win_speed = 1.0;        // the window's speed (c)
  int shape = 1;                 // particle shape order: 1 linear, 2 quadratic
  std::vector<RunHost> runs;
  // per-phase event timing
  bool profiling = false;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  double phase_ms[PIC_NPHASES] = {0, 0, 0, 0, 0};
  int64_t phase_n[PIC_NPHASES] = {0, 0, 0, 0, 0};
  // captured steps: keyed by the launch arguments of the step, each holds the
  // graph and the run views (particle buffers swapped by a sort) after it
  bool use_graph = false;
  struct Captured {
    hipGraphExec_t exec;
    Batch after;
  };
  std::map<std::string, Captured> graphs;
  hipStream_t capture_stream = nullptr;  // the caller's stream may be the legacy default stream,
                                         // which cannot be captured: steps are captured here
  ~pic_ctx() {
    for (auto &m : marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    for (auto &e : event_pool) (void)hipEventDestroy(e);
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second.exec);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
};

namespace {

int validate_run(const pic_run_desc &r, int i, int N) {
  if (r.Nz < 8 || r.Nr < 4 || r.M < 0 || r.M > PIC_MAX_MODES || r.ppc < 0)
    return fail(PIC_E_INVALID, "run %d: grid Nz=%d Nr=%d M=%d ppc=%d out of range", i, r.Nz, r.Nr, r.M, r.ppc);
  if (r.Nz < 2 * N) return fail(PIC_E_INVALID, "run %d: Nz=%d shorter than the %d-tap stencil", i, r.Nz, 2 * N);
  if (!(r.dz > 0) || !(r.dr > 0) || !std::isfinite(r.dz) || !std::isfinite(r.dr))
    return fail(PIC_E_INVALID, "run %d: cell sizes must be positive", i);
  if (!(r.n0 >= 0) || !(r.ramp_len >= 0) || !(r.down_len >= 0) || !std::isfinite(r.ramp_start) ||
      !std::isfinite(r.down_start))
    return fail(PIC_E_INVALID, "run %d: density must be >= 0 and ramps finite", i);
  if (r.n_pulses < 0 || r.n_pulses > PIC_MAX_PULSES) return fail(PIC_E_INVALID, "run %d: n_pulses out of range", i);
  if (r.n_pulses > 0 && r.M < 1) return fail(PIC_E_INVALID, "run %d: a laser needs M >= 1", i);
  for (int p = 0; p < r.n_pulses; ++p)
    if (!(r.pulse[p].w0 > 0) || !(r.pulse[p].tau > 0))
      return fail(PIC_E_INVALID, "run %d: pulse %d needs w0 > 0 and tau > 0", i, p);
  const int64_t np = run_particle_count(r);
  if (np > (int64_t)kIdMask) return fail(PIC_E_INVALID, "run %d: %lld electrons exceed the id range", i, (long long)np);
  // the push addresses a particle array with 32-bit byte offsets
  if (np * 8 > (int64_t)UINT32_MAX)
    return fail(PIC_E_INVALID, "run %d: %lld electrons exceed the 2^29 a run may hold", i, (long long)np);
  if (r.n_tracked < 0 || r.n_tracked > np) return fail(PIC_E_INVALID, "run %d: n_tracked out of range", i);
  if (r.n_steps < 0) return fail(PIC_E_INVALID, "run %d: n_steps < 0", i);
  // the kernels address a node inside a plane with 32-bit signed offsets
  if ((int64_t)(r.Nr + 1) * r.Nz > (int64_t)INT32_MAX)
    return fail(PIC_E_INVALID, "run %d: (Nr+1) Nz = %lld nodes per plane exceed 2^31 - 1", i,
                (long long)(r.Nr + 1) * r.Nz);
  return PIC_OK;
}

// particle shape order of the options: 1 linear (0 or 1), 2 quadratic
int shape_of(const pic_opts &o) { return o.shape == 2 ? 2 : 1; }

// Sort tile: 32 x 8 cells unless given.  A default extent shrinks until the
// push workgroup's LDS (current and field windows) fits the budget of two
// workgroups per CU: the radial extent halves down to 4, then the axial one
// steps down by 2 to 16, then the radial one halves again.
int choose_tiles(const pic_opts &o, int M, int *Tz, int *Tr) {
  *Tz = o.tile_z > 0 ? o.tile_z : 32;
  *Tr = o.tile_r > 0 ? o.tile_r : 8;
  const bool det = o.deterministic != 0;
  const int sh = shape_of(o);
  auto over = [&] { return push_lds_bytes(M, *Tz, *Tr, o.precision, det, sh) > kPushLdsDefault; };
  while (over()) {
    if (o.tile_r <= 0 && *Tr > 4) *Tr /= 2;
    else if (o.tile_z <= 0 && *Tz > 16) *Tz -= 2;
    else if (o.tile_r <= 0 && *Tr > 1) *Tr /= 2;
    else break;
  }
  if (push_lds_bytes(M, *Tz, *Tr, o.precision, det, sh) > kPushLdsMax)
    return fail(PIC_E_INVALID, "tile %dx%d needs %zu bytes of LDS (limit %zu)", *Tz, *Tr,
                push_lds_bytes(M, *Tz, *Tr, o.precision, det, sh), kPushLdsMax);
  return PIC_OK;
}

long long keys_of(const pic_run_desc &r, int Tz, int Tr) {
  const long long ntz = (r.Nz + Tz - 1) / Tz, ntr = (r.Nr + Tr - 1) / Tr;
  return ntz * ntr * (long long)Tz * Tr;
}

Batch batch_of_one(const KRun &k) {
  Batch b;
  std::memset(&b, 0, sizeof b);
  b.n = 1;
  b.run[0] = k;
  return b;
}

RunHost *get_run(pic_ctx *ctx, int run) {
  if (run < 0 || run >= (int)ctx->runs.size()) return nullptr;
  return &ctx->runs[(size_t)run];
}

// live contexts: a destroyed or foreign handle is recognised without touching it
std::mutex g_live_mu;
std::set<const pic_ctx *> g_live;

bool ctx_ok(pic_ctx *ctx) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  return ctx && g_live.count(ctx) && ctx->magic == kMagic;
}
void ctx_register(pic_ctx *ctx) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.insert(ctx);
}
void ctx_unregister(pic_ctx *ctx) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.erase(ctx);
}

template <typename T>
int upload(void *dst, const std::vector<T> &src, hipStream_t s) {
  if (src.empty()) return PIC_OK;
  return hip_ok(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s),
                "hipMemcpyAsync H2D");
}

}  // namespace

extern "C" {

const char *pic_last_error(void) { return g_msg; }

int pic_solver_setup(int32_t solver, int32_t n_coef, int32_t M, double dz, double dr, double cfl_fraction,
                     double fit_band, double *dt, double *courant_limit, double *coef_E, double *coef_B) {
  g_msg[0] = 0;
  if (solver != PIC_SOLVER_DUAL && solver != PIC_SOLVER_YEE) return fail(PIC_E_INVALID, "unknown solver %d", solver);
  const int N = solver == PIC_SOLVER_YEE ? 1 : n_coef;
  if (N < 1 || N > PIC_MAX_COEF || M < 0 || M > PIC_MAX_MODES || !(dz > 0) || !(dr > 0))
    return fail(PIC_E_INVALID, "bad solver setup arguments");
  const double band = fit_band > 0 ? fit_band : 2.0 * kPi / 3.0;
  const double frac = cfl_fraction > 0 ? cfl_fraction : 0.95;
  if (!(frac <= 1.0)) return fail(PIC_E_INVALID, "cfl_fraction must be in (0, 1]");
  const double lim = courant_limit_fitted(solver, N, M, dz, dr, band);
  std::vector<double> CE(N), CB(N);
  const double nu = frac * lim;
  if (N == 1) CE[0] = CB[0] = 1.0;
  else fit_dual(N, nu, band, CE.data(), CB.data());
  if (dt) *dt = nu * dz;
  if (courant_limit) *courant_limit = lim;
  if (coef_E) std::memcpy(coef_E, CE.data(), sizeof(double) * N);
  if (coef_B) std::memcpy(coef_B, CB.data(), sizeof(double) * N);
  return PIC_OK;
}

int pic_courant_limit(int32_t n_coef, const double *coef_E, const double *coef_B, int32_t M, double dz, double dr,
                      double *courant_limit) {
  g_msg[0] = 0;
  if (n_coef < 1 || n_coef > PIC_MAX_COEF || !coef_E || !coef_B || M < 0 || M > PIC_MAX_MODES || !(dz > 0) ||
      !(dr > 0) || !courant_limit)
    return fail(PIC_E_INVALID, "bad arguments");
  *courant_limit = courant_limit_of(coef_E, coef_B, n_coef, M, dz, dr);
  return PIC_OK;
}

int pic_jz_inverse_taps(int32_t n_coef, const double *coef_B, int32_t precision, double *taps, int32_t *n_taps) {
  g_msg[0] = 0;
  if (n_coef < 1 || n_coef > PIC_MAX_COEF || !coef_B || !taps || !n_taps ||
      (precision != PIC_PREC_FP64 && precision != PIC_PREC_FP32))
    return fail(PIC_E_INVALID, "bad arguments");
  int nh = 0;
  const int rc = jz_inverse_taps(coef_B, n_coef, precision == PIC_PREC_FP64 ? 0x1p-53 : 0x1p-24, PIC_MAX_JZ_TAPS,
                                 taps, &nh);
  if (rc == 1) return fail(PIC_E_INVALID, "the z filter of these coefficients has P(k) <= 0: no inverse");
  if (rc == 2) return fail(PIC_E_INVALID, "the inverse z filter needs more than %d taps", PIC_MAX_JZ_TAPS);
  *n_taps = nh;
  return PIC_OK;
}

int pic_load_host(const pic_run_desc *run, double *z, double *x, double *y, double *w, int64_t *id,
                  int64_t *tracked_ids, int64_t *n_out) {
  g_msg[0] = 0;
  if (!run || !n_out) return fail(PIC_E_INVALID, "NULL argument");
  TRY(validate_run(*run, 0, 1));
  *n_out = run_particle_count(*run);
  if (!z && !x && !y && !w && !id && !tracked_ids) return PIC_OK;
  load_electrons(*run, z, x, y, w, id, tracked_ids);
  return PIC_OK;
}

int pic_init(const pic_run_desc *runs, int32_t n_runs, const pic_opts *opts, void *device_workspace,
             size_t *workspace_bytes, void *hip_stream, pic_ctx **out) {
  g_msg[0] = 0;
  if (!runs || n_runs < 1 || !opts || !workspace_bytes) return fail(PIC_E_INVALID, "NULL or empty argument");
  const pic_opts &o = *opts;
  if (o.precision != PIC_PREC_FP64 && o.precision != PIC_PREC_FP32)
    return fail(PIC_E_INVALID, "precision must be 64 or 32");
  if (o.solver != PIC_SOLVER_DUAL && o.solver != PIC_SOLVER_YEE) return fail(PIC_E_INVALID, "unknown solver");
  const int N = o.solver == PIC_SOLVER_YEE ? 1 : o.n_coef;
  if (N < 1 || N > PIC_MAX_COEF) return fail(PIC_E_INVALID, "n_coef must be in 1..%d", PIC_MAX_COEF);
  if (o.cfl_fraction < 0 || o.cfl_fraction > 1 || o.dt < 0 || !std::isfinite(o.dt))
    return fail(PIC_E_INVALID, "cfl_fraction or dt out of range");
  if ((o.coef_E == nullptr) != (o.coef_B == nullptr)) return fail(PIC_E_INVALID, "give both coef_E and coef_B");
  if ((o.run_coef_E == nullptr) != (o.run_coef_B == nullptr))
    return fail(PIC_E_INVALID, "give both run_coef_E and run_coef_B");
  if (o.run_dt)
    for (int i = 0; i < n_runs; ++i)
      if (!(o.run_dt[i] > 0) || !std::isfinite(o.run_dt[i])) return fail(PIC_E_INVALID, "run_dt[%d] out of range", i);
  if (o.sort_interval < 0 || o.tile_z < 0 || o.tile_r < 0) return fail(PIC_E_INVALID, "negative sort options");
  if (o.current != PIC_CURRENT_FILTER && o.current != PIC_CURRENT_EXACT_JZ)
    return fail(PIC_E_INVALID, "current must be PIC_CURRENT_FILTER or PIC_CURRENT_EXACT_JZ");
  if (o.deterministic != 0 && o.deterministic != 1) return fail(PIC_E_INVALID, "deterministic must be 0 or 1");
  if (o.deterministic && o.precision != PIC_PREC_FP64)
    return fail(PIC_E_INVALID, "the deterministic mode is for PIC_PREC_FP64 runs");
  if (o.window_interval < 0 || o.window_guard < 0 || !(o.window_speed >= 0) || !std::isfinite(o.window_speed))
    return fail(PIC_E_INVALID, "window_interval, window_guard and window_speed must be >= 0");
  if (o.window_interval > 0 && (o.use_graph || o.deterministic))
    return fail(PIC_E_INVALID, "the moving window does not run with use_graph or the deterministic mode");
  if (o.shape < 0 || o.shape > 2) return fail(PIC_E_INVALID, "shape must be 0, 1 (linear) or 2 (quadratic)");
  for (int i = 0; i < n_runs; ++i) {
    TRY(validate_run(runs[i], i, N));
    if (particle_capacity(runs[i], o) * 8 > (int64_t)UINT32_MAX)
      return fail(PIC_E_INVALID, "run %d: the moving window's particle slots exceed the 2^29 a run may hold", i);
    if (o.window_interval > 0 && o.window_guard >= runs[i].Nz)
      return fail(PIC_E_INVALID, "run %d: window_guard must be below Nz", i);
    if (runs[i].M != runs[0].M) return fail(PIC_E_INVALID, "all runs of one context must share M");
  }
  int Tz, Tr;
  TRY(choose_tiles(o, runs[0].M, &Tz, &Tr));

  // workspace size
  std::vector<Layout> lays;
  std::vector<size_t> offs;
  size_t total = 0;
  for (int i = 0; i < n_runs; ++i) {
    lays.push_back(layout_of(runs[i], o.precision, N, Tz, Tr, keys_of(runs[i], Tz, Tr), o.deterministic != 0,
                             particle_capacity(runs[i], o)));
    offs.push_back(total);
    total = align_up(total + lays.back().total);
  }
  if (!device_workspace) {
    *workspace_bytes = total;
    return PIC_OK;
  }
  if (!out) return fail(PIC_E_INVALID, "NULL out");
  if (*workspace_bytes < total)
    return fail(PIC_E_NOMEM, "workspace of %zu bytes, %zu needed", *workspace_bytes, total);
  if (((uintptr_t)device_workspace) % kAlign) return fail(PIC_E_INVALID, "workspace must be 256-byte aligned");

  pic_ctx *ctx = new (std::nothrow) pic_ctx();
  if (!ctx) return fail(PIC_E_NOMEM, "host allocation failed");
  ctx->prec = o.precision;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->ws = (unsigned char *)device_workspace;
  ctx->sort_interval = o.sort_interval > 0 ? o.sort_interval : kDefaultSortInterval;
  ctx->use_graph = o.use_graph != 0;
  ctx->current = o.current;
  ctx->det = o.deterministic != 0;
  ctx->win_K = o.window_interval;
  ctx->win_guard = o.window_guard;
  ctx->win_speed = o.window_speed > 0 ? o.window_speed : 1.0;
  ctx->shape = shape_of(o);
  ctx->runs.resize((size_t)n_runs);
  const hipStream_t s = ctx->stream;
  const bool f64 = o.precision == PIC_PREC_FP64;
  const double band = o.fit_band > 0 ? o.fit_band : 2.0 * kPi / 3.0;
  const double frac = o.cfl_fraction > 0 ? o.cfl_fraction : 0.95;

  int rc = prepare_kernels(o.precision, runs[0].M, Tz, Tr, ctx->det, shape_of(o));
  for (int i = 0; i < n_runs && rc == PIC_OK; ++i) {
    RunHost &R = ctx->runs[(size_t)i];
    R.d = runs[i];
    R.N = N;
    const pic_run_desc &d = R.d;
    // ---- coefficients and dt (Sec. III.A) ----
    R.CE.assign(N, 1.0);
    R.CB.assign(N, 1.0);
    const double *ce = o.run_coef_E ? o.run_coef_E + (size_t)i * N : o.coef_E;
    const double *cb = o.run_coef_B ? o.run_coef_B + (size_t)i * N : o.coef_B;
    const double dt_fix = o.run_dt ? o.run_dt[i] : o.dt;
    if (ce) {
      R.CE.assign(ce, ce + N);
      R.CB.assign(cb, cb + N);
      R.nu_lim = courant_limit_of(R.CE.data(), R.CB.data(), N, d.M, d.dz, d.dr);
      R.dt = dt_fix > 0 ? dt_fix : frac * R.nu_lim * d.dz;
    } else if (dt_fix > 0) {
      if (N > 1) fit_dual(N, dt_fix / d.dz, band, R.CE.data(), R.CB.data());
      R.nu_lim = courant_limit_of(R.CE.data(), R.CB.data(), N, d.M, d.dz, d.dr);
      R.dt = dt_fix;
    } else {
      R.nu_lim = courant_limit_fitted(o.solver, N, d.M, d.dz, d.dr, band);
      R.dt = frac * R.nu_lim * d.dz;
      if (N > 1) fit_dual(N, R.dt / d.dz, band, R.CE.data(), R.CB.data());
    }
    if (R.dt / d.dz > R.nu_lim) {
      rc = fail(PIC_E_CFL, "run %d: c dt/dz = %.6g above the Courant limit %.6g", i, R.dt / d.dz, R.nu_lim);
      break;
    }
    // z filter taps p_l = sum_{l' > |l|} C^B_{l'}, so that D_B = D_Yee o P
    R.P.assign(2 * N - 1, 0.0);
    for (int l = 0; l < N; ++l) {
      double p = 0.0;
      for (int lp = l + 1; lp <= N; ++lp) p += R.CB[(size_t)lp - 1];
      R.P[(size_t)(N - 1 + l)] = p;
      R.P[(size_t)(N - 1 - l)] = p;
    }
    // P^{-1} as a cut symmetric stencil for the exact J_z correction
    R.H.clear();
    if (o.current == PIC_CURRENT_EXACT_JZ) {
      double h[PIC_MAX_JZ_TAPS];
      int nh = 0;
      const int hr = jz_inverse_taps(R.CB.data(), N, f64 ? 0x1p-53 : 0x1p-24, PIC_MAX_JZ_TAPS, h, &nh);
      if (hr) {
        rc = fail(PIC_E_INVALID, hr == 1 ? "run %d: the z filter has P(k) <= 0, so J_z cannot be corrected exactly"
                                         : "run %d: the inverse z filter needs more than the maximum of taps",
                  i);
        break;
      }
      R.H.assign(h, h + nh);
    }
    // ---- device view ----
    const Layout &L = lays[(size_t)i];
    unsigned char *base = ctx->ws + offs[(size_t)i];
    R.offset = offs[(size_t)i];
    R.bytes = L.total;
    KRun &k = R.k;
    std::memset(&k, 0, sizeof k);
    k.Nz = d.Nz;
    k.Nr = d.Nr;
    k.M = d.M;
    k.N = N;
    k.dz = d.dz;
    k.dr = d.dr;
    k.dt = R.dt;
    k.np = run_particle_count(d);
    R.cap = particle_capacity(d, o);
    k.window = ctx->win_K > 0 ? 1 : 0;
    k.shape = ctx->shape;
    k.plane = (long long)(d.Nr + 1) * d.Nz;
    k.E = base + L.E;
    k.B[0] = base + L.B0;
    k.B[1] = base + L.B1;
    k.Bbar = base + L.Bbar;
    k.J[0] = base + L.J0;
    k.J[1] = base + L.J1;
    k.rho = base + L.rho;
    k.pz = base + L.pz;
    k.pfz = base + L.pfz;
    k.px = base + L.px;
    k.py = base + L.py;
    k.pux = base + L.pux;
    k.puy = base + L.puy;
    k.puz = base + L.puz;
    k.pw = base + L.pw;
    k.pid = (uint32_t *)(base + L.pid);
    k.sz = base + L.sz;
    k.sfz = base + L.sfz;
    k.sx = base + L.sx;
    k.sy = base + L.sy;
    k.sux = base + L.sux;
    k.suy = base + L.suy;
    k.suz = base + L.suz;
    k.sw = base + L.sw;
    k.spid = (uint32_t *)(base + L.spid);
    k.perm = (uint64_t *)(base + L.perm);
    k.cell_count = (int32_t *)(base + L.ccount);
    k.cell_start = (int32_t *)(base + L.cstart);
    k.scan_tmp = (int32_t *)(base + L.scan);
    k.Tz = Tz;
    k.Tr = Tr;
    k.ntz = (d.Nz + Tz - 1) / Tz;
    k.ntr = (d.Nr + Tr - 1) / Tr;
    k.n_keys = keys_of(d, Tz, Tr);
    k.W = (double *)(base + L.W);
    k.Wc = (double *)(base + L.Wc);
    k.tracked = (const int32_t *)(base + L.tracked);
    k.n_tracked = d.n_tracked;
    k.CE = base + L.CE;
    k.CB = base + L.CB;
    k.P = base + L.P;
    k.H = base + L.H;
    k.NH = (int)R.H.size();
    k.red = (double *)(base + L.red);
    k.work = (int32_t *)(base + L.work);
    k.flags = (uint32_t *)(base + L.work + 32);
    k.Jfix = ctx->det ? (unsigned long long *)(base + L.Jfix) : nullptr;
    k.qscale = 1.0;
    R.dev_gamma = (double *)(base + L.gam);
    R.dev_ids = (int64_t *)(base + L.ids);

    // ---- coefficients ----
    if (f64) {
      if ((rc = upload(base + L.CE, R.CE, s)) || (rc = upload(base + L.CB, R.CB, s)) || (rc = upload(base + L.P, R.P, s)) ||
          (!R.H.empty() && (rc = upload(base + L.H, R.H, s))))
        break;
    } else {
      std::vector<float> a(R.CE.begin(), R.CE.end()), b(R.CB.begin(), R.CB.end()), c(R.P.begin(), R.P.end()),
          hf(R.H.begin(), R.H.end());
      if ((rc = upload(base + L.CE, a, s)) || (rc = upload(base + L.CB, b, s)) || (rc = upload(base + L.P, c, s)) ||
          (!hf.empty() && (rc = upload(base + L.H, hf, s))))
        break;
      if ((rc = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
    }
    // ---- electrons (host FP64 loading, then the run's precision) ----
    const int64_t np = k.np;
    std::vector<double> z(np), x(np), y(np), w(np);
    std::vector<int64_t> ids(np), tr((size_t)(d.n_tracked > 0 ? d.n_tracked : 0));
    load_electrons(d, z.data(), x.data(), y.data(), w.data(), ids.data(), tr.empty() ? nullptr : tr.data());
    std::vector<uint32_t> pid(np);
    for (int64_t p = 0; p < np; ++p) pid[(size_t)p] = (uint32_t)ids[(size_t)p];
    if (ctx->det) {
      // 2^K with 4 max|q| 2^K < 2^30: every scaled contribution fits the
      // integer split of the deterministic deposit (|contribution| <= 4 |q|)
      double wmax = 0.0;
      for (int64_t p = 0; p < np; ++p) wmax = std::max(wmax, std::fabs(w[(size_t)p]));
      int e = 0;
      if (wmax > 0) std::frexp(wmax, &e);
      k.qscale = wmax > 0 ? std::ldexp(1.0, 28 - e) : 1.0;
      if ((rc = launch_zero(k.Jfix, lays[(size_t)i].Jfix ? (size_t)2 * 3 * (2 * d.M + 1) * (size_t)k.plane * 8 : 0,
                            s)))
        break;
    }
    for (size_t t = 0; t < tr.size(); ++t) pid[(size_t)tr[t]] |= kTrackedBit;
    std::vector<int32_t> tr32(tr.begin(), tr.end());
    R.tr_ids = tr;
    R.gam0.assign(tr.size(), 1.0);  // cold start
    if (f64) {
      std::vector<double> zero(np, 0.0);
      if ((rc = upload(k.pz, z, s)) || (rc = upload(k.px, x, s)) || (rc = upload(k.py, y, s)) ||
          (rc = upload(k.pux, zero, s)) || (rc = upload(k.puy, zero, s)) || (rc = upload(k.puz, zero, s)) ||
          (rc = upload(k.pw, w, s)) || (rc = upload(k.pid, pid, s)) || (rc = upload((void *)k.tracked, tr32, s)))
        break;
      if ((rc = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
    } else {
      // z as int32 cell + FP32 offset; an offset that rounds to 1 carries
      std::vector<int32_t> iz(np);
      std::vector<float> fz(np), xf(np), yf(np), wf(np), zero(np, 0.0f);
      for (int64_t p = 0; p < np; ++p) {
        double c = std::floor(z[(size_t)p]);
        float f = (float)(z[(size_t)p] - c);
        if (f >= 1.0f) {
          f = 0.0f;
          c += 1.0;
          if (c >= d.Nz) c -= d.Nz;
        }
        iz[(size_t)p] = (int32_t)c;
        fz[(size_t)p] = f;
        xf[(size_t)p] = (float)x[(size_t)p];
        yf[(size_t)p] = (float)y[(size_t)p];
        wf[(size_t)p] = (float)w[(size_t)p];
      }
      if ((rc = upload(k.pz, iz, s)) || (rc = upload(k.pfz, fz, s)) || (rc = upload(k.px, xf, s)) ||
          (rc = upload(k.py, yf, s)) || (rc = upload(k.pux, zero, s)) || (rc = upload(k.puy, zero, s)) ||
          (rc = upload(k.puz, zero, s)) || (rc = upload(k.pw, wf, s)) || (rc = upload(k.pid, pid, s)) ||
          (rc = upload((void *)k.tracked, tr32, s)))
        break;
      if ((rc = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
    }
    // ---- fields: laser E^0, B^0 (Eq. (18)), then B^{-1/2}, B^{+1/2} ----
    {
      const size_t nvec = (size_t)3 * (2 * d.M + 1) * (size_t)k.plane;
      std::vector<double> Eh(nvec, 0.0), Bh(nvec, 0.0);
      laser_fields(d, Eh.data(), Bh.data());
      if (f64) {
        if ((rc = upload(k.E, Eh, s)) || (rc = upload(k.B[0], Bh, s)) || (rc = upload(k.B[1], Bh, s)) ||
            (rc = upload(k.Bbar, Bh, s)))
          break;
        if ((rc = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
      } else {
        std::vector<float> Ef(Eh.begin(), Eh.end()), Bf(Bh.begin(), Bh.end());
        if ((rc = upload(k.E, Ef, s)) || (rc = upload(k.B[0], Bf, s)) || (rc = upload(k.B[1], Bf, s)) ||
            (rc = upload(k.Bbar, Bf, s)))
          break;
        if ((rc = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
      }
    }
    const size_t rs = f64 ? 8 : 4;
    const size_t vecb = (size_t)3 * (2 * d.M + 1) * (size_t)k.plane * rs;
    if ((rc = launch_zero(k.work, 64, s)) || (rc = launch_zero(k.J[0], vecb, s)) || (rc = launch_zero(k.J[1], vecb, s)) ||
        (rc = launch_zero(k.W, (size_t)(d.n_tracked > 0 ? d.n_tracked : 1) * (d.M + 1) * 8, s)) ||
        (rc = launch_zero(k.Wc, (size_t)(d.n_tracked > 0 ? d.n_tracked : 1) * 2 * 8, s)))
      break;
    // B[0] = B^0 + (dt/2) curl_E E^0 = B^{-1/2};  B[1] = B^0 - (dt/2) curl_E E^0 = B^{+1/2}
    Batch b = batch_of_one(k);
    for (int h = 0; h < 2 && rc == PIC_OK; ++h) {
      b.bout[0] = k.B[h];
      b.bin[0] = k.B[h];
      b.avg[0] = nullptr;
      b.tau[0] = (h == 0 ? -0.5 : 0.5) * R.dt;
      rc = launch_bfield(b, ctx->prec, s);
    }
    if (rc) break;
    if ((rc = launch_sort(b, ctx->prec, s))) break;  // the push kernel works tile by tile
    k = b.run[0];
    if ((rc = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
  }
  if (rc != PIC_OK) {
    if (rc == PIC_E_DEVICE && g_msg[0] == 0) fail(rc, "%s", last_device_error());
    ctx->magic = 0;
    delete ctx;
    return rc;
  }
  ctx_register(ctx);
  *out = ctx;
  return PIC_OK;
}

}  // extern "C"

extern "C" int check_sort_flags(pic_ctx *ctx);

namespace {

hipEvent_t take_event(pic_ctx *ctx) {
  hipEvent_t e = nullptr;
  if (!ctx->event_pool.empty()) {
    e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// Launch one phase, bracketed by events when profiling.
template <typename F>
int timed(pic_ctx *ctx, int phase, F &&launch) {
  if (!ctx->profiling) return launch();
  hipEvent_t a = take_event(ctx), b = take_event(ctx);
  if (!a || !b) return fail(PIC_E_DEVICE, "hipEventCreate failed");
  TRY(hip_ok(hipEventRecord(a, ctx->stream), "hipEventRecord"));
  int rc = launch();
  TRY(hip_ok(hipEventRecord(b, ctx->stream), "hipEventRecord"));
  ctx->marks.push_back({phase, a, b});
  return rc;
}

// Moving window, before a step whose count of steps taken n is a positive
// multiple of K: the run's box advances by s = floor(v n dt / dz) - S cells.
// The fresh plasma of the s new absolute columns is appended to the particle
// arrays in the box's current coordinates, the fields move back (E, B, Bbar;
// J is zero between steps), and k.shift = s makes the step's sort move every
// electron back s cells and drop those outside the box.  *moved: a move was
// enqueued (the step must sort and then read back the electron count).
int window_move(pic_ctx *ctx, RunHost &R, hipStream_t s, bool *moved) {
  *moved = false;
  const int64_t n = R.steps;
  if (ctx->win_K <= 0 || n <= 0 || n % ctx->win_K != 0) return PIC_OK;
  const int64_t target = (int64_t)std::floor(ctx->win_speed * (double)n * R.dt / R.d.dz);
  const int64_t sft = target - R.win_S;
  if (sft <= 0) return PIC_OK;
  const pic_run_desc &d = R.d;
  KRun &k = R.k;
  const int64_t cols = std::min<int64_t>(sft, d.Nz), a1 = target + d.Nz;
  const int64_t nf = cols * (int64_t)(d.Nr - 1) * d.ppc;
  if (k.np + nf > R.cap)
    return fail(PIC_E_NOMEM, "moving window: %lld electrons after the move exceed the %lld slots",
                (long long)(k.np + nf), (long long)R.cap);
  if (nf > 0 && a1 * (int64_t)(d.Nr - 1) * d.ppc - 1 > (int64_t)kIdMask)
    return fail(PIC_E_INVALID, "moving window: the plasma ids of absolute column %lld exceed the id range",
                (long long)(a1 - 1));
  if (nf > 0) {
    std::vector<double> z((size_t)nf), x((size_t)nf), y((size_t)nf), w((size_t)nf);
    std::vector<int64_t> id((size_t)nf);
    load_columns(d, a1 - cols, a1, R.win_S, z.data(), x.data(), y.data(), w.data(), id.data());
    // in the cell order the sort will give them (near enough: the cell of
    // r is taken without the sort's rounding care), so that the sort's
    // blocks count them in LDS; the slots they land in are the sort's choice
    {
      std::vector<int64_t> key((size_t)nf);
      const int64_t TT = (int64_t)k.Tz * k.Tr;
      for (size_t p = 0; p < (size_t)nf; ++p) {
        const int64_t iz = std::min<int64_t>(std::max<int64_t>((int64_t)std::floor(z[p]) - sft, 0), d.Nz - 1);
        const int64_t ir = std::min<int64_t>((int64_t)std::sqrt(x[p] * x[p] + y[p] * y[p]), d.Nr - 1);
        key[p] = ((ir / k.Tr) * k.ntz + iz / k.Tz) * TT + (ir % k.Tr) * k.Tz + iz % k.Tz;
      }
      std::vector<size_t> ord((size_t)nf);
      for (size_t p = 0; p < ord.size(); ++p) ord[p] = p;
      std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
      auto permute = [&](auto &v) {
        auto t = v;
        for (size_t p = 0; p < ord.size(); ++p) v[p] = t[ord[p]];
      };
      permute(z);
      permute(x);
      permute(y);
      permute(w);
      permute(id);
    }
    std::vector<uint32_t> pid(id.begin(), id.end());
    const size_t at = (size_t)k.np;
    if (ctx->prec == PIC_PREC_FP64) {
      std::vector<double> zero((size_t)nf, 0.0);
      TRY(upload((double *)k.pz + at, z, s));
      TRY(upload((double *)k.px + at, x, s));
      TRY(upload((double *)k.py + at, y, s));
      TRY(upload((double *)k.pux + at, zero, s));
      TRY(upload((double *)k.puy + at, zero, s));
      TRY(upload((double *)k.puz + at, zero, s));
      TRY(upload((double *)k.pw + at, w, s));
      TRY(upload(k.pid + at, pid, s));
      TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
    } else {
      // int32 cell + FP32 offset, as pic_init converts (the cell is not wrapped)
      std::vector<int32_t> iz((size_t)nf);
      std::vector<float> fz((size_t)nf), xf((size_t)nf), yf((size_t)nf), wf((size_t)nf), zero((size_t)nf, 0.0f);
      for (size_t p = 0; p < (size_t)nf; ++p) {
        double c = std::floor(z[p]);
        float f = (float)(z[p] - c);
        if (f >= 1.0f) {
          f = 0.0f;
          c += 1.0;
        }
        iz[p] = (int32_t)c;
        fz[p] = f;
        xf[p] = (float)x[p];
        yf[p] = (float)y[p];
        wf[p] = (float)w[p];
      }
      TRY(upload((int32_t *)k.pz + at, iz, s));
      TRY(upload((float *)k.pfz + at, fz, s));
      TRY(upload((float *)k.px + at, xf, s));
      TRY(upload((float *)k.py + at, yf, s));
      TRY(upload((float *)k.pux + at, zero, s));
      TRY(upload((float *)k.puy + at, zero, s));
      TRY(upload((float *)k.puz + at, zero, s));
      TRY(upload((float *)k.pw + at, wf, s));
      TRY(upload(k.pid + at, pid, s));
      TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
    }
    k.np += nf;
  }
  k.shift = (int)std::min<int64_t>(sft, (int64_t)d.Nz + 1);  // beyond Nz every electron is dropped alike
  TRY(launch_window_shift(k, ctx->prec, ctx->win_guard, s));
  R.win_S = target;
  *moved = true;
  return PIC_OK;
}

// Enqueue one step of the runs `ids` (at most kMaxBatch, all at the same step
// count): sort when due, then push, E update and B update, one launch per
// phase for all of them -- or the replay of that step's captured graph.
int step_batch(pic_ctx *ctx, const std::vector<int> &ids) {
  hipStream_t s = ctx->stream;  // where the launches go: the caller's stream, or the capture stream
  const int prec = ctx->prec;
  const int64_t step = ctx->runs[(size_t)ids[0]].steps;
  const int par = (int)(step & 1);
  bool sort = step > 0 && step % ctx->sort_interval == 0;
  bool moved[kMaxBatch] = {};
  for (size_t i = 0; i < ids.size(); ++i) {
    TRY(window_move(ctx, ctx->runs[(size_t)ids[i]], s, &moved[i]));
    if (moved[i]) sort = true;
  }
  Batch b;
  std::memset(&b, 0, sizeof b);  // every byte defined: the batch is a capture key
  b.n = (int)ids.size();
  b.par = par;
  b.det = ctx->det ? 1 : 0;
  for (int i = 0; i < b.n; ++i) {
    const RunHost &R = ctx->runs[(size_t)ids[(size_t)i]];
    b.run[i] = R.k;
    b.bout[i] = R.k.B[par];
    b.bin[i] = R.k.B[par ^ 1];
    b.avg[i] = R.k.Bbar;
    b.tau[i] = R.dt;
  }
  auto launches = [&](bool events) {
    auto ph = [&](int phase, auto &&f) { return events ? timed(ctx, phase, f) : f(); };
    if (sort) TRY(ph(PIC_PHASE_SORT, [&] { return launch_sort(b, prec, s); }));
    TRY(ph(PIC_PHASE_PUSH, [&] {
      const int rc = launch_push(b, prec, s);
      return (rc || !b.det) ? rc : launch_fix_convert(b, s);  // deterministic: the integer sums into J
    }));
    TRY(ph(PIC_PHASE_EFIELD, [&] { return launch_efield(b, prec, s); }));
    TRY(ph(PIC_PHASE_BFIELD, [&] { return launch_bfield(b, prec, s); }));
    return PIC_OK;
  };
  if (!ctx->use_graph) {
    TRY(launches(true));
  } else {
    std::string key((const char *)&b, sizeof b);
    key.push_back(sort ? 1 : 0);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
      if (!ctx->capture_stream)
        TRY(hip_ok(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking), "hipStreamCreateWithFlags"));
      s = ctx->capture_stream;
      TRY(hip_ok(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture"));
      const int rc = launches(false);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(s, &g);
      s = ctx->stream;
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      TRY(hip_ok(e, "hipStreamEndCapture"));
      pic_ctx::Captured c;
      const hipError_t ei = hipGraphInstantiate(&c.exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      TRY(hip_ok(ei, "hipGraphInstantiate"));
      c.after = b;  // run views after the step (a sort swaps particle buffers)
      it = ctx->graphs.emplace(std::move(key), c).first;
    }
    TRY(timed(ctx, PIC_PHASE_STEP, [&] { return hip_ok(hipGraphLaunch(it->second.exec, s), "hipGraphLaunch"); }));
    b = it->second.after;
  }
  for (int i = 0; i < b.n; ++i) {
    RunHost &R = ctx->runs[(size_t)ids[(size_t)i]];
    R.k = b.run[i];
    R.steps++;
    if (moved[i]) {  // the sort kept the electrons in the box: cell_start[n_keys] of them
      int32_t alive = 0;
      TRY(hip_ok(hipMemcpyAsync(&alive, R.k.cell_start + R.k.n_keys, 4, hipMemcpyDeviceToHost, s), "D2H"));
      TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
      TRY(check_sort_flags(ctx));
      if (alive < 0 || alive > R.k.np) return fail(PIC_E_DEVICE, "moving window: bad electron count %d", alive);
      R.k.np = alive;
      R.k.shift = 0;
    }
  }
  return PIC_OK;
}

// Sort every run of the context now (outside the step cadence).
int sort_runs_now(pic_ctx *ctx) {
  for (size_t g = 0; g < ctx->runs.size(); g += kMaxBatch) {
    Batch b;
    std::memset(&b, 0, sizeof b);
    b.n = (int)std::min(ctx->runs.size() - g, (size_t)kMaxBatch);
    for (int i = 0; i < b.n; ++i) b.run[i] = ctx->runs[g + (size_t)i].k;
    TRY(launch_sort(b, ctx->prec, ctx->stream));
    for (int i = 0; i < b.n; ++i) ctx->runs[g + (size_t)i].k = b.run[i];
  }
  return PIC_OK;
}

// Candidate sort tiles of the autotuner (those whose push workgroup fits the LDS).
constexpr int kTuneTiles[][2] = {{32, 8}, {32, 6}, {32, 4}, {30, 4}, {24, 8}, {24, 4}, {20, 4},
                                 {16, 8}, {16, 4}, {64, 4}, {64, 2}, {48, 4}, {32, 2}};

// Fold finished marks into the per-phase sums (the stream must be idle).
int collect_marks(pic_ctx *ctx) {
  for (auto &m : ctx->marks) {
    float ms = 0.f;
    TRY(hip_ok(hipEventElapsedTime(&ms, m.a, m.b), "hipEventElapsedTime"));
    ctx->phase_ms[m.phase] += ms;
    ctx->phase_n[m.phase] += 1;
    ctx->event_pool.push_back(m.a);
    ctx->event_pool.push_back(m.b);
  }
  ctx->marks.clear();
  return PIC_OK;
}

}  // namespace

extern "C" {

int pic_step(pic_ctx *ctx, int64_t n_steps) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  if (n_steps < 0) return fail(PIC_E_INVALID, "n_steps < 0");
  const hipStream_t s = ctx->stream;
  std::vector<int> ids;
  for (int64_t n = 0; n < n_steps; ++n) {
    // the runs that still have steps to take, all at the same step count
    ids.clear();
    for (size_t r = 0; r < ctx->runs.size(); ++r) {
      const RunHost &R = ctx->runs[r];
      if (R.d.n_steps == 0 || R.steps < R.d.n_steps) ids.push_back((int)r);
    }
    if (ids.empty()) break;
    for (size_t g = 0; g < ids.size(); g += kMaxBatch) {
      const std::vector<int> grp(ids.begin() + (long)g, ids.begin() + (long)std::min(ids.size(), g + kMaxBatch));
      TRY(step_batch(ctx, grp));
    }
    // keep the number of outstanding event pairs bounded
    if (ctx->profiling && ctx->marks.size() > 4096) {
      TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
      TRY(collect_marks(ctx));
    }
  }
  return PIC_OK;
}

int pic_autotune(const pic_run_desc *runs, int32_t n_runs, pic_opts *opts, void *device_workspace,
                 size_t *workspace_bytes, void *hip_stream, int32_t trial_steps, pic_tune_report *report) {
  g_msg[0] = 0;
  if (!runs || n_runs < 1 || !opts || !workspace_bytes) return fail(PIC_E_INVALID, "NULL or empty argument");
  if (trial_steps < 4 || trial_steps > 64) return fail(PIC_E_INVALID, "trial_steps must be in 4..64");
  if (opts->precision != PIC_PREC_FP64 && opts->precision != PIC_PREC_FP32)
    return fail(PIC_E_INVALID, "precision must be 64 or 32");
  std::vector<pic_run_desc> rd(runs, runs + n_runs);
  for (auto &r : rd) r.n_steps = 0;  // trials take as many steps as they need
  std::vector<std::pair<int, int>> cand;
  if (opts->tile_z > 0 || opts->tile_r > 0) {
    int Tz, Tr;
    TRY(choose_tiles(*opts, rd[0].M, &Tz, &Tr));
    cand.push_back({Tz, Tr});
  } else {
    for (const auto &t : kTuneTiles)
      if (push_lds_bytes(rd[0].M, t[0], t[1], opts->precision, opts->deterministic != 0, shape_of(*opts)) <=
              kPushLdsMax &&
          cand.size() < PIC_MAX_TUNE)
        cand.push_back({t[0], t[1]});
  }
  pic_opts o = *opts;
  o.use_graph = 0;
  o.sort_interval = 1 << 30;  // no sort inside the timed steps
  size_t need = 0;
  for (const auto &c : cand) {
    o.tile_z = c.first;
    o.tile_r = c.second;
    size_t b = 0;
    TRY(pic_init(rd.data(), n_runs, &o, nullptr, &b, nullptr, nullptr));
    need = std::max(need, b);
  }
  if (!device_workspace) {
    *workspace_bytes = need;
    return PIC_OK;
  }
  if (*workspace_bytes < need) return fail(PIC_E_NOMEM, "workspace of %zu bytes, %zu needed", *workspace_bytes, need);
  const hipStream_t s = (hipStream_t)hip_stream;
  const int T = trial_steps;
  std::vector<hipEvent_t> ev((size_t)T + 2, nullptr);
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
      return fail(PIC_E_DEVICE, "hipEventCreate failed");
    }
  pic_tune_report rep;
  std::memset(&rep, 0, sizeof rep);
  rep.best = -1;
  double best = 0.0;
  int rc = PIC_OK;
  for (size_t i = 0; i < cand.size() && rc == PIC_OK; ++i) {
    o.tile_z = cand[i].first;
    o.tile_r = cand[i].second;
    pic_ctx *ctx = nullptr;
    size_t b = *workspace_bytes;
    if ((rc = pic_init(rd.data(), n_runs, &o, device_workspace, &b, hip_stream, &ctx))) break;
    // T untimed steps (kernels loaded, caches warm, the electrons and the
    // pulse no longer in their loaded state), then a timed sort: the timed
    // steps start from a freshly sorted state
    rc = pic_step(ctx, T);
    if (!rc) rc = hip_ok(hipEventRecord(ev[0], s), "hipEventRecord");
    if (!rc) rc = sort_runs_now(ctx);
    if (!rc) rc = hip_ok(hipEventRecord(ev[1], s), "hipEventRecord");
    for (int k = 0; k < T && !rc; ++k) {
      rc = pic_step(ctx, 1);
      if (!rc) rc = hip_ok(hipEventRecord(ev[(size_t)k + 2], s), "hipEventRecord");
    }
    if (!rc) rc = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
    double t_sort = 0.0, sum = 0.0, cost = 0.0;
    int bestK = 1;
    for (int k = 0; k <= T && !rc; ++k) {
      float ms = 0.f;
      rc = hip_ok(hipEventElapsedTime(&ms, ev[(size_t)k], ev[(size_t)k + 1]), "hipEventElapsedTime");
      if (k == 0) {
        t_sort = ms;
        continue;
      }
      sum += ms;
      const double c = (t_sort + sum) / k;  // mean step cost when sorting every k steps
      if (k == 1 || c < cost) {
        cost = c;
        bestK = k;
      }
    }
    const int rd_rc = pic_destroy(ctx);
    if (rc) break;
    if (rd_rc) {
      rc = rd_rc;
      break;
    }
    rep.tile_z[rep.n] = cand[i].first;
    rep.tile_r[rep.n] = cand[i].second;
    rep.interval[rep.n] = bestK;
    rep.ms_per_step[rep.n] = cost;
    if (rep.best < 0 || cost < best) {
      best = cost;
      rep.best = rep.n;
    }
    rep.n++;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  opts->tile_z = rep.tile_z[rep.best];
  opts->tile_r = rep.tile_r[rep.best];
  opts->sort_interval = rep.interval[rep.best];
  if (report) *report = rep;
  return PIC_OK;
}

// After a synchronisation of the context's stream: PIC_E_STATE if a cell
// sort of any run has raised an integrity flag (the flags are sticky).
int check_sort_flags(pic_ctx *ctx) {
  for (size_t i = 0; i < ctx->runs.size(); ++i) {
    uint32_t f = 0;
    TRY(hip_ok(hipMemcpyAsync(&f, ctx->runs[i].k.flags, sizeof f, hipMemcpyDeviceToHost, ctx->stream),
               "hipMemcpyAsync"));
    TRY(hip_ok(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"));
    if (f) {
      char msg[320];
      sort_flags_text(f, (int)i, msg, sizeof msg);
      return fail(PIC_E_STATE, "%s", msg);
    }
  }
  return PIC_OK;
}

int pic_profile(pic_ctx *ctx, int32_t enable) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  TRY(hip_ok(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"));
  TRY(collect_marks(ctx));
  ctx->profiling = enable != 0;
  if (enable)
    for (int p = 0; p < PIC_NPHASES; ++p) { ctx->phase_ms[p] = 0; ctx->phase_n[p] = 0; }
  return PIC_OK;
}

int pic_profile_read(pic_ctx *ctx, double *ms, int64_t *launches) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  TRY(hip_ok(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"));
  TRY(collect_marks(ctx));
  for (int p = 0; p < PIC_NPHASES; ++p) {
    if (ms) ms[p] = ctx->phase_ms[p];
    if (launches) launches[p] = ctx->phase_n[p];
  }
  return PIC_OK;
}

int pic_run_info_get(pic_ctx *ctx, int32_t run, pic_run_info *info) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  RunHost *R = get_run(ctx, run);
  if (!R || !info) return fail(PIC_E_INVALID, "bad run index or NULL info");
  info->dt = R->dt;
  info->courant_limit = R->nu_lim;
  info->n_particles = R->k.np;
  info->steps_done = R->steps;
  info->n_coef = R->N;
  info->n_tracked = R->d.n_tracked;
  info->tile_z = R->k.Tz;
  info->tile_r = R->k.Tr;
  info->window_cells = R->win_S;
  return PIC_OK;
}

int pic_coefficients(pic_ctx *ctx, int32_t run, double *coef_E, double *coef_B, double *taps) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  RunHost *R = get_run(ctx, run);
  if (!R) return fail(PIC_E_INVALID, "bad run index");
  if (coef_E) std::memcpy(coef_E, R->CE.data(), R->CE.size() * 8);
  if (coef_B) std::memcpy(coef_B, R->CB.data(), R->CB.size() * 8);
  if (taps) std::memcpy(taps, R->P.data(), R->P.size() * 8);
  return PIC_OK;
}

int pic_fields(pic_ctx *ctx, int32_t run, int32_t comp, int32_t m, double *out, size_t out_len) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  RunHost *R = get_run(ctx, run);
  if (!R) return fail(PIC_E_INVALID, "bad run index");
  TRY(check_sort_flags(ctx));
  if (comp < 0 || comp > PIC_BZ_NEW || m < 0 || m > R->d.M || !out) return fail(PIC_E_INVALID, "bad component or mode");
  const KRun &k = R->k;
  const size_t plane = (size_t)k.plane;
  if (out_len < 2 * plane) return fail(PIC_E_NOMEM, "out holds %zu doubles, %zu needed", out_len, 2 * plane);
  const hipStream_t s = ctx->stream;
  const bool f64 = ctx->prec == PIC_PREC_FP64;
  const int NM = 2 * k.M + 1;
  const int qa = m == 0 ? 0 : 2 * m - 1, qb = 2 * m;
  const int par = (int)(R->steps & 1);
  TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
  // copy the (Re, Im) planes of mode m of one component
  std::vector<double> re(plane, 0.0), im(plane, 0.0);
  auto read_plane = [&](const void *base, int c, int q, bool is_f64, std::vector<double> &dst) -> int {
    if (is_f64) {
      const double *src = (const double *)base + ((size_t)c * NM + q) * plane;
      return hip_ok(hipMemcpy(dst.data(), src, plane * 8, hipMemcpyDeviceToHost), "hipMemcpy D2H");
    }
    std::vector<float> t(plane);
    const float *src = (const float *)base + ((size_t)c * NM + q) * plane;
    int rc = hip_ok(hipMemcpy(t.data(), src, plane * 4, hipMemcpyDeviceToHost), "hipMemcpy D2H");
    for (size_t a = 0; a < plane; ++a) dst[a] = t[a];
    return rc;
  };
  auto read_comp = [&](const void *base, int c, bool is_f64) -> int {
    int rc = read_plane(base, c, qa, is_f64, re);
    if (rc == PIC_OK && m > 0) rc = read_plane(base, c, qb, is_f64, im);
    return rc;
  };
  const void *src = nullptr;
  int c = 0;
  bool cur = false, rho = false;
  if (comp <= PIC_EZ) { src = k.E; c = comp; }
  else if (comp <= PIC_BZ) { src = k.Bbar; c = comp - PIC_BR; }
  else if (comp <= PIC_JZ) { src = k.J[(R->steps + 1) & 1]; c = comp - PIC_JR; cur = true; }
  else if (comp == PIC_RHO) { rho = true; }
  else if (comp <= PIC_BZ_OLD) { src = k.B[par]; c = comp - PIC_BR_OLD; }
  else { src = k.B[par ^ 1]; c = comp - PIC_BR_NEW; }
  if (rho) {
    TRY(launch_zero(k.rho, (size_t)NM * plane * 8, s));
    TRY(launch_rho(k, ctx->prec, s));
    TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
    TRY(read_comp(k.rho, 0, true));
  } else {
    TRY(read_comp(src, c, f64));
    if (cur) {  // physical current = raw deposit * row factor
      const double dz = k.dz, dr = k.dr, dt = k.dt;
      for (int j = 0; j <= k.Nr; ++j) {
        const double Vj = j == 0 ? kPi * dr * dr * dz / 4.0 : 2.0 * kPi * (j * dr) * dr * dz;
        double f;
        if (c == 0) f = 1.0 / (dt * 2.0 * kPi * ((j + 0.5) * dr) * dz);
        else if (c == 2) f = 1.0 / (dt * (Vj / dz));
        else f = (m == 0 || j == 0) ? 1.0 / Vj : 1.0 / (dt * 2.0 * kPi * dr * dz);
        // the m >= 1 J_z vanishes on the axis (E_z^m is held at zero there)
        if (c == 2 && m > 0 && j == 0) f = 0.0;
        for (int i = 0; i < k.Nz; ++i) {
          re[(size_t)j * k.Nz + i] *= f;
          im[(size_t)j * k.Nz + i] *= f;
        }
      }
    }
  }
  for (size_t a = 0; a < plane; ++a) {
    out[2 * a] = re[a];
    out[2 * a + 1] = im[a];
  }
  return PIC_OK;
}

int pic_particles(pic_ctx *ctx, int32_t run, double *z, double *x, double *y, double *ux, double *uy, double *uz,
                  double *w, int64_t *id, size_t out_len) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  RunHost *R = get_run(ctx, run);
  if (!R) return fail(PIC_E_INVALID, "bad run index");
  TRY(check_sort_flags(ctx));
  const KRun &k = R->k;
  const size_t np = (size_t)k.np;
  if (out_len < np) return fail(PIC_E_NOMEM, "buffers hold %zu, %zu needed", out_len, np);
  TRY(hip_ok(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"));
  const bool f64 = ctx->prec == PIC_PREC_FP64;
  auto get = [&](const void *src, double *dst) -> int {
    if (!dst || np == 0) return PIC_OK;
    if (f64) return hip_ok(hipMemcpy(dst, src, np * 8, hipMemcpyDeviceToHost), "D2H");
    std::vector<float> t(np);
    int rc = hip_ok(hipMemcpy(t.data(), src, np * 4, hipMemcpyDeviceToHost), "D2H");
    for (size_t a = 0; a < np; ++a) dst[a] = t[a];
    return rc;
  };
  if (z && np) {
    if (f64) TRY(hip_ok(hipMemcpy(z, k.pz, np * 8, hipMemcpyDeviceToHost), "D2H"));
    else {
      std::vector<int32_t> iz(np);
      std::vector<float> fz(np);
      TRY(hip_ok(hipMemcpy(iz.data(), k.pz, np * 4, hipMemcpyDeviceToHost), "D2H"));
      TRY(hip_ok(hipMemcpy(fz.data(), k.pfz, np * 4, hipMemcpyDeviceToHost), "D2H"));
      for (size_t a = 0; a < np; ++a) z[a] = (double)iz[a] + (double)fz[a];
    }
  }
  TRY(get(k.px, x));
  TRY(get(k.py, y));
  TRY(get(k.pux, ux));
  TRY(get(k.puy, uy));
  TRY(get(k.puz, uz));
  TRY(get(k.pw, w));
  if (id && np) {
    std::vector<uint32_t> t(np);
    TRY(hip_ok(hipMemcpy(t.data(), k.pid, np * 4, hipMemcpyDeviceToHost), "D2H"));
    for (size_t a = 0; a < np; ++a) id[a] = (int64_t)(t[a] & kIdMask);
  }
  return PIC_OK;
}

int pic_mode_work(pic_ctx *ctx, int32_t run, double *work, double *gamma, double *gamma_acc, int64_t *ids,
                  double *field_energy, double *kinetic) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  RunHost *R = get_run(ctx, run);
  if (!R) return fail(PIC_E_INVALID, "bad run index");
  TRY(check_sort_flags(ctx));
  const KRun &k = R->k;
  const hipStream_t s = ctx->stream;
  const int M = k.M;
  const int nt = k.n_tracked;
  bool finite = true;
  std::vector<double> W((size_t)nt * (M + 1));
  if (nt > 0) {
    // ids of tracked electrons not in the box (dropped by a moving window) stay -1
    TRY(hip_ok(hipMemsetAsync(R->dev_ids, 0xff, (size_t)nt * 8, s), "hipMemsetAsync"));
    TRY(launch_tracked_gamma(k, ctx->prec, R->dev_gamma, R->dev_ids, s));
    TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
    TRY(hip_ok(hipMemcpy(W.data(), k.W, W.size() * 8, hipMemcpyDeviceToHost), "D2H"));
    std::vector<double> g((size_t)nt);
    std::vector<int64_t> id((size_t)nt);
    TRY(hip_ok(hipMemcpy(g.data(), R->dev_gamma, (size_t)nt * 8, hipMemcpyDeviceToHost), "D2H"));
    TRY(hip_ok(hipMemcpy(id.data(), R->dev_ids, (size_t)nt * 8, hipMemcpyDeviceToHost), "D2H"));
    for (int t = 0; t < nt; ++t) {
      double acc = R->gam0[(size_t)t];
      for (int m = 0; m <= M; ++m) acc += W[(size_t)t * (M + 1) + m];
      const bool present = id[(size_t)t] >= 0;
      if (!std::isfinite(acc) || (present && !std::isfinite(g[(size_t)t]))) finite = false;
      if (gamma_acc) gamma_acc[t] = acc;
      if (gamma) gamma[t] = present ? g[(size_t)t] : std::nan("");
      if (ids) ids[t] = R->tr_ids[(size_t)t];
    }
    if (work) std::memcpy(work, W.data(), W.size() * 8);
  }
  if (field_energy) {
    int nb = 0;
    TRY(launch_energy(k, ctx->prec, (int)(R->steps & 1), kRedBlocks, &nb, s));
    std::vector<double> part((size_t)nb * (M + 1));
    TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
    TRY(hip_ok(hipMemcpy(part.data(), k.red, part.size() * 8, hipMemcpyDeviceToHost), "D2H"));
    for (int m = 0; m <= M; ++m) {
      double acc = 0.0;
      for (int b = 0; b < nb; ++b) acc += part[(size_t)b * (M + 1) + m];
      field_energy[m] = acc;
      if (!std::isfinite(acc)) finite = false;
    }
  }
  if (kinetic) {
    int nb = 0;
    TRY(launch_kinetic(k, ctx->prec, &nb, s));
    std::vector<double> part((size_t)nb);
    TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
    TRY(hip_ok(hipMemcpy(part.data(), k.red, part.size() * 8, hipMemcpyDeviceToHost), "D2H"));
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[(size_t)b];
    *kinetic = acc;
    if (!std::isfinite(acc)) finite = false;
  }
  if (!finite) return fail(PIC_E_NUMERIC, "a diagnostic reduction is not finite");
  return PIC_OK;
}

int pic_cartesian_work(pic_ctx *ctx, int32_t run, double *wz, double *wperp, double *f, double *w_lwfa,
                       double *w_dla) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  RunHost *R = get_run(ctx, run);
  if (!R) return fail(PIC_E_INVALID, "bad run index");
  TRY(check_sort_flags(ctx));
  const KRun &k = R->k;
  const pic_run_desc &d = R->d;
  const bool need_f = f || w_lwfa || w_dla;
  if (need_f && (d.n_pulses < 1 || !(d.n0 > 0) || !(d.pulse[0].w0 > 0)))
    return fail(PIC_E_INVALID, "the Pukhov ratio needs a pulse with w0 > 0 and n0 > 0");
  const int nt = k.n_tracked;
  if (nt == 0) return PIC_OK;
  const hipStream_t s = ctx->stream;
  std::vector<double> Wc((size_t)nt * 2), g((size_t)nt);
  if (need_f) TRY(launch_tracked_gamma(k, ctx->prec, R->dev_gamma, R->dev_ids, s));
  TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
  TRY(hip_ok(hipMemcpy(Wc.data(), k.Wc, Wc.size() * 8, hipMemcpyDeviceToHost), "D2H"));
  if (need_f) TRY(hip_ok(hipMemcpy(g.data(), R->dev_gamma, (size_t)nt * 8, hipMemcpyDeviceToHost), "D2H"));
  const double c = need_f ? -2.0 / (std::sqrt(d.n0) * d.pulse[0].w0 * d.pulse[0].w0) : 0.0;
  bool finite = true;
  for (int t = 0; t < nt; ++t) {
    const double a = Wc[2 * (size_t)t], b = Wc[2 * (size_t)t + 1];
    if (wz) wz[t] = a;
    if (wperp) wperp[t] = b;
    if (!std::isfinite(a) || !std::isfinite(b)) finite = false;
    if (!need_f) continue;
    const double ft = c * std::sqrt(2.0 * g[(size_t)t]);
    if (!std::isfinite(ft)) finite = false;
    if (f) f[t] = ft;
    if (w_lwfa) w_lwfa[t] = a - ft * b;
    if (w_dla) w_dla[t] = (1.0 + ft) * b;
  }
  if (!finite) return fail(PIC_E_NUMERIC, "a work value is not finite");
  return PIC_OK;
}

int pic_divergence(pic_ctx *ctx, int32_t run, double gamma_min, double *out) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  RunHost *R = get_run(ctx, run);
  if (!R) return fail(PIC_E_INVALID, "bad run index");
  TRY(check_sort_flags(ctx));
  if (!out) return fail(PIC_E_INVALID, "out is NULL");
  if (!(gamma_min >= 1.0) || !std::isfinite(gamma_min)) return fail(PIC_E_INVALID, "gamma_min must be >= 1");
  const KRun &k = R->k;
  const hipStream_t s = ctx->stream;
  int nb = 0;
  static_assert(PIC_MAX_MODES + 1 >= 4, "the reduction buffer holds 4 sums per block");
  TRY(launch_divergence(k, ctx->prec, gamma_min * gamma_min - 1.0, kRedBlocks, &nb, s));
  std::vector<double> part((size_t)nb * 4);
  TRY(hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"));
  TRY(hip_ok(hipMemcpy(part.data(), k.red, part.size() * 8, hipMemcpyDeviceToHost), "D2H"));
  for (int c = 0; c < 4; ++c) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[(size_t)b * 4 + c];
    out[c] = acc;
    if (!std::isfinite(acc)) return fail(PIC_E_NUMERIC, "a divergence sum is not finite");
  }
  // charge-weighted RMS angles; 0 when no electron passes the cut
  out[4] = out[0] > 0 ? std::sqrt(out[1] / out[0]) : 0.0;
  out[5] = out[0] > 0 ? std::sqrt(out[2] / out[0]) : 0.0;
  return PIC_OK;
}

int pic_dla_integrate(const pic_dla_model *model, int64_t n, const double *t0, double *x, double *zeta, double *xd,
                      double *zetad, double t_end, double h, void *hip_stream) {
  g_msg[0] = 0;
  if (!model || n < 0 || (n > 0 && (!t0 || !x || !zeta || !xd || !zetad)))
    return fail(PIC_E_INVALID, "bad arrays or count");
  if (!(h > 0) || !std::isfinite(h) || !std::isfinite(t_end)) return fail(PIC_E_INVALID, "bad step or end time");
  const pic_dla_model &m = *model;
  if (!(m.kz > 0) || !std::isfinite(m.kz) || !(m.vphi >= 1.0) || !std::isfinite(m.vphi) || !std::isfinite(m.a0) ||
      !std::isfinite(m.cB) || !std::isfinite(m.wake))
    return fail(PIC_E_INVALID, "model out of range (kz > 0, vphi >= 1, finite factors)");
  TRY(launch_dla(m, (long long)n, t0, x, zeta, xd, zetad, t_end, h, hip_stream));
  return PIC_OK;
}

// ---- checkpoint / restore --------------------------------------------------
// Layout: header, then per run its descriptor, step count, initial tracked
// gamma and coefficients (for validation), then the device state in a fixed
// order: E, B at both half steps, Bbar, both J buffers, rho, the particle
// arrays in their current (sorted) order, the tile ranges of the last sort,
// and the tracked work.

}  // extern "C"

namespace {

struct CkptHeader {
  char magic[8];
  int32_t version, n_runs, precision, tile_z, tile_r, sort_interval, current, deterministic, shape;
};

struct Seg {
  void *dev;
  size_t bytes;
};

std::vector<Seg> state_segments(const RunHost &R, int prec) {
  const KRun &k = R.k;
  const pic_run_desc &d = R.d;
  const size_t rs = prec == PIC_PREC_FP64 ? 8 : 4;
  const size_t NM = (size_t)(2 * d.M + 1);
  const size_t vec = 3 * NM * (size_t)k.plane * rs;
  const size_t np = (size_t)k.np;
  const size_t nt = (size_t)(d.n_tracked > 0 ? d.n_tracked : 0);
  std::vector<Seg> s = {{k.E, vec}, {k.B[0], vec}, {k.B[1], vec}, {k.Bbar, vec}, {k.J[0], vec}, {k.J[1], vec},
                        {k.rho, NM * (size_t)k.plane * 8}, {k.pz, np * (prec == PIC_PREC_FP64 ? 8 : 4)}};
  if (prec != PIC_PREC_FP64) s.push_back({k.pfz, np * 4});
  for (void *p : {k.px, k.py, k.pux, k.puy, k.puz, k.pw}) s.push_back({p, np * rs});
  s.push_back({k.pid, np * 4});
  s.push_back({k.cell_start, (size_t)(k.n_keys + 1) * 4});
  s.push_back({k.W, nt * (size_t)(d.M + 1) * 8});
  s.push_back({k.Wc, nt * 2 * 8});
  return s;
}

size_t run_meta_bytes(const RunHost &R) {
  return sizeof(pic_run_desc) + sizeof(int64_t) + (R.gam0.size() + R.CE.size() + R.CB.size()) * sizeof(double);
}

size_t checkpoint_bytes(pic_ctx *ctx) {
  size_t n = sizeof(CkptHeader);
  for (const RunHost &R : ctx->runs) {
    n += run_meta_bytes(R);
    for (const Seg &g : state_segments(R, ctx->prec)) n += g.bytes;
  }
  return n;
}

CkptHeader header_of(pic_ctx *ctx) {
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, "PICCKPT1", 8);
  h.version = 4;
  h.n_runs = (int32_t)ctx->runs.size();
  h.precision = ctx->prec;
  h.tile_z = ctx->runs.empty() ? 0 : ctx->runs[0].k.Tz;
  h.tile_r = ctx->runs.empty() ? 0 : ctx->runs[0].k.Tr;
  h.sort_interval = ctx->sort_interval;
  h.current = ctx->current;
  h.deterministic = ctx->det ? 1 : 0;
  h.shape = ctx->shape;
  return h;
}

}  // namespace

extern "C" {

int pic_checkpoint(pic_ctx *ctx, void *host_buf, size_t *bytes) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  if (ctx->win_K > 0) return fail(PIC_E_INVALID, "no checkpoint of a moving-window context");
  TRY(check_sort_flags(ctx));
  if (!bytes) return fail(PIC_E_INVALID, "bytes is NULL");
  const size_t need = checkpoint_bytes(ctx);
  if (!host_buf) {
    *bytes = need;
    return PIC_OK;
  }
  if (*bytes < need) return fail(PIC_E_NOMEM, "buffer of %zu bytes, %zu needed", *bytes, need);
  TRY(hip_ok(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"));
  unsigned char *o = (unsigned char *)host_buf;
  const CkptHeader h = header_of(ctx);
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  for (const RunHost &R : ctx->runs) {
    std::memcpy(o, &R.d, sizeof(pic_run_desc));
    o += sizeof(pic_run_desc);
    std::memcpy(o, &R.steps, sizeof(int64_t));
    o += sizeof(int64_t);
    for (const std::vector<double> *v : {&R.gam0, &R.CE, &R.CB}) {
      if (!v->empty()) std::memcpy(o, v->data(), v->size() * sizeof(double));
      o += v->size() * sizeof(double);
    }
    for (const Seg &g : state_segments(R, ctx->prec)) {
      if (g.bytes) TRY(hip_ok(hipMemcpy(o, g.dev, g.bytes, hipMemcpyDeviceToHost), "D2H"));
      o += g.bytes;
    }
  }
  *bytes = need;
  return PIC_OK;
}

int pic_restore(pic_ctx *ctx, const void *host_buf, size_t bytes) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  if (ctx->win_K > 0) return fail(PIC_E_INVALID, "no restore into a moving-window context");
  if (!host_buf) return fail(PIC_E_INVALID, "buffer is NULL");
  const size_t need = checkpoint_bytes(ctx);
  if (bytes != need) return fail(PIC_E_INVALID, "checkpoint of %zu bytes, this context takes %zu", bytes, need);
  const unsigned char *p = (const unsigned char *)host_buf;
  const CkptHeader h = header_of(ctx);
  if (std::memcmp(p, &h, sizeof h) != 0)
    return fail(PIC_E_INVALID,
                "checkpoint header does not match this context (version, runs, precision, tile, interval, current, "
                "deterministic mode, shape order)");
  // validate every run before any device copy
  const unsigned char *q = p + sizeof h;
  for (const RunHost &R : ctx->runs) {
    if (std::memcmp(q, &R.d, sizeof(pic_run_desc)) != 0) return fail(PIC_E_INVALID, "run descriptors differ");
    q += sizeof(pic_run_desc) + sizeof(int64_t) + R.gam0.size() * sizeof(double);
    for (const std::vector<double> *v : {&R.CE, &R.CB}) {
      if (!v->empty() && std::memcmp(q, v->data(), v->size() * sizeof(double)) != 0)
        return fail(PIC_E_INVALID, "solver coefficients differ");
      q += v->size() * sizeof(double);
    }
    for (const Seg &g : state_segments(R, ctx->prec)) q += g.bytes;
  }
  TRY(hip_ok(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"));
  q = p + sizeof h;
  for (RunHost &R : ctx->runs) {
    q += sizeof(pic_run_desc);
    std::memcpy(&R.steps, q, sizeof(int64_t));
    q += sizeof(int64_t);
    if (!R.gam0.empty()) std::memcpy(R.gam0.data(), q, R.gam0.size() * sizeof(double));
    q += (R.gam0.size() + R.CE.size() + R.CB.size()) * sizeof(double);
    for (const Seg &g : state_segments(R, ctx->prec)) {
      if (g.bytes) TRY(hip_ok(hipMemcpy(g.dev, q, g.bytes, hipMemcpyHostToDevice), "H2D"));
      q += g.bytes;
    }
  }
  return PIC_OK;
}

int pic_destroy(pic_ctx *ctx) {
  g_msg[0] = 0;
  if (!ctx_ok(ctx)) return fail(PIC_E_STATE, "invalid or destroyed context");
  ctx_unregister(ctx);
  ctx->magic = 0;
  delete ctx;
  return PIC_OK;
}

}  // extern "C"
