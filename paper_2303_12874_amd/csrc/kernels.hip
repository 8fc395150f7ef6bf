// kernels.hip -- gfx950 kernels of the quasi-3D r-z PIC step with the dual
// Maxwell solver (arXiv 2303.12874, Sec. III).  One step of a run is
//   push:   per sort tile, gather E^n and Bbar^n = (B^{n-1/2} + B^{n+1/2})/2
//           (Eq. (12)) at each electron, Boris push (Eq. (6)), per-mode work
//           of tracked electrons (Eq. (16)), move, charge-conserving deposit
//           of J^{n+1/2} into an LDS window, flushed once per tile;
//   efield: E^{n+1} = E^n + dt (curl_B B^{n+1/2} - J'), J' = (P J_r, P J_phi, J_z)
//           with the z filter P that makes the two-point continuity of the
//           deposit hold for D_B (Gauss's law with [k]_B, Eq. (10));
//           also clears the other current buffer;
//   bfield: B^{n+3/2} = B^{n+1/2} - dt curl_E E^{n+1}, into the buffer that
//           held B^{n-1/2}, and Bbar^{n+1} for the next gather.
//
// Field layout: for component c, mode plane q holds (Nr+1) x Nz reals, z
// fastest, at (c * NM + q) * (Nr+1) * Nz; NM = 2M+1 planes: q = 0 is Re of
// m = 0, q = 2m-1 and 2m are Re and Im of mode m >= 1.  Threads of a
// wavefront sit in consecutive cells (columns), so every plane read is one
// coalesced row segment.  Inside the kernels a node is handled as a record
// of NMP = 2(M+1) reals, (Re, Im) of every mode with Im of m = 0 zero.
// A quantity at z_{i+1/2} is stored at column i, one at r_{j+1/2} at row j.
//
// Every global index is clamped or wrapped into its array, whatever the
// particle data hold, so corrupted particles give NaN fields, not faults.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "pic_internal.h"

namespace pic {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kFieldTile = 128;  // z-columns per field-update workgroup
constexpr int kSortLdsEntries = 4608;  // sort entries of a tile held in LDS (36 KB, with their 9 KB of ranks)
constexpr int kSortRankPerCell = 8;    // mean entries per cell above which a tile's cells are ranked in parallel
constexpr int kDealBlock = 64;         // consecutive tiles dealt to one XCD's ticket counter
constexpr int kDealMinPerGroup = 32;   // tiles per resident workgroup from which tiles are dealt per XCD

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

// Element i of a particle array as a uniform base plus a 32-bit byte offset,
// so that a load or store needs no 64-bit address arithmetic per lane
// (pic_init keeps every particle array under 2^32 bytes).
template <typename T>
__device__ __forceinline__ T &elem(void *base, int i) {
  return *(T *)((char *)base + (unsigned)i * (unsigned)sizeof(T));
}

// Electrons of a tile are stored transposed: with n electrons in (cell, id)
// order L[0..n) and chunk = ceil(n / 256), list column c holds L[c chunk +
// it] for it = 0, 1, ..., and round `it` of the tile's workgroup takes the
// round_count(n, chunk, it) electrons of its columns from consecutive slots,
// thread t the slot t.  round_count = electrons (active threads) of round it.
__device__ __forceinline__ int round_count(int n, int chunk, int it) {
  if (it >= n) return 0;
  const int c = (n - 1 - it) / chunk + 1;
  return c < 256 ? c : 256;
}

// The slots of a round do not hold the columns in their order: slot o holds
// column round_column(o, cnt, S), the columns c = S l + w (w < S) grouped by
// w, l rising.  With S at least the number of columns per cell, the 64 lanes
// of a wavefront (64 consecutive slots, of one w in a full round; a partly
// filled round's wavefront can span two) are in distinct cells, so that
// their LDS atomics do not collide on one address, and every particle load
// and store of a wavefront is one contiguous run of slots.
__device__ __forceinline__ int round_spread(int n, int chunk, long long TT) {
  int S = 1;
  while (S < 4 && (long long)S * chunk * TT < n) S *= 2;
  return S;
}
__device__ __forceinline__ int round_column(int o, int cnt, int S) {
  int w = 0, pre = 0;
  for (; w < S - 1; ++w) {
    const int cw = (cnt - w + S - 1) / S;  // columns S l + w below cnt
    if (o < pre + cw) break;
    pre += cw;
  }
  return S * (o - pre) + w;
}

// largest integer j with j^2 <= r2 (r = sqrt(r2) rounded)
template <typename R>
__device__ __forceinline__ int radial_index(R r2, R r) {
  int j = (int)floor(r);
  if ((R)j * (R)j > r2) j -= 1;
  if ((R)(j + 1) * (R)(j + 1) <= r2) j += 1;
  return j;
}

// 1/sqrt(x) and 1/x for x > 0 from the hardware estimates: FP32 as they are
// (about an ulp), FP64 with one Newton step (close to correct rounding).  One
// reciprocal square root replaces a square root and a division.
template <typename R>
__device__ __forceinline__ R rsqrt_hw(R x) {
  if constexpr (std::is_same<R, double>::value) {
    const double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x * y;
    return fma(y, fma(-h, y, 0.5), y);
  } else {
    return __builtin_amdgcn_rsqf(x);
  }
}
template <typename R>
__device__ __forceinline__ R rcp_hw(R x) {
  if constexpr (std::is_same<R, double>::value) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
  } else {
    return __builtin_amdgcn_rcpf(x);
  }
}

// Relaxed hardware float atomics (no denormal-mode emulation).  The LDS and
// the global forms use different scopes so that the compiler never merges a
// workgroup-local and a device-memory update into one flat-address atomic.
template <typename R>
__device__ __forceinline__ void atomic_add(R *a, R v) {  // device memory
  [[clang::atomic(no_remote_memory, no_fine_grained_memory, ignore_denormal_mode)]] {
    __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}
template <typename R>
__device__ __forceinline__ void lds_add(R *a, R v) {  // LDS
  [[clang::atomic(ignore_denormal_mode)]] {
    __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Deterministic mode: a scaled contribution w c (|w c| < 2^30) as the integer
// pair a = rint(w c), b = rint((w c - a) 2^31), the remainder taken from the
// exact product by an explicit fma (an expression the compiler may contract
// differently in each place it is inlined would round differently), added to
// a pair of 64-bit integer sums (two's complement, so that negative parts
// wrap correctly).  Integer addition is associative: the sums do not depend
// on the order the atomics run in.
__device__ __forceinline__ void fix_split(double w, double c, unsigned long long &a, unsigned long long &b) {
  const double ra = rint(w * c);
  const double rb = rint(fma(w, c, -ra) * 2147483648.0);  // |w c - ra| <= 1/2 + ulp
  a = (unsigned long long)(long long)(int)ra;
  b = (unsigned long long)(long long)(int)rb;
}
__device__ __forceinline__ void fix_add_lds(unsigned long long *p, double w, double c) {
  unsigned long long a, b;
  fix_split(w, c, a, b);
  __hip_atomic_fetch_add(p, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_add(p + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void fix_add_global(unsigned long long *p, unsigned long long a, unsigned long long b) {
  if (a) __hip_atomic_fetch_add(p, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (b) __hip_atomic_fetch_add(p + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- node records -----------------------------------------------------------
// A record of NMP reals starts at a multiple of its own size from a 256-byte
// aligned base, so it is 16-byte aligned when its size is a multiple of 16
// (always for FP64; FP32 with M odd) and 8-byte aligned otherwise.
template <typename R, int NMP>
struct RecVec {
  static constexpr int bytes = NMP * (int)sizeof(R);
  static constexpr int vbytes = (bytes % 16 == 0) ? 16 : 8;
  static constexpr int per = vbytes / (int)sizeof(R);  // reals per vector
  static constexpr int nv = NMP / per;
  using V = typename std::conditional<sizeof(R) == 8, double2,
                                      typename std::conditional<vbytes == 16, float4, float2>::type>::type;
};

template <typename R, int NMP>
__device__ __forceinline__ void store_rec(R *__restrict__ p, const R in[NMP]) {
  using T = RecVec<R, NMP>;
  typename T::V *q = reinterpret_cast<typename T::V *>(p);
#pragma unroll
  for (int a = 0; a < T::nv; ++a) {
    typename T::V x;
    R *xs = reinterpret_cast<R *>(&x);
#pragma unroll
    for (int b = 0; b < T::per; ++b) xs[b] = in[a * T::per + b];
    q[a] = x;
  }
}

// A node of one component from the mode planes (stride `plane`): record slot
// s = 2m (Re), 2m+1 (Im); slot 1 (Im of m = 0) is not stored.  I is the index
// type: 64-bit for device memory, 32-bit for LDS.
template <typename R, int NMP, typename I = long long>
__device__ __forceinline__ void load_node(const R *__restrict__ F, I plane, I node, R out[NMP]) {
  out[0] = F[node];
  out[1] = R(0);
#pragma unroll
  for (int s = 2; s < NMP; ++s) out[s] = F[(s - 1) * plane + node];
}
template <typename R, int NMP>
__device__ __forceinline__ void store_node(R *__restrict__ F, long long plane, long long node, const R in[NMP]) {
  F[node] = in[0];
#pragma unroll
  for (int s = 2; s < NMP; ++s) F[(s - 1) * plane + node] = in[s];
}

// the NMP reals of one component of an LDS field-window record (Re, Im of
// each mode; Im of m = 0 is stored as zero), read as vectors of VB bytes
template <typename R, int NMP, int VB>
__device__ __forceinline__ void load_rec(const R *__restrict__ p, R out[NMP]) {
  constexpr int VR = VB / (int)sizeof(R);
  typedef R V __attribute__((ext_vector_type(VR)));
  static_assert(VR >= 2 && NMP % VR == 0, "record vectors");
#pragma unroll
  for (int k = 0; k < NMP / VR; ++k) {
    const V x = *(const V *)(p + k * VR);
#pragma unroll
    for (int j = 0; j < VR; ++j) out[k * VR + j] = x[j];
  }
}
template <typename R, int N, int VB>
__device__ __forceinline__ void store_rec(R *__restrict__ p, const R in[N]) {
  constexpr int VR = VB / (int)sizeof(R);
  typedef R V __attribute__((ext_vector_type(VR)));
  static_assert(VR >= 2 && N % VR == 0, "record vectors");
#pragma unroll
  for (int k = 0; k < N / VR; ++k) {
    V x;
#pragma unroll
    for (int j = 0; j < VR; ++j) x[j] = in[k * VR + j];
    *(V *)(p + k * VR) = x;
  }
}

// mirror sign of mode m at r_{-1/2}: (-1)^{m+1} for r and phi components,
// (-1)^m for z components (the point (-r, phi) is (r, phi + pi)).
__host__ __device__ constexpr int mirror_sign_m(int m, bool zcomp) { return ((m % 2 == 0) == zcomp) ? 1 : -1; }

// Bilinear interpolation of one component (all modes) from four nodes: pa,
// pb on the lower row (columns ca, cb), pc, pd on the upper row.  VB = 0:
// device memory, plane q of the component at offset q * pstride (Im of m = 0
// not stored); VB > 0: an LDS field-window record component (load_rec).
// With `mirror` the lower row is the image of r_{-1/2} (pa, pb point at row
// r_{1/2}) and each mode takes its mirror sign.
template <typename R, int NMP, bool HALF_R, bool ZCOMP, typename I, int VB = 0>
__device__ __forceinline__ void interp4(const R *pa, const R *pb, const R *pc, const R *pd, I pstride,
                                        bool mirror, R fz, R fr, R out[NMP]) {
  const R w00 = (R(1) - fz) * (R(1) - fr), w10 = fz * (R(1) - fr);
  const R w01 = (R(1) - fz) * fr, w11 = fz * fr;
  // lower-row weights of the modes whose mirror sign is -1
  const R n00 = (HALF_R && mirror) ? -w00 : w00, n10 = (HALF_R && mirror) ? -w10 : w10;
  R a[NMP], b[NMP], c[NMP], d[NMP];
  if constexpr (VB > 0) {
    load_rec<R, NMP, VB>(pa, a);
    load_rec<R, NMP, VB>(pb, b);
    load_rec<R, NMP, VB>(pc, c);
    load_rec<R, NMP, VB>(pd, d);
  } else {
    load_node<R, NMP, I>(pa, pstride, 0, a);
    load_node<R, NMP, I>(pb, pstride, 0, b);
    load_node<R, NMP, I>(pc, pstride, 0, c);
    load_node<R, NMP, I>(pd, pstride, 0, d);
  }
  out[1] = R(0);  // Im of m = 0
#pragma unroll
  for (int s = 0; s < NMP; ++s) {
    if (s == 1) continue;
    const bool neg = HALF_R && mirror_sign_m(s / 2, ZCOMP) < 0;
    out[s] = (neg ? n00 : w00) * a[s] + (neg ? n10 : w10) * b[s] + w01 * c[s] + w11 * d[s];
  }
}

// Quadratic B-spline weights of the three nodes round the nearest node, d
// the offset from that node in cells (in [-1/2, 1/2]).
template <typename R>
__device__ __forceinline__ void qspline(R d, R w[3]) {
  const R lo = R(0.5) - d, hi = R(0.5) + d;
  w[0] = R(0.5) * lo * lo;
  w[1] = R(0.75) - d * d;
  w[2] = R(0.5) * hi * hi;
}

// Quadratic interpolation of one component (all modes) from the 3 x 3
// records of an LDS field window: node (a, b) of the stencil at
// p + b rstride + a nstride (p points at the component in the first node).
// Rows below the axis were staged as mirror images, so no axis rule applies.
template <typename R, int NMP, int VB>
__device__ __forceinline__ void interp9(const R *p, int rstride, int nstride, const R wz[3], const R wr[3],
                                        R out[NMP]) {
#pragma unroll
  for (int s = 0; s < NMP; ++s) out[s] = R(0);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    R t[NMP];
#pragma unroll
    for (int s = 0; s < NMP; ++s) t[s] = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R v[NMP];
      if constexpr (VB > 0) load_rec<R, NMP, VB>(p + b * rstride + a * nstride, v);
      else load_node<R, NMP, int>(p + b * rstride + a * nstride, 1, 0, v);
#pragma unroll
      for (int s = 0; s < NMP; ++s) t[s] += wz[a] * v[s];
    }
#pragma unroll
    for (int s = 0; s < NMP; ++s) out[s] += wr[b] * t[s];
  }
  out[1] = R(0);  // Im of m = 0
}

// The same from device memory (mode planes of stride `plane`): columns c0 ..
// c0+2 (periodic), rows r0 .. r0+2 of the component's radial grid; a row
// below the axis reads its mirror image (integer grid r_{-j} -> r_j, half
// grid r_{-j-1/2} -> r_{j-1/2}) times each mode's mirror sign.
template <typename R, int NMP, bool HALF_R, bool ZCOMP>
__device__ __forceinline__ void interp9_global(const R *F, long long plane, int Nz, int Nr, int c0, int r0,
                                               const R wz[3], const R wr[3], R out[NMP]) {
  int col[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) col[a] = wrap_any(c0 + a, Nz);
#pragma unroll
  for (int s = 0; s < NMP; ++s) out[s] = R(0);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    int row = r0 + b;
    const bool mir = row < 0;
    if (mir) row = HALF_R ? -row - 1 : -row;
    row = clampi(row, 0, Nr);
    R t[NMP];
#pragma unroll
    for (int s = 0; s < NMP; ++s) t[s] = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R v[NMP];
      load_node<R, NMP>(F, plane, (long long)row * Nz + col[a], v);
#pragma unroll
      for (int s = 0; s < NMP; ++s) t[s] += wz[a] * v[s];
    }
#pragma unroll
    for (int s = 0; s < NMP; ++s) out[s] += ((mir && mirror_sign_m(s / 2, ZCOMP) < 0) ? -wr[b] : wr[b]) * t[s];
  }
  out[1] = R(0);
}

// run of a batch that owns block g of the launch
__device__ __forceinline__ int batch_run(const Batch &b, long long g) {
  int r = 0;
#pragma unroll
  for (int i = 1; i < kMaxBatch; ++i) r += (i < b.n && g >= b.off[i]) ? 1 : 0;
  return r;
}

// One workgroup per sort tile of Tz x Tr cells.  The tile's electrons (the
// range the last cell sort assigned to it) are processed in contiguous
// per-thread chunks, spread so that the 64 lanes of a wavefront sit in
// distinct cells and their LDS atomics do not collide.  Two LDS windows, both
// node-major (all planes of a node contiguous, so that every component and
// mode offset is an immediate):
//  * E and Bbar over the tile's field window, staged once, which the gather
//    reads: one record per node of 6 components (E_r, E_phi, E_z, Bbar_r,
//    Bbar_phi, Bbar_z) of NMP reals each, read as vectors, and a pad;
//  * the current of the whole tile over the node window [z0-1, z0+Tz+2) x
//    [r0-1, r0+Tr+2) (every move of less than one cell from a cell of the
//    tile stays inside it), records of 3 NM FP64 sums, added to the global
//    arrays once.
// An electron that drifted out of either window since the last sort gathers
// from, or deposits to, global memory directly.
// DET (FP64 only): the deterministic mode, whose window and device sums are
// integer pairs (fix_split) instead of FP64 values.
// SH: the particle shape order, 1 linear (CIC) or 2 quadratic.
template <typename R, int M, bool DET, int SH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void push_kernel(const Batch bt) {
  constexpr int NM = 2 * M + 1;       // planes per component
  constexpr int NMP = 2 * (M + 1);    // reals per field record in registers
  constexpr int JS = 3 * NM;          // FP64 sums per current-window node
  constexpr bool F64 = std::is_same<R, double>::value;
  constexpr int PREC = F64 ? PIC_PREC_FP64 : PIC_PREC_FP32;
  constexpr int FS = field_node_reals(M, PREC);  // reals per field-window record
  constexpr int VB = field_vec_bytes(M, PREC);   // bytes per vector load of a record, 0: one real at a time
  constexpr int CR = field_comp_reals(M, PREC);  // reals per component of a record
  static_assert(CR == (VB ? NMP : NM), "record component");
  // The tile current is summed in FP64 for both precisions: the LDS FP64
  // atomic add is the fast one on gfx950 (ds_add_f32 costs about 20 times
  // ds_add_f64, and FP32 sums in LDS made the FP32 push several times
  // slower).  In the FP32 form a contribution is the FP64 product of an FP32
  // node weight and an FP32 mode coefficient, which is exact, so the FP64
  // arithmetic adds no precision to the FP32 inputs; it only keeps the sums
  // from rounding (the global current they are added to is FP32).
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double *lds = (double *)lds_raw;
  const int par = bt.par;
  const int TZ = bt.run[0].Tz, TR = bt.run[0].Tr;  // one sort tile for every run of a batch
  const int WZ = current_window_z(TZ, SH), WR = current_window_r(TR, SH);
  const long long TT = (long long)TZ * TR;
  static_assert(!DET || F64, "the deterministic mode is FP64 only");
  static_assert(SH == 1 || SH == 2, "shape order 1 or 2");
  constexpr int JW = DET ? 2 : 1;             // 8-byte words per current sum
  const int RJ = current_window_row(M, TZ, DET, SH);  // words per current-window row (padded)
  const int nlds = RJ * WR;
  const int FZ = field_window_z(TZ, SH), FR = field_window_r(TR, SH);
  const int RF = field_window_row(M, TZ, PREC, SH);  // reals per field-window row
  R *fw = (R *)(lds + field_window_offset_words(M, TZ, TR, DET, SH));  // 16-byte aligned

  // Persistent: each workgroup takes tiles (of all runs of the batch) from
  // ticket counters, zero before the launch, until none are left; the
  // dealing is dynamic, so tiles of uneven cost (the laser region) spread
  // evenly.  Tiles are in their order: run, then tile of the run, z fastest.
  // With deal_xcd they are cut into blocks of kDealBlock, and block b
  // belongs to counter b mod 8.  Workgroups are dispatched to the 8 XCDs
  // round-robin by block index, so a workgroup draws first from the counter
  // of its XCD: neighbouring tiles, which share field-window halo lines and
  // flushed current lines, then run on one XCD and meet in its L2.  A
  // workgroup whose counter is exhausted draws from the next ones in turn.
  // Otherwise (few tiles per workgroup, where the end of the launch weighs
  // more) one counter deals the tiles in their order.
  const int ntiles = (int)bt.off[bt.n];
  __shared__ int ticket;
  const int x0 = (int)(blockIdx.x & 7u);
  int xi = 0;  // (thread 0) counters found exhausted
  auto next_tile = [&]() -> int {
    if (!bt.deal_xcd) return atomicAdd(bt.run[0].work, 1);
    while (xi < 8) {
      const int x = (x0 + xi) & 7;
      const long long k = atomicAdd(bt.run[0].work + x, 1);
      const long long g = ((k / kDealBlock) * 8 + x) * kDealBlock + k % kDealBlock;
      if (g < ntiles) return (int)g;
      ++xi;  // every later ticket of this counter lies past the tiles too
    }
    return ntiles;
  };
  if (threadIdx.x == 0) ticket = next_tile();
  __syncthreads();
  int gt = ticket;
  const int t_hi = ntiles;
  // node e of the field window of tile g (run, then tile of the run): all
  // 6 NM planes, loaded together so that they are in flight at once
  auto stage_load = [&](int g, int e, R v[FS]) {
    const int rg = batch_run(bt, g);
    const KRun &kg = bt.run[rg];
    const int tl = g - (int)bt.off[rg];
    const int fz0g = (tl % kg.ntz) * TZ - 1 - kFieldMarginZ, fr0g = (tl / kg.ntz) * TR - 1 - kFieldMarginR;
    const int row = e / FZ, col = e - row * FZ;
    const int grow = fr0g + row;
    const bool ok = grow >= 0 && grow <= kg.Nr;
    const long long pl = kg.plane;
    // offset inside a plane (32-bit, so that each load is a uniform plane
    // base plus a per-lane offset); every address is valid (row clamped), so
    // the loads need no branch
    const int colw = wrap_any(fz0g + col, kg.Nz);
    const unsigned gg = (unsigned)((ok ? grow : 0) * kg.Nz + colw);
    // quadratic: row r_{-1} (the only row below the axis in the window) is
    // the image of r_1 for a component on the integer radial grid and r_{-1/2}
    // that of r_{1/2} for one on the half grid, times the mirror sign
    const bool mirror = SH == 2 && grow == -1;
    const R *Eg = (const R *)kg.E, *Bg = (const R *)kg.Bbar;
#pragma unroll
    for (int i = 0; i < FS; ++i) v[i] = R(0);  // the pad (and Im of m = 0 in the vector records)
#pragma unroll
    for (int cq = 0; cq < 6 * NM; ++cq) {
      const int c = cq / NM, q = cq % NM;
      if constexpr (SH == 2) {
        const bool half_r = c == 0 || c == 4 || c == 5;  // E_r, B_phi, B_z
        const bool zcomp = c == 2 || c == 5;
        const unsigned at = mirror ? (unsigned)((half_r ? 0 : kg.Nz) + colw) : gg;
        const R t = ((c < 3 ? Eg : Bg) + ((c % 3) * NM + q) * pl)[at];
        const R sg = mirror && mirror_sign_m((q + 1) / 2, zcomp) < 0 ? R(-1) : R(1);
        v[c * CR + ((VB && q > 0) ? q + 1 : q)] = (ok || mirror) ? sg * t : R(0);
      } else {
        const R t = ((c < 3 ? Eg : Bg) + ((c % 3) * NM + q) * pl)[gg];
        v[c * CR + ((VB && q > 0) ? q + 1 : q)] = ok ? t : R(0);
      }
    }
  };
  auto stage_store = [&](int e, const R v[FS]) {
    const int row = e / FZ;
    R *dst = fw + row * RF + (e - row * FZ) * FS;
    if constexpr (VB > 0) {
      store_rec<R, FS, VB>(dst, v);
    } else {
#pragma unroll
      for (int i = 0; i < FS; ++i) dst[i] = v[i];
    }
  };

  // the current window starts at zero; each flush clears what it adds
  for (int e = threadIdx.x; e < nlds; e += blockDim.x) lds[e] = 0.0;
  if (gt < t_hi)
    for (int e = threadIdx.x; e < FZ * FR; e += blockDim.x) {
      R v[FS];
      stage_load(gt, e, v);
      stage_store(e, v);
    }
  __syncthreads();

  while (gt < t_hi) {
  const int rn = batch_run(bt, gt);
  const KRun &k = bt.run[rn];
  const int tile = gt - (int)bt.off[rn];
  const int tz = tile % k.ntz, tr = tile / k.ntz;
  const int zlo = tz * TZ - SH, rlo = tr * TR - SH;  // current-window origin
  const int beg = k.cell_start[tile * TT], end = k.cell_start[(tile + 1) * TT];
  const int Nz = k.Nz, Nr = k.Nr;
  const long long plane = k.plane;
  const long long cstride = plane * NM;  // reals per component
  const R dt = (R)k.dt;
  const R *E = (const R *)k.E;
  const R *Bb = (const R *)k.Bbar;
  const int fz0 = tz * TZ - 1 - kFieldMarginZ, fr0 = tr * TR - 1 - kFieldMarginR;
  R *J = (R *)k.J[par];
  R *X = (R *)k.px, *Y = (R *)k.py, *UX = (R *)k.pux, *UY = (R *)k.puy, *UZ = (R *)k.puz;

  const int n = end - beg;
  const int chunk = (n + 255) / 256;
  // thread t takes slot t of each round (the sort has spread the slots'
  // electrons over the tile's cells, round_column)
  const int slot = threadIdx.x;
  const R dt_dz = (R)(k.dt / k.dz), dt_dr = (R)(k.dt / k.dr);
  // the electron of the next round is loaded while this round's is pushed
  R nw = 0, nz = 0, nfz = 0, nx = 0, ny = 0, nux = 0, nuy = 0, nuz = 0;
  int niz = 0;
  uint32_t nid = 0;
  auto fetch = [&](int pp) {
    nw = elem<R>(k.pw, pp);
    nid = elem<uint32_t>(k.pid, pp);
    if constexpr (F64) {
      nz = elem<double>(k.pz, pp);
    } else {
      niz = elem<int>(k.pz, pp);
      nfz = elem<float>(k.pfz, pp);
    }
    nx = elem<R>(X, pp);
    ny = elem<R>(Y, pp);
    nux = elem<R>(UX, pp);
    nuy = elem<R>(UY, pp);
    nuz = elem<R>(UZ, pp);
  };
  int base = 0;
  int cnt = round_count(n, chunk, 0);
  if (slot < cnt) fetch(beg + slot);
  for (int it = 0; it < chunk; ++it) {
    const int p = beg + base + slot;
    const bool act = slot < cnt;
    const R cw = nw, cz = nz, cfz = nfz, cx = nx, cy = ny, cux = nux, cuy = nuy, cuz = nuz;
    const int ciz = niz;
    const uint32_t cid = nid;
    base += cnt;
    cnt = (it + 1 < chunk) ? round_count(n, chunk, it + 1) : 0;
    if (slot < cnt) fetch(beg + base + slot);
    if (!act) continue;
    const R q = -cw;
    const uint32_t pidw = cid;

    // ---- old position ----
    int i0, dh;  // cell of z, and -1 or 0: the half-z stencil starts at i0 + dh
    R f0, z0 = 0;
    if constexpr (F64) {
      z0 = cz;
      const R fl = floor(z0);
      i0 = (int)fl;
      f0 = z0 - fl;
    } else {
      i0 = ciz;
      f0 = cfz;
    }
    if ((unsigned)i0 >= (unsigned)Nz) i0 = wrap_any(i0, Nz);
    const R x0 = cx, y0 = cy;
    const R r20 = fma(x0, x0, y0 * y0);
    const R ir0 = r20 > R(0) ? rsqrt_hw(r20) : R(0);
    const R r0 = r20 * ir0;  // the cell index below is exact whatever the last bits of r0
    const int j0 = clampi(radial_index(r20, r0), 0, Nr - 2);
    const R c0 = r20 > R(0) ? x0 * ir0 : R(1), s0 = y0 * ir0;

    // ---- gather E^n and Bbar^n = (B^{n-1/2} + B^{n+1/2})/2 (Eq. (12)) ----
    R fh;
    if constexpr (F64) {
      const R zz = z0 - R(0.5);
      const R fl = floor(zz);
      fh = zz - fl;
      dh = fl < floor(z0) ? -1 : 0;
    } else {
      if (f0 >= R(0.5)) {
        dh = 0;
        fh = f0 - R(0.5);
      } else {
        dh = -1;
        fh = f0 + R(0.5);
      }
    }
    const int ci0 = i0, ci1 = wrap_once(i0 + 1, Nz);
    const int ch0 = wrap_once(i0 + dh, Nz), ch1 = wrap_once(ch0 + 1, Nz);
    const R fr = r0 - (R)j0;
    const R rr = r0 - R(0.5);
    const R flr = floor(rr);
    int jh = (int)flr;
    const R frh = rr - flr;
    jh = clampi(jh, -1, Nr - 2);
    const bool mir = jh < 0;

    R er[NMP], ep[NMP], ez[NMP], br[NMP], bp[NMP], bz[NMP];
    // stencil in the field window: columns of i0 (periodic) and of the half-z
    // stencil (i0 - 1 or i0), rows of j0 and of the half-r stencil
    int fc = i0 - fz0;
    fc += (fc < 0) ? Nz : 0;
    fc -= (fc >= Nz) ? Nz : 0;
    if constexpr (SH == 2) {
      // Quadratic: 3 x 3 nodes round the nearest node of each component's
      // grid.  Along z the nearest integer node is i0 + zn and the nearest
      // half node (z_{i+1/2}, column i) is i0; along r likewise j0 + rn and
      // j0.  Weights at offsets f0 - zn, f0 - 1/2, fr - rn, fr - 1/2.
      const int zn = f0 >= R(0.5) ? 1 : 0, rn_ = fr >= R(0.5) ? 1 : 0;
      R wzn[3], wzh[3], wrn[3], wrh[3];
      qspline(f0 - (R)zn, wzn);
      qspline(f0 - R(0.5), wzh);
      qspline(fr - (R)rn_, wrn);
      qspline(fr - R(0.5), wrh);
      const int cn = fc + zn - 1, chh = fc - 1;                // first window column: integer, half z
      const int rnn = j0 + rn_ - 1 - fr0, rhh = j0 - 1 - fr0;  // first window row: integer, half r
      if (chh >= 0 && cn + 2 <= FZ - 1 && rhh >= 0 && rnn + 2 <= FR - 1) {
        interp9<R, NMP, VB>(fw + rhh * RF + cn * FS, RF, FS, wzn, wrh, er);
        interp9<R, NMP, VB>(fw + rnn * RF + cn * FS + CR, RF, FS, wzn, wrn, ep);
        interp9<R, NMP, VB>(fw + rnn * RF + chh * FS + 2 * CR, RF, FS, wzh, wrn, ez);
        interp9<R, NMP, VB>(fw + rnn * RF + chh * FS + 3 * CR, RF, FS, wzh, wrn, br);
        interp9<R, NMP, VB>(fw + rhh * RF + chh * FS + 4 * CR, RF, FS, wzh, wrh, bp);
        interp9<R, NMP, VB>(fw + rhh * RF + cn * FS + 5 * CR, RF, FS, wzn, wrh, bz);
      } else {
        const int gn = i0 + zn - 1, gh = i0 - 1, qn = j0 + rn_ - 1, qh = j0 - 1;
        interp9_global<R, NMP, true, false>(E, plane, Nz, Nr, gn, qh, wzn, wrh, er);
        interp9_global<R, NMP, false, false>(E + cstride, plane, Nz, Nr, gn, qn, wzn, wrn, ep);
        interp9_global<R, NMP, false, true>(E + 2 * cstride, plane, Nz, Nr, gh, qn, wzh, wrn, ez);
        interp9_global<R, NMP, false, false>(Bb, plane, Nz, Nr, gh, qn, wzh, wrn, br);
        interp9_global<R, NMP, true, false>(Bb + cstride, plane, Nz, Nr, gh, qh, wzh, wrh, bp);
        interp9_global<R, NMP, true, true>(Bb + 2 * cstride, plane, Nz, Nr, gn, qh, wzn, wrh, bz);
      }
    } else {
      const int a0 = fc, h0 = fc + dh;
      const int ri0 = j0 - fr0, rh0 = (mir ? 0 : jh) - fr0, rh1 = jh + 1 - fr0;
      if (h0 >= 0 && a0 + 1 <= FZ - 1 && ri0 >= 0 && rh0 >= 0 && ri0 + 1 <= FR - 1 && rh1 <= FR - 1) {
        const R *li0 = fw + ri0 * RF, *li1 = li0 + RF;  // rows of j0, j0 + 1
        const R *lh0 = fw + rh0 * RF, *lh1 = fw + rh1 * RF;  // half-r rows
        const int A0 = a0 * FS, A1 = A0 + FS, H0 = h0 * FS, H1 = H0 + FS;
        interp4<R, NMP, true, false, int, VB>(lh0 + A0, lh0 + A1, lh1 + A0, lh1 + A1, 1, mir, f0, frh, er);
        interp4<R, NMP, false, false, int, VB>(li0 + A0 + CR, li0 + A1 + CR, li1 + A0 + CR, li1 + A1 + CR, 1, false,
                                               f0, fr, ep);
        interp4<R, NMP, false, true, int, VB>(li0 + H0 + 2 * CR, li0 + H1 + 2 * CR, li1 + H0 + 2 * CR,
                                              li1 + H1 + 2 * CR, 1, false, fh, fr, ez);
        interp4<R, NMP, false, false, int, VB>(li0 + H0 + 3 * CR, li0 + H1 + 3 * CR, li1 + H0 + 3 * CR,
                                               li1 + H1 + 3 * CR, 1, false, fh, fr, br);
        interp4<R, NMP, true, false, int, VB>(lh0 + H0 + 4 * CR, lh0 + H1 + 4 * CR, lh1 + H0 + 4 * CR,
                                              lh1 + H1 + 4 * CR, 1, mir, fh, frh, bp);
        interp4<R, NMP, true, true, int, VB>(lh0 + A0 + 5 * CR, lh0 + A1 + 5 * CR, lh1 + A0 + 5 * CR,
                                             lh1 + A1 + 5 * CR, 1, mir, f0, frh, bz);
      } else {
        const long long gi0 = (long long)j0 * Nz, gi1 = gi0 + Nz;
        const long long gh0 = (long long)(mir ? 0 : jh) * Nz, gh1 = (long long)(jh + 1) * Nz;
        const R *er_ = E, *ep_ = E + cstride, *ez_ = E + 2 * cstride;
        const R *br_ = Bb, *bp_ = Bb + cstride, *bz_ = Bb + 2 * cstride;
        interp4<R, NMP, true, false, long long>(er_ + gh0 + ci0, er_ + gh0 + ci1, er_ + gh1 + ci0, er_ + gh1 + ci1,
                                                plane, mir, f0, frh, er);
        interp4<R, NMP, false, false, long long>(ep_ + gi0 + ci0, ep_ + gi0 + ci1, ep_ + gi1 + ci0, ep_ + gi1 + ci1,
                                                 plane, false, f0, fr, ep);
        interp4<R, NMP, false, true, long long>(ez_ + gi0 + ch0, ez_ + gi0 + ch1, ez_ + gi1 + ch0, ez_ + gi1 + ch1,
                                                plane, false, fh, fr, ez);
        interp4<R, NMP, false, false, long long>(br_ + gi0 + ch0, br_ + gi0 + ch1, br_ + gi1 + ch0, br_ + gi1 + ch1,
                                                 plane, false, fh, fr, br);
        interp4<R, NMP, true, false, long long>(bp_ + gh0 + ch0, bp_ + gh0 + ch1, bp_ + gh1 + ch0, bp_ + gh1 + ch1,
                                                plane, mir, fh, frh, bp);
        interp4<R, NMP, true, true, long long>(bz_ + gh0 + ci0, bz_ + gh0 + ci1, bz_ + gh1 + ci0, bz_ + gh1 + ci1,
                                               plane, mir, f0, frh, bz);
      }
    }

    // ---- reconstruct Re sum_m F^m e^{i m phi}, rotate to Cartesian ----
    // Ecyl[m] = (E_r, E_phi, E_z) of mode m at the electron's azimuth (kept
    // for the per-mode work of tracked electrons); the modes are summed in
    // cylindrical components and rotated to (x, y) once.
    R Ecyl[M + 1][3];
    R Ec[3], Bc[3];
    {
      Ecyl[0][0] = er[0];
      Ecyl[0][1] = ep[0];
      Ecyl[0][2] = ez[0];
      R Er = er[0], Ep = ep[0], Ez = ez[0], Br = br[0], Bp = bp[0], Bz = bz[0];
      R ere = c0, eim = s0;  // e^{i m phi}, m = 1, then by recurrence
#pragma unroll
      for (int m = 1; m <= M; ++m) {
        if (m > 1) {
          const R nre = ere * c0 - eim * s0;
          const R nim = ere * s0 + eim * c0;
          ere = nre;
          eim = nim;
        }
        const int a = 2 * m, b = 2 * m + 1;
        Ecyl[m][0] = er[a] * ere - er[b] * eim;
        Ecyl[m][1] = ep[a] * ere - ep[b] * eim;
        Ecyl[m][2] = ez[a] * ere - ez[b] * eim;
        Er += Ecyl[m][0];
        Ep += Ecyl[m][1];
        Ez += Ecyl[m][2];
        Br += br[a] * ere - br[b] * eim;
        Bp += bp[a] * ere - bp[b] * eim;
        Bz += bz[a] * ere - bz[b] * eim;
      }
      Ec[0] = Er * c0 - Ep * s0;
      Ec[1] = Er * s0 + Ep * c0;
      Ec[2] = Ez;
      Bc[0] = Br * c0 - Bp * s0;
      Bc[1] = Br * s0 + Bp * c0;
      Bc[2] = Bz;
    }

    // ---- Boris, q/m = -1 (Eq. (6)) ----
    const R u[3] = {cux, cuy, cuz};
    R um[3], up[3], un[3], tt[3], ss[3], u1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) um[a] = u[a] - R(0.5) * dt * Ec[a];
    const R hb = -R(0.5) * dt * rsqrt_hw(R(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) tt[a] = hb * Bc[a];
    const R t2 = tt[0] * tt[0] + tt[1] * tt[1] + tt[2] * tt[2];
    const R sf = R(2) * rcp_hw(R(1) + t2);
#pragma unroll
    for (int a = 0; a < 3; ++a) ss[a] = sf * tt[a];
    u1[0] = um[0] + (um[1] * tt[2] - um[2] * tt[1]);
    u1[1] = um[1] + (um[2] * tt[0] - um[0] * tt[2]);
    u1[2] = um[2] + (um[0] * tt[1] - um[1] * tt[0]);
    up[0] = um[0] + (u1[1] * ss[2] - u1[2] * ss[1]);
    up[1] = um[1] + (u1[2] * ss[0] - u1[0] * ss[2]);
    up[2] = um[2] + (u1[0] * ss[1] - u1[1] * ss[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) un[a] = up[a] - R(0.5) * dt * Ec[a];
    const R gg_new = R(1) + un[0] * un[0] + un[1] * un[1] + un[2] * un[2];  // gamma^2
    const R inv_g = rsqrt_hw(gg_new);

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
        const double inv = 1.0 / (g_old + sqrt((double)gg_new));
        const double v0 = ((double)um[0] + (double)up[0]) * inv;
        const double v1 = ((double)um[1] + (double)up[1]) * inv;
        const double v2 = ((double)um[2] + (double)up[2]) * inv;
        double *W = k.W + (long long)lo * (M + 1);
        // the same work split by field direction, Eq. (17)
        double ez = 0.0, ep = 0.0;
#pragma unroll
        for (int m = 0; m <= M; ++m) {
          const double fr = Ecyl[m][0], fp = Ecyl[m][1], fz = Ecyl[m][2];
          const double ex = fr * c0 - fp * s0, ey = fr * s0 + fp * c0;  // mode m's E in (x, y)
          W[m] += -k.dt * (ex * v0 + ey * v1 + fz * v2);
          ez += fz;
          ep += ex * v0 + ey * v1;
        }
        double *Wc = k.Wc + (long long)lo * 2;
        Wc[0] += -k.dt * ez * v2;
        Wc[1] += -k.dt * ep;
      }
    }

    // ---- move ----
    int i1;
    R f1;
    R z1 = 0;
    if constexpr (F64) {
      z1 = z0 + un[2] * inv_g * dt_dz;
      const R fl = floor(z1);
      i1 = (int)fl;
      f1 = z1 - fl;
    } else {
      f1 = f0 + un[2] * inv_g * dt_dz;
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
    R x1 = x0 + un[0] * inv_g * dt_dr;
    R y1 = y0 + un[1] * inv_g * dt_dr;
    const R Rw = (R)(Nr - 1);
    R r21 = fma(x1, x1, y1 * y1);
    if (r21 >= Rw * Rw) {  // specular reflection at r = (Nr - 1) dr (Rw^2 is exact)
      R r1 = sqrt(r21);
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
    const R ir1 = r21 > R(0) ? rsqrt_hw(r21) : R(0);
    const R r1 = r21 * ir1;
    int j1 = clampi(radial_index(r21, r1), j0 - 1, j0 + 1);
    j1 = clampi(j1, 0, Nr - 2);
    const R c1 = r21 > R(0) ? x1 * ir1 : R(1), s1 = y1 * ir1;
    const R g1 = r1 - (R)j1;

    // ---- charge-conserving deposit of J^{n+1/2} ----
    {
      const R xm = R(0.5) * (x0 + x1), ym = R(0.5) * (y0 + y1);
      const R rm2 = xm * xm + ym * ym;
      const R irm = rm2 > R(0) ? rsqrt_hw(rm2) : R(0);
      const R cmid = rm2 > R(0) ? xm * irm : R(1), smid = ym * irm;
      const R vphi = rm2 > R(0) ? (cmid * un[1] - smid * un[0]) * inv_g : R(0);
      const int di = clampi(i1 - i0, -1, 1);
      const int dj = j1 - j0;
      const R g0 = fr;
      // Mode coefficients, mode by mode with e^{-i m phi} of the old and new
      // positions by recurrence: the flux phase cq xi, xi = (e0 + e1)/2, of
      // J_z and J_r; for J_phi, m = 0 takes cq v_phi, m >= 1 the closure
      // cq (i/m)(e1 - e0) (its factor r_j and the node volume cancel into the
      // row factor of the E update), which is zero on the axis row, where
      // m = 1 takes cq v_phi e_mid instead (cq = c_m q).
      // (the deterministic mode scales every coefficient by the run's 2^K)
      const double qs = DET ? k.qscale : 1.0;
      auto for_modes = [&](bool axis_row, auto &&body) {
        R e0r = 1, e0i = 0, e1r = 1, e1i = 0;
#pragma unroll
        for (int m = 0; m <= M; ++m) {
          if (m == 1) {
            e0r = c0;
            e0i = -s0;
            e1r = c1;
            e1i = -s1;
          } else if (m > 1) {
            // written with explicit fma, so that the old and new phases are
            // rounded alike: an electron whose x, y did not change gets
            // e1 == e0 bit for bit, and no closure current
            R t = fma(e0r, c0, e0i * s0);
            e0i = fma(e0i, c0, -(e0r * s0));
            e0r = t;
            t = fma(e1r, c1, e1i * s1);
            e1i = fma(e1i, c1, -(e1r * s1));
            e1r = t;
          }
          const R cq = (m == 0 ? R(1) : R(2)) * q;
          const R fa = cq * (R(0.5) * (e0r + e1r)), fb = cq * (R(0.5) * (e0i + e1i));
          R pa, pb, pa0, pb0;
          if (m == 0) {
            pa = pa0 = cq * vphi;
            pb = pb0 = R(0);
          } else {
            pa = -cq * (e1i - e0i) * (R(1) / (R)m);
            pb = cq * (e1r - e0r) * (R(1) / (R)m);
            pa0 = axis_row ? (m == 1 ? cq * vphi * cmid : R(0)) : pa;
            pb0 = axis_row ? (m == 1 ? -cq * vphi * smid : R(0)) : pb;
          }
          body(m, m == 0 ? 0 : 2 * m - 1, 2 * m, (double)fa * qs, (double)fb * qs, (double)pa * qs, (double)pb * qs,
               (double)pa0 * qs, (double)pb0 * qs);
        }
      };
      if constexpr (SH == 2) {
        // Quadratic: a 4 x 4 node window [ib, ib+3] x [jb, jb+3] that holds
        // the 3 x 3 supports round the nearest nodes of both positions (a
        // move of less than a cell changes each nearest node by at most one),
        // quadratic B-spline shapes S0, S1 on it, and the same Esirkepov
        // weights and running sums as the linear deposit.  The window starts
        // at node (i0 - 1, j0 - 1), one before the cell, whenever it holds
        // both supports (each nearest node is the cell's first or second
        // node): then lanes in distinct cells never add to one LDS address in
        // the same instruction (a window started at the nearest node minus
        // one gives two lanes in neighbouring cells the same window in a
        // quarter of the cases).  Otherwise it starts one before the lower
        // nearest node.  Nodes on row r_{-1} (within half a cell of the axis)
        // are summed there in the tile window and folded onto r_1 (J_r: face
        // r_{-1/2} onto r_{1/2}) with the mirror sign when the window is
        // flushed; the device-memory path folds them at once.
        const int n0z = f0 >= R(0.5) ? 1 : 0, n1z = f1 >= R(0.5) ? 1 : 0;
        const int n0r = g0 >= R(0.5) ? 1 : 0, n1r = g1 >= R(0.5) ? 1 : 0;
        // nearest nodes relative to the cell: old n0, new n0 + dn
        const int dn = clampi(di + n1z - n0z, -1, 1), dm = clampi(dj + n1r - n0r, -1, 1);
        const int zlo_ = n0z + (dn < 0 ? dn : 0), zhi_ = n0z + (dn > 0 ? dn : 0);
        const int rlo_ = n0r + (dm < 0 ? dm : 0), rhi_ = n0r + (dm > 0 ? dm : 0);
        const int bz = (zlo_ >= 0 && zhi_ <= 1) ? -1 : zlo_ - 1;  // window start relative to the cell
        const int br = (rlo_ >= 0 && rhi_ <= 1) ? -1 : rlo_ - 1;
        const int oz0 = n0z - 1 - bz, oz1 = oz0 + dn;  // first support node of each position in the window
        const int or0 = n0r - 1 - br, or1 = or0 + dm;
        const int lz = zlo_ - 1 - bz, hz = zhi_ - 1 - bz;  // lower and upper of oz0, oz1 (0 or 1)
        const int lr = rlo_ - 1 - br, hr = rhi_ - 1 - br;
        const int ib = i0 + bz, jb = j0 + br;
        // the first (last) window column or row carries current only from a
        // lane whose lower (upper) support starts there: the wave skips it when
        // no lane's does
        const bool zf = __any(lz == 0), zl = __any(hz == 1), rf = __any(lr == 0), rl = __any(hr == 1);
        R q0z[3], q1z[3], q0r[3], q1r[3];
        qspline(f0 - (R)n0z, q0z);
        qspline(f1 - (R)n1z, q1z);
        qspline(g0 - (R)n0r, q0r);
        qspline(g1 - (R)n1r, q1r);
        R Sz0[4], Sz1[4], Sr0[4], Sr1[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          Sz0[a] = a == oz0 ? q0z[0] : (a == oz0 + 1 ? q0z[1] : (a == oz0 + 2 ? q0z[2] : R(0)));
          Sz1[a] = a == oz1 ? q1z[0] : (a == oz1 + 1 ? q1z[1] : (a == oz1 + 2 ? q1z[2] : R(0)));
          Sr0[a] = a == or0 ? q0r[0] : (a == or0 + 1 ? q0r[1] : (a == or0 + 2 ? q0r[2] : R(0)));
          Sr1[a] = a == or1 ? q1r[0] : (a == or1 + 1 ? q1r[1] : (a == or1 + 2 ? q1r[2] : R(0)));
        }
        // J_z at (ib+a+1/2, jb+b), a = 0..2; J_r at (ib+a, jb+b+1/2), b = 0..2;
        // J_phi at (ib+a, jb+b)
        double wz[4][3], wr[4][3], ws[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          R run = 0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            run += (Sz1[a] - Sz0[a]) * (Sr0[b] + Sr1[b]) * R(0.5);
            wz[b][a] = -(double)run;
          }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          R run = 0;
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            run += (Sr1[b] - Sr0[b]) * (Sz0[a] + Sz1[a]) * R(0.5);
            wr[a][b] = -(double)run;
          }
#pragma unroll
          for (int b = 0; b < 4; ++b) ws[a][b] = (double)(R(0.5) * (Sz0[a] * Sr0[b] + Sz1[a] * Sr1[b]));
        }
        // a lane's shapes cover window columns lz .. hz + 2 and rows
        // lr .. hr + 2; its z fluxes faces lz .. hz + 1, its r fluxes faces
        // lr .. hr + 1 (past those a line's running sum is the whole line's,
        // zero).  Each lane masks itself off the others.
        auto deposit = [&](auto &&dep) {
          for_modes(true, [&](int m, int qa, int qb, double fa, double fb, double pa, double pb, double pa0,
                              double pb0) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              if ((b == 0 && !rf) || (b == 3 && !rl)) continue;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                if ((a == 0 && !zf) || (a == 2 && !zl)) continue;
                if (a < lz || a > hz + 1 || b < lr || b > hr + 2) continue;
                dep(2, qa, b, a, wz[b][a], fa);
                if (m > 0) dep(2, qb, b, a, wz[b][a], fb);
              }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              if ((a == 0 && !zf) || (a == 3 && !zl)) continue;
#pragma unroll
              for (int b = 0; b < 3; ++b) {
                if ((b == 0 && !rf) || (b == 2 && !rl)) continue;
                if (a < lz || a > hz + 2 || b < lr || b > hr + 1) continue;
                dep(0, qa, b, a, wr[a][b], fa);
                if (m > 0) dep(0, qb, b, a, wr[a][b], fb);
              }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              if ((a == 0 && !zf) || (a == 3 && !zl)) continue;
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                if ((b == 0 && !rf) || (b == 3 && !rl)) continue;
                if (a < lz || a > hz + 2 || b < lr || b > hr + 2) continue;
                const bool axis = jb + b == 0;  // the axis row takes the axis coefficients
                dep(1, qa, b, a, ws[a][b], axis ? pa0 : pa);
                if (m > 0) dep(1, qb, b, a, ws[a][b], axis ? pb0 : pb);
              }
            }
          });
        };
        if ((ib - zlo >= 0) && (ib + 3 - zlo < WZ) && (jb - rlo >= 0) && (jb + 3 - rlo < WR)) {
          double *jw = lds + (jb - rlo) * RJ + (ib - zlo) * (JW * JS);
          deposit([&](int c, int qq, int b, int a, double w, double cf) {
            double *p = jw + b * RJ + a * (JW * JS) + JW * (c * NM + qq);
            if constexpr (DET) fix_add_lds((unsigned long long *)p, w, cf);
            else lds_add(p, w * cf);
          });
        } else {
          int col[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) col[a] = wrap_any(ib + a, Nz);
          deposit([&](int c, int qq, int b, int a, double w, double cf) {
            // row r_{-1} onto r_1, face r_{-1/2} onto r_{1/2}, with the
            // mirror sign of the component and mode
            int row = jb + b;
            double sg = 1.0;
            if (row < 0) {
              const int m = (qq + 1) / 2;
              row = c == 0 ? -row - 1 : -row;
              sg = (c == 0 ? mirror_sign_m(m, false) : (c == 1 && m == 0 ? -1 : mirror_sign_m(m, true))) < 0 ? -1.0
                                                                                                                : 1.0;
            }
            const long long at = (c * NM + qq) * plane + (long long)row * Nz + col[a];
            if constexpr (DET) {
              unsigned long long x, y;
              fix_split(sg * w, cf, x, y);  // sg w is exact
              fix_add_global(k.Jfix + 2 * at, x, y);
            } else {
              atomic_add(J + at, (R)(sg * w * cf));
            }
          });
        }
      } else if (!DET && !__any(di != 0 || dj != 0)) {
        // (this path not in the deterministic mode: which path an electron
        // takes would depend on the other electrons of its wavefront, and the
        // two paths round differently)
        // No electron of the wavefront left its cell: each deposits on the
        // 2 x 2 nodes (i0 + a, j0 + b) of its cell.  J_z at (i0+1/2, j0+b)
        // carries (f1 - f0) times the mean radial shape of row b, J_r at
        // (i0+a, j0+1/2) (g1 - g0) times the mean axial shape of column a,
        // J_phi at (i0+a, j0+b) half the summed shape (the 2D Esirkepov
        // weights of a move inside one cell).
        const R df = f1 - f0, dg = g1 - g0;
        const R sz0 = R(1) - f0, sz1 = R(1) - f1, sr0 = R(1) - g0, sr1 = R(1) - g1;
        const double wz0 = (double)(df * (R(0.5) * (sr0 + sr1))), wz1 = (double)(df * (R(0.5) * (g0 + g1)));
        const double wr0 = (double)(dg * (R(0.5) * (sz0 + sz1))), wr1 = (double)(dg * (R(0.5) * (f0 + f1)));
        const double w00 = (double)(R(0.5) * (sz0 * sr0 + sz1 * sr1)), w10 = (double)(R(0.5) * (f0 * sr0 + f1 * sr1));
        const double w01 = (double)(R(0.5) * (sz0 * g0 + sz1 * g1)), w11 = (double)(R(0.5) * (f0 * g0 + f1 * g1));
        auto deposit = [&](auto &&dep) {
          for_modes(j0 == 0, [&](int m, int qa, int qb, double fa, double fb, double pa, double pb, double pa0,
                                 double pb0) {
            dep(2, qa, 0, 0, wz0, fa);
            dep(2, qa, 1, 0, wz1, fa);
            dep(0, qa, 0, 0, wr0, fa);
            dep(0, qa, 0, 1, wr1, fa);
            dep(1, qa, 0, 0, w00, pa0);
            dep(1, qa, 0, 1, w10, pa0);
            dep(1, qa, 1, 0, w01, pa);
            dep(1, qa, 1, 1, w11, pa);
            if (m > 0) {
              dep(2, qb, 0, 0, wz0, fb);
              dep(2, qb, 1, 0, wz1, fb);
              dep(0, qb, 0, 0, wr0, fb);
              dep(0, qb, 0, 1, wr1, fb);
              dep(1, qb, 0, 0, w00, pb0);
              dep(1, qb, 0, 1, w10, pb0);
              dep(1, qb, 1, 0, w01, pb);
              dep(1, qb, 1, 1, w11, pb);
            }
          });
        };
        if ((i0 - zlo >= 0) && (i0 + 1 - zlo < WZ) && (j0 - rlo >= 0) && (j0 + 1 - rlo < WR)) {
          double *jw = lds + (j0 - rlo) * RJ + (i0 - zlo) * (JW * JS);
          deposit([&](int c, int qq, int b, int a, double w, double cf) {
            double *p = jw + b * RJ + a * (JW * JS) + JW * (c * NM + qq);
            if constexpr (DET) fix_add_lds((unsigned long long *)p, w, cf);
            else lds_add(p, w * cf);
          });
        } else {
          const int col1 = wrap_once(i0 + 1, Nz);
          deposit([&](int c, int qq, int b, int a, double w, double cf) {
            const long long at = (c * NM + qq) * plane + (long long)(j0 + b) * Nz + (a ? col1 : i0);
            if constexpr (DET) {
              unsigned long long x, y;
              fix_split(w, cf, x, y);
              fix_add_global(k.Jfix + 2 * at, x, y);
            } else {
              atomic_add(J + at, (R)(w * cf));
            }
          });
        }
      } else {
        // General move: the 3 x 3 node window [ib, ib+2] x [jb, jb+2] that
        // holds both positions; shapes S0, S1 on it, the 2D Esirkepov weights
        // Wz = dSz (Sr0 + Sr1)/2, Wr = dSr (Sz0 + Sz1)/2, and the fluxes minus
        // their running sums.
        const int oz0 = di < 0 ? 1 : 0, oz1 = oz0 + di;  // cells of the two positions in the window
        const int ib = i0 - oz0;
        const int or0 = dj < 0 ? 1 : 0, or1 = or0 + dj;
        const int jb = j0 - or0;
        // the third node column (row) of the window carries current only for an
        // electron that crossed a z (r) cell face; skip it when no lane did
        const bool zx = __any(di != 0), rx = __any(dj != 0);
        R Sz0[3], Sz1[3], Sr0[3], Sr1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          Sz0[a] = (a == oz0) ? R(1) - f0 : ((a == oz0 + 1) ? f0 : R(0));
          Sz1[a] = (a == oz1) ? R(1) - f1 : ((a == oz1 + 1) ? f1 : R(0));
          Sr0[a] = (a == or0) ? R(1) - g0 : ((a == or0 + 1) ? g0 : R(0));
          Sr1[a] = (a == or1) ? R(1) - g1 : ((a == or1 + 1) ? g1 : R(0));
        }
        // J_z at face (ib+a+1/2, jb+b): minus the running sum of Wz behind it;
        // J_r at (ib+a, jb+b+1/2): minus the running sum of Wr below it;
        // J_phi at node (ib+a, jb+b): half the summed shape
        double wz[3][2], wr[3][2], ws[3][3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          R run = 0;
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            run += (Sz1[a] - Sz0[a]) * (Sr0[b] + Sr1[b]) * R(0.5);
            wz[b][a] = -(double)run;
          }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          R run = 0;
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            run += (Sr1[b] - Sr0[b]) * (Sz0[a] + Sz1[a]) * R(0.5);
            wr[a][b] = -(double)run;
          }
#pragma unroll
          for (int b = 0; b < 3; ++b) ws[a][b] = (double)(R(0.5) * (Sz0[a] * Sr0[b] + Sz1[a] * Sr1[b]));
        }
        // the whole deposit, into `dep(c, plane, b, a, w, cf)` (the value w cf): component c (0 r,
        // 1 phi, 2 z), window node (ib + a, jb + b).  A node past the first
        // two columns (rows) takes current only from a lane whose electron
        // crossed a z (r) face: the wave skips it when no lane did, and each
        // other lane masks itself off.
        auto deposit = [&](auto &&dep) {
          for_modes(jb == 0, [&](int m, int qa, int qb, double fa, double fb, double pa, double pb, double pa0,
                                 double pb0) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              if (b == 2 && !rx) continue;
#pragma unroll
              for (int a = 0; a < 2; ++a) {
                if (a == 1 && !zx) continue;
                if ((a == 1 && di == 0) || (b == 2 && dj == 0)) continue;
                dep(2, qa, b, a, wz[b][a], fa);
                if (m > 0) dep(2, qb, b, a, wz[b][a], fb);
              }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              if (a == 2 && !zx) continue;
#pragma unroll
              for (int b = 0; b < 2; ++b) {
                if (b == 1 && !rx) continue;
                if ((a == 2 && di == 0) || (b == 1 && dj == 0)) continue;
                dep(0, qa, b, a, wr[a][b], fa);
                if (m > 0) dep(0, qb, b, a, wr[a][b], fb);
              }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              if (a == 2 && !zx) continue;
#pragma unroll
              for (int b = 0; b < 3; ++b) {
                if (b == 2 && !rx) continue;
                if ((a == 2 && di == 0) || (b == 2 && dj == 0)) continue;
                dep(1, qa, b, a, ws[a][b], (b == 0 ? pa0 : pa));
                if (m > 0) dep(1, qb, b, a, ws[a][b], (b == 0 ? pb0 : pb));
              }
            }
          });
        };
        if ((ib - zlo >= 0) && (ib + 2 - zlo < WZ) && (jb - rlo >= 0) && (jb + 2 - rlo < WR)) {
          double *jw = lds + (jb - rlo) * RJ + (ib - zlo) * (JW * JS);
          deposit([&](int c, int qq, int b, int a, double w, double cf) {
            double *p = jw + b * RJ + a * (JW * JS) + JW * (c * NM + qq);
            if constexpr (DET) fix_add_lds((unsigned long long *)p, w, cf);
            else lds_add(p, w * cf);
          });
        } else {
          int col[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) col[a] = wrap_once(ib + a, Nz);
          deposit([&](int c, int qq, int b, int a, double w, double cf) {
            const long long at = (c * NM + qq) * plane + (long long)(jb + b) * Nz + col[a];
            if constexpr (DET) {
              unsigned long long x, y;
              fix_split(w, cf, x, y);
              fix_add_global(k.Jfix + 2 * at, x, y);
            } else {
              atomic_add(J + at, (R)(w * cf));
            }
          });
        }
      }
    }

    // ---- store (periodic in z; with a moving window unwrapped, and an
    // electron that left the box keeps zero weight until the next move) ----
    if constexpr (F64) {
      if (k.window) {
        if (z1 < R(0) || z1 >= (R)Nz) elem<R>(k.pw, p) = R(0);
      } else {
        if (z1 < R(0)) z1 += (R)Nz;
        if (z1 >= (R)Nz) z1 -= (R)Nz;
      }
      elem<double>(k.pz, p) = z1;
    } else {
      if (k.window) {
        const int i1raw = ciz + (i1 - i0);  // the cell before wrapping
        if (i1raw < 0 || i1raw >= Nz) elem<R>(k.pw, p) = R(0);
        elem<int>(k.pz, p) = i1raw;
      } else {
        elem<int>(k.pz, p) = wrap_once(i1, Nz);
      }
      elem<float>(k.pfz, p) = f1;
    }
    elem<R>(X, p) = x1;
    elem<R>(Y, p) = y1;
    elem<R>(UX, p) = un[0];
    elem<R>(UY, p) = un[1];
    elem<R>(UZ, p) = un[2];
  }

  // ---- flush the tile's current (each thread a window node, all its
  // component planes), clear the window, then stage the next tile's field
  // window ----
  if (threadIdx.x == 0) ticket = next_tile();  // read after the barrier
  __syncthreads();
  const int nt = ticket;
  // quadratic: one window node, row r_{-1} folded onto r_1 (J_r: face
  // r_{-1/2} onto r_{1/2}) with the mirror sign: (-1)^m for J_z, (-1)^(m+1)
  // for J_r, and for J_phi (-1)^m of the closure (its factor r changes sign
  // with the row) and -1 of the m = 0 current
  auto flush_quadratic = [&](int e) {
    const int lr = e / WZ, lc = e - lr * WZ;
    const int row = rlo + lr;
    if (row < -1 || row > Nr) return;  // never deposited to
    const int col = wrap_any(zlo + lc, Nz);
    double *src = lds + lr * RJ + lc * (JW * JS);
#pragma unroll
    for (int cq = 0; cq < JS; ++cq) {
      const int c = cq / NM, m = (cq % NM + 1) / 2;
      int trow = row;
      bool neg = false;
      if (row < 0) {
        trow = c == 0 ? 0 : 1;
        neg = (c == 0 ? mirror_sign_m(m, false) : (c == 1 && m == 0 ? -1 : mirror_sign_m(m, true))) < 0;
      }
      const unsigned off = (unsigned)(trow * Nz + col);
      if constexpr (DET) {
        // the integer pair negated word by word (two's complement) is the
        // pair of the negated value
        unsigned long long *s2 = (unsigned long long *)src;
        const unsigned long long a = s2[2 * cq], b = s2[2 * cq + 1];
        s2[2 * cq] = s2[2 * cq + 1] = 0;
        fix_add_global(k.Jfix + 2 * ((long long)cq * plane + off), neg ? 0ull - a : a, neg ? 0ull - b : b);
      } else {
        const R v = (neg ? R(-1) : R(1)) * (R)src[cq];
        src[cq] = 0.0;
        if (v != R(0)) atomic_add(J + cq * plane + off, v);
      }
    }
  };
  if constexpr (!F64) {
    // FP32: the first half of the wavefronts flush the current window while
    // the other half stage the next tile's field window (separate LDS
    // regions), so that the two phases' memory traffic overlaps
    const int split = (int)(blockDim.x >> 7) << 6;
    if ((int)threadIdx.x < split) {
      if (n > 0)
        for (int e = threadIdx.x; e < WZ * WR; e += split) {
          if constexpr (SH == 2) {
            flush_quadratic(e);
            continue;
          }
          const int lr = e / WZ, lc = e - lr * WZ;
          const int row = rlo + lr;
          if (row < 0 || row > Nr) continue;  // never deposited to
          // a node that takes current lies in [-1, Nz + 1]; the others hold zero
          const unsigned off = (unsigned)(row * Nz + wrap_once(zlo + lc, Nz));
          double *src = lds + lr * RJ + lc * (JW * JS);
#pragma unroll
          for (int cq = 0; cq < JS; ++cq) {
            const R v = (R)src[cq];
            src[cq] = 0.0;
            if (v != R(0)) atomic_add(J + cq * plane + off, v);
          }
        }
    } else if (nt < t_hi) {
      for (int e = (int)threadIdx.x - split; e < FZ * FR; e += (int)blockDim.x - split) {
        R v[FS];
        stage_load(nt, e, v);
        stage_store(e, v);
      }
    }
  } else {
    // FP64: the flush (FP64 device atomics) dominates; every thread flushes,
    // then stages
    if (n > 0)
      for (int e = threadIdx.x; e < WZ * WR; e += blockDim.x) {
        if constexpr (SH == 2) {
          flush_quadratic(e);
          continue;
        }
        const int lr = e / WZ, lc = e - lr * WZ;
        const int row = rlo + lr;
        if (row < 0 || row > Nr) continue;  // never deposited to
        // a node that takes current lies in [-1, Nz + 1]; the others hold zero
        const unsigned off = (unsigned)(row * Nz + wrap_once(zlo + lc, Nz));
        double *src = lds + lr * RJ + lc * (JW * JS);
        if constexpr (DET) {
          unsigned long long *s2 = (unsigned long long *)src;
#pragma unroll
          for (int cq = 0; cq < JS; ++cq) {
            const unsigned long long a = s2[2 * cq], b = s2[2 * cq + 1];
            s2[2 * cq] = s2[2 * cq + 1] = 0;
            fix_add_global(k.Jfix + 2 * ((long long)cq * plane + off), a, b);
          }
        } else {
#pragma unroll
          for (int cq = 0; cq < JS; ++cq) {
            const R v = (R)src[cq];
            src[cq] = 0.0;
            if (v != R(0)) atomic_add(J + cq * plane + off, v);
          }
        }
      }
    if (nt < t_hi)
      for (int e = threadIdx.x; e < FZ * FR; e += blockDim.x) {
        R v[FS];
        stage_load(nt, e, v);
        stage_store(e, v);
      }
  }
  __syncthreads();
  gt = nt;
  }  // tiles
}

// ---------------------------------------------------------------------------
// field update.  One workgroup = kFieldTile consecutive columns of one row j;
// the rows whose z differences or z filter need neighbours (+-N columns) are
// first staged in LDS with coalesced record loads, every other operand is a
// record of the thread's own column.
//
// The E update takes the deposited current through one of two z stencils
// that make it conserve charge with D_B = D_Yee o P: the filter P (2N-1
// taps) on J_r and J_phi (kExact false), or P^{-1} (2 NH - 1 taps) on J_z
// with J_r and J_phi as deposited (kExact true).

template <typename R, int M, bool kExact>
__global__ __launch_bounds__(kFieldTile) void efield_kernel(const Batch bt) {
  constexpr int NMP = 2 * (M + 1);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  R *lds = (R *)lds_raw;
  const int rn = batch_run(bt, blockIdx.x);
  const KRun &k = bt.run[rn];
  const int par = bt.par;
  const int Nz = k.Nz, Nr = k.Nr, N = k.N;
  const int ncol = (Nz + kFieldTile - 1) / kFieldTile;
  const int blk = (int)(blockIdx.x - bt.off[rn]);  // (row j, column block) of this run
  const int j = blk / ncol;
  const int i0 = (blk - j * ncol) * kFieldTile;
  const int t = threadIdx.x;
  const int W = kFieldTile + 2 * N;  // staged columns i0-N .. i0+kFieldTile+N-1
  const int NH = k.NH;               // exact: J_z staged over i0-NH+1 .. i0+kFieldTile+NH-2
  const int WH = kFieldTile + 2 * (NH - 1);
  const long long plane = k.plane, cstride = plane * (NMP - 1);  // NM planes per component
  const long long row = (long long)j * Nz;
  const R *B = (const R *)k.B[par ^ 1];  // B^{n+1/2}
  const R *Jc = (const R *)k.J[par];
  R *Jn = (R *)k.J[par ^ 1];
  R *E = (R *)k.E;
  R *sBp = lds, *sBr = lds + W * NMP, *sJr = lds + 2 * W * NMP, *sJp = lds + 3 * W * NMP;
  R *sJz = lds + 2 * W * NMP;  // exact: in place of sJr, sJp
  // the thread's own-column operands (a column past Nz reads column Nz - 1
  // and is dropped after the barrier).  In FP32 they are loaded first, to be
  // in flight while the rows are staged; in FP64 that costs more in
  // registers than it gains, and they are loaded after the z operators.
  constexpr bool kEarly = sizeof(R) == 4;
  const int i = i0 + t;
  const bool live = i < Nz;
  const long long ic = live ? i : Nz - 1;
  R er[NMP], ep[NMP], ez[NMP], bz[NMP], bzm[NMP], bpm[NMP], jz[NMP];
  R pjr[NMP], pjp[NMP];  // J_r, J_phi as the update takes them
  auto load_own = [&]() {
    load_node<R, NMP>(E + 0 * cstride, plane, row + ic, er);
    load_node<R, NMP>(E + 1 * cstride, plane, row + ic, ep);
    load_node<R, NMP>(E + 2 * cstride, plane, row + ic, ez);
    load_node<R, NMP>(B + 2 * cstride, plane, row + ic, bz);
    if constexpr (kExact) {
      load_node<R, NMP>(Jc + 0 * cstride, plane, row + ic, pjr);
      load_node<R, NMP>(Jc + 1 * cstride, plane, row + ic, pjp);
    } else {
      load_node<R, NMP>(Jc + 2 * cstride, plane, row + ic, jz);
    }
    // half row j-1 (unused in row 0).  FP64 loads it without a branch, row 0
    // reading its own row: the branch leaves part of the two arrays in scratch
    // memory there (24 bytes; 0.158 -> 0.154 ms at 4096 x 256, modes 0..2).
    // FP32 keeps the branch, measured faster (0.391 -> 0.377 ms at
    // 8192 x 512, modes 0..3) despite 12 bytes of scratch.
    if constexpr (!kEarly) {
      const long long rowm = j > 0 ? row - Nz : row;
      load_node<R, NMP>(B + 2 * cstride, plane, rowm + ic, bzm);
      load_node<R, NMP>(B + 1 * cstride, plane, rowm + ic, bpm);
    } else if (j > 0) {
      load_node<R, NMP>(B + 2 * cstride, plane, row - Nz + ic, bzm);
      load_node<R, NMP>(B + 1 * cstride, plane, row - Nz + ic, bpm);
    } else {
#pragma unroll
      for (int s = 0; s < NMP; ++s) bzm[s] = bpm[s] = R(0);
    }
  };
  if constexpr (kEarly) load_own();
  for (int r = t; r < W; r += kFieldTile) {
    const int col = wrap_any(i0 - N + r, Nz);
    R v[NMP];
    load_node<R, NMP>(B + 1 * cstride, plane, row + col, v);  // B_phi (half row j)
    store_rec<R, NMP>(sBp + r * NMP, v);
    load_node<R, NMP>(B + 0 * cstride, plane, row + col, v);  // B_r
    store_rec<R, NMP>(sBr + r * NMP, v);
    if constexpr (!kExact) {
      load_node<R, NMP>(Jc + 0 * cstride, plane, row + col, v);  // J_r
      store_rec<R, NMP>(sJr + r * NMP, v);
      load_node<R, NMP>(Jc + 1 * cstride, plane, row + col, v);  // J_phi
      store_rec<R, NMP>(sJp + r * NMP, v);
    }
  }
  if constexpr (kExact)
    for (int r = t; r < WH; r += kFieldTile) {
      const int col = wrap_any(i0 - (NH - 1) + r, Nz);
      R v[NMP];
      load_node<R, NMP>(Jc + 2 * cstride, plane, row + col, v);  // J_z
      store_rec<R, NMP>(sJz + r * NMP, v);
    }
  __syncthreads();
  if (!live) return;
  const R dt = (R)k.dt, dr = (R)k.dr, idz = (R)(1.0 / k.dz);
  const R *CB = (const R *)k.CB, *P = (const R *)k.P;
  // physical current = raw deposit * factor of the row
  const double dzd = k.dz, drd = k.dr, dtd = k.dt;
  const double Vj = j == 0 ? kPi * drd * drd * dzd / 4.0 : 2.0 * kPi * (j * drd) * drd * dzd;
  const R fz = (R)(1.0 / (dtd * (Vj / dzd)));
  const R frr = (R)(1.0 / (dtd * (2.0 * kPi * ((j + 0.5) * drd) * dzd)));
  const R fp_direct = (R)(1.0 / Vj);
  const R fp_closure = (R)(1.0 / (dtd * 2.0 * kPi * drd * dzd));
  const R rh = ((R)j + R(0.5)) * dr;
  const int c0 = t + N;  // LDS index of column i

  // z operators on the staged rows, all modes at once
  R dbp[NMP], dbr[NMP];
#pragma unroll
  for (int s = 0; s < NMP; ++s) dbp[s] = dbr[s] = R(0);
  for (int l = 1; l <= N; ++l) {  // D_B: sum_l C^B_l (g_{i+l-1/2} - g_{i-l+1/2})
    const R cb = CB[l - 1];
    const R *ap = sBp + (c0 + l - 1) * NMP, *am = sBp + (c0 - l) * NMP;
    const R *bp_ = sBr + (c0 + l - 1) * NMP, *bm = sBr + (c0 - l) * NMP;
#pragma unroll
    for (int s = 0; s < NMP; ++s) {
      dbp[s] += cb * (ap[s] - am[s]);
      dbr[s] += cb * (bp_[s] - bm[s]);
    }
  }
  if constexpr (kExact) {  // symmetric stencil of P^{-1} on J_z
    const R *H = (const R *)k.H;
    const int ch = t + NH - 1;  // LDS index of column i in the J_z rows
    const R h0 = H[0];
#pragma unroll
    for (int s = 0; s < NMP; ++s) jz[s] = h0 * sJz[ch * NMP + s];
    for (int l = 1; l < NH; ++l) {
      const R hl = H[l];
      const R *a1 = sJz + (ch + l) * NMP, *a2 = sJz + (ch - l) * NMP;
#pragma unroll
      for (int s = 0; s < NMP; ++s) jz[s] += hl * (a1[s] + a2[s]);
    }
  } else {
    const R p0 = P[N - 1];
#pragma unroll
    for (int s = 0; s < NMP; ++s) {
      pjr[s] = p0 * sJr[c0 * NMP + s];
      pjp[s] = p0 * sJp[c0 * NMP + s];
    }
    for (int l = 1; l < N; ++l) {  // symmetric filter P
      const R pl = P[N - 1 + l];
      const R *a1 = sJr + (c0 + l) * NMP, *a2 = sJr + (c0 - l) * NMP;
      const R *b1 = sJp + (c0 + l) * NMP, *b2 = sJp + (c0 - l) * NMP;
#pragma unroll
      for (int s = 0; s < NMP; ++s) {
        pjr[s] += pl * (a1[s] + a2[s]);
        pjp[s] += pl * (b1[s] + b2[s]);
      }
    }
  }
  // (FP64: the own-column operands are loaded only now, after the z
  // operators, so that they and the operators' sums are not all live at once)
  if constexpr (!kEarly) load_own();

  const R *bpc = sBp + c0 * NMP, *brc = sBr + c0 * NMP;
#pragma unroll
  for (int m = 0; m <= M; ++m) {
    const int a = 2 * m, b = 2 * m + 1;
    const R mm = (R)m;
    // E_r at (i, j+1/2): (i m / r) B_z - D_B B_phi - P J_r
    if (j < Nr) {
      const R cre = -mm * bz[b] / rh - dbp[a] * idz, cim = mm * bz[a] / rh - dbp[b] * idz;
      er[a] += dt * (cre - pjr[a] * frr);
      er[b] += dt * (cim - pjr[b] * frr);
    } else {
      er[a] = er[b] = R(0);
    }
    // E_phi at (i, j): D_B B_r - dB_z/dr - P J_phi
    if (j == Nr || (j == 0 && m != 1)) {
      ep[a] = ep[b] = R(0);
    } else {
      const R fpf = (m == 0 || j == 0) ? fp_direct : fp_closure;
      R dre, dim_;
      if (j == 0) {
        dre = R(2) * bz[a] / dr;
        dim_ = R(2) * bz[b] / dr;
      } else {
        dre = (bz[a] - bzm[a]) / dr;
        dim_ = (bz[b] - bzm[b]) / dr;
      }
      ep[a] += dt * (dbr[a] * idz - dre - pjp[a] * fpf);
      ep[b] += dt * (dbr[b] * idz - dim_ - pjp[b] * fpf);
    }
    // E_z at (i+1/2, j): (1/r) d(r B_phi)/dr - (i m / r) B_r - J_z
    if (j == Nr || (j == 0 && m != 0)) {
      ez[a] = ez[b] = R(0);
    } else if (j == 0) {
      ez[a] += dt * (R(4) * bpc[a] / dr - jz[a] * fz);
      ez[b] += dt * (R(4) * bpc[b] / dr - jz[b] * fz);
    } else {
      const R rj = (R)j * dr;
      const R jp5 = (R)j + R(0.5), jm5 = (R)j - R(0.5);
      const R cre = (jp5 * bpc[a] - jm5 * bpm[a]) / rj + mm * brc[b] / rj;
      const R cim = (jp5 * bpc[b] - jm5 * bpm[b]) / rj - mm * brc[a] / rj;
      ez[a] += dt * (cre - jz[a] * fz);
      ez[b] += dt * (cim - jz[b] * fz);
    }
  }
  store_node<R, NMP>(E + 0 * cstride, plane, row + i, er);
  store_node<R, NMP>(E + 1 * cstride, plane, row + i, ep);
  store_node<R, NMP>(E + 2 * cstride, plane, row + i, ez);
  // clear the other current buffer for the next deposit
  R zero[NMP];
#pragma unroll
  for (int s = 0; s < NMP; ++s) zero[s] = R(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) store_node<R, NMP>(Jn + c * cstride, plane, row + i, zero);
}

// Bout = Bin - tau curl_E E; with avg != nullptr also avg = (Bin + Bout)/2,
// the time-centred B that the next gather uses (Eq. (12)).  Bout may be Bin.
template <typename R, int M>
__global__ __launch_bounds__(kFieldTile) void bfield_kernel(const Batch bt) {
  constexpr int NMP = 2 * (M + 1);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  R *lds = (R *)lds_raw;
  const int rn = batch_run(bt, blockIdx.x);
  const KRun &k = bt.run[rn];
  R *Bout = (R *)bt.bout[rn];
  const R *Bin = (const R *)bt.bin[rn];
  R *avg = (R *)bt.avg[rn];
  const R tau = (R)bt.tau[rn];
  const int Nz = k.Nz, Nr = k.Nr, N = k.N;
  const int ncol = (Nz + kFieldTile - 1) / kFieldTile;
  const int blk = (int)(blockIdx.x - bt.off[rn]);  // (row j, column block) of this run
  const int j = blk / ncol;
  const int i0 = (blk - j * ncol) * kFieldTile;
  const int t = threadIdx.x;
  const int W = kFieldTile + 2 * N;  // staged columns i0-N+1 .. i0+kFieldTile+N
  const long long plane = k.plane, cstride = plane * (NMP - 1);  // NM planes per component
  const long long row = (long long)j * Nz;
  const R *E = (const R *)k.E;
  R *sEp = lds, *sEr = lds + W * NMP;
  for (int r = t; r < W; r += kFieldTile) {
    const int col = wrap_any(i0 - N + 1 + r, Nz);
    R v[NMP];
    load_node<R, NMP>(E + 1 * cstride, plane, row + col, v);  // E_phi row j
    store_rec<R, NMP>(sEp + r * NMP, v);
    load_node<R, NMP>(E + 0 * cstride, plane, row + col, v);  // E_r (half row j; zero on row Nr)
    store_rec<R, NMP>(sEr + r * NMP, v);
  }
  __syncthreads();
  const int i = i0 + t;
  if (i >= Nz) return;
  const R dr = (R)k.dr, idz = (R)(1.0 / k.dz);
  const R *CE = (const R *)k.CE;
  const int c0 = t + N - 1;  // LDS index of column i
  R dep_[NMP], der[NMP];
#pragma unroll
  for (int s = 0; s < NMP; ++s) dep_[s] = der[s] = R(0);
  for (int l = 1; l <= N; ++l) {  // D_E: sum_l C^E_l (f_{i+l} - f_{i-l+1}), at z_{i+1/2}
    const R ce = CE[l - 1];
    const R *a1 = sEp + (c0 + l) * NMP, *a2 = sEp + (c0 - l + 1) * NMP;
    const R *b1 = sEr + (c0 + l) * NMP, *b2 = sEr + (c0 - l + 1) * NMP;
#pragma unroll
    for (int s = 0; s < NMP; ++s) {
      dep_[s] += ce * (a1[s] - a2[s]);
      der[s] += ce * (b1[s] - b2[s]);
    }
  }
  R bin_r[NMP], bin_p[NMP], bin_z[NMP], ez[NMP], ezp[NMP], epp[NMP];
  load_node<R, NMP>(Bin + 0 * cstride, plane, row + i, bin_r);
  load_node<R, NMP>(Bin + 1 * cstride, plane, row + i, bin_p);
  load_node<R, NMP>(Bin + 2 * cstride, plane, row + i, bin_z);
  load_node<R, NMP>(E + 2 * cstride, plane, row + i, ez);
  const bool up = j < Nr;
  if (up) {
    load_node<R, NMP>(E + 2 * cstride, plane, row + Nz + i, ezp);
    load_node<R, NMP>(E + 1 * cstride, plane, row + Nz + i, epp);
  } else {
#pragma unroll
    for (int s = 0; s < NMP; ++s) ezp[s] = epp[s] = R(0);
  }
  const R *epc = sEp + c0 * NMP, *erc = sEr + c0 * NMP;
  R nbr[NMP], nbp[NMP], nbz[NMP];
#pragma unroll
  for (int m = 0; m <= M; ++m) {
    const int a = 2 * m, b = 2 * m + 1;
    const R mm = (R)m;
    // B_r at (i+1/2, j): (i m / r) E_z - D_E E_phi; on the axis only m = 1 (E_z^1 ~ r)
    if (j == 0 && m != 1) {
      nbr[a] = nbr[b] = R(0);
    } else {
      R cre, cim;
      if (j == 0) {  // i E_z(r_1) / dr
        cre = -ezp[b] / dr;
        cim = ezp[a] / dr;
      } else {
        const R rj = (R)j * dr;
        cre = -mm * ez[b] / rj;
        cim = mm * ez[a] / rj;
      }
      nbr[a] = bin_r[a] - tau * (cre - dep_[a] * idz);
      nbr[b] = bin_r[b] - tau * (cim - dep_[b] * idz);
    }
    if (up) {
      const R rh = ((R)j + R(0.5)) * dr;
      // B_phi at (i+1/2, j+1/2): D_E E_r - dE_z/dr
      nbp[a] = bin_p[a] - tau * (der[a] * idz - (ezp[a] - ez[a]) / dr);
      nbp[b] = bin_p[b] - tau * (der[b] * idz - (ezp[b] - ez[b]) / dr);
      // B_z at (i, j+1/2): (1/r) d(r E_phi)/dr - (i m / r) E_r
      const R rj1 = (R)(j + 1) * dr, rj = (R)j * dr;
      const R cre = (rj1 * epp[a] - rj * epc[a]) / (rh * dr) + mm * erc[b] / rh;
      const R cim = (rj1 * epp[b] - rj * epc[b]) / (rh * dr) - mm * erc[a] / rh;
      nbz[a] = bin_z[a] - tau * cre;
      nbz[b] = bin_z[b] - tau * cim;
    } else {
      nbp[a] = nbp[b] = nbz[a] = nbz[b] = R(0);
    }
  }
  if (avg) {
    R v[NMP];
#pragma unroll
    for (int s = 0; s < NMP; ++s) v[s] = R(0.5) * (bin_r[s] + nbr[s]);
    store_node<R, NMP>(avg + 0 * cstride, plane, row + i, v);
#pragma unroll
    for (int s = 0; s < NMP; ++s) v[s] = R(0.5) * (bin_p[s] + nbp[s]);
    store_node<R, NMP>(avg + 1 * cstride, plane, row + i, v);
#pragma unroll
    for (int s = 0; s < NMP; ++s) v[s] = R(0.5) * (bin_z[s] + nbz[s]);
    store_node<R, NMP>(avg + 2 * cstride, plane, row + i, v);
  }
  store_node<R, NMP>(Bout + 0 * cstride, plane, row + i, nbr);
  store_node<R, NMP>(Bout + 1 * cstride, plane, row + i, nbp);
  store_node<R, NMP>(Bout + 2 * cstride, plane, row + i, nbz);
}

// Deterministic mode, between the push and the E update: each value of the
// step's current J[par] from its integer pair, J = a 2^-K + b 2^-(K+31),
// and the pair cleared for the next step.  One thread per value.
__global__ __launch_bounds__(256) void fix_convert_kernel(const Batch bt) {
  const int rn = batch_run(bt, blockIdx.x);
  const KRun &k = bt.run[rn];
  const long long i = (long long)(blockIdx.x - bt.off[rn]) * 256 + threadIdx.x;
  const long long n = 3 * (2 * k.M + 1) * k.plane;
  if (i >= n) return;
  unsigned long long *p = k.Jfix + 2 * i;
  const long long a = (long long)p[0], b = (long long)p[1];
  p[0] = p[1] = 0;
  const double s = 1.0 / k.qscale;  // a power of two: exact
  ((double *)k.J[bt.par])[i] = (double)a * s + (double)b * (s * 0x1p-31);
}

// ---------------------------------------------------------------------------
// small utility kernels

__global__ void zero_kernel(uint4 *p, size_t n16, unsigned char *tail, size_t ntail) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t a = t; a < n16; a += stride) p[a] = make_uint4(0, 0, 0, 0);
  if (t < ntail) tail[t] = 0;
}

// charge density of the electrons (diagnostic), FP64 records, physical units
template <typename R, int M>
__global__ __launch_bounds__(256) void rho_kernel(KRun k) {
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
  if (r > R(0)) {
    c = x / r;
    s = y / r;
  }
  const double q = -(double)((const R *)k.pw)[p];
  double *rho = (double *)k.rho;
  const double dzd = k.dz, drd = k.dr;
  // quadratic: 3 x 3 nodes round the nearest node, row r_{-1} onto r_1
  // with the sign (-1)^m of a scalar's mode m
  const int zn = (k.shape == 2 && f0 >= R(0.5)) ? 1 : 0, rn = (k.shape == 2 && fr >= R(0.5)) ? 1 : 0;
  double wz[3], wr[3];
  qspline((double)f0 - zn, wz);
  qspline((double)fr - rn, wr);
  double er = 1, ei = 0;
  for (int m = 0; m <= M; ++m) {
    if (m > 0) {
      const double tr = er * c + ei * s, ti = ei * c - er * s;
      er = tr;
      ei = ti;
    }
    const double cm = m == 0 ? 1.0 : 2.0;
    const int qa = m == 0 ? 0 : 2 * m - 1;
    if (k.shape == 2) {
      for (int b = 0; b < 3; ++b) {
        int j = j0 + rn - 1 + b;
        double sg = 1.0;
        if (j < 0) {
          j = -j;
          sg = m % 2 ? -1.0 : 1.0;
        }
        if ((m > 0 && j == 0) || j > Nr) continue;  // the m >= 1 density vanishes on the axis
        const double V = j == 0 ? kPi * drd * drd * dzd / 4.0 : 2.0 * kPi * (j * drd) * drd * dzd;
        for (int a = 0; a < 3; ++a) {
          const long long node = (long long)j * Nz + wrap_any(i0 + zn - 1 + a, Nz);
          const double S = sg * wz[a] * wr[b];
          atomic_add(rho + qa * k.plane + node, cm * q * er * S / V);
          if (m > 0) atomic_add(rho + (qa + 1) * k.plane + node, cm * q * ei * S / V);
        }
      }
      continue;
    }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const int j = j0 + b;
        if (m > 0 && j == 0) continue;  // the m >= 1 density vanishes on the axis
        const double V = j == 0 ? kPi * drd * drd * dzd / 4.0 : 2.0 * kPi * (j * drd) * drd * dzd;
        const double S = (a ? (double)f0 : 1.0 - (double)f0) * (b ? (double)fr : 1.0 - (double)fr);
        const long long node = (long long)j * Nz + wrap_once(i0 + a, Nz);
        atomic_add(rho + qa * k.plane + node, cm * q * er * S / V);
        if (m > 0) atomic_add(rho + (qa + 1) * k.plane + node, cm * q * ei * S / V);
      }
  }
}

// field energy per mode: per-block partial sums red[block * (M+1) + m]
template <typename R, int M>
__global__ __launch_bounds__(256) void energy_kernel(KRun k, int par) {
  constexpr int NM = 2 * M + 1;
  __shared__ double sh[256 * (M + 1)];
  const long long n = k.plane, cs = n * NM;
  const int tid = threadIdx.x;
  double acc[M + 1];
  for (int m = 0; m <= M; ++m) acc[m] = 0.0;
  const R *E = (const R *)k.E, *Bb = (const R *)k.Bbar;
  const double dzd = k.dz, drd = k.dr;
  for (long long idx = (long long)blockIdx.x * blockDim.x + tid; idx < n; idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx / k.Nz);
    const double vn = j == 0 ? kPi * drd * drd * dzd / 4.0 : 2.0 * kPi * (j * drd) * drd * dzd;
    const double vh = j < k.Nr ? 2.0 * kPi * ((j + 0.5) * drd) * drd * dzd : 0.0;
    for (int q = 0; q < NM; ++q) {
      const int m = (q + 1) / 2;
      auto sq = [&](const R *F, int c) {
        const double v = F[c * cs + q * n + idx];
        return v * v;
      };
      acc[m] += vh * (sq(E, 0) + sq(Bb, 1) + sq(Bb, 2)) + vn * (sq(E, 1) + sq(E, 2) + sq(Bb, 0));
    }
  }
  (void)par;
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

// Charge-weighted divergence sums over electrons with |u|^2 >= u2min and
// u_z > 0: w, w atan(ux/uz)^2, w atan(uy/uz)^2 and the count, per block.
template <typename R>
__global__ __launch_bounds__(256) void divergence_kernel(KRun k, double u2min) {
  __shared__ double sh[4][256];
  const int tid = threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const R *UX = (const R *)k.pux, *UY = (const R *)k.puy, *UZ = (const R *)k.puz, *W = (const R *)k.pw;
  for (long long p = (long long)blockIdx.x * blockDim.x + tid; p < k.np; p += (long long)gridDim.x * blockDim.x) {
    const double ux = UX[p], uy = UY[p], uz = UZ[p];
    if (!(uz > 0.0) || ux * ux + uy * uy + uz * uz < u2min) continue;
    const double w = W[p], tx = atan(ux / uz), ty = atan(uy / uz);
    a0 += w;
    a1 += w * tx * tx;
    a2 += w * ty * ty;
    a3 += 1.0;
  }
  sh[0][tid] = a0;
  sh[1][tid] = a1;
  sh[2][tid] = a2;
  sh[3][tid] = a3;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
      for (int c = 0; c < 4; ++c) sh[c][tid] += sh[c][tid + s];
    __syncthreads();
  }
  if (tid < 4) k.red[4 * blockIdx.x + tid] = sh[tid][0];
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
  if (k.shift > 0) {  // a window move: back by `shift` cells, outside the box -> the drop key n_keys
    iz -= k.shift;
    if (iz < 0 || iz >= k.Nz) return (int)k.n_keys;
  }
  iz = wrap_any(iz, k.Nz);
  const R x = ((const R *)k.px)[p], y = ((const R *)k.py)[p];
  const R r2 = fma(x, x, y * y);
  const int ir = clampi(radial_index(r2, sqrt(r2)), 0, k.Nr - 1);
  const int tile = (ir / k.Tr) * k.ntz + iz / k.Tz;
  const int local = (ir % k.Tr) * k.Tz + iz % k.Tz;
  return tile * (k.Tz * k.Tr) + local;
}

// Key and scatter kernels work on blocks of kSortBlock consecutive electrons
// (kSortPer per thread).  In the order of the previous sort such a block spans
// one or two tiles, so keys inside a window of two tiles' cells, starting at
// the tile of the block's first electron, are counted and ranked in LDS, with
// one device-memory atomic per cell and block; the drop key n_keys of a
// window move has a counter of its own after the window; other keys (the
// first sort of the loading order, electrons that changed tiles) take a
// device-memory atomic each.  The keys go to the run's spid buffer, free
// until the gather writes it.
constexpr int kSortPer = 8;
constexpr int kSortBlock = 256 * kSortPer;

template <typename R>
__global__ __launch_bounds__(256) void sort_key_kernel(const Batch bt) {
  extern __shared__ int32_t hist[];  // 2 TT counters, then the drop key's
  const int rn = batch_run(bt, blockIdx.x);
  const KRun &k = bt.run[rn];
  const int TT = k.Tz * k.Tr, HW = 2 * TT;
  const long long p0 = (long long)(blockIdx.x - bt.off[rn]) * kSortBlock;
  const int kb = cell_order<R>(k, p0) / TT * TT;  // window start (p0 < np: blocks cover np)
  for (int d = threadIdx.x; d <= HW; d += blockDim.x) hist[d] = 0;
  __syncthreads();
  int32_t *keys = (int32_t *)k.spid;
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const long long p = p0 + q * 256 + threadIdx.x;
    if (p >= k.np) break;
    const int key = cell_order<R>(k, p);
    keys[p] = key;
    const int d = key - kb;
    if (key >= k.n_keys) atomicAdd(&hist[HW], 1);
    else if (d >= 0 && d < HW) atomicAdd(&hist[d], 1);
    else atomicAdd(&k.cell_count[key], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < HW; d += blockDim.x)
    if (hist[d] > 0 && kb + d < k.n_keys) atomicAdd(&k.cell_count[kb + d], hist[d]);
  if (threadIdx.x == 0 && hist[HW] > 0) atomicAdd(&k.cell_count[k.n_keys], hist[HW]);
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

// each electron's entry (id, source index) into its cell's range, in
// whatever order the atomics run: ranks within the block from LDS atomics,
// then one device-memory atomic per cell of the window reserves the block's
// share of the cell (cell_count holds a copy of cell_start, the fill cursor)
__global__ __launch_bounds__(256) void sort_scatter_kernel(const Batch bt) {
  extern __shared__ int32_t hist[];  // 2 TT + 1 counters (the last the drop key's), then 2 TT + 1 bases
  const int rn = batch_run(bt, blockIdx.x);
  const KRun &k = bt.run[rn];
  const int TT = k.Tz * k.Tr, HW = 2 * TT;
  int32_t *base = hist + HW + 1;
  const long long p0 = (long long)(blockIdx.x - bt.off[rn]) * kSortBlock;
  const int32_t *keys = (const int32_t *)k.spid;
  const int kb = keys[p0] / TT * TT;  // the window of the key kernel
  for (int d = threadIdx.x; d <= HW; d += blockDim.x) hist[d] = 0;
  __syncthreads();
  int key[kSortPer], rank[kSortPer];
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const long long p = p0 + q * 256 + threadIdx.x;
    key[q] = p < k.np ? keys[p] : -1;
    const bool drop = key[q] >= k.n_keys;  // the drop key: its own counter
    const int d = drop ? HW : key[q] - kb;
    rank[q] = (p < k.np && (drop || (d >= 0 && d < HW))) ? atomicAdd(&hist[d], 1) : -1;
  }
  __syncthreads();
  for (int d = threadIdx.x; d <= HW; d += blockDim.x) {
    const long long c = d == HW ? k.n_keys : kb + d;
    base[d] = (hist[d] > 0 && (d == HW || c < k.n_keys)) ? atomicAdd(&k.cell_count[c], hist[d]) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kSortPer; ++q) {
    const long long p = p0 + q * 256 + threadIdx.x;
    if (p >= k.np) break;
    const int dq = key[q] >= k.n_keys ? HW : key[q] - kb;
    const int pos = rank[q] >= 0 ? base[dq] + rank[q] : atomicAdd(&k.cell_count[key[q]], 1);
    if (const uint32_t f = sort_index_flags(pos, k.np, kSortBadSlot)) {
      atomicOr(k.flags, f);
      continue;
    }
    k.perm[pos] = ((uint64_t)(k.pid[p] & kIdMask) << 32) | (uint64_t)p;
  }
}

// entries of one cell [b, e) in ascending id (insertion sort; cells are short)
__device__ __forceinline__ void sort_cell(uint64_t *ent, int b, int e) {
  for (int a = b + 1; a < e; ++a) {
    const uint64_t v = ent[a];
    int t = a - 1;
    while (t >= b && ent[t] > v) {  // ids are unique, so the entry order is the id order
      ent[t + 1] = ent[t];
      --t;
    }
    ent[t + 1] = v;
  }
}

// Order a tile's n entries `ent` by (cell, id), then gather its electrons into
// the transposed order the push kernel reads (see round_count).  Inlined with
// `ent` either in LDS or in device memory, so that every access has a known
// address space.  In LDS (kRank) the entries stay where they are and `pos`
// lists them in (cell, id) order (their ranks, rank_cells); in device memory
// each cell is sorted in place by one thread.  Cell bounds are clamped to the
// tile and a source index out of range is skipped, so that no data can drive
// an access out of bounds.
template <typename R, bool kRank>
__device__ __forceinline__ void sort_tile(const KRun &k, uint64_t *ent, const uint16_t *pos, long long c0, int beg,
                                          int n) {
  const long long TT = (long long)k.Tz * k.Tr;
  if constexpr (!kRank) {
    for (long long c = threadIdx.x; c < TT; c += blockDim.x) {
      const int b = clampi(k.cell_start[c0 + c] - beg, 0, n), e = clampi(k.cell_start[c0 + c + 1] - beg, 0, n);
      sort_cell(ent, b, e);
    }
    __syncthreads();
  }
  const int chunk = (n + 255) / 256;
  const int S = round_spread(n, chunk, TT);
  const int t = threadIdx.x;
  // the gather, kG rounds at a time: every load of the group is issued
  // before its stores, so that the rounds' memory latencies overlap (the
  // source and destination buffers are distinct)
  constexpr bool F64 = std::is_same<R, double>::value;
  using Zw = typename std::conditional<F64, double, int>::type;  // the z word
  constexpr int kG = 4;
  const Zw *__restrict__ PZ = (const Zw *)k.pz;
  const float *__restrict__ PF = (const float *)k.pfz;
  const R *__restrict__ PX = (const R *)k.px, *__restrict__ PY = (const R *)k.py;
  const R *__restrict__ PUX = (const R *)k.pux, *__restrict__ PUY = (const R *)k.puy;
  const R *__restrict__ PUZ = (const R *)k.puz, *__restrict__ PW = (const R *)k.pw;
  const uint32_t *__restrict__ PID = k.pid;
  Zw *__restrict__ SZ = (Zw *)k.sz;
  float *__restrict__ SF = (float *)k.sfz;
  R *__restrict__ SX = (R *)k.sx, *__restrict__ SY = (R *)k.sy, *__restrict__ SUX = (R *)k.sux;
  R *__restrict__ SUY = (R *)k.suy, *__restrict__ SUZ = (R *)k.suz, *__restrict__ SW = (R *)k.sw;
  uint32_t *__restrict__ SID = k.spid;
  int base = 0;
  for (int it0 = 0; it0 < chunk; it0 += kG) {
    int dd[kG];
    long long ss[kG];
    bool ok[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int it = it0 + g;
      const int cnt = it < chunk ? round_count(n, chunk, it) : 0;
      dd[g] = beg + base + t;
      base += cnt;
      int L = t < cnt ? round_column(t, cnt, S) * chunk + it : 0;  // list position
      if constexpr (kRank) L = pos[L];
      ss[g] = t < cnt ? (long long)(ent[L] & 0xffffffffu) : -1;
      ok[g] = ss[g] >= 0 && ss[g] < k.np;
      if (t < cnt && !ok[g]) atomicOr(k.flags, sort_index_flags(ss[g], k.np, kSortBadSource));
    }
    Zw vz[kG];
    float vf[kG];
    R vx[kG], vy[kG], vux[kG], vuy[kG], vuz[kG], vw[kG];
    uint32_t vid[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      if (!ok[g]) continue;
      const long long q = ss[g];
      vz[g] = PZ[q];
      if constexpr (!F64) vf[g] = PF[q];
      vx[g] = PX[q];
      vy[g] = PY[q];
      vux[g] = PUX[q];
      vuy[g] = PUY[q];
      vuz[g] = PUZ[q];
      vw[g] = PW[q];
      vid[g] = PID[q];
    }
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      if (!ok[g]) continue;
      const int d = dd[g];
      SZ[d] = vz[g] - (Zw)k.shift;  // a window move: back by `shift` cells (exact)
      if constexpr (!F64) SF[d] = vf[g];
      SX[d] = vx[g];
      SY[d] = vy[g];
      SUX[d] = vux[g];
      SUY[d] = vuy[g];
      SUZ[d] = vuz[g];
      SW[d] = vw[g];
      SID[d] = vid[g];
    }
  }
}

// (cell, id) order of a tile's n entries held in LDS, all threads at once:
// entry a of the cell range [b, e) (the last cell starting at or before a,
// from the tile's clamped cell starts cs) has the rank r = #{x in [b, e):
// ent[x] < ent[a]} (ids are unique, so the entry order is the id order), and
// pos[b + r] = a.  pos starts as the identity, so that inconsistent data can
// leave it stale but never out of range.
__device__ __forceinline__ void rank_cells(const uint64_t *ent, uint16_t *pos, const int32_t *cs, int TT, int n) {
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    int lo = 0, hi = TT - 1;  // cs[lo] <= a
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cs[mid] <= a) lo = mid;
      else hi = mid - 1;
    }
    const int b = cs[lo], e = cs[lo + 1];
    const uint64_t v = ent[a];
    int r = 0;
    for (int x = b; x < e; ++x) r += ent[x] < v ? 1 : 0;
    if (b + r < n) pos[b + r] = (uint16_t)a;
  }
}

// One workgroup per tile: its entries in LDS, ranked (measured faster with
// 16 electrons per cell: sort 2.60 -> 2.26 ms on the 8192 x 512 run) or, with
// a few per cell, each cell sorted by one thread (faster there: ranking took
// the six-run scan's sort, 4 per cell, from 1.26 to 1.32 ms); in device
// memory, sorted in place, for a tile too dense for the LDS budget.
template <typename R>
__global__ __launch_bounds__(256) void sort_tile_kernel(const Batch bt) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int rn = batch_run(bt, blockIdx.x);
  const KRun &k = bt.run[rn];
  const long long TT = (long long)k.Tz * k.Tr;
  const long long c0 = (long long)(blockIdx.x - bt.off[rn]) * TT;
  const int beg = k.cell_start[c0], end = k.cell_start[c0 + TT];
  const int n = end - beg;
  if (threadIdx.x == 0) {
    uint32_t f = sort_tile_flags(beg, end, k.np);
    if (blockIdx.x == bt.off[rn])  // one block per run
      f |= sort_count_flags(k.cell_start[k.n_keys], k.np, k.shift > 0);
    if (f) atomicOr(k.flags, f);
  }
  if (n <= 0 || beg < 0 || end > k.np) return;
  if (n <= kSortLdsEntries) {
    uint64_t *ent = (uint64_t *)lds_raw;
    for (int a = threadIdx.x; a < n; a += blockDim.x) ent[a] = k.perm[beg + a];
    if (n > kSortRankPerCell * TT) {  // dense cells: ranks, all threads at once
      uint16_t *pos = (uint16_t *)(lds_raw + (size_t)kSortLdsEntries * sizeof(uint64_t));
      int32_t *cs = (int32_t *)(lds_raw + (size_t)kSortLdsEntries * (sizeof(uint64_t) + sizeof(uint16_t)));
      for (int a = threadIdx.x; a < n; a += blockDim.x) pos[a] = (uint16_t)a;
      for (long long c = threadIdx.x; c <= TT; c += blockDim.x) cs[c] = clampi(k.cell_start[c0 + c] - beg, 0, n);
      __syncthreads();
      rank_cells(ent, pos, cs, (int)TT, n);
      __syncthreads();
      sort_tile<R, true>(k, ent, pos, c0, beg, n);
    } else {  // a few entries per cell: each cell sorted in place by one thread
      __syncthreads();
      sort_tile<R, false>(k, ent, nullptr, c0, beg, n);
    }
  } else {
    sort_tile<R, false>(k, k.perm + beg, nullptr, c0, beg, n);
  }
}

// ---------------------------------------------------------------------------
// launch helpers

thread_local char g_err[256] = "";




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

// block offsets of the runs of a batch, `per(k)` blocks each; false if the
// launch would be empty
template <typename F>
bool set_offsets(Batch &b, F per) {
  b.off[0] = 0;
  for (int i = 0; i < b.n; ++i) b.off[i + 1] = b.off[i] + per(b.run[i]);
  for (int i = b.n; i < kMaxBatch; ++i) b.off[i + 1] = b.off[b.n];
  return b.off[b.n] > 0;
}

template <typename R>
constexpr int prec_of() {
  return std::is_same<R, double>::value ? PIC_PREC_FP64 : PIC_PREC_FP32;
}

// the push kernel of (deterministic mode, shape order); the deterministic
// mode is FP64 only (nullptr otherwise)
template <typename R, int M>
auto push_kernel_of(bool det, int sh) -> decltype(&push_kernel<R, M, false, 1>) {
  if (!det) return sh == 2 ? push_kernel<R, M, false, 2> : push_kernel<R, M, false, 1>;
  if constexpr (std::is_same<R, double>::value)
    return sh == 2 ? push_kernel<R, M, true, 2> : push_kernel<R, M, true, 1>;
  return nullptr;
}

template <typename R, int M>
struct PrepL {
  static int run(int Tz, int Tr, bool det, int sh) {
    // dynamic LDS above 64 KB must be allowed per kernel, once, outside any capture
    const auto f = push_kernel_of<R, M>(det, sh);
    if (!f) return PIC_E_INVALID;
    const size_t lds = push_lds_bytes(M, Tz, Tr, prec_of<R>(), det, sh);
    if (lds <= 65536) return PIC_OK;
    return check(hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                 "hipFuncSetAttribute(push_kernel)");
  }
};
template <typename R, int M>
struct PushL {
  static int run(Batch &b, hipStream_t s) {
    if (!set_offsets(b, [](const KRun &k) { return k.np > 0 ? (long long)k.ntz * k.ntr : 0LL; })) return PIC_OK;
    const KRun &k0 = b.run[0];
    const bool det = b.det != 0;
    const int sh = k0.shape;
    const auto f = push_kernel_of<R, M>(det, sh);
    if (!f) return PIC_E_INVALID;
    const size_t lds = push_lds_bytes(M, k0.Tz, k0.Tr, prec_of<R>(), det, sh);
    // persistent grid: as many workgroups as are resident at once (a multiple
    // of 8, one share per XCD), each walking its tiles; the occupancy query
    // is cached per thread for the last (device, kernel, LDS size)
    static thread_local size_t lds_seen = 0;
    static thread_local int dev_seen = -1;
    static thread_local const void *f_seen = nullptr;
    static thread_local long long resident = 0;
    int dev = 0;
    if (int rc = check(hipGetDevice(&dev), "hipGetDevice")) return rc;
    if (lds != lds_seen || dev != dev_seen || (const void *)f != f_seen) {
      int per_cu = 0, cus = 0;
      int rc = check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, lds),
                     "hipOccupancyMaxActiveBlocksPerMultiprocessor");
      if (!rc) rc = check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
      if (rc) return rc;
      resident = (long long)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
      resident = resident >= 8 ? resident & ~7LL : resident;
      lds_seen = lds;
      dev_seen = dev;
      f_seen = (const void *)f;
    }
    const long long grid = b.off[b.n] < resident ? b.off[b.n] : resident;
    // XCD-aware dealing from 32 tiles per workgroup (measured: the
    // 8192 x 512 push, 85 tiles per workgroup, 2.4% faster, the six-run
    // scan's 1%; the 4096 x 256 FP64 push, 17 per workgroup, 3-5% slower)
    b.deal_xcd = b.off[b.n] >= kDealMinPerGroup * grid ? 1 : 0;
    zero_kernel<<<1, 64, 0, s>>>((uint4 *)b.run[0].work, 2, nullptr, 0);  // the 8 ticket counters from 0
    if (int rc = check(hipGetLastError(), "zero_kernel")) return rc;
    void *args[] = {&b};
    return check(hipLaunchKernel((const void *)f, dim3((unsigned)grid), dim3(256), args, lds, s), "push_kernel");
  }
};
template <typename R, int M>
struct EL {
  static int run(Batch &b, hipStream_t s) {
    set_offsets(b, [](const KRun &k) { return (long long)((k.Nz + kFieldTile - 1) / kFieldTile) * (k.Nr + 1); });
    const size_t rec = (size_t)2 * (M + 1) * sizeof(R);
    const size_t wb = (size_t)(kFieldTile + 2 * b.run[0].N);
    if (b.run[0].NH > 0) {  // all runs of a context share the option; their tap counts differ
      int nh = 0;
      for (int r = 0; r < b.n; ++r) nh = b.run[r].NH > nh ? b.run[r].NH : nh;
      const size_t lds = (2 * wb + (size_t)(kFieldTile + 2 * (nh - 1))) * rec;
      efield_kernel<R, M, true><<<(unsigned)b.off[b.n], kFieldTile, lds, s>>>(b);
    } else {
      efield_kernel<R, M, false><<<(unsigned)b.off[b.n], kFieldTile, 4 * wb * rec, s>>>(b);
    }
    return check(hipGetLastError(), "efield_kernel");
  }
};
template <typename R, int M>
struct BL {
  static int run(Batch &b, hipStream_t s) {
    set_offsets(b, [](const KRun &k) { return (long long)((k.Nz + kFieldTile - 1) / kFieldTile) * (k.Nr + 1); });
    const size_t lds = (size_t)2 * (kFieldTile + 2 * b.run[0].N) * 2 * (M + 1) * sizeof(R);
    bfield_kernel<R, M><<<(unsigned)b.off[b.n], kFieldTile, lds, s>>>(b);
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
int record_device_error(int hip_status, const char *what) { return check((hipError_t)hip_status, what); }

int launch_push(Batch &b, int prec, void *stream) {
  return dispatch_M<PushL>(prec, b.run[0].M, b, (hipStream_t)stream);
}
int launch_efield(Batch &b, int prec, void *stream) {
  return dispatch_M<EL>(prec, b.run[0].M, b, (hipStream_t)stream);
}
int launch_bfield(Batch &b, int prec, void *stream) {
  return dispatch_M<BL>(prec, b.run[0].M, b, (hipStream_t)stream);
}
int prepare_kernels(int prec, int M, int Tz, int Tr, bool det, int sh) {
  return dispatch_M<PrepL>(prec, M, Tz, Tr, det, sh);
}
int launch_fix_convert(Batch &b, void *stream) {
  if (!set_offsets(b, [](const KRun &k) { return (3 * (2 * k.M + 1) * k.plane + 255) / 256; })) return PIC_OK;
  fix_convert_kernel<<<(unsigned)b.off[b.n], 256, 0, (hipStream_t)stream>>>(b);
  return check(hipGetLastError(), "fix_convert_kernel");
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
int launch_divergence(const KRun &k, int prec, double u2min, int nblocks_max, int *nblocks, void *stream) {
  long long want = (k.np + 255) / 256;
  int nb = (int)(want < nblocks_max ? want : nblocks_max);
  if (nb < 1) nb = 1;
  *nblocks = nb;
  if (prec == PIC_PREC_FP64) divergence_kernel<double><<<nb, 256, 0, (hipStream_t)stream>>>(k, u2min);
  else divergence_kernel<float><<<nb, 256, 0, (hipStream_t)stream>>>(k, u2min);
  return check(hipGetLastError(), "divergence_kernel");
}
int launch_tracked_gamma(const KRun &k, int prec, double *gamma, int64_t *ids, void *stream) {
  if (k.np == 0 || k.n_tracked == 0) return PIC_OK;
  const unsigned blocks = (unsigned)((k.np + 255) / 256);
  if (prec == PIC_PREC_FP64) tracked_gamma_kernel<double><<<blocks, 256, 0, (hipStream_t)stream>>>(k, gamma, ids);
  else tracked_gamma_kernel<float><<<blocks, 256, 0, (hipStream_t)stream>>>(k, gamma, ids);
  return check(hipGetLastError(), "tracked_gamma_kernel");
}

// ---------------------------------------------------------------------------
// moving window: each of E, B[0], B[1], Bbar back by s columns in place, row
// by row (one workgroup per row of (Nr+1) Nz reals); a chunk's reads
// (columns [c0+s, c0+s+C)) all land before its writes ([c0, c0+C)), and no
// chunk reads what an earlier one wrote
constexpr int kShiftPer = 4;
template <typename R>
__global__ __launch_bounds__(256) void window_shift_kernel(R *a0, R *a1, R *a2, R *a3, long long rows, int Nz, int s,
                                                           int guard) {
  const long long b = blockIdx.x;
  R *base = b < rows ? a0 : (b < 2 * rows ? a1 : (b < 3 * rows ? a2 : a3));
  R *row = base + (b % rows) * (long long)Nz;
  for (int c0 = 0; c0 < Nz; c0 += 256 * kShiftPer) {
    R v[kShiftPer];
#pragma unroll
    for (int j = 0; j < kShiftPer; ++j) {
      const int i = c0 + j * 256 + (int)threadIdx.x;
      v[j] = (i < Nz && s < Nz - i) ? row[i + s] : R(0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kShiftPer; ++j) {
      const int i = c0 + j * 256 + (int)threadIdx.x;
      if (i < Nz) row[i] = i < guard ? R(0) : v[j];
    }
  }
}

int launch_window_shift(const KRun &k, int prec, int guard, void *stream) {
  if (k.shift <= 0) return PIC_OK;
  const long long rows = 3LL * (2 * k.M + 1) * (k.Nr + 1);
  const unsigned blocks = (unsigned)(4 * rows);
  const hipStream_t s = (hipStream_t)stream;
  if (prec == PIC_PREC_FP64)
    window_shift_kernel<double><<<blocks, 256, 0, s>>>((double *)k.E, (double *)k.B[0], (double *)k.B[1],
                                                       (double *)k.Bbar, rows, k.Nz, k.shift, guard);
  else
    window_shift_kernel<float><<<blocks, 256, 0, s>>>((float *)k.E, (float *)k.B[0], (float *)k.B[1],
                                                      (float *)k.Bbar, rows, k.Nz, k.shift, guard);
  return check(hipGetLastError(), "window_shift_kernel");
}

int launch_sort(Batch &b, int prec, void *stream) {
  const hipStream_t s = (hipStream_t)stream;
  int rc;
  for (int i = 0; i < b.n; ++i)
    if ((rc = launch_zero(b.run[i].cell_count, (size_t)(b.run[i].n_keys + 1) * 4, stream))) return rc;
  const auto pblocks = [](const KRun &k) { return (k.np + kSortBlock - 1) / kSortBlock; };
  const size_t hw = ((size_t)2 * b.run[0].Tz * b.run[0].Tr + 1) * sizeof(int32_t);  // a 2-tile window + the drop key
  if (set_offsets(b, pblocks)) {
    if (prec == PIC_PREC_FP64) sort_key_kernel<double><<<(unsigned)b.off[b.n], 256, hw, s>>>(b);
    else sort_key_kernel<float><<<(unsigned)b.off[b.n], 256, hw, s>>>(b);
    if ((rc = check(hipGetLastError(), "sort_key_kernel"))) return rc;
  }
  for (int i = 0; i < b.n; ++i) {
    const KRun &k = b.run[i];
    const long long nk = k.n_keys + 1;
    if ((rc = scan_exclusive(k.cell_count, k.cell_start, nk, k.scan_tmp, s))) return rc;
    if (k.np == 0) continue;
    copy_i32_kernel<<<(unsigned)((nk + 255) / 256), 256, 0, s>>>(k.cell_count, k.cell_start, nk);
    if ((rc = check(hipGetLastError(), "copy_i32_kernel"))) return rc;
  }
  if (!set_offsets(b, pblocks)) return PIC_OK;
  sort_scatter_kernel<<<(unsigned)b.off[b.n], 256, 2 * hw, s>>>(b);
  if ((rc = check(hipGetLastError(), "sort_scatter_kernel"))) return rc;
  set_offsets(b, [](const KRun &k) { return k.np > 0 ? (long long)k.ntz * k.ntr : 0LL; });
  // entries, their ranks and the tile's cell starts (the runs of a batch share the tile)
  const size_t lds = (size_t)kSortLdsEntries * (sizeof(uint64_t) + sizeof(uint16_t)) +
                     ((size_t)b.run[0].Tz * b.run[0].Tr + 1) * sizeof(int32_t);
  if (lds > 65536) {  // tiles of more than about 4800 cells
    const void *f = prec == PIC_PREC_FP64 ? (const void *)sort_tile_kernel<double> : (const void *)sort_tile_kernel<float>;
    if ((rc = check(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                    "hipFuncSetAttribute(sort_tile_kernel)")))
      return rc;
  }
  if (prec == PIC_PREC_FP64) sort_tile_kernel<double><<<(unsigned)b.off[b.n], 256, lds, s>>>(b);
  else sort_tile_kernel<float><<<(unsigned)b.off[b.n], 256, lds, s>>>(b);
  if ((rc = check(hipGetLastError(), "sort_tile_kernel"))) return rc;
  for (int i = 0; i < b.n; ++i) {
    KRun &k = b.run[i];
    if (k.np == 0) continue;
    std::swap(k.pz, k.sz);
    std::swap(k.pfz, k.sfz);
    std::swap(k.px, k.sx);
    std::swap(k.py, k.sy);
    std::swap(k.pux, k.sux);
    std::swap(k.puy, k.suy);
    std::swap(k.puz, k.suz);
    std::swap(k.pw, k.sw);
    std::swap(k.pid, k.spid);
  }
  return PIC_OK;
}

}  // namespace pic
