// noalloc.hip -- pic_divergence_arrays: the divergence reduction of
// pic_divergence over electron arrays the caller holds in device memory,
// with no allocation and no workspace: its per-block partial sums live in a
// file-scope device array of fixed size, one copy per GPU, for callers that
// cannot allocate device memory (code under graph capture, serving loops,
// harnesses that forbid it).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "pic_internal.h"

namespace pic {
namespace {

// Partial sums of the reduction: kNoAllocBlocks blocks of 4 FP64 sums (w,
// w theta_x^2, w theta_y^2, count), 64 KiB per GPU, held until the process
// ends.  Each block writes its own 4 sums, so nothing needs clearing between
// calls; calls that overlap on one GPU race for it.
constexpr int kNoAllocBlocks = 2048;
constexpr long long kNoAllocMaxElectrons = (long long)kNoAllocBlocks * 256 * 64;  // 64 per thread
__device__ __align__(256) double scratch[kNoAllocBlocks * 4];

// The device address of `scratch` on each device, looked up once per device
// with that device current (the name is only a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

int scratch_on_current_device(double **out) {
  int dev = 0;
  if (int rc = record_device_error((int)hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev < 0 || dev >= kMaxDevices) return PIC_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (int rc = record_device_error((int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress"))
      return rc;
    g_scratch[dev] = (double *)p;
  }
  *out = g_scratch[dev];
  return PIC_OK;
}

}  // namespace
}  // namespace pic

using namespace pic;

extern "C" int pic_divergence_arrays(int32_t precision, int64_t n, const void *ux, const void *uy, const void *uz,
                                     const void *w, double gamma_min, double *out, void *hip_stream) {
  set_error(PIC_OK, "%s", "");
  if (precision != PIC_PREC_FP64 && precision != PIC_PREC_FP32) return set_error(PIC_E_INVALID, "precision must be 64 or 32");
  if (!out || n < 0 || (n > 0 && (!ux || !uy || !uz || !w))) return set_error(PIC_E_INVALID, "bad arrays or count");
  if (!(gamma_min >= 1.0) || !std::isfinite(gamma_min)) return set_error(PIC_E_INVALID, "gamma_min must be >= 1");
  if (n > kNoAllocMaxElectrons)
    return set_error(PIC_E_NOMEM, "%lld electrons exceed the %lld one call of pic_divergence_arrays takes",
                         (long long)n, kNoAllocMaxElectrons);
  for (int c = 0; c < 6; ++c) out[c] = 0.0;
  if (n == 0) return PIC_OK;
  double *part = nullptr;
  if (int rc = scratch_on_current_device(&part)) return set_error(rc, "%s", last_device_error());
  // the divergence kernel of pic_divergence, on a view of the caller's arrays
  KRun k{};
  k.np = n;
  k.pux = const_cast<void *>(ux);
  k.puy = const_cast<void *>(uy);
  k.puz = const_cast<void *>(uz);
  k.pw = const_cast<void *>(w);
  k.red = part;
  const hipStream_t s = (hipStream_t)hip_stream;
  int nb = 0;
  if (int rc = launch_divergence(k, precision, gamma_min * gamma_min - 1.0, kNoAllocBlocks, &nb, s))
    return set_error(rc, "%s", last_device_error());
  static thread_local double host[kNoAllocBlocks * 4];  // no per-call host allocation either
  if (int rc = record_device_error((int)hipMemcpyAsync(host, part, (size_t)nb * 4 * sizeof(double),
                                                        hipMemcpyDeviceToHost, s), "hipMemcpyAsync"))
    return set_error(rc, "%s", last_device_error());
  if (int rc = record_device_error((int)hipStreamSynchronize(s), "hipStreamSynchronize"))
    return set_error(rc, "%s", last_device_error());
  for (int c = 0; c < 4; ++c) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += host[b * 4 + c];  // blocks in order: the same sum every call
    if (!std::isfinite(acc)) return set_error(PIC_E_NUMERIC, "a divergence sum is not finite");
    out[c] = acc;
  }
  out[4] = out[0] > 0 ? std::sqrt(out[1] / out[0]) : 0.0;
  out[5] = out[0] > 0 ? std::sqrt(out[2] / out[0]) : 0.0;
  return PIC_OK;
}
