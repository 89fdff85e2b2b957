// Allocation-free form of the l2-ball projection (eq. l2ball_prox), for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// The projection's only scratch is its FP64 partial sums of ||in - center||^2
// (a fixed number of first-stage blocks plus the total, independent of the
// length). Here they live in the file-scope device array `scratch`, one copy
// per GPU, held until the process ends. Host code never uses the array's name
// as an address: on the first call on a device, with that device current,
// hipGetSymbolAddress gives the device address, which is kept per device and
// passed to the kernels. Every call on one GPU shares that GPU's array, so
// calls that overlap on one GPU (two streams, two threads) race; the kernels
// write every partial before reading it, so nothing needs clearing.
#include <mutex>

#include "ops.hpp"

namespace pr {
namespace {

constexpr size_t kNoallocDoubles = 2048;   // 16 KB; the projection uses ball_scratch_bytes()
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kNoallocDoubles];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void** out) {
  int dev = 0;
  PR_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d: at most %d devices are supported", dev, kMaxDevices);
    return PR_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    PR_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned no address for the projection scratch");
      return PR_EHIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" int pr_proj_l2ball_noalloc(const void* in, const void* center, void* out, int64_t len, int32_t prec,
                                      double eps, double* dist, void* stream) {
  clear_error();
  if (len < 0) { set_error("len < 0"); return PR_EINVAL; }
  if (len > 0) { PR_NONNULL(in); PR_NONNULL(center); PR_NONNULL(out); }
  if (prec != PR_F32 && prec != PR_F64) { set_error("prec = %d", prec); return PR_EINVAL; }
  if (!(eps >= 0)) { set_error("eps must be >= 0"); return PR_EINVAL; }
  if (ball_scratch_bytes() > sizeof(scratch)) {
    set_error("the projection needs %zu bytes of scratch, the static array holds %zu", ball_scratch_bytes(),
              sizeof(scratch));
    return PR_EUNSUPPORTED;
  }
  PR_TRY(check_sticky());
  void* sp = nullptr;
  PR_TRY(scratch_address(&sp));
  return proj_l2ball(in, center, out, len, prec, eps, sp, dist, as_stream(stream));
}
