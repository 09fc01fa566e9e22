// bilu_apply_noalloc: the preconditioner apply with its work vectors in a
// fixed device array instead of the handle's workspace, for callers that
// cannot allocate (code under stream capture, serving loops, harnesses that
// forbid it).  The array is file-scope and per device; its address is looked
// up once per device with that device current and kept.
#include <mutex>

#include "internal.h"

namespace bilu {
namespace {

// three vectors (x and y in the permuted numbering, the forward result t)
// of at most kStaticMaxN doubles each: 48 MiB per device
constexpr int64_t kStaticMaxN = int64_t(1) << 21;
static __device__ __align__(256) double scratch[3 * kStaticMaxN];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's array (looked up on its first use on
// the current device).
hipError_t static_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace bilu

using namespace bilu;

extern "C" bilu_status bilu_apply_noalloc(bilu_handle* h, const double* x, double* y) {
  if (!h || !x || !y || x == y) return fail(h, BILU_ERR_INVALID, "bilu_apply_noalloc: bad pointers");
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "bilu_apply_noalloc before bilu_factor");
  const int64_t n = h->n;
  if (n > kStaticMaxN)
    return fail(h, BILU_ERR_INVALID,
                "bilu_apply_noalloc: n = " + std::to_string(n) + " exceeds its limit of " +
                    std::to_string(kStaticMaxN) + " unknowns (use bilu_apply)");
  try {
    double* base = nullptr;
    hipError_t e = static_scratch(&base);
    if (e != hipSuccess) return hip_check(h, e, "bilu_apply_noalloc: device array");
    double* xp = base;
    double* yp = base + kStaticMaxN;
    double* tp = base + 2 * kStaticMaxN;
    launch_gather(h->stream, n, h->d_perm.p, h->sl(), x, xp);
    bilu_status s = apply_permuted(h, xp, yp, tp, false);
    if (s != BILU_OK) return s;
    launch_scatter(h->stream, n, h->perm_col(), h->sr(), yp, y);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_check(h, e, "bilu_apply_noalloc");
    return BILU_OK;
  } catch (...) {
    return fail(h, BILU_ERR_INTERNAL, "bilu_apply_noalloc: unexpected exception");
  }
}
