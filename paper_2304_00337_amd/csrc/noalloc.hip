// Gram product for callers that cannot allocate device memory (bl_gram_noalloc).
//
// The row-block partial sums of the Gram kernels live in one file-scope device array of
// fixed size instead of a per-call hipMalloc.  Its device address is looked up once per GPU
// (with that GPU current) and kept: the array's name in host code is only a host-side
// stand-in and must never be passed to a kernel.  Every call on a GPU shares that GPU's copy,
// so calls that overlap on one GPU (other streams or handles) race; the kernels overwrite
// every partial they later read, so nothing needs clearing between calls.
#include "engine.h"

#include <mutex>

namespace bl {
namespace {

constexpr int64_t kNoAllocDoubles = (int64_t)1 << 21;   // 16 MiB per GPU
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on the first call per device).
int scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(BL_EINVAL, "device index out of range%s");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return set_error(BL_EHIP, "scratch address lookup failed: %s", hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return BL_OK;
}

}  // namespace
}  // namespace bl

using namespace bl;

extern "C" {

int bl_gram_noalloc(bl_solver* s, const void* X, int32_t q, const void* W, int32_t r, int64_t len,
                    void* out_dev) {
  if (!s || !X || !W || !out_dev || q < 1 || r < 1 || len < 1)
    return set_error(BL_EINVAL, "invalid gram arguments%s");
  const int64_t need = (int64_t)gram_blocks(len) * q * r * 2;
  if (need > kNoAllocDoubles)
    return set_error(BL_EINVAL, "q * r too large for the fixed scratch of bl_gram_noalloc (row blocks x q x r x 2 "
                                "must be <= 2^21 doubles)%s");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(BL_EHIP, "no current device%s");
  if (dev != s->device) return set_error(BL_EINVAL, "the handle's device must be the current device%s");
  double* part = nullptr;
  int rc = scratch_address(dev, &part);
  if (rc) return rc;
  const Launch L{nullptr, 1, 0, s->st};
  if (gram(View<const double>{static_cast<const double*>(X), q, 0}, q,
           View<const double>{static_cast<const double*>(W), r, 0}, r, len, part, kNoAllocDoubles,
           static_cast<double*>(out_dev), L) != 0)
    return set_error(BL_EINVAL, "scratch too small%s");
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BL_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return BL_OK;
}

}  // extern "C"
