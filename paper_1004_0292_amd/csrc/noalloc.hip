// y = A x without any device allocation, for callers that cannot allocate: the
// planar staging of x and y that sscg_apply_A keeps in buffers the library
// allocates lives here in one file-scope device array (each device the library runs
// on holds its copy until the process ends). Its address on a device is looked up
// once per device, on that device's first call, and kept; host code uses that
// address, never the array's name (which on the host is only a stand-in).
#include <mutex>

#include "sscg.h"
#include "sscg_internal.h"

namespace {
constexpr size_t kScratchBytes = (size_t)32 << 20;   // x staging in the first half, y in the second
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

extern "C" int sscg_apply_A_noalloc(sscg_ctx *c, const void *x, void *y, int32_t nsrc, int32_t prec) {
  size_t each = 0;
  const int rc = sscg::context_check_apply(c, x, y, nsrc, prec, &each);
  if (rc != SSCG_OK) return rc;
  if (each > kScratchBytes / 2)
    return sscg::context_fail(c, SSCG_EINVAL,
                              "apply_A_noalloc: nsrc * 12 V entries exceed its 16 MiB staging (at most 1048576 "
                              "complex entries in FP64, 2097152 in FP32)");
  const int dev = sscg::context_device(c);
  if (dev < 0 || dev >= kMaxDevices) return sscg::context_fail(c, SSCG_EINVAL, "apply_A_noalloc: device index");
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    return sscg::context_fail(c, SSCG_EDEVICE, "apply_A_noalloc: hipSetDevice failed");
  }
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return sscg::context_fail(c, SSCG_EDEVICE, "apply_A_noalloc: hipGetSymbolAddress of the scratch failed");
      }
      g_scratch[dev] = p;
    }
    base = g_scratch[dev];
  }
  return sscg::apply_A_staged(c, x, y, nsrc, prec, base, static_cast<char *>(base) + kScratchBytes / 2, false);
}
