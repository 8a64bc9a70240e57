// noalloc.hip -- linmin_unmix_noalloc: linmin_unmix with its work areas in a
// fixed device array of this file instead of stream-ordered allocations,
// for callers that cannot allocate device memory.
//
// The array `scratch` exists once per GPU the library runs on, for the life
// of the process.  Host code never passes its name to a kernel or a copy:
// in host code that name is a stand-in, not a device address.  The device
// address is looked up once per device (hipGetSymbolAddress, with that
// device current) on the entry point's first call there, and only that
// address is handed on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/linmin.h"
#include "unmix.h"

namespace {

static __device__ __align__(256) char scratch[LINMIN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch[kMaxDevices];  // device address of scratch on each device, once looked up

// Device address of this device's scratch (dev is the current device).
int scratch_of(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return LINMIN_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return LINMIN_EHIP;
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return LINMIN_OK;
}

}  // namespace

extern "C" int linmin_unmix_noalloc(linmin_lib lib, const float* cube, int64_t P, const float* sigma,
                                    double* out_coeffs, double* out_cov, const linmin_opts* opts, void* stream) {
  linmin_opts o;
  size_t bytes = 0;
  const int rc0 = lm::unmix_check(lib, cube, P, out_coeffs, out_cov, opts, &o, &bytes);
  if (rc0 != LINMIN_OK || P == 0) return rc0;
  if (bytes > (size_t)LINMIN_NOALLOC_SCRATCH_BYTES) return LINMIN_ESCRATCH;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LINMIN_EHIP;
  char* ws = nullptr;
  const int rc1 = scratch_of(dev, &ws);
  if (rc1 != LINMIN_OK) return rc1;
  return lm::unmix_ws(lib, cube, P, sigma, out_coeffs, out_cov, o, static_cast<hipStream_t>(stream), ws);
}
