// unmix.h -- the body of linmin_unmix shared by its entry points (the one
// with stream-ordered work areas and the one with a fixed device array).
// Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/linmin.h"

namespace lm {

// Argument checks of linmin_unmix.  Fills *o (the defaults where opts is
// NULL) and *bytes, the work area one call needs (0 when P == 0).  Returns
// LINMIN_OK or the error linmin_unmix reports.
int unmix_check(linmin_lib lib, const float* cube, int64_t P, const double* out_coeffs, const double* out_cov,
                const linmin_opts* opts, linmin_opts* o, size_t* bytes);

// Enqueue the unmix on st with the work area ws (device, at least the
// bytes of unmix_check, 256-byte aligned).  Allocates nothing.  Every byte
// of ws a kernel reads is written earlier in the same call, so ws may hold
// anything on entry; two calls that share ws must not overlap in time.
int unmix_ws(linmin_lib lib, const float* cube, int64_t P, const float* sigma, double* out_coeffs,
             double* out_cov, const linmin_opts& o, hipStream_t st, char* ws);

}  // namespace lm
