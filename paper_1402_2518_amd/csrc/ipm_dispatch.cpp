// ipm_dispatch.cpp -- choose the compiled interior-point shape for a library.
#include "kernels.h"

namespace lm {

#define LM_SHAPE(t, nc, g) int ipm_entry_##t##_##nc##_##g(const IpmParams& p, int mode, hipStream_t st);
#include "ipm_shapes.def"
#undef LM_SHAPE

int ipm_shape_nc(int n) {
  int best = -1;
#define LM_SHAPE(t, nc, g) \
  if (nc >= n && (best < 0 || nc < best)) best = nc;
#include "ipm_shapes.def"
#undef LM_SHAPE
  return best;
}

int launch_ipm(const IpmParams& p, int mode, bool fp32, hipStream_t st) {
  if (p.P <= 0) return 0;
  const int nc = ipm_shape_nc(p.n);
  if (nc < 0) return -5;
#define LM_SHAPE(t, nc_, g)                                              \
  if (nc_ == nc && (fp32 == (sizeof(t) == 4))) return ipm_entry_##t##_##nc_##_##g(p, mode, st);
#include "ipm_shapes.def"
#undef LM_SHAPE
  return -5;
}

}  // namespace lm
