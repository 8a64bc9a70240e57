// ipm_dispatch.cpp -- choose the compiled interior-point shape for a library.
#include <stdlib.h>
#include <string.h>

#include "kernels.h"

namespace lm {

#define LM_SHAPE(t, nc, g) \
  int ipm_entry_##t##_##nc##_##g(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#define LM_TILE(t) int ipm_tile_entry_##t(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#define LM_RC(t) int ipm_rc_entry_##t(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC

int ipm_shape_nc(int n) {
  int best = -1;
#define LM_SHAPE(t, nc, g) \
  if (nc >= n && (best < 0 || nc < best)) best = nc;
#define LM_TILE(t)
#define LM_RC(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
  return best;
}

// FP64 kernel family: the row-cyclic matrix-core kernel (one pixel per
// wavefront) where such a shape exists for NC, else the four-pixel tile
// kernel, else the lane-group kernel.  LINMIN_FP64_KERNEL=tile skips the
// row-cyclic shapes and =valu forces the lane-group kernel (all three are
// complete implementations; the switch exists to compare them).
static int forced_family() {
  static int forced = -1;
  if (forced < 0) {
    const char* e = getenv("LINMIN_FP64_KERNEL");
    forced = (e && strcmp(e, "valu") == 0) ? 1 : ((e && strcmp(e, "tile") == 0) ? 2 : 0);
  }
  return forced;
}

static bool use_rc(int nc) {
  if (forced_family() != 0 || nc % 16) return false;
  bool have = false;
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t)
#define LM_RC(t) have |= (4 * t == nc);
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
  return have;
}

static bool use_tile(int nc) {
  if (forced_family() == 1 || nc % 4) return false;
  bool have = false;
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t) have |= (4 * t == nc);
#define LM_RC(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
  return have;
}

// lanes per pixel of the lane-group shape for (nc, precision), or -1
static int group_lanes(int nc, bool fp32) {
#define LM_SHAPE(t, nc_, g) \
  if (nc_ == nc && (fp32 == (sizeof(t) == 4))) return g;
#define LM_TILE(t)
#define LM_RC(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
  return -1;
}

int ipm_kernel_class(int n, bool fp32, bool stable) {
  const int nc = ipm_shape_nc(n);
  if (nc < 0) return -1;
  if (!fp32 && use_rc(nc)) return 5000 + nc;
  if (!fp32 && use_tile(nc)) return (stable ? 4000 : 1000) + nc;
  return group_lanes(nc, fp32) > 0 ? (fp32 ? 3000 : 2000) + nc : -1;
}

int ipm_pixels_per_block(int n, bool fp32) {
  const int nc = ipm_shape_nc(n);
  if (nc < 0) return -1;
  if (!fp32 && use_rc(nc)) return 4;    // one pixel per wavefront, four wavefronts
  if (!fp32 && use_tile(nc)) return 16;  // four pixels per wavefront, four wavefronts
  const int g = group_lanes(nc, fp32);
  return g > 0 ? 4 * (64 / g) : -1;
}

static int dispatch(int n, const IpmParams& p, const IpmBatch* b, int mode, bool fp32, hipStream_t st) {
  const int nc = ipm_shape_nc(n);
  if (nc < 0) return -5;
  if (!fp32 && use_rc(nc)) {
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t)
#define LM_RC(t) \
    if (4 * t == nc) return ipm_rc_entry_##t(p, b, mode, st);
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
  }
  if (!fp32 && use_tile(nc)) {
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t) \
    if (4 * t == nc) return ipm_tile_entry_##t(p, b, mode, st);
#define LM_RC(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
  }
#define LM_SHAPE(t, nc_, g)                                              \
  if (nc_ == nc && (fp32 == (sizeof(t) == 4))) return ipm_entry_##t##_##nc_##_##g(p, b, mode, st);
#define LM_TILE(t)
#define LM_RC(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
  return -5;
}

int launch_ipm(const IpmParams& p, int mode, bool fp32, hipStream_t st) {
  if (p.P <= 0) return 0;
  return dispatch(p.n, p, nullptr, mode, fp32, st);
}

int launch_ipm_batch(int n, int constraint, int stable, const IpmBatch& b, int mode, bool fp32, hipStream_t st) {
  if (b.njobs <= 0 || b.blocks <= 0) return 0;
  IpmParams p{};
  p.n = n;
  p.constraint = constraint;
  p.stable = stable;
  return dispatch(n, p, &b, mode, fp32, st);
}

}  // namespace lm
