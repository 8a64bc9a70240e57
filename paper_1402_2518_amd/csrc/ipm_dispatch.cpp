// ipm_dispatch.cpp -- choose the compiled interior-point kernel for a library.
//
// Kernel families (every one a complete implementation of the same method):
//   row-cyclic  FP64, one pixel per wavefront on the 4x4x4 FP64 matrix cores
//   tile        FP64, four pixels per wavefront on the 4x4x4 FP64 matrix cores
//   group       FP64 or FP32, a group of lanes per pixel on the vector units
//   tile32      FP32 (first stage of the mixed form) on the 4x4x1 FP32
//               matrix cores: sixteen pixels per wavefront, or for the
//               larger libraries a pixel's tile columns dealt out over Q
//               blocks (16 / Q pixels per wavefront)
// The default choice per padded size NC is the first family compiled for it
// in the order above (FP32: tile32, then group), a group kernel with the
// first width listed for NC.  A measured table installed with
// linmin_set_kernel overrides it (family and, for group kernels, the width)
// where the chosen shape is compiled; LINMIN_FP64_KERNEL=valu|tile and
// LINMIN_FP32_KERNEL=valu force a family for comparison runs.
#include <stdlib.h>
#include <string.h>

#include <atomic>

#include "kernels.h"

namespace lm {

#define LM_SHAPE(t, nc, g) \
  int ipm_entry_##t##_##nc##_##g(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#define LM_TILE(t) int ipm_tile_entry_##t(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#define LM_RC(t, bb) int ipm_rc_entry_##t##_##bb(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#define LM_TILE32(t) int ipm_tile32_entry_##t(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#define LM_CC32(t, q) \
  int ipm_cc32_entry_##t##_##q(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st);
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
#undef LM_CC32

// quads per pixel of the FP32 column-cyclic shape for nc, or 0
static int cc32_quads(int nc) {
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t)
#define LM_RC(t, bb)
#define LM_TILE32(t)
#define LM_CC32(t, q) \
  if (4 * t == nc) return q;
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
#undef LM_CC32
  return 0;
}

// an FP32 tile shape (sixteen pixels per wavefront) exists for nc
static bool tile32_has(int nc) {
  bool have = false;
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t)
#define LM_RC(t, bb)
#define LM_TILE32(t) have |= (4 * t == nc);
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
  return have;
}

int ipm_shape_nc(int n) {
  int best = -1;
#define LM_SHAPE(t, nc, g) \
  if (nc >= n && (best < 0 || nc < best)) best = nc;
#define LM_TILE(t)
#define LM_RC(t, bb)
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
  return best;
}

// lanes per pixel of the first lane-group shape listed for (nc, precision)
// (the default width), or -1
static int group_lanes(int nc, bool fp32) {
#define LM_SHAPE(t, nc_, g) \
  if (nc_ == nc && (fp32 == (sizeof(t) == 4))) return g;
#define LM_TILE(t)
#define LM_RC(t, bb)
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
  return -1;
}

// a lane-group shape of width g is compiled for (nc, precision)
static bool group_has(int nc, bool fp32, int g) {
#define LM_SHAPE(t, nc_, g_) \
  if (nc_ == nc && (fp32 == (sizeof(t) == 4)) && g_ == g) return true;
#define LM_TILE(t)
#define LM_RC(t, bb)
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
  return false;
}

bool ipm_family_available(int nc, bool fp32, int fam, int lanes) {
  if (fam == kFamGroup && lanes > 0) return group_has(nc, fp32, lanes);
  if (fam != kFamGroup && lanes != 0) return false;
  return ipm_family_available(nc, fp32, fam);
}

bool ipm_family_available(int nc, bool fp32, int fam) {
  bool have = false;
  switch (fam) {
    case kFamRowCyclic:
      if (fp32 || nc % 16) return false;
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t)
#define LM_RC(t, bb) have |= (4 * t == nc);
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
      return have;
    case kFamTile:
      if (fp32 || nc % 4) return false;
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t) have |= (4 * t == nc);
#define LM_RC(t, bb)
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
      return have;
    case kFamTile32:
      if (!fp32 || nc % 4) return false;
      return tile32_has(nc) || cc32_quads(nc) > 0;
    case kFamGroup:
      return group_lanes(nc, fp32) > 0;
  }
  return false;
}

// measured choices: [fp32][nc] = family | lanes << 8, 0 = none (the
// default rule applies)
static std::atomic<int> g_choice[2][kNcMax + 1];

int ipm_set_family(int nc, bool fp32, int fam, int lanes) {
  if (nc < 1 || nc > kNcMax || lanes < 0 || lanes > 64) return -1;
  if (fam != 0 && !ipm_family_available(nc, fp32, fam, lanes)) return -1;
  g_choice[fp32 ? 1 : 0][nc].store(fam == 0 ? 0 : (fam | (lanes << 8)), std::memory_order_relaxed);
  return 0;
}

// the installed choice for (nc, precision) if it is compiled, else 0
static int choice(int nc, bool fp32) {
  if (nc < 1 || nc > kNcMax) return 0;
  const int t = g_choice[fp32 ? 1 : 0][nc].load(std::memory_order_relaxed);
  return (t && ipm_family_available(nc, fp32, t & 0xff, t >> 8)) ? t : 0;
}

static int forced_family(bool fp32) {
  static int forced64 = -1, forced32 = -1;
  if (forced64 < 0) {
    const char* e = getenv("LINMIN_FP64_KERNEL");
    forced64 = (e && strcmp(e, "valu") == 0) ? kFamGroup : ((e && strcmp(e, "tile") == 0) ? kFamTile : 0);
    const char* f = getenv("LINMIN_FP32_KERNEL");
    forced32 = (f && strcmp(f, "valu") == 0) ? kFamGroup : 0;
  }
  return fp32 ? forced32 : forced64;
}

int ipm_family(int nc, bool fp32) {
  const int forced = forced_family(fp32);
  if (forced && ipm_family_available(nc, fp32, forced)) return forced;
  if (const int t = choice(nc, fp32)) return t & 0xff;
  static const int order64[] = {kFamRowCyclic, kFamTile, kFamGroup};
  static const int order32[] = {kFamTile32, kFamGroup};
  if (fp32) {
    for (int f : order32)
      if (ipm_family_available(nc, true, f)) return f;
  } else {
    for (int f : order64)
      if (ipm_family_available(nc, false, f)) return f;
  }
  return 0;
}

int ipm_group_lanes(int nc, bool fp32) {
  const int t = choice(nc, fp32);
  const int forced = forced_family(fp32);
  if ((!forced || !ipm_family_available(nc, fp32, forced)) && (t & 0xff) == kFamGroup && (t >> 8) > 0)
    return t >> 8;
  return group_lanes(nc, fp32);
}

int ipm_choice_code(int n, bool fp32) {
  const int nc = ipm_shape_nc(n);
  if (nc < 0) return -1;
  const int fam = ipm_family(nc, fp32);
  return fam == kFamGroup ? (fam | (ipm_group_lanes(nc, fp32) << 8)) : fam;
}

int ipm_kernel_class(int n, bool fp32, bool stable) { return ipm_kernel_class_of(n, fp32, stable, ipm_choice_code(n, fp32)); }

int ipm_kernel_class_of(int n, bool fp32, bool stable, int code) {
  const int nc = ipm_shape_nc(n);
  if (nc < 0 || code < 0) return -1;
  switch (code & 0xff) {
    case kFamRowCyclic: return 5000 + nc;
    case kFamTile: return (stable ? 4000 : 1000) + nc;
    case kFamTile32: return 6000 + nc;
    case kFamGroup: return (fp32 ? 3000 : 2000) + 10000 * (code >> 8) + nc;
  }
  return -1;
}

int ipm_pixels_per_block_code(int code, int nc) {
  switch (code & 0xff) {
    case kFamRowCyclic: return 4;   // one pixel per wavefront, four wavefronts
    case kFamTile: return 16;       // four pixels per wavefront, four wavefronts
    case kFamTile32:                // sixteen pixels per wavefront, or 16 / Q (column-cyclic), four wavefronts
      return tile32_has(nc) ? 64 : (cc32_quads(nc) > 0 ? 4 * (16 / cc32_quads(nc)) : -1);
    case kFamGroup: return (code >> 8) > 0 ? 4 * (64 / (code >> 8)) : -1;
  }
  return -1;
}

int ipm_pixels_per_block(int n, bool fp32) {
  const int code = ipm_choice_code(n, fp32);
  return code < 0 ? -1 : ipm_pixels_per_block_code(code, ipm_shape_nc(n));
}

// launch the kernel that code (family | group width << 8) names
static int dispatch(int n, const IpmParams& p, const IpmBatch* b, int mode, bool fp32, int code, hipStream_t st) {
  const int nc = ipm_shape_nc(n);
  if (nc < 0 || code < 0 || !ipm_family_available(nc, fp32, code & 0xff, code >> 8)) return -5;
  switch (code & 0xff) {
    case kFamRowCyclic:
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t)
#define LM_RC(t, bb) \
      if (4 * t == nc) return ipm_rc_entry_##t##_##bb(p, b, mode, st);
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
      break;
    case kFamTile:
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t) \
      if (4 * t == nc) return ipm_tile_entry_##t(p, b, mode, st);
#define LM_RC(t, bb)
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
      break;
    case kFamTile32:
#define LM_SHAPE(t, nc_, g)
#define LM_TILE(t)
#define LM_RC(t, bb)
#define LM_TILE32(t) \
      if (4 * t == nc) return ipm_tile32_entry_##t(p, b, mode, st);
#define LM_CC32(t, q) \
      if (4 * t == nc) return ipm_cc32_entry_##t##_##q(p, b, mode, st);
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
#undef LM_CC32
      break;
    case kFamGroup: {
      const int lanes = code >> 8;
#define LM_SHAPE(t, nc_, g) \
      if (nc_ == nc && (fp32 == (sizeof(t) == 4)) && g == lanes) return ipm_entry_##t##_##nc_##_##g(p, b, mode, st);
#define LM_TILE(t)
#define LM_RC(t, bb)
#define LM_TILE32(t)
#include "ipm_shapes.def"
#undef LM_SHAPE
#undef LM_TILE
#undef LM_RC
#undef LM_TILE32
      break;
    }
  }
  return -5;
}

int launch_ipm(const IpmParams& p, int mode, bool fp32, hipStream_t st) {
  if (p.P <= 0) return 0;
  return dispatch(p.n, p, nullptr, mode, fp32, ipm_choice_code(p.n, fp32), st);
}

int ipm_retry_code(int n) {
  const int nc = ipm_shape_nc(n);
  if (nc < 0) return -1;
  if (ipm_family_available(nc, false, kFamTile)) return kFamTile;
  if (ipm_family_available(nc, false, kFamRowCyclic)) return kFamRowCyclic;
  return -1;
}

int launch_ipm_retry(const IpmParams& p, hipStream_t st) {
  if (p.P <= 0) return 0;
  return dispatch(p.n, p, nullptr, kRetry, false, ipm_retry_code(p.n), st);
}

int launch_ipm_batch(int n, int constraint, int stable, const IpmBatch& b, int mode, bool fp32, int code,
                     hipStream_t st) {
  if (b.njobs <= 0 || b.blocks <= 0) return 0;
  IpmParams p{};
  p.n = n;
  p.constraint = constraint;
  p.stable = stable;
  return dispatch(n, p, &b, mode, fp32, code, st);
}

}  // namespace lm
