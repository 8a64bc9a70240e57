// common.h -- device helpers shared by the lib_linmin HIP kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lm {

// ---------------------------------------------------------------------------
// Lane moves inside a group.  Groups of G consecutive lanes (G = 1, 2, 4, 8,
// 16, 32) work on one pixel; every cross-lane operation below stays inside
// the group (DPP within a 16-lane row, one row swap for 32-lane groups), so
// it never mixes pixels.
// ---------------------------------------------------------------------------
constexpr int qp(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }
constexpr int kRowMirror = 0x140;      // lane i <- lane 15-i within a row
constexpr int kRowHalfMirror = 0x141;  // lane i <- lane 7-i within each half-row

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = dpp_i32<CTRL>(lo);
  hi = dpp_i32<CTRL>(hi);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return dpp_i32<CTRL>(v);
}

// Row exchanges without LDS (v_permlane16_swap / v_permlane32_swap).  Rows
// are the four 16-lane groups of the wave.  pair<16>(v) returns, at this
// lane's position inside its row, v of the even row of its row pair (rows
// 0/1, 2/3) in .lo and v of the odd row in .hi; pair<32>(v) returns v of the
// lower 32 lanes in .lo and of the upper 32 in .hi.  Combining .lo and .hi
// with a commutative operation gives the same bits on both partner lanes.
template <typename T>
struct Pair {
  T lo, hi;
};
template <int W>
__device__ __forceinline__ Pair<uint32_t> pair_u32(uint32_t v) {
  static_assert(W == 16 || W == 32, "row pairs are 16 or 32 lanes apart");
  if constexpr (W == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return {r[0], r[1]};
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return {r[0], r[1]};
  }
}
template <int W>
__device__ __forceinline__ Pair<int> pair(int v) {
  const Pair<uint32_t> r = pair_u32<W>((uint32_t)v);
  return {(int)r.lo, (int)r.hi};
}
template <int W>
__device__ __forceinline__ Pair<float> pair(float v) {
  const Pair<uint32_t> r = pair_u32<W>(__float_as_uint(v));
  return {__uint_as_float(r.lo), __uint_as_float(r.hi)};
}
template <int W>
__device__ __forceinline__ Pair<double> pair(double v) {
  const Pair<uint32_t> l = pair_u32<W>((uint32_t)__double2loint(v));
  const Pair<uint32_t> h = pair_u32<W>((uint32_t)__double2hiint(v));
  return {__hiloint2double((int)h.lo, (int)l.lo), __hiloint2double((int)h.hi, (int)l.hi)};
}

// Sum / max / min over the group; every lane of the group gets the same bits
// (each butterfly step adds the same two operands on both partner lanes).
// lane i <- lane i^16 (crosses DPP rows; only used by 32-lane groups)
template <typename T>
__device__ __forceinline__ T xor16(T v) {
  const Pair<T> p = pair<16>(v);
  return ((__lane_id() >> 4) & 1) ? p.lo : p.hi;
}

template <int G, typename T>
__device__ __forceinline__ T gsum(T v) {
  static_assert(G <= 32, "group wider than half a wave");
  if constexpr (G >= 2) v += dpp<qp(1, 0, 3, 2)>(v);
  if constexpr (G >= 4) v += dpp<qp(2, 3, 0, 1)>(v);
  if constexpr (G >= 8) v += dpp<kRowHalfMirror>(v);
  if constexpr (G >= 16) v += dpp<kRowMirror>(v);
  if constexpr (G >= 32) {
    const Pair<T> p = pair<16>(v);
    v = p.lo + p.hi;
  }
  return v;
}
template <int G, typename T>
__device__ __forceinline__ T gmax(T v) {
  if constexpr (G >= 2) v = fmax(v, dpp<qp(1, 0, 3, 2)>(v));
  if constexpr (G >= 4) v = fmax(v, dpp<qp(2, 3, 0, 1)>(v));
  if constexpr (G >= 8) v = fmax(v, dpp<kRowHalfMirror>(v));
  if constexpr (G >= 16) v = fmax(v, dpp<kRowMirror>(v));
  if constexpr (G >= 32) {
    const Pair<T> p = pair<16>(v);
    v = fmax(p.lo, p.hi);
  }
  return v;
}
template <int G, typename T>
__device__ __forceinline__ T gmin(T v) {
  if constexpr (G >= 2) v = fmin(v, dpp<qp(1, 0, 3, 2)>(v));
  if constexpr (G >= 4) v = fmin(v, dpp<qp(2, 3, 0, 1)>(v));
  if constexpr (G >= 8) v = fmin(v, dpp<kRowHalfMirror>(v));
  if constexpr (G >= 16) v = fmin(v, dpp<kRowMirror>(v));
  if constexpr (G >= 32) {
    const Pair<T> p = pair<16>(v);
    v = fmin(p.lo, p.hi);
  }
  return v;
}
template <int G>
__device__ __forceinline__ int gmin_i(int v) {
  if constexpr (G >= 2) v = min(v, dpp<qp(1, 0, 3, 2)>(v));
  if constexpr (G >= 4) v = min(v, dpp<qp(2, 3, 0, 1)>(v));
  if constexpr (G >= 8) v = min(v, dpp<kRowHalfMirror>(v));
  if constexpr (G >= 16) v = min(v, dpp<kRowMirror>(v));
  if constexpr (G >= 32) {
    const Pair<int> p = pair<16>(v);
    v = min(p.lo, p.hi);
  }
  return v;
}
template <int G>
__device__ __forceinline__ int gor_i(int v) {
  if constexpr (G >= 2) v |= dpp<qp(1, 0, 3, 2)>(v);
  if constexpr (G >= 4) v |= dpp<qp(2, 3, 0, 1)>(v);
  if constexpr (G >= 8) v |= dpp<kRowHalfMirror>(v);
  if constexpr (G >= 16) v |= dpp<kRowMirror>(v);
  if constexpr (G >= 32) {
    const Pair<int> p = pair<16>(v);
    v = p.lo | p.hi;
  }
  return v;
}

// Value held by group lane SRC (compile time), delivered to every lane of the
// group.  t is the caller's lane index within the group.
template <int G, int SRC, typename T>
__device__ __forceinline__ T gbcast(T v, int t) {
  static_assert(SRC >= 0 && SRC < G, "source lane outside group");
  if constexpr (G == 1) {
    return v;
  } else if constexpr (G == 2) {
    return dpp<qp(SRC, SRC, 2 + SRC, 2 + SRC)>(v);
  } else {
    v = dpp<qp(SRC & 3, SRC & 3, SRC & 3, SRC & 3)>(v);
    if constexpr (G >= 8) {
      T m = dpp<kRowHalfMirror>(v);
      v = (((t >> 2) & 1) == ((SRC >> 2) & 1)) ? v : m;
    }
    if constexpr (G >= 16) {
      T m = dpp<kRowMirror>(v);
      v = (((t >> 3) & 1) == ((SRC >> 3) & 1)) ? v : m;
    }
    if constexpr (G >= 32) {
      T m = xor16(v);
      v = (((t >> 4) & 1) == ((SRC >> 4) & 1)) ? v : m;
    }
    return v;
  }
}

// Finite (neither infinite nor NaN).  A class test, not v - v == 0: with
// floating-point contraction the compiler may fuse the subtraction with the
// multiply that produced v, which yields v's rounding error instead of zero.
template <typename T>
__device__ __forceinline__ bool isfin(T v) {
  return __builtin_isfinite(v);
}

// Fused multiply-add in the operand precision (no promotion of float).
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Reciprocal from the hardware estimate refined by Newton steps (one for
// float, two for double): a division that does not need IEEE rounding.
__device__ __forceinline__ float rcpT(float x) {
  float y = __builtin_amdgcn_rcpf(x);
  return y * fmaT(-x, y, 2.0f);
}
__device__ __forceinline__ double rcpT(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fmaT(-x, y, 2.0);
  return y * fmaT(-x, y, 2.0);
}

// Orders this wave's LDS writes before its later LDS reads.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Compile-time loop: f(integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Batched launches over several cubes: job j owns the units [start[j],
// start[j + 1]) of the launch (blocks, or pixel chunks of grid-stride
// kernels); start holds njobs + 1 ascending values.  The unit index is
// uniform, so the search runs on the scalar unit.
__device__ __forceinline__ int job_of(const int64_t* __restrict__ start, int njobs, int64_t u) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Copy of a job descriptor that every lane reads at the same address, marked
// wave-uniform word by word so that its fields live in scalar registers.
template <typename S>
__device__ __forceinline__ S uniform_copy(const S* __restrict__ p) {
  static_assert(sizeof(S) % 4 == 0, "descriptor size must be a multiple of 4 bytes");
  constexpr int W = (int)(sizeof(S) / 4);
  uint32_t w[W];
  __builtin_memcpy(w, p, sizeof(S));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  S out;
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

}  // namespace lm
