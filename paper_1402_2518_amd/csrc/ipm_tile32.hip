// ipm_tile32.hip -- the FP32 stage of the mixed form (IPLS, Sec. 2.2, on the
// scaled problem of eq. 6 under eqs. 3-4) with the Newton matrix factored on
// the FP32 matrix cores (v_mfma_f32_4x4x1f32), sixteen pixels per wavefront.
//
// Same method as the other interior-point kernels (ipm_body.h); this file
// holds the layout.  The stage runs Mehrotra steps until mu <= mu_switch and
// hands the iterate to the FP64 kernels.
//
// Mapping.  The 4x4x1 FP32 MFMA works on sixteen independent 4x4 blocks;
// block blk = lane >> 2 owns one pixel and lane c = lane & 3 of the block is
// its column.  Operands (gfx950): A: lane (blk, i) holds A[i]; B: lane
// (blk, j) holds B[j]; C/D: lane (blk, j) holds D[r][j] in register r.
// A tile X is kept "stored" as the accumulator layout: lane c holds column
// c of X in four registers.  Feeding register k of a stored X as A and
// register k of a stored P as B for k = 0..3 accumulates
//     mm(X, P, R) = X^T P + R
// in stored form, so the factorisation H = U^T D U (unit upper block U,
// diagonal D) works on the upper triangle of tiles with no data movement:
// the panel is W_KJ = L_K^{-1} H_KJ (with H_KK = L_K D_K L_K^T, L_K = U_KK^T
// unit lower), U_KJ = D_K^{-1} W_KJ, and the trailing update
// H_IJ -= U_KI^T W_KJ is one mm() with the negated U_KI.
// Vectors use a compact layout: lane c holds element 4 m + c in slot m, the
// same element as the diagonal of register c of tile row m, so adding the
// barrier diagonal needs no data movement either.  The triangular solves
// run on the vector units in that layout (one right-hand side costs four
// FMAs per tile and lane, against four MFMAs), the tile row in flight
// broadcast across the block's four lanes by DPP.
#include "ipm_body.h"

namespace lm {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma41(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// X^T P + R for stored 4x4 tiles
__device__ __forceinline__ v4f mm(const v4f& X, const v4f& P, v4f R) {
  R = mfma41(X[0], P[0], R);
  R = mfma41(X[1], P[1], R);
  R = mfma41(X[2], P[2], R);
  return mfma41(X[3], P[3], R);
}

// value of lane Q of the block on every lane of the block
template <int Q>
__device__ __forceinline__ float qbf(float v) {
  return dpp<qp(Q, Q, Q, Q)>(v);
}

template <int T>
struct Tile32 {
  using real = float;
  static constexpr bool kCompact = true;
  // The Newton identity that carries Gh a from step to step holds only to
  // the accuracy of the solve, which in FP32 is too coarse: form it anew.
  static constexpr bool kRecomputeGrad = true;
  static constexpr int NP = 4 * T;
  static constexpr int C = T;  // compact slots: one per tile row
  static constexpr int NT = T * (T + 1) / 2;
  // tile (K, J), K <= J, of the upper triangle
  static constexpr int id(int K, int J) { return K * T - K * (K - 1) / 2 + (J - K); }

  int c;                // this lane's column in its block
  int nvalid;           // library size n
  const float* sG;      // LDS, NP x NP scaled Gram (FP32)
  // after form_factor(): tile (K, J > K) holds -U_KJ, tile (K, K) holds
  // column c of L_K^{-1} (register r: L_K^{-1}[r][c]), rd[K] holds 1 / d of
  // element c
  v4f H[NT];
  float rd[T];
  bool notpd;

  __device__ __forceinline__ int el(int m) const { return 4 * m + c; }
  __device__ __forceinline__ bool writer() const { return c == 0; }

  template <typename V, typename Op>
  static __device__ __forceinline__ V red(V v, Op op) {
    v = op(v, dpp<qp(1, 0, 3, 2)>(v));
    return op(v, dpp<qp(2, 3, 0, 1)>(v));
  }
  static __device__ __forceinline__ float sum(float v) {
    return red(v, [](float a, float b) { return a + b; });
  }
  static __device__ __forceinline__ float vmin(float v) {
    return red(v, [](float a, float b) { return fminf(a, b); });
  }
  static __device__ __forceinline__ float vmax(float v) {
    return red(v, [](float a, float b) { return fmaxf(a, b); });
  }
  static __device__ __forceinline__ int imin(int v) {
    return red(v, [](int a, int b) { return min(a, b); });
  }
  static __device__ __forceinline__ int ior(int v) {
    return red(v, [](int a, int b) { return a | b; });
  }

  // the four elements of tile row m (slot m of the block's lanes) on every lane
  static __device__ __forceinline__ v4f row(float v) {
    return (v4f){qbf<0>(v), qbf<1>(v), qbf<2>(v), qbf<3>(v)};
  }
  // register c of t (this lane's own element of a tile-row vector)
  __device__ __forceinline__ float own(const v4f& t) const {
    return c == 0 ? t[0] : (c == 1 ? t[1] : (c == 2 ? t[2] : t[3]));
  }
  // Gh[4 I + c][4 J .. 4 J + 3]
  __device__ __forceinline__ v4f grow(int I, int J) const {
    return *reinterpret_cast<const v4f*>(sG + (4 * I + c) * NP + 4 * J);
  }

  // out = Gh v
  __device__ __forceinline__ void gvec(const float (&v)[C], float (&out)[C]) const {
    v4f vb[T];
    static_for<0, T>([&](auto jj) { vb[jj] = row(v[jj]); });
    static_for<0, T>([&](auto ii) {
      constexpr int I = decltype(ii)::value;
      float acc0 = 0.f, acc1 = 0.f;
      static_for<0, T>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        const v4f g = grow(I, J);
        acc0 = fmaT(g[0], vb[J][0], acc0);
        acc1 = fmaT(g[1], vb[J][1], acc1);
        acc0 = fmaT(g[2], vb[J][2], acc0);
        acc1 = fmaT(g[3], vb[J][3], acc1);
      });
      out[I] = acc0 + acc1;
    });
  }

  // H = Gh + diag(D), then H = U^T D U
  __device__ __forceinline__ void form_factor(const float (&D)[C]) {
    // tile (K, J): lane c holds column c, i.e. Gh[4 J + c][4 K .. 4 K + 3]
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      static_for<K, T>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        v4f h = grow(J, K);
        if constexpr (J == K) {
          h[0] += c == 0 ? D[K] : 0.f;
          h[1] += c == 1 ? D[K] : 0.f;
          h[2] += c == 2 ? D[K] : 0.f;
          h[3] += c == 3 ? D[K] : 0.f;
        }
        H[id(K, J)] = h;
      });
    });
    bool bad = false;
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      // 4x4 L D L^T of the diagonal tile on every lane of the block
      const v4f h = H[id(K, K)];
      const float m00 = qbf<0>(h[0]), m10 = qbf<0>(h[1]), m20 = qbf<0>(h[2]), m30 = qbf<0>(h[3]);
      const float m11 = qbf<1>(h[1]), m21 = qbf<1>(h[2]), m31 = qbf<1>(h[3]);
      const float m22 = qbf<2>(h[2]), m32 = qbf<2>(h[3]);
      const float m33 = qbf<3>(h[3]);
      const float d0 = m00;
      const float r0 = rcpT(d0);
      const float l10 = m10 * r0, l20 = m20 * r0, l30 = m30 * r0;
      const float d1 = fmaT(-l10, m10, m11);
      const float r1 = rcpT(d1);
      const float t21 = fmaT(-l20, m10, m21), t31 = fmaT(-l30, m10, m31);
      const float l21 = t21 * r1, l31 = t31 * r1;
      const float d2 = fmaT(-l21, t21, fmaT(-l20, m20, m22));
      const float r2 = rcpT(d2);
      const float t32 = fmaT(-l31, t21, fmaT(-l30, m20, m32));
      const float l32 = t32 * r2;
      const float d3 = fmaT(-l32, t32, fmaT(-l31, t31, fmaT(-l30, m30, m33)));
      const float r3 = rcpT(d3);
      const float dmin = fminf(fminf(d0, d1), fminf(d2, d3));
      const float rs = r0 + r1 + r2 + r3;
      bad |= !(dmin > 0.f) || !isfin(rs);
      const float e0 = c == 0 ? 1.f : 0.f, e1 = c == 1 ? 1.f : 0.f;
      const float e2 = c == 2 ? 1.f : 0.f, e3 = c == 3 ? 1.f : 0.f;
      // row c of L^{-1}: L^T w = e_c
      const float w3 = e3;
      const float w2 = fmaT(-l32, w3, e2);
      const float w1 = fmaT(-l31, w3, fmaT(-l21, w2, e1));
      const float w0 = fmaT(-l30, w3, fmaT(-l20, w2, fmaT(-l10, w1, e0)));
      // column c of L^{-1}: L v = e_c
      const float v0 = e0;
      const float v1 = fmaT(-l10, v0, e1);
      const float v2 = fmaT(-l21, v1, fmaT(-l20, v0, e2));
      const float v3 = fmaT(-l32, v2, fmaT(-l31, v1, fmaT(-l30, v0, e3)));
      const v4f li = (v4f){w0, w1, w2, w3};
      H[id(K, K)] = (v4f){v0, v1, v2, v3};
      rd[K] = c == 0 ? r0 : (c == 1 ? r1 : (c == 2 ? r2 : r3));
      const v4f nr = (v4f){-r0, -r1, -r2, -r3};
      // panel and trailing update, one column J at a time: column J needs
      // -U_KI for I <= J (done, or computed just now) and W_KJ
      static_for<K + 1, T>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        const v4f w = mm(li, H[id(K, J)], (v4f){0.f, 0.f, 0.f, 0.f});
        H[id(K, J)] = w * nr;
        static_for<K + 1, J + 1>([&](auto ii) {
          constexpr int I = decltype(ii)::value;
          H[id(I, J)] = mm(H[id(K, I)], w, H[id(I, J)]);
        });
      });
    });
    notpd = bad;
  }

  // forward solve U^T y = r and z = D^{-1} y, in place (compact layout)
  template <int NR>
  __device__ __forceinline__ void forward(float (&x)[NR][C]) const {
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      const v4f lc = H[id(K, K)];
      static_for<0, NR>([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        // y_K = L_K^{-1} t_K: this lane's column of L_K^{-1} times its own
        // element, summed over the block (every lane gets all of y_K)
        v4f y = lc * x[q][K];
        static_for<0, 4>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          y[r] = sum(y[r]);
        });
        x[q][K] = own(y) * rd[K];
        // the rows below: t_J -= U_KJ^T y_K, this lane's element
        static_for<K + 1, T>([&](auto jj) {
          constexpr int J = decltype(jj)::value;
          const v4f u = H[id(K, J)];
          x[q][J] = fmaT(u[0], y[0], fmaT(u[1], y[1], fmaT(u[2], y[2], fmaT(u[3], y[3], x[q][J]))));
        });
      });
    });
  }

  // backward solve U x = z, in place (compact layout)
  template <int NR>
  __device__ __forceinline__ void backward(float (&x)[NR][C]) const {
    static_for<0, T>([&](auto kk) {
      constexpr int K = T - 1 - decltype(kk)::value;
      static_for<0, NR>([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        // partial sums over this lane's column of -U_KJ x_J, with z_K added
        // on the diagonal lane, summed over the block
        v4f s = (v4f){c == 0 ? x[q][K] : 0.f, c == 1 ? x[q][K] : 0.f, c == 2 ? x[q][K] : 0.f,
                      c == 3 ? x[q][K] : 0.f};
        static_for<K + 1, T>([&](auto jj) {
          constexpr int J = decltype(jj)::value;
          const v4f u = H[id(K, J)];
          s[0] = fmaT(u[0], x[q][J], s[0]);
          s[1] = fmaT(u[1], x[q][J], s[1]);
          s[2] = fmaT(u[2], x[q][J], s[2]);
          s[3] = fmaT(u[3], x[q][J], s[3]);
        });
        static_for<0, 4>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          s[r] = sum(s[r]);
        });
        const v4f l = H[id(K, K)];
        x[q][K] = fmaT(l[0], s[0], fmaT(l[1], s[1], fmaT(l[2], s[2], l[3] * s[3])));
      });
    });
  }

  // w = H^{-1} r, u = H^{-1} 1
  __device__ __forceinline__ void solve2(const float (&r)[C], float (&w)[C], float (&u)[C]) const {
    float x[2][C];
    static_for<0, C>([&](auto mm_) {
      constexpr int m = decltype(mm_)::value;
      x[0][m] = r[m];
      x[1][m] = el(m) < nvalid ? 1.f : 0.f;
    });
    forward<2>(x);
    backward<2>(x);
    static_for<0, C>([&](auto mm_) {
      w[mm_] = x[0][mm_];
      u[mm_] = x[1][mm_];
    });
  }
  // w = H^{-1} r
  __device__ __forceinline__ void solve1(const float (&r)[C], float (&w)[C]) const {
    float x[1][C];
    static_for<0, C>([&](auto mm_) { x[0][mm_] = r[mm_]; });
    forward<1>(x);
    backward<1>(x);
    static_for<0, C>([&](auto mm_) { w[mm_] = x[0][mm_]; });
  }
};

// One workgroup's 64 pixels (four wavefronts of sixteen): workgroup wg of
// the cube described by prm.
template <int T, int MODE, int CONS>
__device__ __forceinline__ void ipm_tile32_body(const IpmParams& prm, int64_t wg) {
  using TL = Tile32<T>;
  constexpr int NP = TL::NP;
  __shared__ __align__(16) float sG[NP * NP];
  const float* Gsrc = static_cast<const float*>(prm.Gh);
  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) sG[i] = Gsrc[i];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p = wg * 64 + wave * 16 + (lane >> 2);

  TL tl;
  tl.c = lane & 3;
  tl.sG = sG;
  tl.nvalid = prm.n;
  ipm_pixel<TL, MODE, CONS>(prm, p, p < prm.P, tl);
}

// waves per SIMD the register budget is sized for: beyond T = 6 the tiles
// (4 registers each) and the nine-slot vectors of sixteen pixels need more
// than half of the 512 registers of a lane
template <int T>
constexpr int kTile32Waves = T <= 6 ? 2 : 1;

template <int T, int MODE, int CONS>
__global__ __launch_bounds__(256, kTile32Waves<T>) void ipm_tile32_kernel(IpmParams prm) {
  ipm_tile32_body<T, MODE, CONS>(prm, blockIdx.x);
}

template <int T, int MODE, int CONS>
__global__ __launch_bounds__(256, kTile32Waves<T>) void ipm_tile32_batch_kernel(const IpmParams* __restrict__ jobs,
                                                                                const int64_t* __restrict__ start,
                                                                                int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const IpmParams prm = uniform_copy(jobs + j);
  ipm_tile32_body<T, MODE, CONS>(prm, (int64_t)blockIdx.x - start[j]);
}

template <int T, int CONS>
static int launch_tile32_c(const IpmParams& p, const IpmBatch* b, hipStream_t st) {
  if (b)
    hipLaunchKernelGGL((ipm_tile32_batch_kernel<T, kStage1, CONS>), dim3((unsigned)b->blocks), dim3(256), 0, st,
                       b->jobs, b->start, b->njobs);
  else
    hipLaunchKernelGGL((ipm_tile32_kernel<T, kStage1, CONS>), dim3((unsigned)((p.P + 63) / 64)), dim3(256), 0, st,
                       p);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// b == nullptr: one cube described by p; else the jobs of b (p only gives
// the constraint option).  Only the first stage of the mixed form runs here.
template <int T>
static int launch_tile32(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  if (mode != kStage1) return -5;
  switch (p.constraint) {
    case kSto: return launch_tile32_c<T, kSto>(p, b, st);
    case kSlo: return launch_tile32_c<T, kSlo>(p, b, st);
    case kPos: return launch_tile32_c<T, kPos>(p, b, st);
  }
  return -1;
}

#if defined(LM_TILE32_T)
#define LM_T32ENTRY2(t) ipm_tile32_entry_##t
#define LM_T32ENTRY(t) LM_T32ENTRY2(t)
int LM_T32ENTRY(LM_TILE32_T)(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  return launch_tile32<LM_TILE32_T>(p, b, mode, st);
}
#endif

}  // namespace lm
