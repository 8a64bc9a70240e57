// ipm_cc32.hip -- the FP32 stage of the mixed form (IPLS, Sec. 2.2, on the
// scaled problem of eq. 6 under eqs. 3-4) for the larger libraries: the
// Newton matrix of a pixel spread column-cyclically over Q blocks of the
// FP32 matrix cores (v_mfma_f32_4x4x1f32), 16 / Q pixels per wavefront.
//
// Same method as the other interior-point kernels (ipm_body.h); this file
// holds the layout.  The tile algebra is that of ipm_tile32.hip (stored
// 4x4 tiles, lane c of a block holds column c; four MFMAs accumulate
// X^T P + R; H = U^T D U on the upper triangle of tiles), with a pixel's
// tile columns dealt out over its Q blocks so that the tiles fit in
// registers where sixteen pixels per wavefront would not.
//
// Mapping.  Block (quad) qd = lane >> 2 of the wavefront belongs to pixel
// qd / Q as its quad q = qd % Q; lane c = lane & 3.  Tile column J = Q r + q
// lives on quad q in column slot r (r < R = T / Q), which holds tiles
// (K, J) for K < Q (r + 1); the entries with K > J are never read.  At
// step K the quad holding column K factors the diagonal tile; every quad
// reads it from LDS and factors it too (the same instructions run on every
// lane anyway), so each computes the panel of its own columns; the panel
// tiles -U_KI that the trailing update needs from other quads pass through
// LDS.  Vectors use a compact layout: slot m of lane (q, c) holds element
// 4 (Q m + q) + c, the diagonal element of register c of column Q m + q.
// The triangular solves run on the vector units; the tile row in flight and
// the quads' partial sums pass through LDS.
#include "ipm_body.h"

namespace lm {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f cc_mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// X^T P + R for stored 4x4 tiles
__device__ __forceinline__ v4f cc_mm(const v4f& X, const v4f& P, v4f R) {
  R = cc_mfma(X[0], P[0], R);
  R = cc_mfma(X[1], P[1], R);
  R = cc_mfma(X[2], P[2], R);
  return cc_mfma(X[3], P[3], R);
}

__device__ __forceinline__ v4f ld4(const float* p) { return *reinterpret_cast<const v4f*>(p); }
__device__ __forceinline__ void st4(float* p, const v4f& v) { *reinterpret_cast<v4f*>(p) = v; }

template <int T, int Q>
struct CC32 {
  static_assert(T % Q == 0, "tile columns must deal out evenly over the quads");
  using real = float;
  static constexpr bool kCompact = true;
  // the Newton identity that carries Gh a holds only to the accuracy of an
  // FP32 solve: form the gradient anew at every step
  static constexpr bool kRecomputeGrad = true;
  static constexpr int R = T / Q;                // column slots per quad
  static constexpr int NP = 4 * T;
  static constexpr int C = R;                    // compact slots
  static constexpr int NS = Q * R * (R + 1) / 2;  // tile slots: sum over r of Q (r + 1)
  static constexpr int sid(int r, int K) { return Q * r * (r + 1) / 2 + K; }
  // exchange area of one pixel in LDS (floats)
  static constexpr int XD = 0;            // diagonal tile, entry (r, c) at 4 c + r
  static constexpr int XU = 16;           // tiles -U_KJ of the current row, column J at XU + 16 J + 4 c
  static constexpr int XV = XU + 16 * T;  // a whole vector (gradient) or the tile row of y (solves)
  static constexpr int XS = XV + NP;      // backward partial sums: [rhs][quad][4]
  static constexpr int XSZ = XS + 8 * Q;

  int c, q;             // lane in its quad, quad in its pixel
  int nvalid;           // library size n
  const float* sG;      // LDS, NP x NP scaled Gram (FP32)
  float* xp;            // LDS, this pixel's exchange area
  // after form_factor(): slot (r, K) with K < J = Q r + q holds -U_KJ, slot
  // (r, J) holds column c of L_J^{-1}, rd[r] holds 1 / d of element c of J
  v4f H[NS];
  float rd[R];
  bool notpd;

  __device__ __forceinline__ int el(int m) const { return 4 * (Q * m + q) + c; }
  __device__ __forceinline__ int col(int r) const { return Q * r + q; }
  __device__ __forceinline__ bool writer() const { return q == 0 && c == 0; }

  // reductions over the pixel's 4 Q lanes, the same bits on every lane
  template <typename V, typename Op>
  static __device__ __forceinline__ V red(V v, Op op) {
    v = op(v, dpp<qp(1, 0, 3, 2)>(v));
    v = op(v, dpp<qp(2, 3, 0, 1)>(v));
    if constexpr (Q >= 2) v = op(v, dpp<kRowHalfMirror>(v));
    if constexpr (Q >= 4) v = op(v, dpp<kRowMirror>(v));
    if constexpr (Q >= 8) {
      const Pair<V> p = pair<16>(v);
      v = op(p.lo, p.hi);
    }
    if constexpr (Q >= 16) {
      const Pair<V> p = pair<32>(v);
      v = op(p.lo, p.hi);
    }
    return v;
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
  // sum over the quad's four lanes
  static __device__ __forceinline__ float qsum(float v) {
    v += dpp<qp(1, 0, 3, 2)>(v);
    return v + dpp<qp(2, 3, 0, 1)>(v);
  }
  __device__ __forceinline__ float own(const v4f& t) const {
    return c == 0 ? t[0] : (c == 1 ? t[1] : (c == 2 ? t[2] : t[3]));
  }
  // Gh[4 I + c][4 J .. 4 J + 3]
  __device__ __forceinline__ v4f grow(int I, int J) const { return ld4(sG + (4 * I + c) * NP + 4 * J); }

  // out = Gh v: the whole vector through LDS, then this lane's rows
  __device__ __forceinline__ void gvec(const float (&v)[C], float (&out)[C]) const {
    asm volatile("" ::: "memory");
    static_for<0, R>([&](auto mm_) { xp[XV + el(mm_)] = v[mm_]; });
    lds_sync();
    v4f vb[T];
    static_for<0, T>([&](auto jj) { vb[jj] = ld4(xp + XV + 4 * decltype(jj)::value); });
    static_for<0, R>([&](auto mm_) {
      constexpr int m = decltype(mm_)::value;
      float acc0 = 0.f, acc1 = 0.f;
      static_for<0, T>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        const v4f g = grow(col(m), J);
        acc0 = fmaT(g[0], vb[J][0], acc0);
        acc1 = fmaT(g[1], vb[J][1], acc1);
        acc0 = fmaT(g[2], vb[J][2], acc0);
        acc1 = fmaT(g[3], vb[J][3], acc1);
      });
      out[m] = acc0 + acc1;
    });
    asm volatile("" ::: "memory");
  }

  // H = Gh + diag(D), then H = U^T D U
  __device__ __forceinline__ void form_factor(const float (&D)[C]) {
    asm volatile("" ::: "memory");
    static_for<0, R>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      const int J = col(r);
      static_for<0, Q * (r + 1)>([&](auto kk) {
        constexpr int K = decltype(kk)::value;
        v4f h = grow(J, K);  // tile (K, J): column c is Gh[4 J + c][4 K ..]
        if (K == J) {
          h[0] += c == 0 ? D[r] : 0.f;
          h[1] += c == 1 ? D[r] : 0.f;
          h[2] += c == 2 ? D[r] : 0.f;
          h[3] += c == 3 ? D[r] : 0.f;
        }
        H[sid(r, K)] = h;
      });
    });
    bool bad = false;
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      constexpr int rK = K / Q, qK = K % Q;
      const bool owner = q == qK;
      // the diagonal tile to every quad of the pixel
      if (owner) st4(xp + XD + 4 * c, H[sid(rK, K)]);
      lds_sync();
      const v4f t0 = ld4(xp + XD), t1 = ld4(xp + XD + 4), t2 = ld4(xp + XD + 8), t3 = ld4(xp + XD + 12);
      const float m00 = t0[0], m10 = t0[1], m20 = t0[2], m30 = t0[3];
      const float m11 = t1[1], m21 = t1[2], m31 = t1[3];
      const float m22 = t2[2], m32 = t2[3];
      const float m33 = t3[3];
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
      // row c of L^{-1} (L^T w = e_c) and column c (L v = e_c)
      const float w3 = e3;
      const float w2 = fmaT(-l32, w3, e2);
      const float w1 = fmaT(-l31, w3, fmaT(-l21, w2, e1));
      const float w0 = fmaT(-l30, w3, fmaT(-l20, w2, fmaT(-l10, w1, e0)));
      const float v0 = e0;
      const float v1 = fmaT(-l10, v0, e1);
      const float v2 = fmaT(-l21, v1, fmaT(-l20, v0, e2));
      const float v3 = fmaT(-l32, v2, fmaT(-l31, v1, fmaT(-l30, v0, e3)));
      const v4f li = (v4f){w0, w1, w2, w3};
      const v4f nr = (v4f){-r0, -r1, -r2, -r3};
      H[sid(rK, K)] = owner ? (v4f){v0, v1, v2, v3} : H[sid(rK, K)];
      rd[rK] = owner ? (c == 0 ? r0 : (c == 1 ? r1 : (c == 2 ? r2 : r3))) : rd[rK];
      if constexpr (K + 1 < T) {
        // panel of this quad's columns J > K; the tiles -U_KJ published
        v4f W[R];
        static_for<rK, R>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          const bool live = col(r) > K;
          v4f w = cc_mm(li, H[sid(r, K)], (v4f){0.f, 0.f, 0.f, 0.f});
          w = live ? w : (v4f){0.f, 0.f, 0.f, 0.f};
          W[r] = w;
          const v4f un = w * nr;
          H[sid(r, K)] = live ? un : H[sid(r, K)];
          if (live) st4(xp + XU + 16 * col(r) + 4 * c, un);
        });
        lds_sync();
        // trailing update: tile (I, J) += (-U_KI)^T W_KJ for K < I <= J (a
        // column with J <= K has W = 0 and stays as it is)
        static_for<K + 1, T>([&](auto ii) {
          constexpr int I = decltype(ii)::value;
          const v4f u = ld4(xp + XU + 16 * I + 4 * c);
          static_for<rK, R>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            if constexpr (I < Q * (r + 1)) H[sid(r, I)] = cc_mm(u, W[r], H[sid(r, I)]);
          });
        });
      }
      __builtin_amdgcn_sched_barrier(0);
    });
    notpd = bad;
    asm volatile("" ::: "memory");
  }

  // forward solve U^T y = r and z = D^{-1} y, in place (compact layout)
  template <int NR>
  __device__ __forceinline__ void forward(float (&x)[NR][C]) const {
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      constexpr int rK = K / Q, qK = K % Q;
      const bool owner = q == qK;
      const v4f lc = H[sid(rK, K)];
      static_for<0, NR>([&](auto qq) {
        constexpr int h = decltype(qq)::value;
        // owner: y_K = L_K^{-1} t_K (this lane's column of L_K^{-1} times
        // its own element, summed over the quad), published
        v4f y = lc * x[h][rK];
        static_for<0, 4>([&](auto i) {
          constexpr int k = decltype(i)::value;
          y[k] = qsum(y[k]);
        });
        const float yc = own(y);
        if (owner) {
          x[h][rK] = yc * rd[rK];
          xp[XV + 4 * h + c] = yc;
        }
      });
      if constexpr (K + 1 < T) {
        lds_sync();
        static_for<0, NR>([&](auto qq) {
          constexpr int h = decltype(qq)::value;
          const v4f yb = ld4(xp + XV + 4 * h);
          // the columns J > K of this quad: t_J -= U_KJ^T y_K
          static_for<rK, R>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            const v4f u = H[sid(r, K)];
            const float t = fmaT(u[0], yb[0], fmaT(u[1], yb[1], fmaT(u[2], yb[2], fmaT(u[3], yb[3], x[h][r]))));
            x[h][r] = col(r) > K ? t : x[h][r];
          });
        });
      }
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // backward solve U x = z, in place (compact layout)
  template <int NR>
  __device__ __forceinline__ void backward(float (&x)[NR][C]) const {
    static_for<0, T>([&](auto kk) {
      constexpr int K = T - 1 - decltype(kk)::value;
      constexpr int rK = K / Q, qK = K % Q;
      const bool owner = q == qK;
      static_for<0, NR>([&](auto qq) {
        constexpr int h = decltype(qq)::value;
        // this quad's part of z_K + sum over J > K of (-U_KJ) x_J
        v4f s = (v4f){0.f, 0.f, 0.f, 0.f};
        if (owner) {
          s[0] = c == 0 ? x[h][rK] : 0.f;
          s[1] = c == 1 ? x[h][rK] : 0.f;
          s[2] = c == 2 ? x[h][rK] : 0.f;
          s[3] = c == 3 ? x[h][rK] : 0.f;
        }
        static_for<rK, R>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          const v4f u = H[sid(r, K)];
          const float xv = col(r) > K ? x[h][r] : 0.f;
          s[0] = fmaT(u[0], xv, s[0]);
          s[1] = fmaT(u[1], xv, s[1]);
          s[2] = fmaT(u[2], xv, s[2]);
          s[3] = fmaT(u[3], xv, s[3]);
        });
        static_for<0, 4>([&](auto i) {
          constexpr int k = decltype(i)::value;
          s[k] = qsum(s[k]);
        });
        xp[XS + (h * Q + q) * 4 + c] = own(s);
      });
      lds_sync();
      const v4f lc = H[sid(rK, K)];
      static_for<0, NR>([&](auto qq) {
        constexpr int h = decltype(qq)::value;
        v4f t = ld4(xp + XS + h * Q * 4);
        static_for<1, Q>([&](auto qi) { t += ld4(xp + XS + (h * Q + decltype(qi)::value) * 4); });
        const float xk = fmaT(lc[0], t[0], fmaT(lc[1], t[1], fmaT(lc[2], t[2], lc[3] * t[3])));
        x[h][rK] = owner ? xk : x[h][rK];
      });
      // the partial sums of this step are read before the next step writes
      // them (in-order LDS of one wavefront)
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  __device__ __forceinline__ void solve2(const float (&r)[C], float (&w)[C], float (&u)[C]) const {
    float x[2][C];
    static_for<0, C>([&](auto mm_) {
      constexpr int m = decltype(mm_)::value;
      x[0][m] = r[m];
      x[1][m] = el(m) < nvalid ? 1.f : 0.f;
    });
    asm volatile("" ::: "memory");
    forward<2>(x);
    backward<2>(x);
    asm volatile("" ::: "memory");
    static_for<0, C>([&](auto mm_) {
      w[mm_] = x[0][mm_];
      u[mm_] = x[1][mm_];
    });
  }
  __device__ __forceinline__ void solve1(const float (&r)[C], float (&w)[C]) const {
    float x[1][C];
    static_for<0, C>([&](auto mm_) { x[0][mm_] = r[mm_]; });
    asm volatile("" ::: "memory");
    forward<1>(x);
    backward<1>(x);
    asm volatile("" ::: "memory");
    static_for<0, C>([&](auto mm_) { w[mm_] = x[0][mm_]; });
  }
};

// pixels per workgroup (four wavefronts) and waves per SIMD by shape: one
// wave per SIMD, because the tiles and the method's vectors take more than
// half of the 512 registers of a lane
template <int T, int Q>
constexpr int kCcPixels = 4 * (16 / Q);
template <int T, int Q>
constexpr int kCcWaves = 1;

// One workgroup's pixels: workgroup wg of the cube described by prm.
template <int T, int Q, int MODE, int CONS>
__device__ __forceinline__ void ipm_cc32_body(const IpmParams& prm, int64_t wg) {
  using TL = CC32<T, Q>;
  constexpr int NP = TL::NP;
  constexpr int PB = kCcPixels<T, Q>;
  __shared__ __align__(16) float sG[NP * NP];
  __shared__ __align__(16) float sx[PB * TL::XSZ];
  const float* Gsrc = static_cast<const float*>(prm.Gh);
  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) sG[i] = Gsrc[i];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qd = lane >> 2;
  const int pib = wave * (16 / Q) + qd / Q;  // pixel in the workgroup
  const int64_t p = wg * PB + pib;
  TL tl;
  tl.c = lane & 3;
  tl.q = qd % Q;
  tl.nvalid = prm.n;
  tl.sG = sG;
  tl.xp = sx + pib * TL::XSZ;
  ipm_pixel<TL, MODE, CONS>(prm, p, p < prm.P, tl);
}

template <int T, int Q, int MODE, int CONS>
__global__ __launch_bounds__(256, (kCcWaves<T, Q>)) void ipm_cc32_kernel(IpmParams prm) {
  ipm_cc32_body<T, Q, MODE, CONS>(prm, blockIdx.x);
}

template <int T, int Q, int MODE, int CONS>
__global__ __launch_bounds__(256, (kCcWaves<T, Q>)) void ipm_cc32_batch_kernel(const IpmParams* __restrict__ jobs,
                                                                              const int64_t* __restrict__ start,
                                                                              int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const IpmParams prm = uniform_copy(jobs + j);
  ipm_cc32_body<T, Q, MODE, CONS>(prm, (int64_t)blockIdx.x - start[j]);
}

template <int T, int Q, int CONS>
static int launch_cc32_c(const IpmParams& p, const IpmBatch* b, hipStream_t st) {
  constexpr int PB = kCcPixels<T, Q>;
  if (b)
    hipLaunchKernelGGL((ipm_cc32_batch_kernel<T, Q, kStage1, CONS>), dim3((unsigned)b->blocks), dim3(256), 0, st,
                       b->jobs, b->start, b->njobs);
  else
    hipLaunchKernelGGL((ipm_cc32_kernel<T, Q, kStage1, CONS>), dim3((unsigned)((p.P + PB - 1) / PB)), dim3(256), 0,
                       st, p);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// b == nullptr: one cube described by p; else the jobs of b (p only gives
// the constraint option).  Only the first stage of the mixed form runs here.
template <int T, int Q>
static int launch_cc32(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  if (mode != kStage1) return -5;
  switch (p.constraint) {
    case kSto: return launch_cc32_c<T, Q, kSto>(p, b, st);
    case kSlo: return launch_cc32_c<T, Q, kSlo>(p, b, st);
    case kPos: return launch_cc32_c<T, Q, kPos>(p, b, st);
  }
  return -1;
}

#if defined(LM_CC32_T) && defined(LM_CC32_Q)
#define LM_CENTRY2(t, q) ipm_cc32_entry_##t##_##q
#define LM_CENTRY(t, q) LM_CENTRY2(t, q)
int LM_CENTRY(LM_CC32_T, LM_CC32_Q)(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  return launch_cc32<LM_CC32_T, LM_CC32_Q>(p, b, mode, st);
}
#endif

}  // namespace lm
