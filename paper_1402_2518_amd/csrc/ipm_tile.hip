// ipm_tile.hip -- FP64 interior-point solve (IPLS, Sec. 2.2) with the Newton
// matrix held as 4x4 tiles on the matrix cores (v_mfma_f64_4x4x4f64).
//
// Same method as ipm.hip (Mehrotra predictor-corrector on the scaled QP of
// eq. 6 under eqs. 3-4, then the finishing step that certifies the free set);
// only the mapping differs.
//
// Mapping.  The 4x4x4 FP64 MFMA works on four independent 4x4 blocks per
// wavefront; block b = (lane >> 2) & 3 owns one pixel, so a wavefront solves
// four pixels.  Inside a block, lane (x, z) = (lane >> 4, lane & 3).
// Operand layouts (gfx950): A: lane (x=k, z=i) holds A[i][k]; B: lane
// (x=k, z=j) holds B[k][j]; C/D: lane (x=i, z=j) holds D[i][j].
// A tile X is kept "stored": lane (x, z) holds X[z][x].  Then one register
// is A = X and B = X^T at once, and
//     mfma(stored P, stored Q, stored R) = stored(Q P^T + R),
// so the trailing update of a block factorisation, H_IJ -= L_IK W_JK^T, is
// one MFMA on stored tiles with no data movement.  The Newton matrix is
// factored as L D L^T with unit lower L and diagonal D, column block by
// column block: the 4x4 diagonal block is factored redundantly on the 16
// lanes of its block (after an exchange through LDS) into L_KK diag(d) L_KK^T,
// the panel is W_JK = H_JK L_KK^{-T} and L_JK = W_JK diag(d)^{-1}, and the
// trailing update subtracts L_IK W_JK^T.  Keeping L_KK^{-1} and 1/d apart
// rather than forming the block inverse keeps the factorisation stable when
// a diagonal block is nearly singular (linearly dependent spectra, such as
// the +/- pairs of the additional spectra, with small lambda/a): the error
// of the update then scales with 1/sqrt(d), not 1/d.  No square roots.
// Vectors that feed the MFMA use the
// "x layout": lane (x, z) holds element 4I + x of right-hand side z, so up
// to four right-hand sides ride along (the solve carries u = H^{-1} 1 next to
// the Newton right-hand side).  Elementwise work uses a compact layout: lane
// (x, z) holds element 16m + 4z + x of slot m.
#include "common.h"
#include "kernels.h"

namespace lm {

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// quad broadcast: lane (x, z) <- lane (x, R) of the same block
template <int R>
__device__ __forceinline__ double qb(double v) {
  return dpp<qp(R, R, R, R)>(v);
}

// Reductions over the 16 lanes of a block (same bits on every lane): a quad
// butterfly with DPP, then the row pair (x ^ 1) and the half-wave pair
// (x ^ 2) through row swaps.
template <typename T, typename Op>
__device__ __forceinline__ T bred(T v, Op op) {
  v = op(v, dpp<qp(1, 0, 3, 2)>(v));
  v = op(v, dpp<qp(2, 3, 0, 1)>(v));
  Pair<T> p = pair<16>(v);
  v = op(p.lo, p.hi);
  p = pair<32>(v);
  return op(p.lo, p.hi);
}
__device__ __forceinline__ double bsum(double v) {
  return bred(v, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double bmin(double v) {
  return bred(v, [](double a, double b) { return fmin(a, b); });
}
__device__ __forceinline__ double bmax(double v) {
  return bred(v, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ int bmin_i(int v) {
  return bred(v, [](int a, int b) { return min(a, b); });
}
__device__ __forceinline__ int bor_i(int v) {
  return bred(v, [](int a, int b) { return a | b; });
}

// Reciprocal to about single precision squared (one Newton step), for
// step-to-boundary ratios, which only need a few digits.
__device__ __forceinline__ double rcp1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return y * fmaT(-x, y, 2.0);
}

template <typename T>
__device__ __forceinline__ bool fin(T v) {
  return isfin(v);
}

template <int T>
struct Tile {
  static constexpr int NP = 4 * T;
  static constexpr int C = (T + 3) / 4;  // compact slots
  static constexpr int NT = T * (T + 1) / 2;
  static constexpr int id(int I, int J) { return I * (I + 1) / 2 + J; }

  int x, z, blk;            // lane coordinates
  const double* sG;         // LDS, NP x NP scaled Gram
  double* xch;              // LDS, 16 doubles of this pixel (tile exchange)
  // Stored tiles of the lower triangle.  After factor(): L D L^T with unit
  // lower L and diagonal D; H[id(K, K)] holds L_KK^{-1} below its diagonal
  // and 1/d on it (zero above), H[id(I, K)] = -L_IK (I > K).
  double H[NT];
  bool notpd;

  // compact -> x layout (every right-hand side slot gets the same vector)
  __device__ __forceinline__ void to_x(const double (&v)[C], double (&xl)[T]) const {
    static_for<0, T>([&](auto ii) {
      constexpr int I = decltype(ii)::value;
      xl[I] = qb<I % 4>(v[I / 4]);
    });
  }
  // x layout, right-hand side R -> compact
  template <int R>
  __device__ __forceinline__ void from_x(const double (&xl)[T], double (&v)[C]) const {
    double tb[4 * C];
    static_for<0, 4 * C>([&](auto ii) {
      constexpr int I = decltype(ii)::value;
      if constexpr (I < T) tb[I] = qb<R>(xl[I]);
      else tb[I] = 0.0;
    });
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      v[m] = z == 0 ? tb[4 * m] : (z == 1 ? tb[4 * m + 1] : (z == 2 ? tb[4 * m + 2] : tb[4 * m + 3]));
    });
  }

  // v = Gh * xa: x layout in, compact layout out (each tile row is moved to
  // its compact slot as soon as it is done)
  __device__ __forceinline__ void gmul(const double (&xa)[T], double (&v)[C]) const {
    static_for<0, C>([&](auto mm) { v[mm] = 0.0; });
    static_for<0, T>([&](auto ii) {
      constexpr int I = decltype(ii)::value;
      double acc = 0.0;
      static_for<0, T>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        acc = mfma4(sG[(4 * I + z) * NP + 4 * J + x], xa[J], acc);
      });
      const double e = qb<0>(acc);  // element 4I + x of right-hand side 0
      v[I / 4] = (z == I % 4) ? e : v[I / 4];
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // H = Gh + diag(D), D in x layout
  __device__ __forceinline__ void form(const double (&xD)[T]) {
    static_for<0, T>([&](auto ii) {
      constexpr int I = decltype(ii)::value;
      static_for<0, I + 1>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        double v = sG[(4 * I + z) * NP + 4 * J + x];
        if constexpr (I == J) v += (x == z) ? xD[I] : 0.0;
        H[id(I, J)] = v;
      });
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // The symmetric 4x4 tile M held in stored form (lane (x, z) holds
  // M[z][x]) as L diag(d) L^T with unit lower L: the block's 16 lanes
  // exchange the tile through LDS and factor it redundantly.  Each lane
  // returns entry (z, x) of L^{-1} (1 on the diagonal, 0 above it) in li and
  // 1 / d_x in rx.
  __device__ __forceinline__ void ldl4(double h, bool& bad, double& li, double& rx) const {
    xch[z * 4 + x] = h;
    lds_sync();
    const double m00 = xch[0], m10 = xch[4], m11 = xch[5], m20 = xch[8], m21 = xch[9];
    const double m22 = xch[10], m30 = xch[12], m31 = xch[13], m32 = xch[14], m33 = xch[15];
    const double d0 = m00;
    const double r0 = rcpT(d0);
    const double l10 = m10 * r0, l20 = m20 * r0, l30 = m30 * r0;
    const double d1 = fmaT(-l10, m10, m11);
    const double r1 = rcpT(d1);
    const double t21 = fmaT(-l20, m10, m21), t31 = fmaT(-l30, m10, m31);
    const double l21 = t21 * r1, l31 = t31 * r1;
    const double d2 = fmaT(-l21, t21, fmaT(-l20, m20, m22));
    const double r2 = rcpT(d2);
    const double t32 = fmaT(-l31, t21, fmaT(-l30, m20, m32));
    const double l32 = t32 * r2;
    const double d3 = fmaT(-l32, t32, fmaT(-l31, t31, fmaT(-l30, m30, m33)));
    const double r3 = rcpT(d3);
    // pivots positive and finite; for a sum, s - s == 0 is a safe finiteness
    // test (no product to contract with) and keeps the factor's register
    // footprint lower than a class test here
    const double dmin = fmin(fmin(d0, d1), fmin(d2, d3));
    const double ds = d0 + d1 + d2 + d3;
    bad |= !(dmin > 0.0) || !(ds == ds && ds - ds == 0.0);
    // column x of L^{-1}: L v = e_x
    const double e0 = x == 0 ? 1.0 : 0.0, e1 = x == 1 ? 1.0 : 0.0;
    const double e2 = x == 2 ? 1.0 : 0.0, e3 = x == 3 ? 1.0 : 0.0;
    const double v1 = fmaT(-l10, e0, e1);
    const double v2 = fmaT(-l21, v1, fmaT(-l20, e0, e2));
    const double v3 = fmaT(-l32, v2, fmaT(-l31, v1, fmaT(-l30, e0, e3)));
    li = z == 0 ? e0 : (z == 1 ? v1 : (z == 2 ? v2 : v3));
    rx = x == 0 ? r0 : (x == 1 ? r1 : (x == 2 ? r2 : r3));
  }

  // tiled right-looking L D L^T of H
  __device__ __forceinline__ void factor() {
    bool bad = false;
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      double li, rx;
      ldl4(H[id(K, K)], bad, li, rx);
      const double nrx = -rx;
      H[id(K, K)] = (x == z) ? rx : li;
      // Panel W_JK = H_JK L_KK^{-T}, -L_JK = -W_JK diag(d)^{-1}, and trailing
      // update H_IJ -= L_IK W_JK^T, one column J at a time from the last:
      // column J needs -L_IK for I >= J (done) and W_JK, so only one W tile
      // is live.
      static_for<K + 1, T>([&](auto jj) {
        constexpr int J = T + K - decltype(jj)::value;
        const double w = mfma4(li, H[id(J, K)], 0.0);
        H[id(J, K)] = w * nrx;
        static_for<J, T>([&](auto ii) {
          constexpr int I = decltype(ii)::value;
          H[id(I, J)] = mfma4(w, H[id(I, K)], H[id(I, J)]);
        });
      });
    });
    notpd = bad;
  }

  // solve L D L^T X = R in place (x layout, one right-hand side per z)
  __device__ __forceinline__ void solve(double (&xr)[T]) const {
    // L y = r: the unit lower diagonal block, then the blocks below it
    static_for<0, T>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      const double lu = (x == z) ? 1.0 : H[id(J, J)];
      xr[J] = mfma4(lu, xr[J], 0.0);
      static_for<J + 1, T>([&](auto ii) {
        constexpr int I = decltype(ii)::value;
        xr[I] = mfma4(H[id(I, J)], xr[J], xr[I]);
      });
    });
    // diag(d)^{-1} y
    static_for<0, T>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      const double dg = (x == z) ? H[id(J, J)] : 0.0;
      xr[J] = mfma4(dg, xr[J], 0.0);
    });
    // L^T x = diag(d)^{-1} y; a transposed tile comes from lane (z, x)
    const int src = 16 * z + 4 * blk + x;
    static_for<0, T>([&](auto kk) {
      constexpr int I = T - 1 - decltype(kk)::value;
      const double lut = __shfl((x == z) ? 1.0 : H[id(I, I)], src);
      xr[I] = mfma4(lut, xr[I], 0.0);
      static_for<0, I>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        const double lt = __shfl(H[id(I, J)], src);
        xr[J] = mfma4(lt, xr[I], xr[J]);
      });
    });
  }

  // -M^{-1}[z][x] for the symmetric 4x4 tile M held in stored form (lane
  // (x, z) holds M[z][x]).  The block's 16 lanes exchange the tile through
  // LDS, factor it redundantly as L diag(d) L^T (unit lower L), and each lane
  // solves M y = -e_x for its own column, keeping entry z.
  __device__ __forceinline__ double ninv4(double h, bool& bad) const {
    xch[z * 4 + x] = h;
    lds_sync();
    const double m00 = xch[0], m10 = xch[4], m11 = xch[5], m20 = xch[8], m21 = xch[9];
    const double m22 = xch[10], m30 = xch[12], m31 = xch[13], m32 = xch[14], m33 = xch[15];
    const double d0 = m00;
    const double r0 = rcpT(d0);
    const double l10 = m10 * r0, l20 = m20 * r0, l30 = m30 * r0;
    const double d1 = fmaT(-l10, m10, m11);
    const double r1 = rcpT(d1);
    const double t21 = fmaT(-l20, m10, m21), t31 = fmaT(-l30, m10, m31);
    const double l21 = t21 * r1, l31 = t31 * r1;
    const double d2 = fmaT(-l21, t21, fmaT(-l20, m20, m22));
    const double r2 = rcpT(d2);
    const double t32 = fmaT(-l31, t21, fmaT(-l30, m20, m32));
    const double l32 = t32 * r2;
    const double d3 = fmaT(-l32, t32, fmaT(-l31, t31, fmaT(-l30, m30, m33)));
    const double r3 = rcpT(d3);
    // pivots positive and finite; for a sum, s - s == 0 is a safe finiteness
    // test (no product to contract with) and keeps the factor's register
    // footprint lower than a class test here
    const double dmin = fmin(fmin(d0, d1), fmin(d2, d3));
    const double ds = d0 + d1 + d2 + d3;
    bad |= !(dmin > 0.0) || !(ds == ds && ds - ds == 0.0);
    // L v = -e_x, y = L^{-T} diag(r) v
    const double e0 = x == 0 ? -1.0 : 0.0, e1 = x == 1 ? -1.0 : 0.0;
    const double e2 = x == 2 ? -1.0 : 0.0, e3 = x == 3 ? -1.0 : 0.0;
    const double v1 = fmaT(-l10, e0, e1);
    const double v2 = fmaT(-l21, v1, fmaT(-l20, e0, e2));
    const double v3 = fmaT(-l32, v2, fmaT(-l31, v1, fmaT(-l30, e0, e3)));
    const double y3 = v3 * r3;
    const double y2 = fmaT(-l32, y3, v2 * r2);
    const double y1 = fmaT(-l31, y3, fmaT(-l21, y2, v1 * r1));
    const double y0 = fmaT(-l30, y3, fmaT(-l20, y2, fmaT(-l10, y1, e0 * r0)));
    return z == 0 ? y0 : (z == 1 ? y1 : (z == 2 ? y2 : y3));
  }

  // tiled right-looking block L D L^T of H with explicit inverses of the
  // 4x4 diagonal blocks D_K (panel -L_IK = -H_IK D_K^{-1})
  __device__ __forceinline__ void factor_inv() {
    bool bad = false;
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      const double ndinv = ninv4(H[id(K, K)], bad);
      H[id(K, K)] = -ndinv;
      // Panel -L_JK = -H_JK D_K^{-1} and trailing update H_IJ -= L_IK H_JK^T,
      // one column J at a time from the last: column J needs -L_IK for I >= J
      // (done) and the unscaled H_JK, so only one unscaled tile is live.
      static_for<K + 1, T>([&](auto jj) {
        constexpr int J = T + K - decltype(jj)::value;
        const double u = H[id(J, K)];
        H[id(J, K)] = mfma4(ndinv, u, 0.0);
        static_for<J, T>([&](auto ii) {
          constexpr int I = decltype(ii)::value;
          H[id(I, J)] = mfma4(u, H[id(I, K)], H[id(I, J)]);
        });
      });
    });
    notpd = bad;
  }

  // solve with the factor of factor_inv (identity diagonal blocks of L)
  __device__ __forceinline__ void solve_inv(double (&xr)[T]) const {
    // L y = r
    static_for<0, T>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      static_for<J + 1, T>([&](auto ii) {
        constexpr int I = decltype(ii)::value;
        xr[I] = mfma4(H[id(I, J)], xr[J], xr[I]);
      });
    });
    // D^{-1} y
    static_for<0, T>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      xr[J] = mfma4(H[id(J, J)], xr[J], 0.0);
    });
    // L^T x = D^{-1} y; the transposed tile comes from lane (z, x)
    const int src = 16 * z + 4 * blk + x;
    static_for<0, T>([&](auto kk) {
      constexpr int I = T - 1 - decltype(kk)::value;
      static_for<0, I>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        const double lt = __shfl(H[id(I, J)], src);
        xr[J] = mfma4(lt, xr[I], xr[J]);
      });
    });
  }
};

// One workgroup's 16 pixels: workgroup wg of the cube described by prm.
// ST: the stable factorisation (factor/solve) rather than explicit inverses
// of the diagonal blocks (factor_inv/solve_inv).
template <int T, int MODE, int CONS, bool ST>
__device__ __forceinline__ void ipm_tile_body(const IpmParams& prm, int64_t wg) {
  using TL = Tile<T>;
  constexpr int NP = TL::NP;
  constexpr int C = TL::C;
  __shared__ double sG[NP * NP];
  __shared__ double sx[16 * 18];
  const double* Gsrc = static_cast<const double*>(prm.Gh);
  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) sG[i] = Gsrc[i];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = (lane >> 2) & 3, x = lane >> 4, z = lane & 3;
  const int pib = wave * 4 + blk;
  const int64_t p = wg * 16 + pib;
  const bool inrange = p < prm.P;
  const int n = prm.n;

  TL tl;
  tl.x = x;
  tl.z = z;
  tl.blk = blk;
  tl.sG = sG;
  tl.xch = sx + pib * 18;

  bool vm[C];
  static_for<0, C>([&](auto mm) { vm[mm] = (16 * mm + 4 * z + x) < n; });
  auto el = [&](int m) { return 16 * m + 4 * z + x; };
  // x-layout validity of element 4I + x
  auto vx = [&](int I) { return 4 * I + x < n; };

  uint32_t flags = 0;
  double bh[C];
  bool nonfin = false;
  static_for<0, C>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    const double v = (inrange && vm[m]) ? prm.bh[p * n + el(m)] : 0.0;
    if (!fin(v)) nonfin = true;
    bh[m] = v;
  });
  if (inrange && prm.c && !fin(prm.c[p])) nonfin = true;
  nonfin = bor_i((int)nonfin) != 0;
  if (nonfin) {
    flags |= kPxNonfinite;
    static_for<0, C>([&](auto mm) { bh[mm] = 0.0; });
  }
  double bhmax = 0.0;
  static_for<0, C>([&](auto mm) { bhmax = fmax(bhmax, fabs(bh[mm])); });
  bhmax = bmax(bhmax);

  // constraint besides a >= 0: sum-to-one, sum-lower-than-one (slack s of
  // 1^T a <= 1 with multiplier nu: one more complementarity pair), or
  // positivity only (no sum row, nu = 0)
  constexpr bool slo = CONS == kSlo, pos = CONS == kPos;
  const double inv_np = 1.0 / (n + (slo ? 1 : 0));  // complementarity pairs
  double a[C], lam[C], nu = slo ? prm.lambda0 : 0.0, s = slo ? inv_np : 0.0;
  int it = 0;
  bool start = inrange && !nonfin;
  if constexpr (MODE == kStage2) {
    if (inrange) {
      const uint8_t f = prm.st_flag[p];
      flags |= f & 0x7fu;
      start = start && (f & 0x80u);
      it = prm.st_it[p];
      nu = prm.st_nu[p];
      s = slo ? prm.st_s[p] : 0.0;
    }
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const bool ok = inrange && vm[m];
      a[m] = ok ? prm.st_a[p * n + el(m)] : 0.0;
      lam[m] = ok ? prm.st_lam[p * n + el(m)] : 0.0;
    });
  } else {
    static_for<0, C>([&](auto mm) {
      a[mm] = vm[mm] ? inv_np : 0.0;
      lam[mm] = vm[mm] ? prm.lambda0 : 0.0;
    });
  }
  const double tol_mu = prm.tol_mu, tol_d = prm.tol_d, tol_p = prm.tol_p, eta = prm.eta, tau = prm.tau;
  const double inv_n = 1.0 / n;
  constexpr double BIG = 1e30;

  enum { kIpm = 0, kPol = 1, kDone = 2 };
  int phase = start ? kIpm : kDone;
  bool converged = false, certified = false, cand = false;
  bool sfree = pos;  // finishing step: the sum row is absent (slack free or no sum constraint)
  uint32_t freem = 0;  // bit m: compact slot m is free
  int kp = 0;
  double pa[C], pnu = 0.0;

  double g[C], rd[C], D[C], dx[C], u[C], dla[C];
  double rp = 0.0, mu = 0.0;
  double xl[T];
  // gradient of the quadratic at the starting point
  tl.to_x(a, xl);
  tl.gmul(xl, g);
  for (;;) {
    // Gh is re-read from LDS each step rather than held in registers across
    // iterations (it would not fit next to the factor).
    asm volatile("" ::: "memory");
    // ---- phase decisions ---------------------------------------------------
    // g = Gh a is carried from step to step (see the update below).  Where
    // dependent spectra make the Newton matrix nearly singular, the carried
    // g drifts from Gh a, so a pixel whose residuals pass the stopping tests
    // confirms them with an explicit product before it stops; the finishing
    // step's candidate gets its own product as well.
    auto residuals = [&](double& rdm) {
      double sa = 0.0, sal = 0.0;
      rdm = 0.0;
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        rd[m] = vm[m] ? (g[m] - bh[m] - lam[m] + nu) : 0.0;
        sa += a[m];
        sal = fmaT(a[m], lam[m], sal);
        rdm = fmax(rdm, fabs(rd[m]));
      });
      rp = pos ? 0.0 : bsum(sa) + s - 1.0;
      mu = (bsum(sal) + s * nu) * inv_np;
      rdm = bmax(rdm);
    };
    auto stops = [&](double rdm) {
      if constexpr (MODE == kStage1)
        return mu <= fmax(tol_mu, prm.mu_switch);
      else
        return mu <= tol_mu && rdm <= tol_d * (1.0 + bhmax) && fabs(rp) <= tol_p;
    };
    double rdm = 0.0;
    bool conv = false;
    if (phase == kIpm) {
      residuals(rdm);
      conv = stops(rdm);
    }
    const bool confirm = MODE != kStage1 && phase == kIpm && conv;
    double gp[C];
    if (__builtin_amdgcn_ballot_w64(confirm || (phase == kPol && cand)) != 0) {
      double v[C];
      static_for<0, C>([&](auto mm) { v[mm] = confirm ? a[mm] : pa[mm]; });
      tl.to_x(v, xl);
      tl.gmul(xl, gp);
    }
    if (confirm) {
      static_for<0, C>([&](auto mm) { g[mm] = gp[mm]; });
      residuals(rdm);
      conv = stops(rdm);
    }
    if (phase == kIpm) {
      if (conv) {
        converged = true;
        phase = kPol;
        cand = false;
        static_for<0, C>([&](auto mm) {
          if (vm[mm] && a[mm] > lam[mm]) freem |= 1u << mm;
        });
        sfree = pos || (slo && s > nu);
      } else if (it >= prm.maxit) {
        flags |= kPxMaxit;
        phase = kDone;
      }
    } else if (phase == kPol && cand) {
      double wa = INFINITY, wl = INFINITY, pl[C];
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        const bool fr = (freem >> m) & 1u;
        pl[m] = (vm[m] && !fr) ? gp[m] - bh[m] + pnu : 0.0;
        if (vm[m] && fr) wa = fmin(wa, pa[m]);
        if (vm[m] && !fr) wl = fmin(wl, pl[m]);
      });
      wa = bmin(wa);
      wl = bmin(wl);
      // sum-lower-than-one: the slack is one more index (free: its value
      // 1 - 1^T a must be >= 0; at its bound: the multiplier nu must be)
      double spa = 0.0;
      static_for<0, C>([&](auto mm) { spa += pa[mm]; });
      const double sv = 1.0 - bsum(spa);
      const bool slA = slo && sfree && sv < fmin(wa, -tau);
      const bool slL = slo && !sfree && pnu < fmin(wl, -tau);
      if (slA) wa = sv;
      if (slL) wl = pnu;
      if (wa >= -tau && wl >= -tau) {
        certified = true;
        phase = kDone;
        static_for<0, C>([&](auto mm) {
          a[mm] = pa[mm];
          lam[mm] = pl[mm];
        });
        nu = pnu;
        s = (slo && sfree) ? sv : 0.0;
      } else if (kp >= prm.max_polish) {
        phase = kDone;
      } else if ((wa < -tau && wa <= wl) ? slA : slL) {
        sfree = !sfree;
        ++kp;
        cand = false;
      } else {
        const bool flipA = (wa < -tau) && (wa <= wl);
        const double target = flipA ? wa : wl;
        int idx = 1 << 30;
        static_for<0, C>([&](auto mm) {
          constexpr int m = decltype(mm)::value;
          const bool fr = (freem >> m) & 1u;
          const bool c = flipA ? (vm[m] && fr && pa[m] == target) : (vm[m] && !fr && pl[m] == target);
          if (c) idx = min(idx, el(m));
        });
        idx = bmin_i(idx);
        static_for<0, C>([&](auto mm) {
          if (el(mm) == idx) freem ^= 1u << mm;
        });
        ++kp;
        cand = false;
      }
    }
    if (__builtin_amdgcn_ballot_w64(phase != kDone) == 0) break;

    // ---- Newton (or finishing-step) matrix and its factorisation ----------
    double ia[C];  // 1 / a
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      ia[m] = rcpT(a[m]);
      const double dp = ((freem >> m) & 1u) ? 0.0 : BIG;
      const double di = (phase == kPol) ? dp : ((phase == kIpm) ? lam[m] * ia[m] : 1.0);
      D[m] = vm[m] ? di : 0.0;
    });
    tl.to_x(D, xl);
    tl.form(xl);
    if constexpr (ST) tl.factor(); else tl.factor_inv();
    if (phase != kDone && tl.notpd) {
      if (phase == kIpm) flags |= kPxNotPd;
      phase = kDone;
    }

    // ---- first solve: [rhs, 1] (predictor / finishing), u = H^{-1} 1 ------
    {
      double rc[C];
      static_for<0, C>([&](auto mm) {
        rc[mm] = (phase == kPol) ? bh[mm] : (vm[mm] ? -rd[mm] - lam[mm] : 0.0);
      });
      tl.to_x(rc, xl);
      static_for<0, T>([&](auto ii) {
        constexpr int I = decltype(ii)::value;
        const double one = vx(I) ? 1.0 : 0.0;
        xl[I] = (z == 1) ? one : xl[I];
      });
    }
    if constexpr (ST) tl.solve(xl); else tl.solve_inv(xl);
    tl.template from_x<0>(xl, dx);
    tl.template from_x<1>(xl, u);
    double su = 0.0, sw = 0.0;
    static_for<0, C>([&](auto mm) {
      su += u[mm];
      sw += dx[mm];
    });
    su = bsum(su);
    sw = bsum(sw);
    const double isu = rcpT(su);
    if (phase == kPol) {
      // equality-constrained problem on the free set: a = w - nu u, 1^T a = 1
      pnu = sfree ? 0.0 : (sw - 1.0) * isu;
      static_for<0, C>([&](auto mm) {
        pa[mm] = (vm[mm] && ((freem >> mm) & 1u)) ? fmaT(-pnu, u[mm], dx[mm]) : 0.0;
      });
      cand = fin(pnu);
      if (!cand) phase = kDone;
    }
    const bool two = __builtin_amdgcn_ballot_w64(phase == kIpm) != 0;
    if (!two) continue;

    // ---- predictor step and centring --------------------------------------
    // sum row: dnu = (1^T w + r_p - rcs/nu) / (1^T u + s/nu) with the slack
    // pair (rcs = s nu in the predictor), (1^T w + r_p) / 1^T u without it;
    // none for positivity only; ds = (-rcs - s dnu) / nu
    const double son = slo ? s / nu : 0.0;
    const double dnu_aff = pos ? 0.0 : (slo ? (sw + rp - s) / (su + son) : (sw + rp) * isu);
    const double ds_aff = slo ? -s - son * dnu_aff : 0.0;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      dx[m] = vm[m] ? fmaT(-dnu_aff, u[m], dx[m]) : 0.0;
      dla[m] = vm[m] ? -lam[m] - D[m] * dx[m] : 0.0;
    });
    double st_aff = INFINITY;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const double q1 = -a[m] * rcp1(dx[m]), q2 = -lam[m] * rcp1(dla[m]);
      st_aff = (vm[m] && dx[m] < 0.0) ? fmin(st_aff, q1) : st_aff;
      st_aff = (vm[m] && dla[m] < 0.0) ? fmin(st_aff, q2) : st_aff;
    });
    st_aff = fmin(bmin(st_aff), 1.0);
    if (slo) {
      if (ds_aff < 0.0) st_aff = fmin(st_aff, -s / ds_aff);
      if (dnu_aff < 0.0) st_aff = fmin(st_aff, -nu / dnu_aff);
    }
    double smu = 0.0;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (vm[m]) smu = fmaT(a[m] + st_aff * dx[m], lam[m] + st_aff * dla[m], smu);
    });
    const double smu_s = slo ? (s + st_aff * ds_aff) * (nu + st_aff * dnu_aff) : 0.0;
    const double ratio = (bsum(smu) + smu_s) * inv_np * rcpT(mu);
    const double sig = ratio * ratio * ratio;

    // ---- corrector (second-order term dropped after a short affine step) ---
    const double soc = st_aff >= 0.1 ? 1.0 : 0.0;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const double rcv = fmaT(soc * dx[m], dla[m], a[m] * lam[m]) - sig * mu;
      dla[m] = vm[m] ? rcv * ia[m] : 0.0;  // rc / a
      dx[m] = vm[m] ? -rd[m] - dla[m] : 0.0;
    });
    tl.to_x(dx, xl);
    if constexpr (ST) tl.solve(xl); else tl.solve_inv(xl);
    tl.template from_x<0>(xl, dx);
    double sw2 = 0.0;
    static_for<0, C>([&](auto mm) { sw2 += dx[mm]; });
    sw2 = bsum(sw2);
    const double rcs = slo ? fmaT(soc * ds_aff, dnu_aff, s * nu) - sig * mu : 0.0;
    const double dnu = pos ? 0.0 : (slo ? (sw2 + rp - rcs / nu) / (su + son) : (sw2 + rp) * isu);
    const double ds = slo ? (-rcs - s * dnu) / nu : 0.0;
    double dl[C];
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      dx[m] = vm[m] ? fmaT(-dnu, u[m], dx[m]) : 0.0;
      dl[m] = vm[m] ? -dla[m] - D[m] * dx[m] : 0.0;
    });
    double step = INFINITY;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const double q1 = -a[m] * rcp1(dx[m]), q2 = -lam[m] * rcp1(dl[m]);
      step = (vm[m] && dx[m] < 0.0) ? fmin(step, q1) : step;
      step = (vm[m] && dl[m] < 0.0) ? fmin(step, q2) : step;
    });
    step = bmin(step);
    if (slo) {
      if (ds < 0.0) step = fmin(step, -s / ds);
      if (dnu < 0.0) step = fmin(step, -nu / dnu);
    }
    const double alpha = fmin(1.0, eta * step);
    if (phase == kIpm && fin(alpha)) {
      // the Newton equations give Gh da = -r_d + dlambda - dnu 1 exactly, so
      // the gradient follows the step without another product with Gh
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        const double rdm = g[m] - bh[m] - lam[m] + nu;  // r_d before the step
        g[m] = vm[m] ? fmaT(alpha, dl[m] - rdm - dnu, g[m]) : 0.0;
        a[m] = fmaT(alpha, dx[m], a[m]);
        lam[m] = fmaT(alpha, dl[m], lam[m]);
      });
      nu = fmaT(alpha, dnu, nu);
      s = fmaT(alpha, ds, s);
    }
    if (phase == kIpm) ++it;
  }

  if (converged && !certified && inrange && !nonfin) flags |= kPxInexact;
  if (certified) {
    bool deg = false;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (vm[m]) deg |= ((freem >> m) & 1u) ? (a[m] < prm.deg_tol) : (lam[m] < prm.deg_tol);
    });
    if (slo) deg |= sfree ? (s < prm.deg_tol) : (nu < prm.deg_tol);
    if (bor_i((int)deg)) flags |= kPxDegenerate;
  }
  double sgm = 1.0;
  if (inrange && prm.sigma) sgm = (double)prm.sigma[p];
  if (!(sgm > 0.0) || !fin(sgm)) flags |= kPxBadSigma;
  const double qnan = __builtin_nan("");
  if (inrange) {
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (vm[m]) {
        const int64_t o = p * n + el(m);
        prm.out_a[o] = nonfin ? qnan : a[m];
        if (prm.dcov) {
          double dv;
          if (nonfin) dv = qnan;
          else if (certified) dv = ((freem >> m) & 1u) ? 0.0 : (double)INFINITY;
          else dv = lam[m] / a[m];
          prm.dcov[o] = dv;
        }
      }
    });
    if (prm.dcorner && x == 0 && z == 0) {
      // corner of the bordered matrix of the covariance: 0 on a binding sum
      // row, -s/nu for the slack pair of an uncertified iterate, -inf when
      // there is no sum row
      double cr;
      if (certified) cr = sfree ? -(double)INFINITY : 0.0;
      else cr = pos ? -(double)INFINITY : (slo ? -s / nu : 0.0);
      prm.dcorner[p] = cr;
    }
  }
  if (prm.objective) {
    tl.to_x(a, xl);
    tl.gmul(xl, g);
    double ba = 0.0, aga = 0.0;
    static_for<0, C>([&](auto mm) {
      ba = fmaT(bh[mm], a[mm], ba);
      aga = fmaT(a[mm], g[mm], aga);
    });
    ba = bsum(ba);
    aga = bsum(aga);
    if (inrange && x == 0 && z == 0) {
      double F = (prm.c[p] - 2.0 * prm.gamma * ba + prm.gamma * aga) / (sgm * sgm);
      if (nonfin || (flags & kPxBadSigma)) F = qnan;
      prm.objective[p] = F;
    }
  }
  if (inrange && x == 0 && z == 0) {
    if (prm.status) prm.status[p] = (uint8_t)flags;
    if (prm.iters) prm.iters[p] = it;
  }
}

// waves per SIMD the register budget is sized for: two up to T = 9; beyond,
// the tiles alone need more than half of the 512 registers of a lane
template <int T>
constexpr int kTileWaves = T <= 9 ? 2 : 1;

template <int T, int MODE, int CONS, bool ST>
__global__ __launch_bounds__(256, kTileWaves<T>) void ipm_tile_kernel(IpmParams prm) {
  ipm_tile_body<T, MODE, CONS, ST>(prm, blockIdx.x);
}

// Several cubes in one launch (one job per cube, blocks assigned by start).
template <int T, int MODE, int CONS, bool ST>
__global__ __launch_bounds__(256, kTileWaves<T>) void ipm_tile_batch_kernel(const IpmParams* __restrict__ jobs,
                                                                             const int64_t* __restrict__ start,
                                                                             int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const IpmParams prm = uniform_copy(jobs + j);
  ipm_tile_body<T, MODE, CONS, ST>(prm, (int64_t)blockIdx.x - start[j]);
}

template <int T, int MODE, int CONS, bool ST>
static void launch_tile_m(const IpmParams& p, const IpmBatch* b, hipStream_t st) {
  if (b)
    hipLaunchKernelGGL((ipm_tile_batch_kernel<T, MODE, CONS, ST>), dim3((unsigned)b->blocks), dim3(256), 0, st,
                       b->jobs, b->start, b->njobs);
  else
    hipLaunchKernelGGL((ipm_tile_kernel<T, MODE, CONS, ST>), dim3((unsigned)((p.P + 15) / 16)), dim3(256), 0, st, p);
}

template <int T, int CONS, bool ST>
static int launch_tile_c(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  if (mode == kFull)
    launch_tile_m<T, kFull, CONS, ST>(p, b, st);
  else if (mode == kStage2)
    launch_tile_m<T, kStage2, CONS, ST>(p, b, st);
  else
    return -5;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int T, bool ST>
static int launch_tile_s(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  switch (p.constraint) {
    case kSto: return launch_tile_c<T, kSto, ST>(p, b, mode, st);
    case kSlo: return launch_tile_c<T, kSlo, ST>(p, b, mode, st);
    case kPos: return launch_tile_c<T, kPos, ST>(p, b, mode, st);
  }
  return -1;
}

// b == nullptr: one cube described by p; else the jobs of b (p only gives
// the constraint option and the factorisation, shared by every job).  The
// explicit-inverse factorisation is built up to T = 9 only, for libraries
// whose scaled Gram matrix is well conditioned.
template <int T>
static int launch_tile(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  if constexpr (T <= 9) {
    if (!p.stable) return launch_tile_s<T, false>(p, b, mode, st);
  }
  return launch_tile_s<T, true>(p, b, mode, st);
}

#if defined(LM_TILE_T)
#define LM_TENTRY2(t) ipm_tile_entry_##t
#define LM_TENTRY(t) LM_TENTRY2(t)
int LM_TENTRY(LM_TILE_T)(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  return launch_tile<LM_TILE_T>(p, b, mode, st);
}
#endif

}  // namespace lm
