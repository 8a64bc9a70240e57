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
#include "ipm_body.h"

namespace lm {

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

template <int T, bool ST>
struct Tile {
  using real = double;
  using xreg = double;
  static constexpr bool kCompact = false;
  static constexpr bool kRecomputeGrad = false;
  static constexpr int NP = 4 * T;
  static constexpr int C = (T + 3) / 4;  // compact slots
  static constexpr int NX = T;           // solve registers: one per tile row
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
  int nvalid;               // library size n

  // compact layout: lane (x, z) holds element 16m + 4z + x of slot m
  __device__ __forceinline__ int el(int m) const { return 16 * m + 4 * z + x; }
  __device__ __forceinline__ bool xvalid(int I) const { return 4 * I + x < nvalid; }
  __device__ __forceinline__ int rhs() const { return z; }
  __device__ __forceinline__ bool writer() const { return x == 0 && z == 0; }

  static __device__ __forceinline__ double sum(double v) { return bsum(v); }
  static __device__ __forceinline__ double vmin(double v) { return bmin(v); }
  static __device__ __forceinline__ double vmax(double v) { return bmax(v); }
  static __device__ __forceinline__ int imin(int v) { return bmin_i(v); }
  static __device__ __forceinline__ int ior(int v) { return bor_i(v); }

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
  // exchange the tile through LDS and factor it redundantly (ldl4_lds).
  __device__ __forceinline__ void ldl4(double h, bool& bad, double& li, double& rx) const {
    xch[z * 4 + x] = h;
    lds_sync();
    ldl4_lds(xch, x, z, bad, li, rx);
  }

  // tiled right-looking L D L^T of H
  __device__ __forceinline__ void factor_st() {
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
  __device__ __forceinline__ void solve_st(double (&xr)[T]) const {
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

  __device__ __forceinline__ void factor() {
    if constexpr (ST) factor_st(); else factor_inv();
  }
  __device__ __forceinline__ void solve(double (&xr)[T]) const {
    if constexpr (ST) solve_st(xr); else solve_inv(xr);
  }
};

// One workgroup's 16 pixels: workgroup wg of the cube described by prm.
// ST: the stable factorisation (factor_st/solve_st) rather than explicit
// inverses of the diagonal blocks (factor_inv/solve_inv).
template <int T, int MODE, int CONS, bool ST>
__device__ __forceinline__ void ipm_tile_body(const IpmParams& prm, int64_t wg) {
  using TL = Tile<T, ST>;
  constexpr int NP = TL::NP;
  __shared__ double sG[NP * NP];
  __shared__ double sx[16 * 18];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = (lane >> 2) & 3, x = lane >> 4, z = lane & 3;
  const int pib = wave * 4 + blk;
  const int64_t p = wg * 16 + pib;
  if constexpr (MODE == kRetry) {
    // most workgroups hold no pixel to solve again
    if (!__syncthreads_or(p < prm.P && (prm.status[p] & kPxRetry) != 0)) return;
  }
  const double* Gsrc = static_cast<const double*>(prm.Gh);
  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) sG[i] = Gsrc[i];
  __syncthreads();

  TL tl;
  tl.x = x;
  tl.z = z;
  tl.blk = blk;
  tl.sG = sG;
  tl.xch = sx + pib * 18;
  tl.nvalid = prm.n;
  ipm_pixel<TL, MODE, CONS>(prm, p, p < prm.P, tl);
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
  else if (mode == kRetry)
    launch_tile_m<T, kRetry, CONS, ST>(p, b, st);
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
