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
// so the Cholesky trailing update H_IJ -= L_IK L_JK^T is one MFMA on the
// stored tiles with no data movement, and the panel is L_IK = H_IK W^T with
// W = inverse of the 4x4 diagonal factor.  Vectors that feed the MFMA use the
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

// sum over the 16 lanes of a block (same bits on every lane)
__device__ __forceinline__ double bsum(double v) {
  v += dpp<qp(1, 0, 3, 2)>(v);
  v += dpp<qp(2, 3, 0, 1)>(v);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
__device__ __forceinline__ double bmin(double v) {
  v = fmin(v, dpp<qp(1, 0, 3, 2)>(v));
  v = fmin(v, dpp<qp(2, 3, 0, 1)>(v));
  v = fmin(v, __shfl_xor(v, 16));
  v = fmin(v, __shfl_xor(v, 32));
  return v;
}
__device__ __forceinline__ double bmax(double v) {
  v = fmax(v, dpp<qp(1, 0, 3, 2)>(v));
  v = fmax(v, dpp<qp(2, 3, 0, 1)>(v));
  v = fmax(v, __shfl_xor(v, 16));
  v = fmax(v, __shfl_xor(v, 32));
  return v;
}
__device__ __forceinline__ int bmin_i(int v) {
  v = min(v, dpp<qp(1, 0, 3, 2)>(v));
  v = min(v, dpp<qp(2, 3, 0, 1)>(v));
  v = min(v, __shfl_xor(v, 16));
  v = min(v, __shfl_xor(v, 32));
  return v;
}
__device__ __forceinline__ int bor_i(int v) {
  v |= dpp<qp(1, 0, 3, 2)>(v);
  v |= dpp<qp(2, 3, 0, 1)>(v);
  v |= __shfl_xor(v, 16);
  v |= __shfl_xor(v, 32);
  return v;
}

template <typename T>
__device__ __forceinline__ bool fin(T v) {
  return v == v && v - v == T(0);
}

template <int T>
struct Tile {
  static constexpr int NP = 4 * T;
  static constexpr int C = (T + 3) / 4;  // compact slots
  static constexpr int NT = T * (T + 1) / 2;
  static constexpr int id(int I, int J) { return I * (I + 1) / 2 + J; }

  int x, z, blk;            // lane coordinates
  const double* sG;         // LDS, NP x NP scaled Gram
  double* xch;              // LDS, 32 doubles of this pixel
  double H[NT];             // stored tiles (lower), then the Cholesky factor
  double W[T], WT[T];       // inverse diagonal factors, stored and transposed
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

  // xg = Gh * xa (x layout in and out)
  __device__ __forceinline__ void gmul(const double (&xa)[T], double (&xg)[T]) const {
    static_for<0, T>([&](auto ii) {
      constexpr int I = decltype(ii)::value;
      double acc = 0.0;
      static_for<0, T>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        acc = mfma4(sG[(4 * I + z) * NP + 4 * J + x], xa[J], acc);
      });
      xg[I] = acc;
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

  // tiled right-looking Cholesky H = L L^T
  __device__ __forceinline__ void factor() {
    notpd = false;
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      // 4x4 diagonal factor, computed redundantly on every lane of the block
      xch[z * 4 + x] = H[id(K, K)];
      lds_sync();
      double m[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) m[q] = xch[q];
      bool bad = false;
      double l[4][4], w[4][4], r[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) l[i][j] = 0.0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double d = m[j * 4 + j];
#pragma unroll
        for (int q = 0; q < j; ++q) d = fmaT(-l[j][q], l[j][q], d);
        if (!(d > 0.0) || !fin(d)) {
          bad = true;
          d = 1.0;
        }
        // 1/sqrt(d): hardware estimate refined by two Newton steps
        double y = __builtin_amdgcn_rsq(d);
        y = y * fmaT(-0.5 * d, y * y, 1.5);
        y = y * fmaT(-0.5 * d, y * y, 1.5);
        l[j][j] = d * y;
        r[j] = y;
#pragma unroll
        for (int i = j + 1; i < 4; ++i) {
          double v = m[i * 4 + j];
#pragma unroll
          for (int q = 0; q < j; ++q) v = fmaT(-l[i][q], l[j][q], v);
          l[i][j] = v * r[j];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) w[i][j] = 0.0;
        w[i][i] = r[i];
#pragma unroll
        for (int j = 0; j < i; ++j) {
          double v = 0.0;
#pragma unroll
          for (int q = j; q < i; ++q) v = fmaT(l[i][q], w[q][j], v);
          w[i][j] = -v * r[i];
        }
      }
      notpd |= bad;
      if (x == 0 && z == 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) xch[16 + q] = w[q / 4][q % 4];
      }
      lds_sync();
      W[K] = xch[16 + z * 4 + x];
      WT[K] = xch[16 + x * 4 + z];
      // panel L_IK = H_IK W^T
      static_for<K + 1, T>([&](auto ii) {
        constexpr int I = decltype(ii)::value;
        H[id(I, K)] = mfma4(W[K], H[id(I, K)], 0.0);
      });
      // trailing update H_IJ -= L_IK L_JK^T
      static_for<K + 1, T>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        const double nl = -H[id(J, K)];
        static_for<J, T>([&](auto ii) {
          constexpr int I = decltype(ii)::value;
          H[id(I, J)] = mfma4(nl, H[id(I, K)], H[id(I, J)]);
        });
      });
    });
  }

  // solve L L^T X = R in place (x layout, one right-hand side per z)
  __device__ __forceinline__ void solve(double (&xr)[T]) const {
    static_for<0, T>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      const double y = mfma4(W[J], xr[J], 0.0);
      xr[J] = y;
      const double ny = -y;
      static_for<J + 1, T>([&](auto ii) {
        constexpr int I = decltype(ii)::value;
        xr[I] = mfma4(H[id(I, J)], ny, xr[I]);
      });
    });
    const int src = 16 * z + 4 * blk + x;  // transpose partner (x,z) <-> (z,x)
    static_for<0, T>([&](auto kk) {
      constexpr int I = T - 1 - decltype(kk)::value;
      const double xv = mfma4(WT[I], xr[I], 0.0);
      xr[I] = xv;
      const double nx = -xv;
      static_for<0, I>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        const double lt = __shfl(H[id(I, J)], src);
        xr[J] = mfma4(lt, nx, xr[J]);
      });
    });
  }
};

template <int T, int MODE>
__global__ __launch_bounds__(256, 2) void ipm_tile_kernel(IpmParams prm) {
  using TL = Tile<T>;
  constexpr int NP = TL::NP;
  constexpr int C = TL::C;
  __shared__ double sG[NP * NP];
  __shared__ double sx[16 * 32];
  const double* Gsrc = static_cast<const double*>(prm.Gh);
  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) sG[i] = Gsrc[i];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int blk = (lane >> 2) & 3, x = lane >> 4, z = lane & 3;
  const int pib = wave * 4 + blk;
  const int64_t p = (int64_t)blockIdx.x * 16 + pib;
  const bool inrange = p < prm.P;
  const int n = prm.n;

  TL tl;
  tl.x = x;
  tl.z = z;
  tl.blk = blk;
  tl.sG = sG;
  tl.xch = sx + pib * 32;

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

  double a[C], lam[C], nu = 0.0;
  int it = 0;
  bool start = inrange && !nonfin;
  if constexpr (MODE == kStage2) {
    if (inrange) {
      const uint8_t f = prm.st_flag[p];
      flags |= f & 0x7fu;
      start = start && (f & 0x80u);
      it = prm.st_it[p];
      nu = prm.st_nu[p];
    }
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const bool ok = inrange && vm[m];
      a[m] = ok ? prm.st_a[p * n + el(m)] : 0.0;
      lam[m] = ok ? prm.st_lam[p * n + el(m)] : 0.0;
    });
  } else {
    static_for<0, C>([&](auto mm) {
      a[mm] = vm[mm] ? 1.0 / n : 0.0;
      lam[mm] = vm[mm] ? prm.lambda0 : 0.0;
    });
  }
  const double tol_mu = prm.tol_mu, tol_d = prm.tol_d, tol_p = prm.tol_p, eta = prm.eta, tau = prm.tau;
  constexpr double BIG = 1e30;

  enum { kIpm = 0, kPol = 1, kDone = 2 };
  int phase = start ? kIpm : kDone;
  bool converged = false, certified = false, cand = false;
  uint32_t freem = 0;  // bit m: compact slot m is free
  int kp = 0;
  double pa[C], pnu = 0.0;

  double g[C], rd[C], D[C], dx[C], u[C], dla[C];
  double rp = 0.0, mu = 0.0;
  double xl[T], xg[T];
  for (;;) {
    // ---- Gram products and phase decisions --------------------------------
    {
      double v[C];
      static_for<0, C>([&](auto mm) { v[mm] = (phase == kPol) ? pa[mm] : a[mm]; });
      tl.to_x(v, xl);
      tl.gmul(xl, xg);
      tl.template from_x<0>(xg, g);
    }
    if (phase == kIpm) {
      double sa = 0.0, sal = 0.0, rdm = 0.0;
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        rd[m] = vm[m] ? (g[m] - bh[m] - lam[m] + nu) : 0.0;
        sa += a[m];
        sal = fmaT(a[m], lam[m], sal);
        rdm = fmax(rdm, fabs(rd[m]));
      });
      rp = bsum(sa) - 1.0;
      mu = bsum(sal) / n;
      rdm = bmax(rdm);
      bool conv;
      if constexpr (MODE == kStage1)
        conv = mu <= fmax(tol_mu, prm.mu_switch);
      else
        conv = mu <= tol_mu && rdm <= tol_d * (1.0 + bhmax) && fabs(rp) <= tol_p;
      if (conv) {
        converged = true;
        phase = kPol;
        cand = false;
        static_for<0, C>([&](auto mm) {
          if (vm[mm] && a[mm] > lam[mm]) freem |= 1u << mm;
        });
      } else if (it >= prm.maxit) {
        flags |= kPxMaxit;
        phase = kDone;
      }
    } else if (phase == kPol && cand) {
      double wa = INFINITY, wl = INFINITY, pl[C];
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        const bool fr = (freem >> m) & 1u;
        pl[m] = (vm[m] && !fr) ? g[m] - bh[m] + pnu : 0.0;
        if (vm[m] && fr) wa = fmin(wa, pa[m]);
        if (vm[m] && !fr) wl = fmin(wl, pl[m]);
      });
      wa = bmin(wa);
      wl = bmin(wl);
      if (wa >= -tau && wl >= -tau) {
        certified = true;
        phase = kDone;
        static_for<0, C>([&](auto mm) {
          a[mm] = pa[mm];
          lam[mm] = pl[mm];
        });
        nu = pnu;
      } else if (kp >= prm.max_polish) {
        phase = kDone;
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
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const double dp = ((freem >> m) & 1u) ? 0.0 : BIG;
      const double di = (phase == kPol) ? dp : ((phase == kIpm) ? lam[m] / a[m] : 1.0);
      D[m] = vm[m] ? di : 0.0;
    });
    tl.to_x(D, xl);
    tl.form(xl);
    tl.factor();
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
    tl.solve(xl);
    tl.template from_x<0>(xl, dx);
    tl.template from_x<1>(xl, u);
    double su = 0.0, sw = 0.0;
    static_for<0, C>([&](auto mm) {
      su += u[mm];
      sw += dx[mm];
    });
    su = bsum(su);
    sw = bsum(sw);
    if (phase == kPol) {
      // equality-constrained problem on the free set: a = w - nu u, 1^T a = 1
      pnu = (sw - 1.0) / su;
      static_for<0, C>([&](auto mm) {
        pa[mm] = (vm[mm] && ((freem >> mm) & 1u)) ? fmaT(-pnu, u[mm], dx[mm]) : 0.0;
      });
      cand = fin(pnu);
      if (!cand) phase = kDone;
    }
    const bool two = __builtin_amdgcn_ballot_w64(phase == kIpm) != 0;
    if (!two) continue;

    // ---- predictor step and centring --------------------------------------
    const double dnu_aff = (sw + rp) / su;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      dx[m] = vm[m] ? fmaT(-dnu_aff, u[m], dx[m]) : 0.0;
      dla[m] = vm[m] ? -lam[m] - D[m] * dx[m] : 0.0;
    });
    double st_aff = INFINITY;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (vm[m] && dx[m] < 0.0) st_aff = fmin(st_aff, -a[m] / dx[m]);
      if (vm[m] && dla[m] < 0.0) st_aff = fmin(st_aff, -lam[m] / dla[m]);
    });
    st_aff = fmin(bmin(st_aff), 1.0);
    double smu = 0.0;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (vm[m]) smu = fmaT(a[m] + st_aff * dx[m], lam[m] + st_aff * dla[m], smu);
    });
    const double ratio = (bsum(smu) / n) / mu;
    const double sig = ratio * ratio * ratio;

    // ---- corrector (second-order term dropped after a short affine step) ---
    const double soc = st_aff >= 0.1 ? 1.0 : 0.0;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const double rcv = fmaT(soc * dx[m], dla[m], a[m] * lam[m]) - sig * mu;
      dla[m] = vm[m] ? rcv / a[m] : 0.0;  // rc / a
      dx[m] = vm[m] ? -rd[m] - dla[m] : 0.0;
    });
    tl.to_x(dx, xl);
    tl.solve(xl);
    tl.template from_x<0>(xl, dx);
    double sw2 = 0.0;
    static_for<0, C>([&](auto mm) { sw2 += dx[mm]; });
    sw2 = bsum(sw2);
    const double dnu = (sw2 + rp) / su;
    double dl[C];
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      dx[m] = vm[m] ? fmaT(-dnu, u[m], dx[m]) : 0.0;
      dl[m] = vm[m] ? -dla[m] - D[m] * dx[m] : 0.0;
    });
    double step = INFINITY;
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (vm[m] && dx[m] < 0.0) step = fmin(step, -a[m] / dx[m]);
      if (vm[m] && dl[m] < 0.0) step = fmin(step, -lam[m] / dl[m]);
    });
    step = bmin(step);
    const double alpha = fmin(1.0, eta * step);
    if (phase == kIpm && fin(alpha)) {
      static_for<0, C>([&](auto mm) {
        a[mm] = fmaT(alpha, dx[mm], a[mm]);
        lam[mm] = fmaT(alpha, dl[mm], lam[mm]);
      });
      nu = fmaT(alpha, dnu, nu);
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
  }
  if (prm.objective) {
    tl.to_x(a, xl);
    tl.gmul(xl, xg);
    tl.template from_x<0>(xg, g);
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

template <int T>
static int launch_tile(const IpmParams& p, int mode, hipStream_t st) {
  const int64_t blocks = (p.P + 15) / 16;
  const dim3 grid((unsigned)blocks), block(256);
  if (mode == kFull)
    hipLaunchKernelGGL((ipm_tile_kernel<T, kFull>), grid, block, 0, st, p);
  else if (mode == kStage2)
    hipLaunchKernelGGL((ipm_tile_kernel<T, kStage2>), grid, block, 0, st, p);
  else
    return -5;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

#if defined(LM_TILE_T)
#define LM_TENTRY2(t) ipm_tile_entry_##t
#define LM_TENTRY(t) LM_TENTRY2(t)
int LM_TENTRY(LM_TILE_T)(const IpmParams& p, int mode, hipStream_t st) { return launch_tile<LM_TILE_T>(p, mode, st); }
#endif

}  // namespace lm
