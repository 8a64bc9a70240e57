// ipm_body.h -- the per-pixel interior-point solve of IPLS (Sec. 2.2) on
// the scaled problem of eq. 6 under eqs. 3-4, shared by the matrix-core
// kernels of lib_linmin.  The Newton matrix lives in a layout policy TL
// (which lanes hold which tiles and vector elements); this file holds the
// method: Mehrotra predictor-corrector steps, the stopping tests, the
// finishing step that certifies the free set, and the per-pixel outputs
// (or, for the first stage of the mixed form, the hand-over state).
//
// A policy TL provides
//   real                arithmetic type of the solve (double, or float for
//                       the first stage of the mixed form)
//   C                   elementwise slots per lane
//   el(m)               element held by slot m on this lane (may be >= n)
//   writer()            the one lane of the pixel that writes its scalars
//   kCompact            true: the policy works on elementwise slots directly
//                       (gvec, form_factor, solve2, solve1 below); false: it
//                       works on solve registers ("x layout", NX registers of
//                       type xreg) and provides
//     xvalid(I), rhs()  element validity of solve register I; this lane's
//                       right-hand-side column (a solve carries up to four)
//     to_x, from_x<R>   elementwise slots <-> solve registers (every column /
//                       column R)
//     gmul(xl, v)       v = Gh * xl
//     form(xD), factor(), solve(xl)
//                       H = Gh + diag(D); L D L^T of H; H^{-1} on the
//                       columns of xl
//   notpd               the last factorisation failed
//   kRecomputeGrad      form Gh a explicitly at every step instead of
//                       carrying it through the Newton identity
//   sum, vmin, vmax, imin, ior
//                       reductions over the pixel's elements with the same
//                       bits on every lane of the pixel
#pragma once
#include "common.h"
#include "kernels.h"

namespace lm {

// Reciprocal to about single precision squared (one Newton step), for
// step-to-boundary ratios, which only need a few digits.
__device__ __forceinline__ double rcp1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return y * fmaT(-x, y, 2.0);
}
__device__ __forceinline__ float rcp1(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ __forceinline__ bool fin(T v) {
  return isfin(v);
}

__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// quad broadcast: lane (x, z) <- lane (x, R) of the same block
template <int R>
__device__ __forceinline__ double qb(double v) {
  return dpp<qp(R, R, R, R)>(v);
}

// L diag(d) L^T (unit lower L, no square roots) of the symmetric 4x4 tile M
// held row-major at xch (16 doubles in LDS, M[i][j] at xch[4 i + j]), on
// every lane that calls it.  Lane (x, z) returns entry (z, x) of L^{-1} (1 on
// the diagonal, 0 above it) in li and 1 / d_x in rx; bad is set when a pivot
// is not positive and finite.
__device__ __forceinline__ void ldl4_lds(const double* xch, int x, int z, bool& bad, double& li, double& rx) {
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

// The operations of the method on elementwise slots, for either kind of
// policy (see the top of this file).
template <typename TL, typename V>
__device__ __forceinline__ void tl_gvec(const TL& tl, const V& v, V& out) {
  if constexpr (TL::kCompact) {
    tl.gvec(v, out);
  } else {
    typename TL::xreg xl[TL::NX];
    tl.to_x(v, xl);
    tl.gmul(xl, out);
  }
}
template <typename TL, typename V>
__device__ __forceinline__ void tl_form_factor(TL& tl, const V& D) {
  if constexpr (TL::kCompact) {
    tl.form_factor(D);
  } else {
    typename TL::xreg xl[TL::NX];
    tl.to_x(D, xl);
    tl.form(xl);
    tl.factor();
  }
}
// w = H^{-1} r and u = H^{-1} 1 (over the valid elements)
template <typename TL, typename V>
__device__ __forceinline__ void tl_solve2(const TL& tl, const V& r, V& w, V& u) {
  if constexpr (TL::kCompact) {
    tl.solve2(r, w, u);
  } else {
    constexpr int NX = TL::NX;
    using X = typename TL::xreg;
    X xl[NX];
    tl.to_x(r, xl);
    static_for<0, NX>([&](auto ii) {
      constexpr int I = decltype(ii)::value;
      const X one = tl.xvalid(I) ? X(1) : X(0);
      xl[I] = (tl.rhs() == 1) ? one : xl[I];
    });
    tl.solve(xl);
    tl.template from_x<0>(xl, w);
    tl.template from_x<1>(xl, u);
  }
}
// w = H^{-1} r
template <typename TL, typename V>
__device__ __forceinline__ void tl_solve1(const TL& tl, const V& r, V& w) {
  if constexpr (TL::kCompact) {
    tl.solve1(r, w);
  } else {
    typename TL::xreg xl[TL::NX];
    tl.to_x(r, xl);
    tl.solve(xl);
    tl.template from_x<0>(xl, w);
  }
}

// Pixel p of the launch described by prm (inrange: p < P; the lanes of an
// out-of-range pixel still take part in the wavefront's matrix-core
// instructions).  CONS: constraint option; MODE: full solve, or a stage of
// the mixed form.
template <typename TL, int MODE, int CONS>
__device__ __forceinline__ void ipm_pixel(const IpmParams& prm, int64_t p, bool inrange, TL& tl) {
  constexpr int C = TL::C;
  using R = typename TL::real;
  const int n = prm.n;
  bool vm[C];
  static_for<0, C>([&](auto mm) { vm[mm] = tl.el(mm) < n; });
  auto el = [&](int m) { return tl.el(m); };

  uint32_t flags = 0;
  // the pass that solves again in FP64 what the mixed form left uncertified
  // touches only those pixels
  bool redo = true;
  if constexpr (MODE == kRetry) redo = inrange && (prm.status[p] & kPxRetry) != 0;
  R bh[C];
  bool nonfin = false;
  static_for<0, C>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    const double v = (inrange && vm[m]) ? prm.bh[p * n + el(m)] : 0.0;
    if (!fin(v)) nonfin = true;
    bh[m] = (R)v;
  });
  if (inrange && prm.c && !fin(prm.c[p])) nonfin = true;
  nonfin = TL::ior((int)nonfin) != 0;
  if (nonfin) {
    flags |= kPxNonfinite;
    static_for<0, C>([&](auto mm) { bh[mm] = R(0); });
  }
  R bhmax = R(0);
  static_for<0, C>([&](auto mm) { bhmax = fmax(bhmax, fabs(bh[mm])); });
  bhmax = TL::vmax(bhmax);

  // constraint besides a >= 0: sum-to-one, sum-lower-than-one (slack s of
  // 1^T a <= 1 with multiplier nu: one more complementarity pair), or
  // positivity only (no sum row, nu = 0)
  constexpr bool slo = CONS == kSlo, pos = CONS == kPos;
  const R inv_np = R(1) / R(n + (slo ? 1 : 0));  // complementarity pairs
  R a[C], lam[C], nu = slo ? (R)prm.lambda0 : R(0), s = slo ? inv_np : R(0);
  int it = 0;
  bool start = inrange && !nonfin && redo;
  if constexpr (MODE == kStage2) {
    if (inrange) {
      const uint8_t f = prm.st_flag[p];
      flags |= f & 0x7fu;
      start = start && (f & 0x80u);
      it = prm.st_it[p];
      nu = (R)prm.st_nu[p];
      s = slo ? (R)prm.st_s[p] : R(0);
    }
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const bool ok = inrange && vm[m];
      a[m] = ok ? (R)prm.st_a[p * n + el(m)] : R(0);
      lam[m] = ok ? (R)prm.st_lam[p * n + el(m)] : R(0);
    });
  } else {
    static_for<0, C>([&](auto mm) {
      a[mm] = vm[mm] ? inv_np : R(0);
      lam[mm] = vm[mm] ? (R)prm.lambda0 : R(0);
    });
  }
  const R tol_mu = (R)prm.tol_mu, tol_d = (R)prm.tol_d, tol_p = (R)prm.tol_p, eta = (R)prm.eta, tau = (R)prm.tau;
  const R mu_stage1 = (R)fmax(prm.tol_mu, prm.mu_switch);
  constexpr R BIG = R(1e30);

  enum { kIpm = 0, kPol = 1, kDone = 2 };
  constexpr bool kPolish = MODE != kStage1;  // the first stage of the mixed form stops before the finishing step
  int phase = start ? kIpm : kDone;
  bool converged = false, certified = false, cand = false;
  bool sfree = pos;  // finishing step: the sum row is absent (slack free or no sum constraint)
  uint32_t freem = 0;  // bit m: compact slot m is free
  int kp = 0;
  bool stalled = false;  // first stage of the mixed form: the last step was too short
  R pa[C], pnu = R(0);

  R g[C], rd[C], D[C], dx[C], u[C], dla[C];
  R rp = R(0), mu = R(0);
  // gradient of the quadratic at the starting point
  tl_gvec(tl, a, g);
  for (;;) {
    // Gh is re-read from LDS each step rather than held in registers across
    // iterations (it would not fit next to the factor).
    asm volatile("" ::: "memory");
    // ---- phase decisions ---------------------------------------------------
    // g = Gh a is carried from step to step (see the update below), or
    // formed anew at every step (TL::kRecomputeGrad).  Where dependent
    // spectra make the Newton matrix nearly singular, the carried g drifts
    // from Gh a, so a pixel whose residuals pass the stopping tests confirms
    // them with an explicit product before it stops; the finishing step's
    // candidate gets its own product as well.
    if constexpr (TL::kRecomputeGrad) {
      if (__builtin_amdgcn_ballot_w64(phase == kIpm) != 0) tl_gvec(tl, a, g);
    }
    auto residuals = [&](R& rdm) {
      R sa = R(0), sal = R(0);
      rdm = R(0);
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        rd[m] = vm[m] ? (g[m] - bh[m] - lam[m] + nu) : R(0);
        sa += a[m];
        sal = fmaT(a[m], lam[m], sal);
        rdm = fmax(rdm, fabs(rd[m]));
      });
      rp = pos ? R(0) : TL::sum(sa) + s - R(1);
      mu = (TL::sum(sal) + s * nu) * inv_np;
      rdm = TL::vmax(rdm);
    };
    auto stops = [&](R rdm) {
      if constexpr (MODE == kStage1)
        return mu <= mu_stage1 || stalled || it >= kStage1MaxIt;
      else
        return mu <= tol_mu && rdm <= tol_d * (R(1) + bhmax) && fabs(rp) <= tol_p;
    };
    R rdm = R(0);
    bool conv = false;
    if (phase == kIpm) {
      residuals(rdm);
      conv = stops(rdm);
    }
    const bool confirm = MODE != kStage1 && !TL::kRecomputeGrad && phase == kIpm && conv;
    R gp[C];
    if (__builtin_amdgcn_ballot_w64(confirm || ((kPolish && phase == kPol) && cand)) != 0) {
      R v[C];
      static_for<0, C>([&](auto mm) { v[mm] = confirm ? a[mm] : pa[mm]; });
      tl_gvec(tl, v, gp);
    }
    if (confirm) {
      static_for<0, C>([&](auto mm) { g[mm] = gp[mm]; });
      residuals(rdm);
      conv = stops(rdm);
    }
    if (phase == kIpm) {
      if (conv && MODE == kStage1) {
        converged = true;
        phase = kDone;
      } else if (conv) {
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
    } else if ((kPolish && phase == kPol) && cand) {
      R wa = R(INFINITY), wl = R(INFINITY), pl[C];
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        const bool fr = (freem >> m) & 1u;
        pl[m] = (vm[m] && !fr) ? gp[m] - bh[m] + pnu : R(0);
        if (vm[m] && fr) wa = fmin(wa, pa[m]);
        if (vm[m] && !fr) wl = fmin(wl, pl[m]);
      });
      wa = TL::vmin(wa);
      wl = TL::vmin(wl);
      // sum-lower-than-one: the slack is one more index (free: its value
      // 1 - 1^T a must be >= 0; at its bound: the multiplier nu must be)
      R spa = R(0);
      static_for<0, C>([&](auto mm) { spa += pa[mm]; });
      const R sv = R(1) - TL::sum(spa);
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
        s = (slo && sfree) ? sv : R(0);
      } else if (kp >= prm.max_polish) {
        phase = kDone;
      } else if ((wa < -tau && wa <= wl) ? slA : slL) {
        sfree = !sfree;
        ++kp;
        cand = false;
      } else {
        const bool flipA = (wa < -tau) && (wa <= wl);
        const R target = flipA ? wa : wl;
        int idx = 1 << 30;
        static_for<0, C>([&](auto mm) {
          constexpr int m = decltype(mm)::value;
          const bool fr = (freem >> m) & 1u;
          const bool c = flipA ? (vm[m] && fr && pa[m] == target) : (vm[m] && !fr && pl[m] == target);
          if (c) idx = min(idx, el(m));
        });
        idx = TL::imin(idx);
        static_for<0, C>([&](auto mm) {
          if (el(mm) == idx) freem ^= 1u << mm;
        });
        ++kp;
        cand = false;
      }
    }
    if (__builtin_amdgcn_ballot_w64(phase != kDone) == 0) break;

    // ---- Newton (or finishing-step) matrix and its factorisation ----------
    R ia[C];  // 1 / a
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      ia[m] = rcpT(a[m]);
      const R dp = ((freem >> m) & 1u) ? R(0) : BIG;
      const R di = ((kPolish && phase == kPol)) ? dp : ((phase == kIpm) ? lam[m] * ia[m] : R(1));
      D[m] = vm[m] ? di : R(0);
    });
    tl_form_factor(tl, D);
    if (phase != kDone && tl.notpd) {
      if (phase == kIpm) flags |= kPxNotPd;
      phase = kDone;
    }

    // ---- first solve: [rhs, 1] (predictor / finishing), u = H^{-1} 1 ------
    {
      R rc[C];
      static_for<0, C>([&](auto mm) {
        rc[mm] = ((kPolish && phase == kPol)) ? bh[mm] : (vm[mm] ? -rd[mm] - lam[mm] : R(0));
      });
      tl_solve2(tl, rc, dx, u);
    }
    R su = R(0), sw = R(0);
    static_for<0, C>([&](auto mm) {
      su += u[mm];
      sw += dx[mm];
    });
    su = TL::sum(su);
    sw = TL::sum(sw);
    const R isu = rcpT(su);
    if ((kPolish && phase == kPol)) {
      // equality-constrained problem on the free set: a = w - nu u, 1^T a = 1
      pnu = sfree ? R(0) : (sw - R(1)) * isu;
      static_for<0, C>([&](auto mm) {
        pa[mm] = (vm[mm] && ((freem >> mm) & 1u)) ? fmaT(-pnu, u[mm], dx[mm]) : R(0);
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
    const R son = slo ? s / nu : R(0);
    const R dnu_aff = pos ? R(0) : (slo ? (sw + rp - s) / (su + son) : (sw + rp) * isu);
    const R ds_aff = slo ? -s - son * dnu_aff : R(0);
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      dx[m] = vm[m] ? fmaT(-dnu_aff, u[m], dx[m]) : R(0);
      dla[m] = vm[m] ? -lam[m] - D[m] * dx[m] : R(0);
    });
    R st_aff = R(INFINITY);
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const R q1 = -a[m] * rcp1(dx[m]), q2 = -lam[m] * rcp1(dla[m]);
      st_aff = (vm[m] && dx[m] < R(0)) ? fmin(st_aff, q1) : st_aff;
      st_aff = (vm[m] && dla[m] < R(0)) ? fmin(st_aff, q2) : st_aff;
    });
    st_aff = fmin(TL::vmin(st_aff), R(1));
    if (slo) {
      if (ds_aff < R(0)) st_aff = fmin(st_aff, -s / ds_aff);
      if (dnu_aff < R(0)) st_aff = fmin(st_aff, -nu / dnu_aff);
    }
    R smu = R(0);
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (vm[m]) smu = fmaT(a[m] + st_aff * dx[m], lam[m] + st_aff * dla[m], smu);
    });
    const R smu_s = slo ? (s + st_aff * ds_aff) * (nu + st_aff * dnu_aff) : R(0);
    const R ratio = (TL::sum(smu) + smu_s) * inv_np * rcpT(mu);
    const R sig = ratio * ratio * ratio;

    // ---- corrector (second-order term dropped after a short affine step) ---
    const R soc = st_aff >= R(0.1) ? R(1) : R(0);
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const R rcv = fmaT(soc * dx[m], dla[m], a[m] * lam[m]) - sig * mu;
      dla[m] = vm[m] ? rcv * ia[m] : R(0);  // rc / a
      dx[m] = vm[m] ? -rd[m] - dla[m] : R(0);
    });
    {
      R rc2[C];
      static_for<0, C>([&](auto mm) { rc2[mm] = dx[mm]; });
      tl_solve1(tl, rc2, dx);
    }
    R sw2 = R(0);
    static_for<0, C>([&](auto mm) { sw2 += dx[mm]; });
    sw2 = TL::sum(sw2);
    const R rcs = slo ? fmaT(soc * ds_aff, dnu_aff, s * nu) - sig * mu : R(0);
    const R dnu = pos ? R(0) : (slo ? (sw2 + rp - rcs / nu) / (su + son) : (sw2 + rp) * isu);
    const R ds = slo ? (-rcs - s * dnu) / nu : R(0);
    R dl[C];
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      dx[m] = vm[m] ? fmaT(-dnu, u[m], dx[m]) : R(0);
      dl[m] = vm[m] ? -dla[m] - D[m] * dx[m] : R(0);
    });
    R step = R(INFINITY);
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const R q1 = -a[m] * rcp1(dx[m]), q2 = -lam[m] * rcp1(dl[m]);
      step = (vm[m] && dx[m] < R(0)) ? fmin(step, q1) : step;
      step = (vm[m] && dl[m] < R(0)) ? fmin(step, q2) : step;
    });
    step = TL::vmin(step);
    if (slo) {
      if (ds < R(0)) step = fmin(step, -s / ds);
      if (dnu < R(0)) step = fmin(step, -nu / dnu);
    }
    const R alpha = fmin(R(1), eta * step);
    if constexpr (MODE == kStage1) stalled = !(alpha >= R(kStage1MinStep));
    if (phase == kIpm && fin(alpha)) {
      // the Newton equations give Gh da = -r_d + dlambda - dnu 1 exactly, so
      // the gradient follows the step without another product with Gh
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        if constexpr (!TL::kRecomputeGrad) {
          const R rdm = g[m] - bh[m] - lam[m] + nu;  // r_d before the step
          g[m] = vm[m] ? fmaT(alpha, dl[m] - rdm - dnu, g[m]) : R(0);
        }
        a[m] = fmaT(alpha, dx[m], a[m]);
        lam[m] = fmaT(alpha, dl[m], lam[m]);
      });
      nu = fmaT(alpha, dnu, nu);
      s = fmaT(alpha, ds, s);
    }
    if (phase == kIpm) ++it;
  }

  if constexpr (MODE == kStage1) {
    // hand the iterate over to the FP64 stage; a loss of positive
    // definiteness in this precision is retried in FP64 from the last
    // accepted iterate
    if (inrange) {
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        if (vm[m]) {
          prm.st_a[p * n + el(m)] = (double)a[m];
          prm.st_lam[p * n + el(m)] = (double)lam[m];
        }
      });
      if (tl.writer()) {
        prm.st_nu[p] = (double)nu;
        if (slo) prm.st_s[p] = (double)s;
        prm.st_it[p] = it;
        prm.st_flag[p] = (uint8_t)((flags & ~(kPxMaxit | kPxNotPd)) | (nonfin ? 0u : 0x80u));
      }
    }
  } else {
    if (converged && !certified && inrange && !nonfin) flags |= kPxInexact;
    if (certified) {
      bool deg = false;
      static_for<0, C>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        if (vm[m]) deg |= ((freem >> m) & 1u) ? (a[m] < prm.deg_tol) : (lam[m] < prm.deg_tol);
      });
      if (slo) deg |= sfree ? (s < prm.deg_tol) : (nu < prm.deg_tol);
      if (TL::ior((int)deg)) flags |= kPxDegenerate;
    }
    double sgm = 1.0;
    if (inrange && prm.sigma) sgm = (double)prm.sigma[p];
    if (!(sgm > 0.0) || !fin(sgm)) flags |= kPxBadSigma;
    const double qnan = __builtin_nan("");
    const bool wout = inrange && redo;
    if (wout) {
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
      if (prm.dcorner && tl.writer()) {
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
      tl_gvec(tl, a, g);
      double ba = 0.0, aga = 0.0;
      static_for<0, C>([&](auto mm) {
        ba = fmaT(bh[mm], a[mm], ba);
        aga = fmaT(a[mm], g[mm], aga);
      });
      ba = TL::sum(ba);
      aga = TL::sum(aga);
      if (wout && tl.writer()) {
        double F = (prm.c[p] - 2.0 * prm.gamma * ba + prm.gamma * aga) / (sgm * sgm);
        if (nonfin || (flags & kPxBadSigma)) F = qnan;
        prm.objective[p] = F;
      }
    }
    if (wout && tl.writer()) {
      if (prm.status) prm.status[p] = (uint8_t)flags;
      if (prm.iters) prm.iters[p] = it;
    }
  }
}

}  // namespace lm
