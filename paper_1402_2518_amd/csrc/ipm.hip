// ipm.hip -- per-pixel primal-dual interior-point solve (IPLS, Sec. 2.2) of
//   min 1/2 a^T Gh a - bh^T a   s.t.  a >= 0 (eq. 3),  1^T a = 1 (eq. 4)
// on the renormalised problem of Sec. 2.3 (eq. 6), scaled by gamma = max G_ii,
// with a finishing step that certifies the optimal partition, and the
// quantities the covariance pass needs (end of Sec. 2.3).
//
// Mapping onto gfx950.  A pixel is owned by a group of G consecutive lanes
// (G = 1..16, one DPP row at most).  Lane t of the group holds rows
// i = s*G + t (slots s = 0..S-1) of the lower triangle of the Newton matrix
// in registers, each slot padded to the longest row of the slot.  The
// bordered system [[H, 1], [1^T, 0]] is factored as L D L^T by a
// right-looking sweep: at step k the group publishes column k to LDS, every
// lane reads it back (a broadcast read) and updates its own rows.  The border
// row (the sum-to-one constraint) is carried as one extra distributed row.
// Triangular solves run row by row with DPP broadcasts and butterfly
// reductions inside the group.  Everything that depends on the step k, the
// slot s or the column j is a compile-time index, so the matrix never leaves
// registers.  The scaled Gram matrix (shared by every pixel) sits in LDS.
//
// Iteration (Mehrotra predictor-corrector, one common step length, eta):
//   r_d = Gh a - bh - lambda + nu 1,  r_p = 1^T a - 1,  mu = a^T lambda / n
//   H = Gh + diag(lambda / a)
//   predictor rc = a*lambda; corrector rc = a*lambda + da_aff*dl_aff - sigma mu
//   (the second-order term is dropped when the affine step is below 0.1)
//   [H 1; 1^T 0] [da; dnu] = [-r_d - rc/a; -r_p],  dl = -rc/a - D da
// Finishing step: free set F = {a_i > lambda_i}; solve the problem with
// a_A = 0 exactly (diagonal BIG on A), check a_F >= -tau and
// lambda_A >= -tau, otherwise move the worst index across and repeat.
#include "common.h"
#include "kernels.h"

namespace lm {

template <int NC, int G>
struct Lay {
  static constexpr int S = (NC + G - 1) / G;
  static constexpr int len(int s) { return ((s + 1) * G < NC) ? (s + 1) * G : NC; }
  static constexpr int off(int s) {
    int o = 0;
    for (int q = 0; q < s; ++q) o += len(q);
    return o;
  }
  static constexpr int HSZ = off(S);
};

template <int B, int E, typename F>
__device__ __forceinline__ void static_for_rev(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, E - 1>{});
    static_for_rev<B, E - 1>(f);
  }
}

template <typename T>
__device__ __forceinline__ bool finite(T v) {
  return isfin(v);
}

// One pixel's factor/solve machinery on its group of G lanes.
template <typename T, int NC, int G>
struct Px {
  using LY = Lay<NC, G>;
  static constexpr int S = LY::S;
  static constexpr int HSZ = LY::HSZ;
  static constexpr int CB = NC + 1;

  int t, n;
  const T* sG;  // LDS, NC x NC
  T* colbuf;    // LDS, 2 x CB
  T* abuf;      // LDS, NC
  bool vm[S];   // row s*G+t < n
  T h[HSZ];
  T bord[S], dinv[S];
  T dN;
  bool notpd;

  __device__ __forceinline__ int row(int s) const { return s * G + t; }
  __device__ __forceinline__ int rowc(int s) const {
    const int i = s * G + t;
    return i < NC ? i : NC - 1;
  }

  // g = Gh a on the own rows (a gathered through LDS)
  __device__ __forceinline__ void matvec(const T (&a)[S], T (&g)[S]) {
    static_for<0, S>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      if (row(s) < NC) abuf[row(s)] = vm[s] ? a[s] : T(0);
    });
    lds_sync();
    static_for<0, S>([&](auto ss) { g[ss] = T(0); });
    static_for<0, NC>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const T aj = abuf[j];
      static_for<0, S>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        g[s] = fmaT(sG[rowc(s) * NC + j], aj, g[s]);
      });
    });
    static_for<0, S>([&](auto ss) { g[ss] = vm[ss] ? g[ss] : T(0); });
  }

  // H = Gh + diag(D) on the own rows (rows beyond NC are zero)
  __device__ __forceinline__ void form(const T (&D)[S]) {
    static_for<0, S>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      const bool in = row(s) < NC;
      const int r = rowc(s);
      static_for<0, LY::len(s)>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        h[LY::off(s) + j] = in ? sG[r * NC + j] : T(0);
      });
      static_for<0, G>([&](auto tt) {
        constexpr int j = s * G + decltype(tt)::value;
        if constexpr (j < LY::len(s)) h[LY::off(s) + j] += (t == tt) ? D[s] : T(0);
      });
    });
  }

  // L D L^T of [[H, 1], [1^T, corner]] (first n rows, border last); corner
  // 0 for sum-to-one, -s/nu with the slack pair of sum-lower-than-one, and a
  // huge negative value when there is no sum row (the border solution is then
  // zero to rounding)
  __device__ __forceinline__ void factor(T corner) {
    dN = corner;
    notpd = false;
    static_for<0, S>([&](auto ss) {
      dinv[ss] = T(1);
      bord[ss] = vm[ss] ? T(1) : T(0);
    });
    static_for<0, NC>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      constexpr int sk = k / G, tk = k % G;
      if (k < n) {
        T* buf = colbuf + (k & 1) * CB;
        static_for<sk, S>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          if (row(s) < NC) buf[row(s)] = h[LY::off(s) + k];
        });
        if (t == tk) buf[NC] = bord[sk];
        lds_sync();
        const T d = buf[k];
        const T cb = buf[NC];
        const bool bad = !(d > T(0)) || !finite(d);
        notpd |= bad;
        const T rcp = bad ? T(1) : rcpT(d);
        dinv[sk] = (t == tk) ? rcp : dinv[sk];
        const T lb = cb * rcp;
        dN -= lb * cb;
        static_for<sk, S>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          const T hk = h[LY::off(s) + k];
          T l = hk * rcp;
          if constexpr (s == sk) l = (t > tk) ? l : T(0);
          static_for<k + 1, LY::len(s)>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            h[LY::off(s) + j] = fmaT(-l, buf[j], h[LY::off(s) + j]);
          });
          h[LY::off(s) + k] = l;
          const T bupd = fmaT(-lb, hk, bord[s]);
          if constexpr (s == sk)
            bord[s] = (t > tk) ? bupd : ((t == tk) ? lb : bord[s]);
          else
            bord[s] = bupd;
        });
      }
    });
    if (!(dN < T(0)) || !finite(dN)) notpd = true;
  }

  // Solve [[H,1],[1^T,corner]] [x; xN] = [r; rN] in place; returns xN.
  __device__ __forceinline__ T solve(T (&r)[S], T rN) {
    static_for<0, NC>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      constexpr int sk = k / G, tk = k % G;
      if (k < n) {
        const T yk = gbcast<G, tk>(r[sk], t);
        static_for<sk, S>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          r[s] = fmaT(-h[LY::off(s) + k], yk, r[s]);
        });
      }
    });
    T part = T(0);
    static_for<0, S>([&](auto ss) { part = fmaT(bord[ss], r[ss], part); });
    const T yN = rN - gsum<G>(part);
    const T xN = notpd ? T(0) : yN / dN;
    static_for<0, S>([&](auto ss) {
      r[ss] *= dinv[ss];
      r[ss] = fmaT(-bord[ss], xN, r[ss]);
    });
    static_for_rev<0, NC>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      constexpr int sk = k / G, tk = k % G;
      if (k < n) {
        T pp = T(0);
        static_for<sk, S>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          pp = fmaT(h[LY::off(s) + k], r[s], pp);
        });
        pp = gsum<G>(pp);
        r[sk] = (t == tk) ? r[sk] - pp : r[sk];
      }
    });
    return xN;
  }
};

// largest step in (0, inf] keeping x + step*dx >= 0 on the valid rows
template <typename T, int S, int G>
__device__ __forceinline__ T max_step(const T (&x)[S], const T (&dx)[S], const bool (&vm)[S]) {
  T m = T(INFINITY);
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (vm[s] && dx[s] < T(0)) m = fmin(m, -x[s] / dx[s]);
  return gmin<G>(m);
}

// One workgroup's pixels: block blk of the cube described by prm.
template <typename T, int NC, int G, int MODE>
__device__ __forceinline__ void ipm_body(const IpmParams& prm, int64_t blk) {
  using PX = Px<T, NC, G>;
  constexpr int S = PX::S;
  constexpr int GPW = 64 / G;
  constexpr int GPB = 4 * GPW;
  constexpr int CB = PX::CB;
  constexpr int GST = 2 * CB + NC;
  __shared__ T sG[NC * NC];
  __shared__ T sbuf[GPB * GST];

  const T* Gsrc = static_cast<const T*>(prm.Gh);
  for (int i = threadIdx.x; i < NC * NC; i += blockDim.x) sG[i] = Gsrc[i];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = lane % G, grp = lane / G;
  const int gib = wave * GPW + grp;
  const int64_t p = blk * GPB + gib;
  const bool inrange = p < prm.P;
  const int n = prm.n;

  PX px;
  px.t = t;
  px.n = n;
  px.sG = sG;
  px.colbuf = sbuf + gib * GST;
  px.abuf = px.colbuf + 2 * CB;
  static_for<0, S>([&](auto ss) { px.vm[ss] = (ss * G + t) < n; });
  const bool(&vm)[S] = px.vm;

  uint32_t flags = 0;
  // scaled projections of the pixel (non-finite input -> NONFINITE)
  T bh[S];
  bool nonfin = false;
  static_for<0, S>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    const double v = (inrange && vm[s]) ? prm.bh[p * n + s * G + t] : 0.0;
    if (!finite(v)) nonfin = true;
    bh[s] = (T)v;
  });
  if (inrange && prm.c && !finite(prm.c[p])) nonfin = true;
  nonfin = gor_i<G>((int)nonfin) != 0;
  if (nonfin) {
    flags |= kPxNonfinite;
    static_for<0, S>([&](auto ss) { bh[ss] = T(0); });
  }
  T bhmax = T(0);
  static_for<0, S>([&](auto ss) { bhmax = fmax(bhmax, fabs(bh[ss])); });
  bhmax = gmax<G>(bhmax);

  // interior-point state; sum-lower-than-one adds the slack s of 1^T a <= 1
  // and its multiplier nu as one more complementarity pair, positivity only
  // has no sum row
  const bool slo = prm.constraint == kSlo, pos = prm.constraint == kPos;
  const T inv_np = T(1) / T(n + (slo ? 1 : 0));
  T a[S], lam[S], nu = slo ? (T)prm.lambda0 : T(0), sl = slo ? inv_np : T(0);
  int it = 0;
  bool start = inrange && !nonfin;
  if constexpr (MODE == kStage2) {
    if (inrange) {
      const uint8_t f = prm.st_flag[p];
      flags |= f & 0x7fu;
      start = start && (f & 0x80u);
      it = prm.st_it[p];
      nu = (T)prm.st_nu[p];
      sl = slo ? (T)prm.st_s[p] : T(0);
    }
    static_for<0, S>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      const bool ok = inrange && vm[s];
      a[s] = ok ? (T)prm.st_a[p * n + s * G + t] : T(0);
      lam[s] = ok ? (T)prm.st_lam[p * n + s * G + t] : T(0);
    });
  } else {
    static_for<0, S>([&](auto ss) {
      a[ss] = vm[ss] ? inv_np : T(0);
      lam[ss] = vm[ss] ? (T)prm.lambda0 : T(0);
    });
  }
  const T tol_mu = (T)(MODE == kStage1 ? fmax(prm.tol_mu, prm.mu_switch) : prm.tol_mu);
  const T tol_d = (T)prm.tol_d, tol_p = (T)prm.tol_p, eta = (T)prm.eta, tau = (T)prm.tau;
  constexpr T BIG = T(MODE == kStage1 ? 1e30f : 1e30);

  // phases of a group: interior-point iterations, finishing step, done
  enum { kIpm = 0, kPol = 1, kDone = 2 };
  int phase = start ? kIpm : kDone;
  bool converged = false, certified = false, cand = false;
  bool sfree = pos;    // finishing step: no sum row (slack free or no sum constraint)
  uint32_t freem = 0;  // finishing step: bit s set when row s*G+t is free
  int kp = 0;          // finishing-step corrections so far
  bool stalled = false;  // first stage of the mixed form: the last step was too short
  T pa[S], pnu = T(0);

  T g[S], rd[S], D[S], x[S], dla[S];
  T rp = T(0), mu = T(0);
  for (;;) {
    // ---- products with the scaled Gram matrix and the phase decisions ----
    static_for<0, S>([&](auto ss) { x[ss] = (phase == kPol) ? pa[ss] : a[ss]; });
    px.matvec(x, g);
    if (phase == kIpm) {
      T sa = T(0), sal = T(0), rdm = T(0);
      static_for<0, S>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        rd[s] = vm[s] ? (g[s] - bh[s] - lam[s] + nu) : T(0);
        sa += a[s];
        sal = fmaT(a[s], lam[s], sal);
        rdm = fmax(rdm, fabs(rd[s]));
      });
      rp = pos ? T(0) : gsum<G>(sa) + sl - T(1);
      mu = (gsum<G>(sal) + sl * nu) * inv_np;
      rdm = gmax<G>(rdm);
      bool conv;
      if constexpr (MODE == kStage1)
        conv = mu <= tol_mu || stalled || it >= kStage1MaxIt;
      else
        conv = mu <= tol_mu && rdm <= tol_d * (T(1) + bhmax) && fabs(rp) <= tol_p;
      if (conv) {
        converged = true;
        if constexpr (MODE == kStage1) {
          phase = kDone;
        } else {
          phase = kPol;
          cand = false;
          static_for<0, S>([&](auto ss) {
            if (vm[ss] && a[ss] > lam[ss]) freem |= 1u << ss;
          });
          sfree = pos || (slo && sl > nu);
        }
      } else if (it >= prm.maxit) {
        flags |= kPxMaxit;
        phase = kDone;
      }
    } else if (phase == kPol && cand) {
      // KKT check of the candidate from the previous solve
      T wa = T(INFINITY), wl = T(INFINITY), pl[S];
      static_for<0, S>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        const bool fr = (freem >> s) & 1u;
        pl[s] = (vm[s] && !fr) ? g[s] - bh[s] + pnu : T(0);
        if (vm[s] && fr) wa = fmin(wa, pa[s]);
        if (vm[s] && !fr) wl = fmin(wl, pl[s]);
      });
      wa = gmin<G>(wa);
      wl = gmin<G>(wl);
      // sum-lower-than-one: the slack is one more index (free: its value
      // 1 - 1^T a must be >= 0; at its bound: the multiplier nu must be)
      T spa = T(0);
      static_for<0, S>([&](auto ss) { spa += pa[ss]; });
      const T sv = T(1) - gsum<G>(spa);
      const bool slA = slo && sfree && sv < fmin(wa, -tau);
      const bool slL = slo && !sfree && pnu < fmin(wl, -tau);
      if (slA) wa = sv;
      if (slL) wl = pnu;
      if (wa >= -tau && wl >= -tau) {
        certified = true;
        phase = kDone;
        static_for<0, S>([&](auto ss) {
          a[ss] = pa[ss];
          lam[ss] = pl[ss];
        });
        nu = pnu;
        sl = (slo && sfree) ? sv : T(0);
      } else if (kp >= prm.max_polish) {
        phase = kDone;
      } else if ((wa < -tau && wa <= wl) ? slA : slL) {
        sfree = !sfree;
        ++kp;
        cand = false;
      } else {
        const bool flipA = (wa < -tau) && (wa <= wl);
        const T target = flipA ? wa : wl;
        int idx = 1 << 30;
        static_for<0, S>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          const bool fr = (freem >> s) & 1u;
          const bool c = flipA ? (vm[s] && fr && pa[s] == target) : (vm[s] && !fr && pl[s] == target);
          if (c) idx = min(idx, s * G + t);
        });
        idx = gmin_i<G>(idx);
        static_for<0, S>([&](auto ss) {
          if (ss * G + t == idx) freem ^= 1u << ss;
        });
        ++kp;
        cand = false;
      }
    }
    if (__builtin_amdgcn_ballot_w64(phase != kDone) == 0) break;

    // ---- Newton matrix (IPM) or free-set matrix (finishing step) ----------
    static_for<0, S>([&](auto ss) {
      const T dp = (((freem >> ss) & 1u) ? T(0) : BIG);
      const T di = (phase == kPol) ? dp : ((phase == kIpm) ? lam[ss] / a[ss] : T(1));
      D[ss] = vm[ss] ? di : T(0);
    });
    px.form(D);
    const T corner = (phase == kPol) ? (sfree ? -BIG : T(0)) : (pos ? -BIG : (slo ? -sl / nu : T(0)));
    px.factor(corner);
    if (phase != kDone && px.notpd) {
      if (phase == kIpm) flags |= kPxNotPd;
      phase = kDone;
    }

    // ---- solves: predictor then corrector (IPM), one solve (finishing) ----
    T rN;
    if (phase == kPol) {
      static_for<0, S>([&](auto ss) { x[ss] = bh[ss]; });
      rN = sfree ? T(0) : T(1);
    } else {
      static_for<0, S>([&](auto ss) { x[ss] = vm[ss] ? -rd[ss] - lam[ss] : T(0); });
      rN = slo ? sl - rp : -rp;  // slack pair: + rcs / nu with rcs = s nu
    }
    const bool two = __builtin_amdgcn_ballot_w64(phase == kIpm) != 0;
    T sig = T(0), ds_aff = T(0), dnu_aff = T(0), rcs = T(0);
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const T xN = px.solve(x, rN);
      if (pass == 0) {
        if (phase == kPol) {
          static_for<0, S>([&](auto ss) { pa[ss] = (vm[ss] && ((freem >> ss) & 1u)) ? x[ss] : T(0); });
          pnu = xN;
          cand = finite(xN);
          if (!cand) phase = kDone;
        }
        // predictor step length and centring parameter
        static_for<0, S>([&](auto ss) { dla[ss] = vm[ss] ? -lam[ss] - D[ss] * x[ss] : T(0); });
        T st_aff = fmin(max_step<T, S, G>(a, x, vm), max_step<T, S, G>(lam, dla, vm));
        st_aff = fmin(st_aff, T(1));
        if (slo) {
          dnu_aff = xN;
          ds_aff = -sl - (sl / nu) * dnu_aff;
          if (ds_aff < T(0)) st_aff = fmin(st_aff, -sl / ds_aff);
          if (dnu_aff < T(0)) st_aff = fmin(st_aff, -nu / dnu_aff);
        }
        T smu = T(0);
        static_for<0, S>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          if (vm[s]) smu = fmaT(a[s] + st_aff * x[s], lam[s] + st_aff * dla[s], smu);
        });
        const T smu_s = slo ? (sl + st_aff * ds_aff) * (nu + st_aff * dnu_aff) : T(0);
        const T ratio = ((gsum<G>(smu) + smu_s) * inv_np) / mu;
        sig = ratio * ratio * ratio;
        // corrector right-hand side; dla <- rc / a.  The second-order term
        // is dropped after a short affine step (guards against cycling).
        const T soc = st_aff >= T(0.1) ? T(1) : T(0);
        static_for<0, S>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          const T rc = fmaT(soc * x[s], dla[s], a[s] * lam[s]) - sig * mu;
          dla[s] = vm[s] ? rc / a[s] : T(0);
          x[s] = vm[s] ? -rd[s] - dla[s] : T(0);
        });
        rcs = slo ? fmaT(soc * ds_aff, dnu_aff, sl * nu) - sig * mu : T(0);
        rN = slo ? rcs / nu - rp : -rp;
        if (!two) break;
      } else {
        // corrector direction and the common step
        T dl[S];
        static_for<0, S>([&](auto ss) { dl[ss] = vm[ss] ? -dla[ss] - D[ss] * x[ss] : T(0); });
        T step = fmin(max_step<T, S, G>(a, x, vm), max_step<T, S, G>(lam, dl, vm));
        const T ds = slo ? (-rcs - sl * xN) / nu : T(0);
        if (slo) {
          if (ds < T(0)) step = fmin(step, -sl / ds);
          if (xN < T(0)) step = fmin(step, -nu / xN);
        }
        const T alpha = fmin(T(1), eta * step);
        if constexpr (MODE == kStage1) stalled = !(alpha >= T(kStage1MinStep));
        if (phase == kIpm && finite(alpha)) {
          static_for<0, S>([&](auto ss) {
            a[ss] = fmaT(alpha, x[ss], a[ss]);
            lam[ss] = fmaT(alpha, dl[ss], lam[ss]);
          });
          nu = fmaT(alpha, xN, nu);
          sl = fmaT(alpha, ds, sl);
        }
        if (phase == kIpm) ++it;
      }
    }
  }

  if constexpr (MODE == kStage1) {
    // hand the iterate over to the FP64 stage
    if (inrange) {
      static_for<0, S>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        if (vm[s]) {
          prm.st_a[p * n + s * G + t] = (double)a[s];
          prm.st_lam[p * n + s * G + t] = (double)lam[s];
        }
      });
      if (t == 0) {
        prm.st_nu[p] = (double)nu;
        if (slo) prm.st_s[p] = (double)sl;
        prm.st_it[p] = it;
        // a loss of positive definiteness in FP32 is retried in FP64 from
        // the last accepted iterate
        const bool more = !nonfin;
        prm.st_flag[p] = (uint8_t)((flags & ~(kPxMaxit | kPxNotPd)) | (more ? 0x80u : 0u));
      }
    }
  } else {
    if (converged && !certified && inrange && !nonfin) flags |= kPxInexact;
    if (certified) {
      bool deg = false;
      static_for<0, S>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        if (vm[s]) deg |= ((freem >> s) & 1u) ? (a[s] < (T)prm.deg_tol) : (lam[s] < (T)prm.deg_tol);
      });
      if (slo) deg |= sfree ? (sl < (T)prm.deg_tol) : (nu < (T)prm.deg_tol);
      if (gor_i<G>((int)deg)) flags |= kPxDegenerate;
    }
    double sgm = 1.0;
    if (inrange && prm.sigma) sgm = (double)prm.sigma[p];
    if (!(sgm > 0.0) || !finite(sgm)) flags |= kPxBadSigma;
    const double qnan = __builtin_nan("");
    if (inrange) {
      static_for<0, S>([&](auto ss) {
        constexpr int s = decltype(ss)::value;
        if (vm[s]) {
          const int64_t o = p * n + s * G + t;
          prm.out_a[o] = nonfin ? qnan : (double)a[s];
          if (prm.dcov) {
            double dv;
            if (nonfin)
              dv = qnan;
            else if (certified)
              dv = ((freem >> s) & 1u) ? 0.0 : (double)INFINITY;
            else
              dv = (double)lam[s] / (double)a[s];
            prm.dcov[o] = dv;
          }
        }
      });
      if (prm.dcorner && t == 0) {
        // corner of the covariance's bordered matrix: 0 on a binding sum row,
        // -s/nu for the slack pair of an uncertified iterate, -inf without a
        // sum row
        double cr;
        if (certified) cr = sfree ? -(double)INFINITY : 0.0;
        else cr = pos ? -(double)INFINITY : (slo ? -(double)sl / (double)nu : 0.0);
        prm.dcorner[p] = cr;
      }
    }
    if (prm.objective) {
      px.matvec(a, g);
      T ba = T(0), aga = T(0);
      static_for<0, S>([&](auto ss) {
        ba = fmaT(bh[ss], a[ss], ba);
        aga = fmaT(a[ss], g[ss], aga);
      });
      ba = gsum<G>(ba);
      aga = gsum<G>(aga);
      if (inrange && t == 0) {
        double F = (prm.c[p] - 2.0 * prm.gamma * (double)ba + prm.gamma * (double)aga) / (sgm * sgm);
        if (nonfin || (flags & kPxBadSigma)) F = qnan;
        prm.objective[p] = F;
      }
    }
    if (inrange && t == 0) {
      if (prm.status) prm.status[p] = (uint8_t)flags;
      if (prm.iters) prm.iters[p] = it;
    }
  }
}

// ---------------------------------------------------------------------------
// Launch of one compiled shape.  The build compiles this file once per entry
// of ipm_shapes.def (LM_T, LM_NC, LM_G defined), so shapes build in parallel;
// ipm_dispatch.cpp picks the shape for a library at run time.
// ---------------------------------------------------------------------------
template <typename T, int NC, int G, int MODE>
__global__ __launch_bounds__(256) void ipm_kernel(IpmParams prm) {
  ipm_body<T, NC, G, MODE>(prm, blockIdx.x);
}

// Several cubes in one launch (one job per cube, blocks assigned by start).
template <typename T, int NC, int G, int MODE>
__global__ __launch_bounds__(256) void ipm_batch_kernel(const IpmParams* __restrict__ jobs,
                                                        const int64_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const IpmParams prm = uniform_copy(jobs + j);
  ipm_body<T, NC, G, MODE>(prm, (int64_t)blockIdx.x - start[j]);
}

template <typename T, int NC, int G, int MODE>
static void launch_mode(const IpmParams& p, const IpmBatch* b, hipStream_t st) {
  constexpr int GPB = 4 * (64 / G);
  if (b)
    hipLaunchKernelGGL((ipm_batch_kernel<T, NC, G, MODE>), dim3((unsigned)b->blocks), dim3(256), 0, st, b->jobs,
                       b->start, b->njobs);
  else
    hipLaunchKernelGGL((ipm_kernel<T, NC, G, MODE>), dim3((unsigned)((p.P + GPB - 1) / GPB)), dim3(256), 0, st, p);
}

// b == nullptr: one cube described by p; else the jobs of b.
template <typename T, int NC, int G>
static int launch_shape(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (mode != kStage1) return -5;
    launch_mode<T, NC, G, kStage1>(p, b, st);
  } else {
    if (mode == kFull)
      launch_mode<T, NC, G, kFull>(p, b, st);
    else if (mode == kStage2)
      launch_mode<T, NC, G, kStage2>(p, b, st);
    else
      return -5;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

#if defined(LM_T) && defined(LM_NC) && defined(LM_G)
#define LM_ENTRY2(t, nc, g) ipm_entry_##t##_##nc##_##g
#define LM_ENTRY(t, nc, g) LM_ENTRY2(t, nc, g)
int LM_ENTRY(LM_T, LM_NC, LM_G)(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  return launch_shape<LM_T, LM_NC, LM_G>(p, b, mode, st);
}
#endif

}  // namespace lm
