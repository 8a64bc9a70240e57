// ipm_rc.hip -- FP64 interior-point solve (IPLS, Sec. 2.2) for the larger
// libraries: a pixel's Newton matrix spread row-cyclically over B of the four
// blocks of v_mfma_f64_4x4x4f64 (B = 4: one pixel per wavefront; B = 2: two).
//
// Same method and per-pixel logic as ipm_tile.hip (ipm_body.h); only the
// mapping of the Newton matrix and of the vectors differs.
//
// Mapping.  lane = 16 x + 4 b + z; block b of the MFMA belongs to pixel b / B
// as its block bp = b % B.  Block bp holds the tile rows I = B r + bp of the
// pixel's N x N Newton matrix (4x4 tiles, T = NC / 4 tile rows, R = T / B row
// slots): slot (r, J) is tile (B r + bp, J) for J <= B r + B - 1,
// kept "stored" as in ipm_tile.hip (lane (x, z) holds X[z][x]), so that one
// MFMA on slot (r, .) works on four tile rows of the same column at once.
// Slots above the tile diagonal hold zeros; the factored diagonal blocks are
// kept apart (dg).  The factorisation is the stable block L D L^T of
// ipm_tile.hip: every block factors the 4x4 diagonal tile of column K (it
// is exchanged through LDS), computes the panel W_JK = H_JK L_KK^{-T} of its
// own rows, and the trailing update H_IJ -= L_IK W_JK^T takes W_JK of row J,
// which lives in block J mod B, from LDS.  The 4x4x4 FP64 MFMA has no block
// broadcast of its A operand on gfx950 (its CBSZ/ABID fields are ignored),
// hence the exchange.  Vectors use the x layout: lane (x, z) of block bp
// holds element 4 (B r + bp) + x of right-hand side z in register r; the
// elementwise work of the method uses the same registers with every column z
// holding the same vector.  Forward solve: column by column, the finished
// tile of row J broadcast to the other blocks by DPP; backward solve: row
// by row, the B blocks' partial sums over their own rows added by DPP.
#include "ipm_body.h"

namespace lm {

constexpr int kRowRor4 = 0x124;   // lane i <- lane i - 4 within a row: block b <- block b - 1
constexpr int kRowRor8 = 0x128;   // block b <- block b - 2
constexpr int kRowRor12 = 0x12c;  // block b <- block b + 1

template <int T, int B>
struct RC {
  using real = double;
  using xreg = double;
  static constexpr bool kCompact = false;
  static constexpr bool kRecomputeGrad = false;
  static_assert(B == 2 || B == 4, "a pixel spans two or four blocks");
  static_assert(T % B == 0, "row-cyclic tiles need a multiple of B tile rows");
  static constexpr int R = T / B;                 // row slots per block
  static constexpr int NP = 4 * T;                // padded library size
  static constexpr int C = (R + 3) / 4;           // elementwise slots
  static constexpr int NX = R;                    // solve registers
  static constexpr int NS = B * R * (R + 1) / 2;  // tile slots: sum over r of B r + B
  static constexpr int sid(int r, int J) { return B * r * (r + 1) / 2 + J; }
  static constexpr int WX = 16 * B;               // doubles of one row slot's panel in LDS

  int x, z, b;              // lane coordinates; b: block within the pixel
  int hb;                   // the block's index in the wavefront (0..3)
  int nvalid;               // library size n
  const double* sG;         // LDS, NP x NP scaled Gram
  double* xch;              // LDS, 16 doubles of this pixel (diagonal tile)
  double* wx;               // LDS, R x WX doubles of this pixel (panel / vector exchange)
  double H[NS];             // after factor(): -L below the tile diagonal, zeros elsewhere
  double dg[R];             // diagonal block of row B r + b: L^{-1} below its diagonal, 1/d on it
  bool notpd;

  // compact layout: slot m of lane (x, b, z) holds element 4 (B (z + 4 m) + b) + x,
  // i.e. x-layout register z + 4 m of the lane's block
  __device__ __forceinline__ int el(int m) const { return 4 * (B * (z + 4 * m) + b) + x; }
  __device__ __forceinline__ int elx(int r) const { return 4 * (B * r + b) + x; }
  __device__ __forceinline__ bool xvalid(int I) const { return elx(I) < nvalid; }
  __device__ __forceinline__ int rhs() const { return z; }
  __device__ __forceinline__ bool writer() const { return x == 0 && z == 0 && b == 0; }

  // Reductions over the pixel's elements, the same bits on every lane: a
  // butterfly over the quad (z), then (B = 4) the row mirror (block b <-> 3 -
  // b; the quad now holds equal values, so the reversal of z is harmless) and
  // the half-row mirror (b <-> b ^ 1), then the row exchanges (x).
  template <typename V, typename Op>
  static __device__ __forceinline__ V red(V v, Op op) {
    v = op(v, dpp<qp(1, 0, 3, 2)>(v));
    v = op(v, dpp<qp(2, 3, 0, 1)>(v));
    if constexpr (B == 4) v = op(v, dpp<kRowMirror>(v));
    v = op(v, dpp<kRowHalfMirror>(v));
    Pair<V> p = pair<16>(v);
    v = op(p.lo, p.hi);
    p = pair<32>(v);
    return op(p.lo, p.hi);
  }
  static __device__ __forceinline__ double sum(double v) {
    return red(v, [](double a, double c) { return a + c; });
  }
  static __device__ __forceinline__ double vmin(double v) {
    return red(v, [](double a, double c) { return fmin(a, c); });
  }
  static __device__ __forceinline__ double vmax(double v) {
    return red(v, [](double a, double c) { return fmax(a, c); });
  }
  static __device__ __forceinline__ int imin(int v) {
    return red(v, [](int a, int c) { return min(a, c); });
  }
  static __device__ __forceinline__ int ior(int v) {
    return red(v, [](int a, int c) { return a | c; });
  }

  // v of the other block of the pixel (B = 2; same x, z)
  __device__ __forceinline__ double partner(double v) const {
    const double lo = dpp<kRowRor4>(v), hi = dpp<kRowRor12>(v);
    return b == 1 ? lo : hi;
  }
  // sum of v over the pixel's blocks (same x, z), the same bits on each
  __device__ __forceinline__ double bsum(double v) const {
    if constexpr (B == 4) {
      v += dpp<kRowRor4>(v);
      return v + dpp<kRowRor8>(v);
    } else {
      return v + partner(v);
    }
  }
  // v of block SRC on every block of the pixel (same x, z); adding zeros is exact
  template <int SRC>
  __device__ __forceinline__ double bcast(double v) const {
    return bsum((b == SRC) ? v : 0.0);
  }

  // compact -> x layout (every right-hand side column gets the same vector)
  __device__ __forceinline__ void to_x(const double (&v)[C], double (&xl)[NX]) const {
    static_for<0, R>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      xl[r] = qb<r % 4>(v[r / 4]);
    });
  }
  // x layout, right-hand side RHS -> compact
  template <int RHS>
  __device__ __forceinline__ void from_x(const double (&xl)[NX], double (&v)[C]) const {
    static_for<0, C>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      double t[4];
      static_for<0, 4>([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        if constexpr (q + 4 * m < R) t[q] = qb<RHS>(xl[q + 4 * m]);
        else t[q] = 0.0;
      });
      v[m] = z == 0 ? t[0] : (z == 1 ? t[1] : (z == 2 ? t[2] : t[3]));
    });
  }

  // v = Gh * xa (every column of xa holds the same vector, x layout): the
  // blocks exchange their elements through LDS, then each forms its own rows
  __device__ __forceinline__ void gmul(const double (&xa)[NX], double (&v)[C]) const {
    asm volatile("" ::: "memory");
    static_for<0, R>([&](auto rr) {
      if (z == 0) wx[elx(rr)] = xa[rr];
    });
    lds_sync();
    double acc[NX];
    static_for<0, R>([&](auto rr) { acc[rr] = 0.0; });
    static_for<0, T>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      const double xj = wx[4 * J + x];
      static_for<0, R>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        const int I = B * r + b;
        acc[r] = mfma4(sG[(4 * I + z) * NP + 4 * J + x], xj, acc[r]);
      });
    });
    from_x<0>(acc, v);
    asm volatile("" ::: "memory");
  }

  // H = Gh + diag(D), D in x layout; zeros above the tile diagonal
  __device__ __forceinline__ void form(const double (&xD)[NX]) {
    static_for<0, R>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      const int I = B * r + b;
      static_for<0, B * r + B>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        double v = sG[(4 * I + z) * NP + 4 * J + x];
        if constexpr (J >= B * r) {  // the slot holds the diagonal tile or zeros on some blocks
          v += (J == I && x == z) ? xD[r] : 0.0;
          v = (J <= I) ? v : 0.0;
        }
        H[sid(r, J)] = v;
      });
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // every block's factor of the diagonal tile d (held on block C only):
  // exchange through LDS, then the 4x4 L D L^T
  template <int C>
  __device__ __forceinline__ void diag_factor(double d, bool& bad, double& li, double& rx) const {
    asm volatile("" ::: "memory");
    if (b == C) xch[z * 4 + x] = d;
    lds_sync();
    ldl4_lds(xch, x, z, bad, li, rx);
  }

  // right-looking block L D L^T, one tile column K at a time.  The next
  // column's diagonal tile is updated first, from its own block's panel
  // tile, so that its exchange does not wait for the panel broadcast.
  __device__ __forceinline__ void factor() {
    bool bad = false;
    double dcur = H[sid(0, 0)];
    static_for<0, T>([&](auto kk) {
      constexpr int K = decltype(kk)::value;
      constexpr int rK = K / B, cK = K % B;
      __builtin_amdgcn_sched_barrier(0);
      double li, rx;
      diag_factor<cK>(dcur, bad, li, rx);
      const double nrx = -rx;
      dg[rK] = (b == cK) ? ((x == z) ? rx : li) : dg[rK];
      H[sid(rK, K)] = (b > cK) ? H[sid(rK, K)] : 0.0;
      if constexpr (K + 1 < T) {
        // panel of every row slot at or below the diagonal one, published for
        // the other blocks; rows at or above K carry zeros
        constexpr int J1 = K + 1, r1 = J1 / B;
        double wdiag = 0.0;
        static_for<rK, R>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          const double w = mfma4(li, H[sid(r, K)], 0.0);
          H[sid(r, K)] = w * nrx;
          wx[r * WX + 4 * (B * x + b) + z] = w;
          if constexpr (r == r1) wdiag = w;
        });
        // (the slot of the next diagonal tile gets the same update below and
        // is cleared at the next step)
        dcur = mfma4(wdiag, H[sid(r1, K)], H[sid(r1, J1)]);
        lds_sync();
        // trailing update of the columns right of K
        static_for<K + 1, T>([&](auto jj) {
          constexpr int J = decltype(jj)::value;
          constexpr int rJ = J / B, cJ = J % B;
          const double w = wx[rJ * WX + 4 * (B * x + cJ) + z];
          static_for<rJ, R>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            H[sid(r, J)] = mfma4(w, H[sid(r, K)], H[sid(r, J)]);
          });
        });
      }
    });
    notpd = bad;
  }

  // solve L D L^T X = R in place (x layout, one right-hand side per z)
  __device__ __forceinline__ void solve(double (&xl)[NX]) const {
    // L y = r: tile row J is finished on block J mod B (its diagonal block),
    // then broadcast and applied to every row below it
    static_for<0, T>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      constexpr int rJ = J / B, cJ = J % B;
      const double lu = (x == z) ? 1.0 : dg[rJ];
      const double t = mfma4(lu, xl[rJ], 0.0);
      xl[rJ] = (b == cJ) ? t : xl[rJ];
      if constexpr (J + 1 < T) {
        const double yb = bcast<cJ>(xl[rJ]);
        static_for<rJ, R>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          xl[r] = mfma4(H[sid(r, J)], yb, xl[r]);
        });
      }
    });
    // diag(d)^{-1} y
    static_for<0, R>([&](auto rr) {
      const double dv = (x == z) ? dg[rr] : 0.0;
      xl[rr] = mfma4(dv, xl[rr], 0.0);
    });
    // L^T x = diag(d)^{-1} y, row by row from the last: each block sums the
    // contributions of its own finished rows (transposed tiles come from lane
    // (z, x) of the same block), the B partial sums are added by DPP
    const int src = 16 * z + 4 * hb + x;
    static_for<0, T>([&](auto kk) {
      constexpr int J = T - 1 - decltype(kk)::value;
      constexpr int rJ = J / B, cJ = J % B;
      double acc = 0.0;
      if constexpr (J + 1 < T) {
        static_for<rJ, R>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          const double lt = __shfl(H[sid(r, J)], src);
          acc = mfma4(lt, xl[r], acc);
        });
        acc = bsum(acc);
      }
      const double lut = __shfl((x == z) ? 1.0 : dg[rJ], src);
      const double t = mfma4(lut, xl[rJ] + acc, 0.0);
      xl[rJ] = (b == cJ) ? t : xl[rJ];
    });
  }
};

// One workgroup of WPB wavefronts, 4 / B pixels each: workgroup wg of the
// cube described by prm.
template <int T, int B, int MODE, int CONS, int WPB>
__device__ __forceinline__ void ipm_rc_body(const IpmParams& prm, int64_t wg) {
  using TL = RC<T, B>;
  constexpr int NP = TL::NP;
  constexpr int PPW = 4 / B, PPB = WPB * PPW;  // pixels per wavefront, per workgroup
  __shared__ double sG[NP * NP];
  __shared__ double sx[PPB * 16];
  __shared__ double sw[PPB * TL::R * TL::WX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hb = (lane >> 2) & 3;
  const int pix = wave * PPW + hb / B;  // pixel in the workgroup
  const int64_t p = wg * PPB + pix;
  if constexpr (MODE == kRetry) {
    // most workgroups hold no pixel to solve again
    if (!__syncthreads_or(p < prm.P && (prm.status[p] & kPxRetry) != 0)) return;
  }
  const double* Gsrc = static_cast<const double*>(prm.Gh);
  for (int i = threadIdx.x; i < NP * NP; i += blockDim.x) sG[i] = Gsrc[i];
  __syncthreads();

  TL tl;
  tl.x = lane >> 4;
  tl.hb = hb;
  tl.b = hb % B;
  tl.z = lane & 3;
  tl.nvalid = prm.n;
  tl.sG = sG;
  tl.xch = sx + pix * 16;
  tl.wx = sw + pix * TL::R * TL::WX;
  ipm_pixel<TL, MODE, CONS>(prm, p, p < prm.P, tl);
}

// wavefronts per workgroup and per SIMD by shape (LM_RC_WAVES > 0 overrides
// the latter, for comparisons)
#ifndef LM_RC_WAVES
#define LM_RC_WAVES 0
#endif
template <int T, int B>
constexpr int kRcWpb = 4;
template <int T, int B>
constexpr int kRcWaves = LM_RC_WAVES > 0 ? LM_RC_WAVES : (T / B <= 4 ? 2 : 1);
template <int T, int B>
constexpr int kRcPixels = kRcWpb<T, B> * (4 / B);  // pixels per workgroup

template <int T, int B, int MODE, int CONS>
__global__ __launch_bounds__((64 * kRcWpb<T, B>), (kRcWaves<T, B>)) void ipm_rc_kernel(IpmParams prm) {
  ipm_rc_body<T, B, MODE, CONS, kRcWpb<T, B>>(prm, blockIdx.x);
}

template <int T, int B, int MODE, int CONS>
__global__ __launch_bounds__((64 * kRcWpb<T, B>), (kRcWaves<T, B>)) void ipm_rc_batch_kernel(
    const IpmParams* __restrict__ jobs, const int64_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const IpmParams prm = uniform_copy(jobs + j);
  ipm_rc_body<T, B, MODE, CONS, kRcWpb<T, B>>(prm, (int64_t)blockIdx.x - start[j]);
}

template <int T, int B, int MODE, int CONS>
static void launch_rc_m(const IpmParams& p, const IpmBatch* b, hipStream_t st) {
  constexpr int W = kRcWpb<T, B>, PB = kRcPixels<T, B>;
  if (b)
    hipLaunchKernelGGL((ipm_rc_batch_kernel<T, B, MODE, CONS>), dim3((unsigned)b->blocks), dim3(64 * W), 0, st,
                       b->jobs, b->start, b->njobs);
  else
    hipLaunchKernelGGL((ipm_rc_kernel<T, B, MODE, CONS>), dim3((unsigned)((p.P + PB - 1) / PB)), dim3(64 * W), 0,
                       st, p);
}

template <int T, int B, int CONS>
static int launch_rc_c(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  if (mode == kFull)
    launch_rc_m<T, B, kFull, CONS>(p, b, st);
  else if (mode == kStage2)
    launch_rc_m<T, B, kStage2, CONS>(p, b, st);
  else if (mode == kRetry)
    launch_rc_m<T, B, kRetry, CONS>(p, b, st);
  else
    return -5;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// b == nullptr: one cube described by p; else the jobs of b (p only gives
// the constraint option, shared by every job).  Always the stable
// factorisation.
template <int T, int B>
static int launch_rc(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  switch (p.constraint) {
    case kSto: return launch_rc_c<T, B, kSto>(p, b, mode, st);
    case kSlo: return launch_rc_c<T, B, kSlo>(p, b, mode, st);
    case kPos: return launch_rc_c<T, B, kPos>(p, b, mode, st);
  }
  return -1;
}

#if defined(LM_RC_T) && defined(LM_RC_B)
#define LM_RENTRY2(t, b) ipm_rc_entry_##t##_##b
#define LM_RENTRY(t, b) LM_RENTRY2(t, b)
int LM_RENTRY(LM_RC_T, LM_RC_B)(const IpmParams& p, const IpmBatch* b, int mode, hipStream_t st) {
  return launch_rc<LM_RC_T, LM_RC_B>(p, b, mode, st);
}
#endif

}  // namespace lm
