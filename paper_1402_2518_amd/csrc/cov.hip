// cov.hip -- coefficient covariance "provided by the Hessian" (end of Sec. 2.3).
//
// For pixel p the solver leaves a per-coefficient diagonal d_i:
//   certified solution: d_i = 0 on the free set, +inf on the active set;
//   otherwise:          d_i = lambda_i / a_i at the last interior iterate.
// With I = {i : d_i finite} the covariance is
//   Cov_II = (s_p^2 / gamma) * [K^{-1}]_II,   K = [[Gh_II + diag(d_I), 1], [1^T, 0]],
// and zero outside I; the upper-left block of K^{-1} equals
// H^{-1} - u u^T / 1^T u with H = Gh_II + diag(d_I), u = H^{-1} 1.
// K is inverted by the symmetric sweep operator (pivots in order, the border
// last; the sweep keeps the matrix symmetric, so the pivot column doubles as
// the pivot row); afterwards the matrix holds -K^{-1}.
//
// Three paths by the size q = |I| + 1 of K.  cov_small_kernel (q <= 16) and
// cov_mid_kernel (16 < q <= 32) put 16 lanes (one DPP row) on a pixel, four
// pixels per wavefront; lane t keeps rows t (and t + 16) of K in registers,
// and each pivot row reaches the other lanes by DPP row broadcasts, so the
// sweep has no memory traffic.  Pivots and columns stop at the largest border
// in the wavefront.  The output is written one row of the pixel's block at a
// time with consecutive lanes on consecutive addresses; by symmetry an entry
// (r, c) is read from the lane that owns row c.  cov_small_kernel sees every
// pixel and flags the larger ones, cov_mid_kernel packs the flagged pixels
// four to a wavefront, and cov_big_kernel sweeps what is left (q > 32) one
// wavefront per pixel with K in LDS.  Noisy mixtures of a few spectra have
// free sets of about 5 to 20 coefficients.
#include "common.h"
#include "kernels.h"

namespace lm {

namespace {

// number of set bits of (lo, hi) strictly below position i (0 <= i < 128)
__device__ __forceinline__ int rank128(uint64_t lo, uint64_t hi, int i) {
  if (i < 64) return __builtin_popcountll(lo & ((1ull << i) - 1ull));
  return __builtin_popcountll(lo) + __builtin_popcountll(hi & ((1ull << (i - 64)) - 1ull));
}
__device__ __forceinline__ bool bit128(uint64_t lo, uint64_t hi, int i) {
  return i < 64 ? ((lo >> i) & 1ull) != 0 : ((hi >> (i - 64)) & 1ull) != 0;
}

// value of lane K of this lane's 16-lane row
template <int K>
__device__ __forceinline__ double rowbcast(double v) {
  return dpp<0x150 + K>(v);
}

// r += be * (r on lane K of this lane's 16-lane row): one 64-bit FMA with a
// row broadcast on its first source.  The compiler does not see the DPP
// inside the asm, so the asm brings the two wait states a DPP read needs
// after a vector write of its source register.  A scalar write of EXEC needs
// five; the sweeps change EXEC only outside their pivot loops (the guards
// there are scalar branches), which a test checks on the built code.
template <int K>
__device__ __forceinline__ void fmac_bcast(double& r, double be) {
  asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
               : "+v"(r)
               : "v"(be), "i"(K));
}
// r += be * (src on lane K of this lane's 16-lane row)
template <int K>
__device__ __forceinline__ void fmac_bcast_from(double& r, double src, double be) {
  asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
               : "+v"(r)
               : "v"(src), "v"(be), "i"(K));
}

}  // namespace

// Covariance of pixel p on the calling 16-lane row (live = the row has a
// pixel).  Every lane of the wavefront must call it together (ballots); the
// rows' pixels are independent.  Writes big[p] = 0 when |I| + 1 <= Q (done),
// 1 otherwise (left for a larger path).  dv, idx: this row's LDS scratch of
// Q entries each.
template <int Q>
__device__ __forceinline__ void cov_group(int n, int64_t p, bool live, const double* __restrict__ Gh, int ldg,
                                          const double* __restrict__ dcov, const double* __restrict__ corner,
                                          const float* __restrict__ sigma,
                                          double gamma, const uint8_t* __restrict__ status, int layout,
                                          double* __restrict__ out, uint8_t* __restrict__ big, double* dv,
                                          int* idx) {
  static_assert(Q == 16 || Q == 32, "one or two rows of K per lane");
  constexpr int H = Q / 16;           // rows of K per lane: t and t + 16
  const int lane = threadIdx.x & 63;
  const int t = lane & 15;            // lane within the pixel's row
  const int gb = lane & 48;           // first lane of the row in the wavefront
  const int ns = (n + 15) >> 4;  // 16-column slots of a row of the output

  // included set: bit i of (mlo, mhi), the same on the 16 lanes of a pixel
  uint64_t mlo = 0, mhi = 0;
  for (int s = 0; s < ns; ++s) {
    const int i = 16 * s + t;
    const double d = (live && i < n) ? dcov[p * n + i] : 0.0;
    const bool inc = live && i < n && isfin(d);
    const uint64_t bits = (__builtin_amdgcn_ballot_w64(inc) >> gb) & 0xFFFFull;
    if (s < 4) mlo |= bits << (16 * s);
    else mhi |= bits << (16 * (s - 4));
    if (inc) {
      const int r = rank128(mlo, mhi, i);
      if (r < Q) {
        idx[r] = i;
        dv[r] = d;
      }
    }
  }
  const int m = __builtin_popcountll(mlo) + __builtin_popcountll(mhi);
  // sum row: present unless the corner is -inf (no sum constraint binding)
  const double cval = live ? corner[p] : 0.0;
  const int bord = cval == -(double)INFINITY ? 0 : 1;
  const int q = m + bord;
  const bool small = live && q <= Q;
  if (live && t == 0) big[p] = small ? 0 : 1;
  lds_sync();

  // rows t + 16 h of K; padding beyond the border is the identity
  double R[H][Q];
  static_for<0, H>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    const int row = t + 16 * h;
    const int ir = (small && row < m) ? idx[row] : 0;
    static_for<0, Q>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      double v;
      if (!small) v = (row == c) ? 1.0 : 0.0;
      else if (row < m && c < m) v = Gh[(int64_t)ir * ldg + idx[c]] + (row == c ? dv[row] : 0.0);
      else if (bord && row <= m && c <= m) v = (row == c) ? cval : 1.0;
      else v = (row == c) ? 1.0 : 0.0;
      R[h][c] = v;
    });
  });

  // sweep pivots 0 .. border of every pixel of the wavefront (a pivot past a
  // pixel's border meets an identity row and leaves its border block alone);
  // columns past the largest border are untouched identity and are skipped
  int mmax = small ? q - 1 : -1;
  mmax = max(mmax, __shfl_xor(mmax, 16));
  mmax = max(mmax, __shfl_xor(mmax, 32));
  // the same on every lane: keep it scalar, so the guards below are scalar
  // branches rather than per-lane masks
  mmax = __builtin_amdgcn_readfirstlane(mmax);
  bool singular = false;
  // Each row keeps the scale of its own pivot step deferred: at pivot k the
  // pivot row is left as it is (its pivot entry becomes -1) and rs = 1/akk
  // is kept for it; the sweep is linear in each row, so the later steps
  // apply to the unscaled row unchanged, and every row is scaled once at the
  // end.  Each entry update is then one FMA that reads the pivot row's entry
  // from lane kt of the DPP row (fmac_bcast).
  double rs0 = 1.0, rs1 = 1.0;  // deferred scales of rows t and t + 16
  static_for<0, Q>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    constexpr int kh = k / 16, kt = k % 16;
    if (k <= mmax) {
      const double akk = rowbcast<kt>(R[kh][k]);
      if (!(akk != 0.0) || akk != akk) singular = true;
      const double r = 1.0 / akk;
      // rows other than the pivot lose f = R_k / akk times the pivot row
      // (be = -f); the pivot column becomes f (-1 on the deferred pivot row)
      const bool p0 = t == k, p1 = H == 2 && t + 16 == k;
      const double f0 = R[0][k] * r;
      const double f1 = H == 2 ? R[H - 1][k] * r : 0.0;
      const double be0 = p0 ? 0.0 : -f0, be1 = p1 ? 0.0 : -f1;
      rs0 = p0 ? r : rs0;
      rs1 = p1 ? r : rs1;
      static_for<0, Q>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        if (j <= mmax) {
          if constexpr (j != k) {
            // the pivot row's entry is not changed by the step (be = 0 on
            // its lane), so the order of the rows does not matter
            if constexpr (kh == 0) fmac_bcast<kt>(R[0][j], be0);
            else fmac_bcast_from<kt>(R[0][j], R[kh][j], be0);
            if constexpr (H == 2) {
              if constexpr (kh == 1) fmac_bcast<kt>(R[H - 1][j], be1);
              else fmac_bcast_from<kt>(R[H - 1][j], R[0][j], be1);
            }
          }
        }
      });
      R[0][k] = p0 ? -1.0 : f0;
      if constexpr (H == 2) R[H - 1][k] = p1 ? -1.0 : f1;
    }
  });
  static_for<0, Q>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    R[0][c] *= rs0;
    if constexpr (H == 2) R[H - 1][c] *= rs1;
  });
  if (!small) return;

  // output; entry (r, c) of -K^{-1} is R[c / 16][r] on lane c % 16 (symmetry)
  bool bad = status && (status[p] & (kPxNonfinite | kPxBadSigma));
  const double s = sigma ? (double)sigma[p] : 1.0;
  if (!(s > 0.0) || !isfin(s)) bad = true;
  const bool nanout = bad || singular;
  const double qnan = __builtin_nan("");
  const double scale = -s * s / gamma;
  const int64_t per = layout == 1 ? (int64_t)n * n : (layout == 2 ? (int64_t)n * (n + 1) / 2 : n);
  double* o = out + p * per;
  constexpr int NS = (128 + 15) / 16;  // column slots of the widest library
  int rj[NS];
  bool inj[NS];
  static_for<0, NS>([&](auto ss) {
    constexpr int sl = decltype(ss)::value;
    const int j = 16 * sl + t;
    inj[sl] = j < n && bit128(mlo, mhi, j);
    rj[sl] = inj[sl] ? rank128(mlo, mhi, j) : 0;
  });
  if (layout == 3) {
    // diagonal: entry (r, r) sits on lane r % 16; broadcast it and let the
    // column with position r keep it
    double dgv[NS];
    static_for<0, NS>([&](auto ss) { dgv[decltype(ss)::value] = 0.0; });
    static_for<0, Q>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      if (r < m) {
        const double kd = rowbcast<r % 16>(R[r / 16][r]);
        static_for<0, NS>([&](auto ss) {
          constexpr int sl = decltype(ss)::value;
          dgv[sl] = (inj[sl] && rj[sl] == r) ? kd : dgv[sl];
        });
      }
    });
    static_for<0, NS>([&](auto ss) {
      constexpr int sl = decltype(ss)::value;
      const int j = 16 * sl + t;
      if (j < n) o[j] = nanout ? qnan : (inj[sl] ? scale * dgv[sl] : 0.0);
    });
    return;
  }
  const bool full = layout == 1;
  // rows outside I are zero
  for (int i = 0; i < n; ++i) {
    if (bit128(mlo, mhi, i)) continue;
    const int64_t row = full ? (int64_t)i * n : (int64_t)i * (i + 1) / 2;
    const int len = full ? n : i + 1;
    for (int sl = 0; 16 * sl < len; ++sl) {
      const int j = 16 * sl + t;
      if (j < len) o[row + j] = nanout ? qnan : 0.0;
    }
  }
  // rows in I, by position r (compile-time, so R[.][r] is a register)
  static_for<0, Q>([&](auto rr) {
    constexpr int r = decltype(rr)::value;
    if (r < m) {
      const int i = idx[r];
      const int64_t row = full ? (int64_t)i * n : (int64_t)i * (i + 1) / 2;
      const int len = full ? n : i + 1;
      static_for<0, NS>([&](auto ss) {
        constexpr int sl = decltype(ss)::value;
        if (16 * sl < len) {
          const int j = 16 * sl + t;
          double v = __shfl(R[0][r], gb + (rj[sl] & 15));
          if constexpr (H == 2) {
            const double v1 = __shfl(R[1][r], gb + (rj[sl] & 15));
            v = rj[sl] >= 16 ? v1 : v;
          }
          if (j < len) o[row + j] = nanout ? qnan : (inj[sl] ? scale * v : 0.0);
        }
      });
    }
  });
}

// every pixel; those with |I| + 1 > 16 are flagged for the next paths
__device__ __forceinline__ void cov_small_body(const CovJob& J, int64_t blk) {
  __shared__ double dvs[16][16];
  __shared__ int idxs[16][16];
  const int g = threadIdx.x >> 4;
  const int64_t p = blk * 16 + g;
  cov_group<16>(J.n, p, p < J.P, J.Gh, J.ldg, J.dcov, J.corner, J.sigma, J.gamma, J.status, J.layout, J.out, J.big,
                dvs[g], idxs[g]);
}

__global__ __launch_bounds__(256) void cov_small_kernel(CovJob J) { cov_small_body(J, blockIdx.x); }

__global__ __launch_bounds__(256) void cov_small_batch_kernel(const CovJob* __restrict__ jobs,
                                                              const int64_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const CovJob J = uniform_copy(jobs + j);
  cov_small_body(J, (int64_t)blockIdx.x - start[j]);
}

// flagged pixels only, four per wavefront: the wavefront takes the 64 flags
// of the chunk at base and hands the set ones to its rows in order
__device__ __forceinline__ void cov_mid_chunk(const CovJob& J, int64_t base, double (*dvs)[32], int (*idxs)[32]) {
  const int lane = threadIdx.x & 63;
  const int g = threadIdx.x >> 4, gi = (lane >> 4) & 3;
  const bool flagged = base + lane < J.P && J.big[base + lane] != 0;
  uint64_t todo = __builtin_amdgcn_ballot_w64(flagged);
  while (todo) {
    uint64_t rest = todo;
    for (int k = 0; k < gi; ++k) rest &= rest - 1ull;
    const bool has = rest != 0ull;
    const int64_t p = base + (has ? __builtin_ctzll(rest) : 0);
    cov_group<32>(J.n, p, has, J.Gh, J.ldg, J.dcov, J.corner, J.sigma, J.gamma, J.status, J.layout, J.out, J.big,
                  dvs[g], idxs[g]);
    for (int k = 0; k < 4; ++k) todo &= todo - 1ull;
  }
}

__global__ __launch_bounds__(256, 2) void cov_mid_kernel(CovJob J) {
  __shared__ double dvs[16][32];
  __shared__ int idxs[16][32];
  const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * wpb;
  for (int64_t base = ((int64_t)blockIdx.x * wpb + wave) * 64; base < J.P; base += nw * 64)
    cov_mid_chunk(J, base, dvs, idxs);
}

// chunks u in [0, start[njobs]) over the jobs, 64 pixels each
__global__ __launch_bounds__(256, 2) void cov_mid_batch_kernel(const CovJob* __restrict__ jobs,
                                                               const int64_t* __restrict__ start, int njobs) {
  __shared__ double dvs[16][32];
  __shared__ int idxs[16][32];
  const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * wpb, total = start[njobs];
  for (int64_t u = (int64_t)blockIdx.x * wpb + wave; u < total; u += nw) {
    const int j = job_of(start, njobs, u);
    const CovJob J = uniform_copy(jobs + j);
    cov_mid_chunk(J, (u - start[j]) * 64, dvs, idxs);
  }
}

// one wavefront per pixel in LDS for what the register paths left: the
// wavefront's slot holds a qcap x qcap matrix and three qcap vectors
__device__ __forceinline__ void cov_big_chunk(const CovJob& J, int64_t base, double* slot, int qcap) {
  const int lane = threadIdx.x & 63;
  const int n = J.n, ldg = J.ldg, layout = J.layout;
  const double* __restrict__ Gh = J.Gh;
  const double* __restrict__ dcov = J.dcov;
  double* __restrict__ out = J.out;
  double* A = slot;                  // q x q, column-major (ld = q)
  double* colk = A + qcap * qcap;    // pivot column before the step
  double* dv = colk + qcap;          // d of the included indices, by position
  int* idx = (int*)(dv + qcap);      // included index at each position
  const double qnan = __builtin_nan("");
  const int64_t per = layout == 1 ? (int64_t)n * n : (layout == 2 ? (int64_t)n * (n + 1) / 2 : n);
  const int j0 = lane, j1 = lane + 64;  // the output columns of this lane
  {
    const bool flagged = base + lane < J.P && J.big[base + lane];
    uint64_t todo = __builtin_amdgcn_ballot_w64(flagged);
    while (todo) {
      const int64_t p = base + __builtin_ctzll(todo);
      todo &= todo - 1ull;
      const double d0 = j0 < n ? dcov[p * n + j0] : 0.0;
      const double d1 = j1 < n ? dcov[p * n + j1] : 0.0;
      double* o = out + p * per;
      bool bad = J.status && (J.status[p] & (kPxNonfinite | kPxBadSigma));
      const double s = J.sigma ? (double)J.sigma[p] : 1.0;
      if (!(s > 0.0) || !isfin(s)) bad = true;
      const bool in0 = j0 < n && isfin(d0), in1 = j1 < n && isfin(d1);
      const uint64_t lo = __builtin_amdgcn_ballot_w64(in0), hi = __builtin_amdgcn_ballot_w64(in1);
      const int m = __builtin_popcountll(lo) + __builtin_popcountll(hi);
      const double cval = J.corner[p];
      const int bord = cval == -(double)INFINITY ? 0 : 1;
      const int q = m + bord;
      const int r0 = rank128(lo, hi, j0), r1 = rank128(lo, hi, j1);
      if (in0) {
        idx[r0] = j0;
        dv[r0] = d0;
      }
      if (in1) {
        idx[r1] = j1;
        dv[r1] = d1;
      }
      lds_sync();
      // K into LDS; element e = a + q b walks by 64 with an incremental (a, b)
      const int qq = q * q, da = 64 % q, db = 64 / q;
      const int a0 = lane % q, b0 = lane / q;
      {
        int a = a0, b = b0;
        for (int e = lane; e < qq; e += 64) {
          double v;
          if (a < m && b < m) {
            v = Gh[(int64_t)idx[a] * ldg + idx[b]];
            if (a == b) v += dv[a];
          } else {
            v = (a == m && b == m) ? cval : 1.0;  // border row and corner
          }
          A[e] = v;
          a += da;
          b += db;
          if (a >= q) {
            a -= q;
            ++b;
          }
        }
      }
      lds_sync();
      bool singular = false;
      for (int k = 0; k < q; ++k) {
        for (int i = lane; i < q; i += 64) colk[i] = A[k * q + i];
        lds_sync();
        const double akk = colk[k];
        if (!(akk != 0.0) || akk != akk) singular = true;
        const double r = 1.0 / akk;
        int a = a0, b = b0;
        for (int e = lane; e < qq; e += 64) {
          const double aik = colk[a], akj = colk[b];
          double v;
          if (a == k && b == k) v = -r;
          else if (a == k) v = akj * r;
          else if (b == k) v = aik * r;
          else v = A[e] - aik * akj * r;
          A[e] = v;
          a += da;
          b += db;
          if (a >= q) {
            a -= q;
            ++b;
          }
        }
        lds_sync();
      }
      const bool nanout = bad || singular;
      const double scale = -s * s / J.gamma;
      if (layout == 3) {
        if (j0 < n) o[j0] = nanout ? qnan : (in0 ? scale * A[r0 * q + r0] : 0.0);
        if (j1 < n) o[j1] = nanout ? qnan : (in1 ? scale * A[r1 * q + r1] : 0.0);
      } else {
        int64_t row = 0;  // offset of row i in the pixel's block
        for (int i = 0; i < n; ++i) {
          const bool ini = bit128(lo, hi, i);
          const int ri = ini ? rank128(lo, hi, i) : 0;
          const int len = layout == 1 ? n : i + 1;
          if (j0 < len) o[row + j0] = nanout ? qnan : ((ini && in0) ? scale * A[r0 * q + ri] : 0.0);
          if (j1 < len) o[row + j1] = nanout ? qnan : ((ini && in1) ? scale * A[r1 * q + ri] : 0.0);
          row += len;
        }
      }
      lds_sync();
    }
  }
}

__global__ __launch_bounds__(256) void cov_big_kernel(CovJob J) {
  extern __shared__ double smem[];
  const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const int qcap = J.n + 1;
  double* slot = smem + wave * (qcap * qcap + 4 * qcap);
  const int64_t nw = (int64_t)gridDim.x * wpb;
  for (int64_t base = ((int64_t)blockIdx.x * wpb + wave) * 64; base < J.P; base += nw * 64)
    cov_big_chunk(J, base, slot, qcap);
}

__global__ __launch_bounds__(256) void cov_big_batch_kernel(const CovJob* __restrict__ jobs,
                                                            const int64_t* __restrict__ start, int njobs, int qcap) {
  extern __shared__ double smem[];
  const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  double* slot = smem + wave * (qcap * qcap + 4 * qcap);
  const int64_t nw = (int64_t)gridDim.x * wpb, total = start[njobs];
  for (int64_t u = (int64_t)blockIdx.x * wpb + wave; u < total; u += nw) {
    const int j = job_of(start, njobs, u);
    const CovJob J = uniform_copy(jobs + j);
    cov_big_chunk(J, (u - start[j]) * 64, slot, qcap);
  }
}

// LDS bytes of one wavefront of the big path for borders up to qcap
static size_t big_slot_bytes(int qcap) { return sizeof(double) * (size_t)(qcap * qcap + 4 * qcap); }

// wavefronts per workgroup of the big path: up to 4, at most 64 KB per workgroup
static int big_waves(int qcap) {
  int wpb = (int)((64 * 1024) / big_slot_bytes(qcap));
  if (wpb > 4) wpb = 4;
  if (wpb < 1) wpb = 1;
  return wpb;
}

int launch_cov(int n, int64_t P, const double* Gh, int ldg, const double* dcov, const double* corner,
               const float* sigma, double gamma, const uint8_t* status, int layout, double* out, uint8_t* big,
               hipStream_t st) {
  if (P <= 0) return 0;
  if (n < 1 || n > 128) return -5;
  const CovJob J{n, P, Gh, ldg, dcov, corner, sigma, gamma, status, layout, out, big};
  const int64_t sblocks = (P + 15) / 16;
  hipLaunchKernelGGL(cov_small_kernel, dim3((unsigned)sblocks), dim3(256), 0, st, J);
  if (hipGetLastError() != hipSuccess) return -3;
  if (n + 1 <= 16) return 0;  // every pixel fit the first path
  int64_t mblocks = (P + 4 * 64 - 1) / (4 * 64);
  if (mblocks > 4096) mblocks = 4096;
  hipLaunchKernelGGL(cov_mid_kernel, dim3((unsigned)mblocks), dim3(256), 0, st, J);
  if (hipGetLastError() != hipSuccess) return -3;
  if (n + 1 <= 32) return 0;
  const int qcap = n + 1, wpb = big_waves(qcap);
  if (big_slot_bytes(qcap) * wpb > 160 * 1024) return -5;
  int64_t blocks = (P + 64 * wpb - 1) / (64 * wpb);  // one 64-pixel chunk per wavefront
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(cov_big_kernel, dim3((unsigned)blocks), dim3(64 * wpb), wpb * big_slot_bytes(qcap), st, J);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_cov_batch(const CovBatch& small, const CovBatch& mid, const CovBatch& big, hipStream_t st) {
  if (small.njobs > 0 && small.units > 0) {
    hipLaunchKernelGGL(cov_small_batch_kernel, dim3((unsigned)small.units), dim3(256), 0, st, small.jobs, small.start,
                       small.njobs);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  if (mid.njobs > 0 && mid.units > 0) {
    int64_t mblocks = (mid.units + 3) / 4;
    if (mblocks > 4096) mblocks = 4096;
    hipLaunchKernelGGL(cov_mid_batch_kernel, dim3((unsigned)mblocks), dim3(256), 0, st, mid.jobs, mid.start, mid.njobs);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  if (big.njobs > 0 && big.units > 0) {
    const int qcap = big.qcap, wpb = big_waves(qcap);
    if (qcap < 2 || qcap > 129 || big_slot_bytes(qcap) * wpb > 160 * 1024) return -5;
    int64_t blocks = (big.units + wpb - 1) / wpb;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(cov_big_batch_kernel, dim3((unsigned)blocks), dim3(64 * wpb), wpb * big_slot_bytes(qcap), st,
                       big.jobs, big.start, big.njobs, qcap);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  return 0;
}

}  // namespace lm
