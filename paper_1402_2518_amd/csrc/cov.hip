// cov.hip -- coefficient covariance "provided by the Hessian" (end of Sec. 2.3).
//
// For pixel p the solver leaves a per-coefficient diagonal d_i:
//   certified solution: d_i = 0 on the free set, +inf on the active set;
//   otherwise:          d_i = lambda_i / a_i at the last interior iterate.
// With I = {i : d_i finite} the covariance is
//   Cov_II = (s_p^2 / gamma) * [K^{-1}]_II,   K = [[Gh_II + diag(d_I), 1], [1^T, 0]],
// and zero outside I; the upper-left block of K^{-1} equals
// H^{-1} - u u^T / 1^T u with H = Gh_II + diag(d_I), u = H^{-1} 1.
// K is inverted in LDS by the symmetric sweep operator (pivots in order, the
// border last; the sweep keeps the matrix symmetric, so the pivot column
// doubles as the pivot row).  One wavefront per pixel, four per workgroup;
// the output block of each pixel is written with consecutive lanes on
// consecutive addresses.
#include "common.h"
#include "kernels.h"

namespace lm {

__global__ __launch_bounds__(256) void cov_kernel(int n, int64_t P, const double* __restrict__ Gh, int ldg,
                                                  const double* __restrict__ dcov,
                                                  const float* __restrict__ sigma, double gamma,
                                                  const uint8_t* __restrict__ status, int layout,
                                                  double* __restrict__ out) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q_max = n + 1;
  const int stride = q_max * q_max + q_max + q_max;  // doubles per wave (ints packed after)
  double* A = smem + wave * stride;                  // q x q, column-major
  double* colk = A + q_max * q_max;                  // pivot column before the step
  int* pos = (int*)(colk + q_max);                   // n: position of i in I, or -1
  int* idx = pos + n;                                // positions -> index
  const double qnan = __builtin_nan("");
  const int64_t per = layout == 1 ? (int64_t)n * n : (layout == 2 ? (int64_t)n * (n + 1) / 2 : n);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  const int wpb = blockDim.x >> 6;
  for (int64_t p = (int64_t)blockIdx.x * wpb + wave; p < P; p += (int64_t)gridDim.x * wpb) {
    const double* d = dcov + p * n;
    double* o = out + p * per;
    bool bad = status && (status[p] & (kPxNonfinite | kPxBadSigma));
    const double s = sigma ? (double)sigma[p] : 1.0;
    if (!(s > 0.0) || !isfin(s)) bad = true;
    // included set by ballot compaction
    int m = 0;
    for (int base = 0; base < n; base += 64) {
      const int i = base + lane;
      const double di = i < n ? d[i] : 0.0;
      const bool inc = i < n && isfin(di);
      const uint64_t mask = __builtin_amdgcn_ballot_w64(inc);
      const int at = m + __builtin_popcountll(mask & below);
      if (i < n) pos[i] = inc ? at : -1;
      if (inc) idx[at] = i;
      m += __builtin_popcountll(mask);
    }
    const int q = m + 1;
    lds_sync();
    for (int e = lane; e < q * q; e += 64) {
      const int i = e % q, j = e / q;
      double v;
      if (i < m && j < m) {
        v = Gh[(int64_t)idx[i] * ldg + idx[j]];
        if (i == j) v += d[idx[i]];
      } else {
        v = (i == m && j == m) ? 0.0 : 1.0;
      }
      A[e] = v;
    }
    lds_sync();
    // sweep every pivot: afterwards A = -K^{-1}
    bool singular = false;
    for (int k = 0; k < q; ++k) {
      for (int i = lane; i < q; i += 64) colk[i] = A[k * q + i];
      lds_sync();
      const double akk = colk[k];
      if (!(akk != 0.0) || akk != akk) singular = true;
      const double r = 1.0 / akk;
      for (int e = lane; e < q * q; e += 64) {
        const int i = e % q, j = e / q;
        const double aik = colk[i], akj = colk[j];
        double v;
        if (i == k && j == k) v = -r;
        else if (i == k) v = akj * r;
        else if (j == k) v = aik * r;
        else v = A[e] - aik * akj * r;
        A[e] = v;
      }
      lds_sync();
    }
    const bool nanout = bad || singular;
    const double scale = -s * s / gamma;
    if (layout == 3) {
      for (int i = lane; i < n; i += 64) {
        const int pi = pos[i];
        o[i] = nanout ? qnan : (pi < 0 ? 0.0 : scale * A[pi * q + pi]);
      }
    } else if (layout == 1) {
      for (int e = lane; e < n * n; e += 64) {
        const int i = e / n, j = e - (e / n) * n;
        const int pi = pos[i], pj = pos[j];
        o[e] = nanout ? qnan : ((pi < 0 || pj < 0) ? 0.0 : scale * A[pj * q + pi]);
      }
    } else {
      const int tot = n * (n + 1) / 2;
      for (int e = lane; e < tot; e += 64) {
        int i = (int)((__builtin_sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (i * (i + 1) / 2 > e) --i;
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        const int j = e - i * (i + 1) / 2;
        const int pi = pos[i], pj = pos[j];
        o[e] = nanout ? qnan : ((pi < 0 || pj < 0) ? 0.0 : scale * A[pj * q + pi]);
      }
    }
    lds_sync();
  }
}

int launch_cov(int n, int64_t P, const double* Gh, int ldg, const double* dcov, const float* sigma,
               double gamma, const uint8_t* status, const double* out_a, int layout, double* out,
               hipStream_t st) {
  (void)out_a;
  if (P <= 0) return 0;
  const int q_max = n + 1;
  const size_t per_wave = sizeof(double) * (size_t)(q_max * q_max + 2 * q_max);
  int wpb = (int)((160 * 1024) / per_wave);
  if (wpb > 4) wpb = 4;
  if (wpb < 1) return -5;
  int64_t blocks = (P + wpb - 1) / wpb;
  if (blocks > 32768) blocks = 32768;
  hipLaunchKernelGGL(cov_kernel, dim3((unsigned)blocks), dim3(64 * wpb), wpb * per_wave, st, n, P, Gh, ldg, dcov,
                     sigma, gamma, status, layout, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lm
