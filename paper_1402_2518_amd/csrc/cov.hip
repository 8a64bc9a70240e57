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
// border last), one wavefront per pixel, one matrix column per lane.
#include "common.h"
#include "kernels.h"

namespace lm {

__global__ __launch_bounds__(64) void cov_kernel(int n, int64_t P, const double* __restrict__ Gh, int ldg,
                                                 const double* __restrict__ dcov,
                                                 const float* __restrict__ sigma, double gamma,
                                                 const uint8_t* __restrict__ status, int layout,
                                                 double* __restrict__ out) {
  extern __shared__ double smem[];
  const int q_max = n + 1;
  double* A = smem;                        // q x q, column-major
  double* colk = A + q_max * q_max;        // pivot column before the step
  int* pos = (int*)(colk + q_max);         // n: position of i in I, or -1
  int* idx = pos + n;                      // q: index of each position
  const int lane = threadIdx.x;
  const double qnan = __builtin_nan("");
  const int64_t per = layout == 1 ? (int64_t)n * n : (layout == 2 ? (int64_t)n * (n + 1) / 2 : n);

  for (int64_t p = blockIdx.x; p < P; p += gridDim.x) {
    const double* d = dcov + p * n;
    double* o = out + p * per;
    // included set (prefix count, done by lane 0: n <= 128)
    bool bad = status && (status[p] & (kPxNonfinite | kPxBadSigma));
    const double s = sigma ? (double)sigma[p] : 1.0;
    if (!(s > 0.0) || !(s == s) || s - s != 0.0) bad = true;
    if (lane == 0) {
      int m = 0;
      for (int i = 0; i < n; ++i) {
        const double di = d[i];
        const bool inc = (di == di) && (di - di == 0.0);
        pos[i] = inc ? m : -1;
        if (inc) idx[m++] = i;
      }
      idx[n] = m;  // count
    }
    __syncthreads();
    const int m = idx[n];
    const int q = m + 1;
    // K, column-major
    for (int j = lane; j < q; j += 64) {
      for (int i = 0; i < q; ++i) {
        double v;
        if (i < m && j < m) {
          v = Gh[(int64_t)idx[i] * ldg + idx[j]];
          if (i == j) v += d[idx[i]];
        } else if (i == m && j == m) {
          v = 0.0;
        } else {
          v = 1.0;
        }
        A[j * q + i] = v;
      }
    }
    __syncthreads();
    // sweep every pivot: afterwards A = -K^{-1}
    bool singular = false;
    for (int k = 0; k < q; ++k) {
      for (int i = lane; i < q; i += 64) colk[i] = A[k * q + i];
      __syncthreads();
      const double akk = colk[k];
      if (!(akk != 0.0) || akk != akk) singular = true;
      const double r = 1.0 / akk;
      for (int j = lane; j < q; j += 64) {
        const double akj = A[j * q + k];
        for (int i = 0; i < q; ++i) {
          const double aik = colk[i];
          const double aij = A[j * q + i];
          double v;
          if (i == k && j == k) v = -r;
          else if (i == k) v = akj * r;
          else if (j == k) v = aik * r;
          else v = aij - aik * akj * r;
          A[j * q + i] = v;
        }
      }
      __syncthreads();
    }
    const double scale = s * s / gamma;
    // outputs, rows written by consecutive lanes
    if (layout == 3) {
      for (int i = lane; i < n; i += 64) {
        const int pi = pos[i];
        o[i] = (bad || singular) ? qnan : (pi < 0 ? 0.0 : -scale * A[pi * q + pi]);
      }
    } else {
      for (int i = 0; i < n; ++i) {
        const int pi = pos[i];
        const int jend = layout == 1 ? n : i + 1;
        double* orow = layout == 1 ? o + (int64_t)i * n : o + (int64_t)i * (i + 1) / 2;
        for (int j = lane; j < jend; j += 64) {
          const int pj = pos[j];
          double v = (pi < 0 || pj < 0) ? 0.0 : -scale * A[pj * q + pi];
          orow[j] = (bad || singular) ? qnan : v;
        }
      }
    }
    __syncthreads();
  }
}

int launch_cov(int n, int64_t P, const double* Gh, int ldg, const double* dcov, const float* sigma,
               double gamma, const uint8_t* status, const double* out_a, int layout, double* out,
               hipStream_t st) {
  (void)out_a;
  if (P <= 0) return 0;
  const size_t lds = sizeof(double) * ((size_t)(n + 1) * (n + 1) + (n + 1)) + sizeof(int) * (size_t)(2 * n + 1);
  const int64_t want = P < 4096 * 16 ? P : 4096 * 16;
  hipLaunchKernelGGL(cov_kernel, dim3((unsigned)want), dim3(64), lds, st, n, P, Gh, ldg, dcov, sigma,
                     gamma, status, layout, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lm
