// detect.hip -- detection post-processing of unmixing results and the
// restriction of a pixel to chosen spectra (second pass).
//
//   * RMS of each pixel's fit, the root mean square over the L channels of
//     the residual y - a S in reflectance units (Sec. 3.1), computed from the
//     residual itself: a pixel per 16-lane group, its coefficients staged in
//     LDS, the library read through the L2 cache;
//   * 1-sigma error of each coefficient: square root of the covariance
//     diagonal (end of Sec. 2.3);
//   * the threshold of eq. 8 per endmember from coefficients of pixels where
//     it is known present / absent: two passes over the P x N coefficients
//     (means, then centred second moments), partial sums per workgroup in a
//     fixed order, so the result does not depend on scheduling;
//   * the detection rules of Sec. 4: coefficient above the threshold,
//     1-sigma error below the coefficient, RMS below the noise level;
//   * the second pass of the conclusion (unmix with the detected spectra
//     only): excluded spectra get a projection bh_i = -M with M larger than
//     any multiplier the restricted problem needs, which makes a_i = 0 at the
//     optimum and leaves the other coefficients at the restricted minimiser.
#include "common.h"
#include "kernels.h"

namespace lm {

__global__ __launch_bounds__(256) void sigma1_kernel(int n, int64_t P, const double* __restrict__ cov, int layout,
                                                     double* __restrict__ sigma1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * n) return;
  const int64_t p = t / n;
  const int i = (int)(t - p * n);
  double v;
  if (layout == 1) v = cov[p * n * n + (int64_t)i * n + i];
  else if (layout == 2) v = cov[p * ((int64_t)n * (n + 1) / 2) + (int64_t)i * (i + 1) / 2 + i];
  else v = cov[p * n + i];
  sigma1[t] = v != v ? v : sqrt(fmax(v, 0.0));
}

// 16 pixels per workgroup, one per 16-lane group; lane t takes channels
// t, t + 16, ...
__global__ __launch_bounds__(256) void rms_kernel(int n, int64_t P, int L, const float* __restrict__ Y,
                                                  const double* __restrict__ A, const float* __restrict__ S,
                                                  double* __restrict__ rms) {
  __shared__ double sa[16][128];
  const int g = threadIdx.x >> 4, t = threadIdx.x & 15;
  const int64_t p = (int64_t)blockIdx.x * 16 + g;
  const bool live = p < P;
  for (int i = t; i < n; i += 16) sa[g][i] = live ? A[p * n + i] : 0.0;
  __syncthreads();
  double acc = 0.0;
  if (live) {
    const float* y = Y + p * (int64_t)L;
    for (int l = t; l < L; l += 16) {
      double r = (double)y[l];
      for (int i = 0; i < n; ++i) r = fmaT(-sa[g][i], (double)S[(int64_t)i * L + l], r);
      acc = fmaT(r, r, acc);
    }
  }
  acc = gsum<16>(acc);
  if (live && t == 0) rms[p] = sqrt(acc / L);
}

// Per-column partial sums over a workgroup's rows: class 0 = present,
// class 1 = absent.  pass 0: counts and sums; pass 1: sums of squared
// deviations from the means in mean[2n].
__global__ __launch_bounds__(128) void thr_partial_kernel(int n, int64_t P, int64_t rows_per_block,
                                                          const double* __restrict__ A,
                                                          const uint8_t* __restrict__ present, int pass,
                                                          const double* __restrict__ mean,
                                                          double* __restrict__ part) {
  const int i = threadIdx.x;
  if (i >= n) return;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < P ? r0 + rows_per_block : P;
  double c0 = 0.0, c1 = 0.0, s0 = 0.0, s1 = 0.0;
  const double m0 = pass ? mean[i] : 0.0, m1 = pass ? mean[n + i] : 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double a = A[r * n + i];
    const bool pr = present[r * n + i] != 0;
    if (pass == 0) {
      if (pr) {
        c0 += 1.0;
        s0 += a;
      } else {
        c1 += 1.0;
        s1 += a;
      }
    } else {
      const double d = a - (pr ? m0 : m1);
      if (pr) s0 = fmaT(d, d, s0);
      else s1 = fmaT(d, d, s1);
    }
  }
  double* o = part + (int64_t)blockIdx.x * 4 * n;
  o[i] = c0;
  o[n + i] = c1;
  o[2 * n + i] = s0;
  o[3 * n + i] = s1;
}

// Reduce the partials in workgroup order.  pass 0: counts and means into
// stat[4n] (c0, c1, mean0, mean1); pass 1: the thresholds of eq. 8.
__global__ __launch_bounds__(128) void thr_final_kernel(int n, int blocks, const double* __restrict__ part, int pass,
                                                        double* __restrict__ stat, double* __restrict__ thr) {
  const int i = threadIdx.x;
  if (i >= n) return;
  double c0 = 0.0, c1 = 0.0, s0 = 0.0, s1 = 0.0;
  for (int b = 0; b < blocks; ++b) {
    const double* o = part + (int64_t)b * 4 * n;
    c0 += o[i];
    c1 += o[n + i];
    s0 += o[2 * n + i];
    s1 += o[3 * n + i];
  }
  if (pass == 0) {
    stat[i] = c0;
    stat[n + i] = c1;
    stat[2 * n + i] = c0 > 0.0 ? s0 / c0 : 0.0;
    stat[3 * n + i] = c1 > 0.0 ? s1 / c1 : 0.0;
  } else {
    const double n0 = stat[i], n1 = stat[n + i];
    const double mean0 = stat[2 * n + i], mean1 = stat[3 * n + i];
    thr[i] = (n0 > 0.0 && n1 > 0.0)
                 ? 0.5 * (mean0 - 2.0 * sqrt(s0 / n0) + mean1 + 6.0 * sqrt(s1 / n1))
                 : __builtin_nan("");
  }
}

__global__ __launch_bounds__(256) void detect_kernel(int n, int64_t P, const double* __restrict__ A,
                                                     const double* __restrict__ sigma1,
                                                     const double* __restrict__ rms, const double* __restrict__ thr,
                                                     double rms_max, uint8_t* __restrict__ det) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * n) return;
  const int64_t p = t / n;
  const int i = (int)(t - p * n);
  const double a = A[t];
  det[t] = (a > thr[i] && sigma1[t] < a && rms[p] < rms_max) ? 1 : 0;
}

// Second pass: bh_i = -M for the spectra pixel p does not keep.  M bounds
// the multiplier an excluded index needs at the restricted optimum: with
// the scaled Gram entries |Gh_ij| <= 1, |(Gh a)_i| <= max(1^T a,
// sqrt(c / gamma)) (a fit never exceeds the pixel's norm) and |nu| <= 1 +
// max |bh| on the kept indices, so M = 4 (1 + max |bh| + sqrt(c / gamma))
// keeps every excluded multiplier positive.  A pixel that keeps nothing gets
// a non-finite projection (reported as such by the solve).
__global__ __launch_bounds__(256) void keep_kernel(int n, int64_t P, const uint8_t* __restrict__ keep,
                                                   const double* __restrict__ c, double gamma,
                                                   double* __restrict__ bh) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double bmax = 0.0;
  int kept = 0;
  for (int i = 0; i < n; ++i) {
    bmax = fmax(bmax, fabs(bh[p * n + i]));
    kept += keep[p * n + i] != 0;
  }
  const double M = 4.0 * (1.0 + bmax + sqrt(fmax(c[p], 0.0) / gamma));
  for (int i = 0; i < n; ++i)
    if (!keep[p * n + i]) bh[p * n + i] = kept ? -M : __builtin_nan("");
}

int launch_error_maps(int n, int64_t P, int L, const float* Y, const double* A, const float* S, const double* cov,
                      int layout, double* rms, double* sigma1, hipStream_t st) {
  if (P <= 0) return 0;
  if (n > 128) return -1;
  if (sigma1) {
    const int64_t total = P * n;
    hipLaunchKernelGGL(sigma1_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, P, cov, layout,
                       sigma1);
  }
  if (rms) hipLaunchKernelGGL(rms_kernel, dim3((unsigned)((P + 15) / 16)), dim3(256), 0, st, n, P, L, Y, A, S, rms);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

size_t thresholds_workspace_bytes(int n, int64_t P) {
  const int64_t blocks = P < 1024 * 256 ? (P + 255) / 256 : 1024;
  return sizeof(double) * (size_t)(4 * n * (blocks > 0 ? blocks : 1) + 4 * n);
}

int launch_thresholds(int n, int64_t P, const double* A, const uint8_t* present, double* thr, double* ws,
                      hipStream_t st) {
  if (n < 1 || n > 128) return -1;
  int64_t blocks = P < 1024 * 256 ? (P + 255) / 256 : 1024;
  if (blocks < 1) blocks = 1;
  const int64_t rows = (P + blocks - 1) / blocks;
  double* part = ws;
  double* stat = ws + 4 * n * blocks;
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(thr_partial_kernel, dim3((unsigned)blocks), dim3(128), 0, st, n, P, rows > 0 ? rows : 1, A,
                       present, pass, stat + 2 * n, part);
    hipLaunchKernelGGL(thr_final_kernel, dim3(1), dim3(128), 0, st, n, (int)blocks, part, pass, stat, thr);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_detect(int n, int64_t P, const double* A, const double* sigma1, const double* rms, const double* thr,
                  double rms_max, uint8_t* det, hipStream_t st) {
  if (P <= 0) return 0;
  const int64_t total = P * n;
  hipLaunchKernelGGL(detect_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, P, A, sigma1, rms,
                     thr, rms_max, det);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_keep(int n, int64_t P, const uint8_t* keep, const double* c, double gamma, double* bh, hipStream_t st) {
  if (P <= 0) return 0;
  hipLaunchKernelGGL(keep_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, n, P, keep, c, gamma, bh);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lm
