// setup.hip -- one-off library preparation (renormalisation, Sec. 2.3).
//
//   Ci = C^{-1}                         (Cholesky of the noise covariance)
//   W  = C^{-1} S^T        (L x N)      so that b = W^T x, G = S W = S C^{-1} S^T
//   gamma = max_i G_ii,  Gh = G / gamma (padded to NC x NC, identity on the
//   padding), Wh = W / gamma
// The Gram matrix itself is formed on MFMA by the projection kernel (gemm.hip)
// with the library rows as the "pixels".  These kernels run once per library
// and are sized for clarity, not speed.
#include "common.h"
#include "kernels.h"

namespace lm {

// In-place Cholesky C = U U^T (lower) and Ci = C^{-1}; one block.
__global__ __launch_bounds__(256) void chol_inverse_kernel(double* C, int L, double* Ci, int* err) {
  __shared__ double piv;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < L; ++k) {
    if (threadIdx.x == 0) {
      const double d = C[(int64_t)k * L + k];
      if (!(d > 0.0) || d != d || d - d != 0.0) bad = 1;
      piv = bad ? 1.0 : sqrt(d);
      C[(int64_t)k * L + k] = piv;
    }
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < L; i += blockDim.x) C[(int64_t)i * L + k] /= piv;
    __syncthreads();
    for (int idx = threadIdx.x; idx < (L - k - 1) * (L - k - 1); idx += blockDim.x) {
      const int i = k + 1 + idx / (L - k - 1), j = k + 1 + idx % (L - k - 1);
      if (j <= i) C[(int64_t)i * L + j] -= C[(int64_t)i * L + k] * C[(int64_t)j * L + k];
    }
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) *err = 1;
    return;
  }
  // columns of C^{-1}: solve U U^T x = e_j, one column per thread
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    double* x = Ci + (int64_t)j * L;  // column j stored as row j (Ci is symmetric)
    for (int i = 0; i < L; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) s -= C[(int64_t)i * L + q] * x[q];
      x[i] = s / C[(int64_t)i * L + i];
    }
    for (int i = L - 1; i >= 0; --i) {
      double s = x[i];
      for (int q = i + 1; q < L; ++q) s -= C[(int64_t)q * L + i] * x[q];
      x[i] = s / C[(int64_t)i * L + i];
    }
  }
}

// W[l][n] = sum_m Ci[l][m] S[n][m]  (or S[n][l] when Ci is NULL); ldw columns, zero padded
__global__ void w_kernel(const float* S, int L, int N, const double* Ci, double* W, int ldw) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L * ldw) return;
  const int l = (int)(idx / ldw), n = (int)(idx % ldw);
  double v = 0.0;
  if (n < N) {
    if (Ci) {
      for (int m = 0; m < L; ++m) v += Ci[(int64_t)l * L + m] * (double)S[(int64_t)n * L + m];
    } else {
      v = (double)S[(int64_t)n * L + l];
    }
  }
  W[idx] = v;
}

// gamma, scaled padded Gram (FP64 and FP32) and scaled W; one block.
__global__ __launch_bounds__(256) void gram_finish_kernel(const double* G, int N, const double* W, int L,
                                                          int ldw, int NC, double* Gh64, float* Gh32,
                                                          double* Wh, double* gamma_out, int* err) {
  __shared__ double gam;
  if (threadIdx.x == 0) {
    double m = 0.0;
    bool ok = true;
    for (int i = 0; i < N; ++i) {
      const double d = G[(int64_t)i * N + i];
      if (d != d || d - d != 0.0) ok = false;
      m = d > m ? d : m;
    }
    if (!ok || !(m > 0.0)) {
      *err = 2;
      m = 1.0;
    }
    gam = m;
    *gamma_out = m;
  }
  __syncthreads();
  const double r = 1.0 / gam;
  for (int idx = threadIdx.x; idx < NC * NC; idx += blockDim.x) {
    const int i = idx / NC, j = idx % NC;
    double v;
    if (i < N && j < N) v = 0.5 * (G[(int64_t)i * N + j] + G[(int64_t)j * N + i]) * r;
    else v = (i == j) ? 1.0 : 0.0;
    Gh64[idx] = v;
    Gh32[idx] = (float)v;
  }
  for (int64_t idx = threadIdx.x; idx < (int64_t)L * ldw; idx += blockDim.x) Wh[idx] = W[idx] * r;
}

int launch_setup(const float* S, int L, int N, const double* C, double* Ci, double* W, int* err,
                 hipStream_t st) {
  // C is overwritten with its Cholesky factor
  if (C) {
    hipLaunchKernelGGL(chol_inverse_kernel, dim3(1), dim3(256), 0, st, const_cast<double*>(C), L, Ci, err);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  const int ldw = 16 * ((N + 15) / 16);
  const int64_t tot = (int64_t)L * ldw;
  hipLaunchKernelGGL(w_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, S, L, N,
                     C ? (const double*)Ci : nullptr, W, ldw);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_gram_finish(const double* G, int N, const double* W, int L, int NC, double* Gh64, float* Gh32,
                       double* Wh, int ldw, double* gamma_dev, int* err, hipStream_t st) {
  hipLaunchKernelGGL(gram_finish_kernel, dim3(1), dim3(256), 0, st, G, N, W, L, ldw, NC, Gh64, Gh32, Wh,
                     gamma_dev, err);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lm
