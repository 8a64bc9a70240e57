// gemm.hip -- per-pixel projections on FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// Renormalised projections of Sec. 2.3 (eq. 6 expanded): for every pixel p
//   bh[p][n] = sum_l Y[p][l] * Wh[l][n]         (Wh = C^{-1} S^T / gamma)
//   c[p]     = sum_l Y[p][l]^2                   (C = I)
// One wavefront computes 16 pixels x 16*NT columns.  Operand layouts of the
// 16x16x4 FP64 MFMA on gfx950: A lane l = (row l%16, k l/16); B lane l =
// (k l/16, col l%16); D lane l register r = (row 4r + l/16, col l%16).
// The K dimension is walked in chunks of 16 channels; within a chunk, step s
// gives lane group g = l/16 the channel c0 + 4g + s, the same channel for its
// A and B operands, so each lane reads four consecutive channels of its pixel.
#include "common.h"
#include "kernels.h"

namespace lm {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int NT>
__device__ __forceinline__ void gemm_proj_body(const float* __restrict__ Y, int64_t P, int L,
                                               const double* __restrict__ W, int ldw, int N,
                                               double* __restrict__ B, double* __restrict__ c, int64_t blk) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t p0 = (blk * 4 + wave) * 16;
  if (p0 >= P) return;
  const int row = lane & 15, g = lane >> 4;
  const int64_t p = p0 + row;
  const bool prow = p < P;
  const float* yrow = Y + (prow ? p : 0) * (int64_t)L;
  d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  double sq = 0.0;
  for (int c0 = 0; c0 < L; c0 += 16) {
    const int ch0 = c0 + 4 * g;
    // Every load of the chunk is issued unconditionally from a clamped
    // channel and the values past L are zeroed afterwards: a guarded load
    // becomes a branch that waits for its own result, which serialises the
    // chunk's memory latency.  y = 0 makes the clamped W row irrelevant.
    float yf[4];
    double w[4][NT];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t ch = min(ch0 + s, L - 1);
      yf[s] = yrow[ch];
#pragma unroll
      for (int t = 0; t < NT; ++t) w[s][t] = W[ch * ldw + t * 16 + row];
    }
    double y[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      y[s] = (prow && ch0 + s < L) ? (double)yf[s] : 0.0;
      sq = __builtin_fma(y[s], y[s], sq);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[s], w[s][t], acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 16 + row;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t pr = p0 + 4 * r + g;
      if (pr < P && col < N) B[pr * N + col] = acc[t][r];
    }
  }
  if (c) {
    sq += __shfl_xor(sq, 16);
    sq += __shfl_xor(sq, 32);
    if (g == 0 && prow) c[p] = sq;
  }
}

template <int NT>
__global__ __launch_bounds__(256) void gemm_proj_f64(const float* __restrict__ Y, int64_t P, int L,
                                                     const double* __restrict__ W, int ldw, int N,
                                                     double* __restrict__ B, double* __restrict__ c) {
  gemm_proj_body<NT>(Y, P, L, W, ldw, N, B, c, blockIdx.x);
}

// Several cubes in one launch (libraries with the same column-block count).
template <int NT>
__global__ __launch_bounds__(256) void gemm_proj_batch_f64(const ProjJob* __restrict__ jobs,
                                                           const int64_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const ProjJob J = uniform_copy(jobs + j);
  gemm_proj_body<NT>(J.Y, J.P, J.L, J.W, J.ldw, J.N, J.B, J.c, (int64_t)blockIdx.x - start[j]);
}

// c[p] = y_p^T Ci y_p for a full L x L inverse noise covariance Ci (ldc
// columns, zero padded): MFMA tiles of (Y Ci) dotted with Y on the fly.
__device__ __forceinline__ void quadform_body(const float* __restrict__ Y, int64_t P, int L,
                                              const double* __restrict__ Ci, int ldc, double* __restrict__ c,
                                              int64_t blk) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t p0 = (blk * 4 + wave) * 16;
  if (p0 >= P) return;
  const int row = lane & 15, g = lane >> 4;
  const int64_t p = p0 + row;
  const bool prow = p < P;
  const float* yrow = Y + (prow ? p : 0) * (int64_t)L;
  double part[4] = {0.0, 0.0, 0.0, 0.0};  // per output row 4r+g
  for (int t0 = 0; t0 < L; t0 += 16) {
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < L; c0 += 16) {
      const int ch0 = c0 + 4 * g;
      // unconditional loads from clamped indices, zeroed afterwards (as in
      // the projections above)
      const int col = min(t0 + row, L - 1);
      float yf[4];
      double w[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t ch = min(ch0 + s, L - 1);
        yf[s] = yrow[ch];
        w[s] = Ci[ch * ldc + col];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double y = (prow && ch0 + s < L) ? (double)yf[s] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(y, (t0 + row < L) ? w[s] : 0.0, acc, 0, 0, 0);
      }
    }
    const int col = t0 + row;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t pr = p0 + 4 * r + g;
      const double yv = (pr < P && col < L) ? (double)Y[pr * L + col] : 0.0;
      part[r] = __builtin_fma(acc[r], yv, part[r]);
    }
  }
  // reduce over the 16 columns held by lanes sharing g
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double v = part[r];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    const int64_t pr = p0 + 4 * r + g;
    if (row == 0 && pr < P) c[pr] = v;
  }
}

__global__ __launch_bounds__(256) void quadform_f64(const float* __restrict__ Y, int64_t P, int L,
                                                    const double* __restrict__ Ci, int ldc,
                                                    double* __restrict__ c) {
  quadform_body(Y, P, L, Ci, ldc, c, blockIdx.x);
}

__global__ __launch_bounds__(256) void quadform_batch_f64(const ProjJob* __restrict__ jobs,
                                                          const int64_t* __restrict__ start, int njobs) {
  const int j = job_of(start, njobs, blockIdx.x);
  const ProjJob J = uniform_copy(jobs + j);
  quadform_body(J.Y, J.P, J.L, J.Ci, J.ldc, J.c, (int64_t)blockIdx.x - start[j]);
}

int launch_gemm_proj_f64(const float* Y, int64_t P, int L, const double* W, int ldw, int N,
                         double* B, double* c, hipStream_t st) {
  if (P <= 0) return 0;
  const int nt = (N + 15) / 16;
  const int64_t blocks = (P + 63) / 64;
  dim3 grid((unsigned)blocks), block(256);
  switch (nt) {
#define CASE(K) \
  case K: hipLaunchKernelGGL(gemm_proj_f64<K>, grid, block, 0, st, Y, P, L, W, ldw, N, B, c); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_quadform_f64(const float* Y, int64_t P, int L, const double* Ci, int ldc, double* c,
                        hipStream_t st) {
  if (P <= 0) return 0;
  const int64_t blocks = (P + 63) / 64;
  hipLaunchKernelGGL(quadform_f64, dim3((unsigned)blocks), dim3(256), 0, st, Y, P, L, Ci, ldc, c);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int proj_pixels_per_block() { return 64; }

int launch_gemm_proj_batch(int N, const ProjJob* jobs, const int64_t* start, int njobs, int64_t blocks,
                           hipStream_t st) {
  if (njobs <= 0 || blocks <= 0) return 0;
  const int nt = (N + 15) / 16;
  dim3 grid((unsigned)blocks), block(256);
  switch (nt) {
#define CASE(K) \
  case K: hipLaunchKernelGGL(gemm_proj_batch_f64<K>, grid, block, 0, st, jobs, start, njobs); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_quadform_batch(const ProjJob* jobs, const int64_t* start, int njobs, int64_t blocks, hipStream_t st) {
  if (njobs <= 0 || blocks <= 0) return 0;
  hipLaunchKernelGGL(quadform_batch_f64, dim3((unsigned)blocks), dim3(256), 0, st, jobs, start, njobs);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace lm
