// kernels.h -- launch interface between the C ABI (linmin.cpp) and the HIP
// kernels of lib_linmin.  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lm {

// Mode of an interior-point launch.
enum IpmMode : int {
  kFull = 0,    // start -> iterate to tolerance -> finishing step -> outputs
  kStage1 = 1,  // start -> iterate until mu <= mu_switch -> save state
  kStage2 = 2,  // load state -> iterate to tolerance -> finishing step -> outputs
  kRetry = 3,   // mixed form, after stage 2: pixels whose status says the
                // finishing step did not certify (or the iterations stopped
                // early) are solved again in FP64 from the start; the others
                // are left as they are
};

// Per-pixel status bits (same meaning as LINMIN_PX_* in linmin.h).
enum : uint32_t {
  kPxMaxit = 1u,
  kPxNonfinite = 2u,
  kPxBadSigma = 4u,
  kPxNotPd = 8u,
  kPxDegenerate = 16u,
  kPxInexact = 32u,
};

// Constraint besides a >= 0 (same values as LINMIN_STO / SLO / POS).
enum : int {
  kSto = 0,  // 1^T a = 1
  kSlo = 1,  // 1^T a <= 1
  kPos = 2,  // none
};

struct IpmParams {
  int n;                // library size N
  int64_t P;            // pixels in this launch
  const void* Gh;       // NC x NC scaled Gram, padded (identity on padded diagonal), FP64 or FP32
  const double* bh;     // P x n scaled projections bh = b / gamma
  const double* c;      // P: x'^T x' (NULL when no objective is wanted)
  const float* sigma;   // P or NULL (s_p = 1)
  double gamma;         // max_i G_ii
  int maxit;
  int max_polish;
  int constraint;       // kSto, kSlo or kPos
  int stable;           // tile kernels: 1 = factorisation safe for nearly singular diagonal blocks
  double tol_mu, tol_d, tol_p, eta, lambda0, tau, deg_tol, mu_switch;
  // hand-over state between the FP32 and FP64 stages
  double* st_a;         // P x n
  double* st_lam;       // P x n
  double* st_nu;        // P
  double* st_s;         // P: slack of 1^T a <= 1 (kSlo)
  int32_t* st_it;       // P
  uint8_t* st_flag;     // P (status bits so far; bit 7: still iterating)
  // outputs
  double* out_a;        // P x n
  uint8_t* status;      // P or NULL
  int32_t* iters;       // P or NULL
  double* objective;    // P or NULL
  double* dcov;         // P x n or NULL: per-coefficient diagonal for the covariance pass
  double* dcorner;      // P or NULL: corner of the covariance's bordered matrix (-inf: no border)
};

// Jobs of a batched interior-point launch: one IpmParams per cube, every
// cube of one launch with the same compiled shape and options.
struct IpmBatch {
  const IpmParams* jobs;  // device, njobs
  const int64_t* start;   // device, njobs + 1: first block of each job, then the total
  int njobs;
  int64_t blocks;         // total workgroups of the launch
};

// The FP32 stage of the mixed form also hands its iterate over after this
// many steps, or after a step shorter than this fraction of the way to the
// boundary: the single-precision Newton directions have stopped making
// progress, and the FP64 stage continues from the last accepted iterate.
constexpr int kStage1MaxIt = 60;
constexpr double kStage1MinStep = 1e-3;

// Interior-point kernel families (ipm_dispatch.cpp).
enum : int { kFamRowCyclic = 1, kFamTile = 2, kFamGroup = 3, kFamTile32 = 4 };
constexpr int kNcMax = 128;
bool ipm_family_available(int nc, bool fp32, int fam);
bool ipm_family_available(int nc, bool fp32, int fam, int lanes);  // lanes: group width, 0 = default
int ipm_family(int nc, bool fp32);                   // family used for padded size nc
int ipm_group_lanes(int nc, bool fp32);              // width of the group kernel used for nc
int ipm_set_family(int nc, bool fp32, int fam, int lanes);  // fam 0 = default rule; -1 if not compiled

// ipm_dispatch.cpp: picks the compiled shape for n and precision.
int ipm_shape_nc(int n);                      // padded size NC used for a library of size n
int ipm_choice_code(int n, bool fp32);        // kernel used now: family | group width << 8
int ipm_pixels_per_block(int n, bool fp32);   // pixels of one workgroup for that kernel
int ipm_pixels_per_block_code(int code, int nc);  // for kernel code at padded size nc
int ipm_kernel_class(int n, bool fp32, bool stable);  // launches of equal class can share a batch
int ipm_kernel_class_of(int n, bool fp32, bool stable, int code);  // the same for kernel code
int launch_ipm(const IpmParams& p, int mode, bool fp32, hipStream_t st);
// the kRetry pass of the mixed form on the FP64 matrix-core kernel for p.n
int launch_ipm_retry(const IpmParams& p, hipStream_t st);
int ipm_retry_code(int n);                    // its kernel code
constexpr uint32_t kPxRetry = kPxInexact | kPxMaxit | kPxNotPd;  // status bits that send a pixel to kRetry
// batched: every job of b has a library with ipm_kernel_class(n, fp32,
// stable) equal to that of n, planned for the kernel code names (fixed when
// the batch was planned); constraint and stable as in IpmParams
int launch_ipm_batch(int n, int constraint, int stable, const IpmBatch& b, int mode, bool fp32, int code,
                     hipStream_t st);

// gemm.hip
// One cube of a batched projection launch: bh = Y W (and c = y^T y, or
// y^T Ci y by the quadratic-form launch when Ci is given).
struct ProjJob {
  const float* Y;
  int64_t P;
  int L;
  const double* W;
  int ldw;
  int N;
  double* B;
  double* c;
  const double* Ci;  // L x ldc inverse noise covariance, or NULL
  int ldc;
};
int proj_pixels_per_block();  // pixels of one projection workgroup (both kernels)
// batched: libraries of one launch share (N + 15) / 16; start: first block of
// each job, then the total
int launch_gemm_proj_batch(int N, const ProjJob* jobs, const int64_t* start, int njobs, int64_t blocks,
                           hipStream_t st);
int launch_quadform_batch(const ProjJob* jobs, const int64_t* start, int njobs, int64_t blocks, hipStream_t st);
int launch_gemm_proj_f64(const float* Y, int64_t P, int L, const double* W, int ldw, int N,
                         double* B, double* c, hipStream_t st);
int launch_quadform_f64(const float* Y, int64_t P, int L, const double* Ci, int ldc, double* c,
                        hipStream_t st);

// cov.hip
// One cube of a covariance pass (the arguments of launch_cov).
struct CovJob {
  int n;
  int64_t P;
  const double* Gh;
  int ldg;
  const double* dcov;
  const double* corner;
  const float* sigma;
  double gamma;
  const uint8_t* status;
  int layout;
  double* out;
  uint8_t* big;
};
// Jobs of one batched covariance path.  units: workgroups of 16 pixels for
// the first path, 64-pixel chunks for the other two; start: first unit of
// each job, then the total.  The first path takes every job, the second the
// jobs with n + 1 > 16, the third those with n + 1 > 32 (qcap: their largest
// n + 1).
struct CovBatch {
  const CovJob* jobs;
  const int64_t* start;
  int njobs;
  int64_t units;
  int qcap;
};
int launch_cov_batch(const CovBatch& small, const CovBatch& mid, const CovBatch& big, hipStream_t st);
// corner: P values (0: sum row, finite < 0: sum row with that corner, -inf:
// no sum row); big: P bytes of workspace (pixels routed to larger paths)
int launch_cov(int n, int64_t P, const double* Gh, int ldg, const double* dcov, const double* corner,
               const float* sigma, double gamma, const uint8_t* status_or_null, int layout,
               double* out_cov, uint8_t* big, hipStream_t st);

// detect.hip
int launch_error_maps(int n, int64_t P, int L, const float* Y, const double* A, const float* S, const double* cov,
                      int layout, double* rms, double* sigma1, hipStream_t st);
size_t thresholds_workspace_bytes(int n, int64_t P);
int launch_thresholds(int n, int64_t P, const double* A, const uint8_t* present, double* thr, double* ws,
                      hipStream_t st);
int launch_detect(int n, int64_t P, const double* A, const double* sigma1, const double* rms, const double* thr,
                  double rms_max, uint8_t* det, hipStream_t st);
int launch_keep(int n, int64_t P, const uint8_t* keep, const double* c, double gamma, double* bh, hipStream_t st);

// setup.hip
int launch_setup(const float* S_dev, int L, int N, const double* C_dev /* L x L or NULL */,
                 double* Ci_dev /* L x L out, when C given */, double* W_dev /* L x N out */,
                 int* err_dev, hipStream_t st);
int launch_gram_finish(const double* G_dev, int N, const double* W_dev, int L, int NC,
                       double* Gh64, float* Gh32, double* Wh, int ldw, double* gamma_dev,
                       int* err_dev, hipStream_t st);

}  // namespace lm
