// linmin.cpp -- C ABI of lib_linmin (declared in include/linmin.h).
//
// Host side only: argument checks, device memory, and the order of kernel
// launches.  All arithmetic of the path runs in the HIP kernels:
//   create:  setup.hip (C^{-1}, W), gemm.hip (Gram on MFMA), setup.hip (scale)
//   unmix:   gemm.hip (projections) -> ipm.hip (IPLS + finishing step)
//            -> cov.hip (covariance)
// The one host computation is linmin_extra_spectra, which fills a host array
// a caller appends to its library before linmin_create_library.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "../../include/linmin.h"
#include "kernels.h"
#include "unmix.h"

struct linmin_lib_s {
  int L, N, NC, ldw, dev;
  int stable;    // Gh has an eigenvalue below kNearlySingular: tile kernels use the stable factorisation
  double gamma;
  double* Wh;    // L x ldw, W / gamma
  double* Gh64;  // NC x NC, G / gamma padded with identity
  float* Gh32;   // NC x NC
  double* G;     // N x N, unscaled Gram
  double* Ci;    // L x L inverse noise covariance, or NULL for C = I
  float* S;      // N x L library as given (the residual of the RMS map)
};

namespace {

int hip_ok(hipError_t e) { return e == hipSuccess ? LINMIN_OK : LINMIN_EHIP; }

#define TRY(x)                   \
  do {                           \
    int rc_ = (x);               \
    if (rc_ != LINMIN_OK) {      \
      rc = rc_;                  \
      goto fail;                 \
    }                            \
  } while (0)

int from_launch(int r) {
  if (r == 0) return LINMIN_OK;
  if (r == -5) return LINMIN_EUNSUPPORTED;
  if (r == -1) return LINMIN_EINVAL;
  return LINMIN_EHIP;
}

void free_lib(linmin_lib l) {
  if (!l) return;
  (void)hipFree(l->Wh);
  (void)hipFree(l->Gh64);
  (void)hipFree(l->Gh32);
  (void)hipFree(l->G);
  (void)hipFree(l->Ci);
  (void)hipFree(l->S);
  delete l;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Below this smallest eigenvalue of the scaled Gram matrix Gh = G / gamma
// (largest diagonal 1), a diagonal block of the Newton matrix Gh + diag(D)
// can be so nearly singular that an explicit 4x4 block inverse loses the
// next pivots: its error is about eps / lambda_min, which must stay well
// below lambda_min, i.e. lambda_min >> sqrt(eps) = 1.5e-8.
constexpr double kNearlySingular = 1e-7;

// Kernel choice at library set-up: whether Gh - tau I is not positive
// definite (a Cholesky factorisation of it breaks down), i.e. Gh has an
// eigenvalue below tau.  G is N x N row-major and symmetric.
bool nearly_singular(const double* G, int N, double gamma, double tau) {
  std::vector<double> Lc((size_t)N * N, 0.0);
  for (int j = 0; j < N; ++j) {
    double d = G[(size_t)j * N + j] / gamma - tau;
    for (int k = 0; k < j; ++k) d -= Lc[(size_t)j * N + k] * Lc[(size_t)j * N + k];
    if (!(d > 0.0) || !isfinite(d)) return true;
    d = sqrt(d);
    Lc[(size_t)j * N + j] = d;
    for (int i = j + 1; i < N; ++i) {
      double v = G[(size_t)i * N + j] / gamma;
      for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * N + k] * Lc[(size_t)j * N + k];
      Lc[(size_t)i * N + j] = v / d;
    }
  }
  return false;
}

struct Work {
  size_t bh, c, dcov, dcorner, big, st_a, st_lam, st_nu, st_s, st_it, st_flag, status, total;
};

Work plan(const linmin_lib_s* lib, int64_t P, const linmin_opts& o, bool want_cov) {
  Work w{};
  const size_t n = (size_t)lib->N, p = (size_t)P;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  w.bh = take(sizeof(double) * p * n);
  w.c = take(sizeof(double) * p);
  w.dcov = want_cov ? take(sizeof(double) * p * n) : (size_t)-1;
  w.big = want_cov ? take(p) : (size_t)-1;
  w.dcorner = want_cov ? take(sizeof(double) * p) : (size_t)-1;
  if (o.precision == LINMIN_MIXED) {
    w.st_a = take(sizeof(double) * p * n);
    w.st_lam = take(sizeof(double) * p * n);
    w.st_nu = take(sizeof(double) * p);
    w.st_s = take(sizeof(double) * p);
    w.st_it = take(sizeof(int32_t) * p);
    w.st_flag = take(p);
  } else {
    w.st_a = w.st_lam = w.st_nu = w.st_s = w.st_it = w.st_flag = (size_t)-1;
  }
  w.status = (o.status == nullptr) ? take(p) : (size_t)-1;
  w.total = off;
  return w;
}

// Interior-point arguments of one cube; ws is the cube's work area laid out
// by plan(), status the per-pixel status array (caller's or in ws).
lm::IpmParams make_ipm(const linmin_lib_s* lib, int64_t P, const float* sigma, double* out_coeffs, uint8_t* status,
                       int32_t* iters, double* objective, const linmin_opts& o, const Work& w, char* ws,
                       bool want_cov) {
  auto at = [&](size_t off) -> char* { return off == (size_t)-1 ? nullptr : ws + off; };
  lm::IpmParams prm{};
  prm.n = lib->N;
  prm.P = P;
  prm.bh = (double*)at(w.bh);
  prm.c = (double*)at(w.c);
  prm.sigma = sigma;
  prm.gamma = lib->gamma;
  prm.maxit = o.maxit;
  prm.max_polish = o.max_polish;
  prm.constraint = o.constraint;
  prm.stable = lib->stable;
  prm.tol_mu = o.tol_mu;
  prm.tol_d = o.tol_d;
  prm.tol_p = o.tol_p;
  prm.eta = o.eta;
  prm.lambda0 = o.lambda0;
  prm.tau = o.tau;
  prm.deg_tol = o.deg_tol;
  prm.mu_switch = o.mu_switch;
  prm.out_a = out_coeffs;
  prm.status = status;
  prm.iters = iters;
  prm.objective = objective;
  prm.dcov = want_cov ? (double*)at(w.dcov) : nullptr;
  prm.dcorner = want_cov ? (double*)at(w.dcorner) : nullptr;
  if (o.precision == LINMIN_MIXED) {
    prm.st_a = (double*)at(w.st_a);
    prm.st_lam = (double*)at(w.st_lam);
    prm.st_nu = (double*)at(w.st_nu);
    prm.st_s = (double*)at(w.st_s);
    prm.st_it = (int32_t*)at(w.st_it);
    prm.st_flag = (uint8_t*)at(w.st_flag);
  }
  prm.Gh = lib->Gh64;
  return prm;
}

int check_opts(const linmin_opts& o) {
  if (o.precision != LINMIN_FP64 && o.precision != LINMIN_MIXED) return LINMIN_EINVAL;
  if (o.cov_layout < LINMIN_COV_NONE || o.cov_layout > LINMIN_COV_DIAG) return LINMIN_EINVAL;
  if (o.maxit < 0 || o.max_polish < 0 || !(o.eta > 0.0 && o.eta < 1.0) || !(o.lambda0 > 0.0)) return LINMIN_EINVAL;
  if (o.constraint != LINMIN_STO && o.constraint != LINMIN_SLO && o.constraint != LINMIN_POS) return LINMIN_EINVAL;
  return LINMIN_OK;
}

}  // namespace

namespace lm {

// Checks of linmin_unmix and its variants: fills *o (defaults where opts is
// NULL) and *bytes (the work area one call needs, 0 when P == 0).
int unmix_check(linmin_lib lib, const float* cube, int64_t P, const double* out_coeffs, const double* out_cov,
                const linmin_opts* opts, linmin_opts* o, size_t* bytes) {
  *bytes = 0;
  if (!lib || P < 0) return LINMIN_EINVAL;
  if (opts) *o = *opts;
  else linmin_default_opts(o);
  const int rc0 = check_opts(*o);
  if (rc0 != LINMIN_OK) return rc0;
  if (P == 0) return LINMIN_OK;
  if (!cube || !out_coeffs) return LINMIN_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LINMIN_EHIP;
  if (dev != lib->dev) return LINMIN_EINVAL;
  *bytes = plan(lib, P, *o, out_cov != nullptr && o->cov_layout != LINMIN_COV_NONE).total;
  return LINMIN_OK;
}

// The unmix itself (projections, interior point, covariance) on stream st
// with the work area ws of at least unmix_check's bytes, laid out by plan().
// Nothing here allocates; every byte of ws that a kernel reads was written
// earlier in the same call, so ws may hold anything on entry.
int unmix_ws(linmin_lib lib, const float* cube, int64_t P, const float* sigma, double* out_coeffs,
             double* out_cov, const linmin_opts& o, hipStream_t st, char* ws) {
  const bool want_cov = out_cov != nullptr && o.cov_layout != LINMIN_COV_NONE;
  const Work w = plan(lib, P, o, want_cov);
  auto at = [&](size_t off) -> char* { return off == (size_t)-1 ? nullptr : ws + off; };
  double* bh = (double*)at(w.bh);
  double* c = (double*)at(w.c);
  uint8_t* status = o.status ? o.status : (uint8_t*)at(w.status);
  int rc = LINMIN_OK;

  hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(o.stage_events);
  auto mark = [&](int i) {
    if (ev && hipEventRecord(ev[i], st) != hipSuccess) return LINMIN_EHIP;
    return LINMIN_OK;
  };
  // projections bh = Y Wh and c = y^T C^{-1} y
  rc = mark(0);
  if (rc == LINMIN_OK) rc = from_launch(launch_gemm_proj_f64(cube, P, lib->L, lib->Wh, lib->ldw, lib->N, bh, c, st));
  if (rc == LINMIN_OK && lib->Ci) rc = from_launch(launch_quadform_f64(cube, P, lib->L, lib->Ci, lib->L, c, st));
  if (rc == LINMIN_OK && o.keep) rc = from_launch(launch_keep(lib->N, P, o.keep, c, lib->gamma, bh, st));
  if (rc == LINMIN_OK) rc = mark(1);
  if (rc == LINMIN_OK) {
    IpmParams prm = make_ipm(lib, P, sigma, out_coeffs, status, o.iters, o.objective, o, w, ws, want_cov);
    if (o.precision == LINMIN_MIXED) {
      prm.Gh = lib->Gh32;
      rc = from_launch(launch_ipm(prm, kStage1, true, st));
      if (rc == LINMIN_OK) {
        prm.Gh = lib->Gh64;
        rc = from_launch(launch_ipm(prm, kStage2, false, st));
      }
      // what the finishing step could not certify after the hand-over is
      // solved again in FP64 from the start
      if (rc == LINMIN_OK) rc = from_launch(launch_ipm_retry(prm, st));
    } else {
      prm.Gh = lib->Gh64;
      rc = from_launch(launch_ipm(prm, kFull, false, st));
    }
  }
  if (rc == LINMIN_OK) rc = mark(2);
  if (rc == LINMIN_OK && want_cov)
    rc = from_launch(launch_cov(lib->N, P, lib->Gh64, lib->NC, (double*)at(w.dcov), (double*)at(w.dcorner), sigma,
                                lib->gamma, status, o.cov_layout, out_cov, (uint8_t*)at(w.big), st));
  if (rc == LINMIN_OK) rc = mark(3);
  return rc;
}

}  // namespace lm

extern "C" {

void linmin_default_opts(linmin_opts* o) {
  if (!o) return;
  o->precision = LINMIN_FP64;
  o->cov_layout = LINMIN_COV_FULL;
  o->maxit = 200;
  o->max_polish = 16;
  o->constraint = LINMIN_STO;
  o->tol_mu = 1e-13;
  o->tol_d = 1e-12;
  o->tol_p = 1e-13;
  o->eta = 0.99;
  o->lambda0 = 0.1;
  o->tau = 1e-11;
  o->deg_tol = 1e-9;
  o->mu_switch = 1e-10;
  o->status = nullptr;
  o->iters = nullptr;
  o->objective = nullptr;
  o->stage_events = nullptr;
  o->keep = nullptr;
}

const char* linmin_strerror(int code) {
  switch (code) {
    case LINMIN_OK: return "success";
    case LINMIN_EINVAL: return "invalid argument";
    case LINMIN_ENOMEM: return "out of memory";
    case LINMIN_EHIP: return "HIP runtime or kernel launch failure";
    case LINMIN_ENOTSPD: return "matrix not symmetric positive definite";
    case LINMIN_EUNSUPPORTED: return "unsupported option combination";
    case LINMIN_ESCRATCH: return "work area larger than the no-allocation scratch array";
    default: return "unknown error";
  }
}

int linmin_set_kernel(int N, int stage, int family, int lanes) {
  if (N < 1 || N > LINMIN_N_MAX || (stage != LINMIN_STAGE_FP64 && stage != LINMIN_STAGE_FP32)) return LINMIN_EINVAL;
  if (family < LINMIN_KERNEL_DEFAULT || family > LINMIN_KERNEL_TILE32 || lanes < 0 || lanes > 64) return LINMIN_EINVAL;
  if (lanes != 0 && family != LINMIN_KERNEL_GROUP) return LINMIN_EINVAL;
  const int nc = lm::ipm_shape_nc(N);
  if (nc < 0) return LINMIN_EUNSUPPORTED;
  static_assert(LINMIN_KERNEL_ROWCYCLIC == lm::kFamRowCyclic && LINMIN_KERNEL_TILE == lm::kFamTile &&
                    LINMIN_KERNEL_GROUP == lm::kFamGroup && LINMIN_KERNEL_TILE32 == lm::kFamTile32,
                "kernel family codes");
  return lm::ipm_set_family(nc, stage == LINMIN_STAGE_FP32, family, lanes) == 0 ? LINMIN_OK : LINMIN_EUNSUPPORTED;
}

int linmin_get_kernel(int N, int stage, int* lanes) {
  if (N < 1 || N > LINMIN_N_MAX || (stage != LINMIN_STAGE_FP64 && stage != LINMIN_STAGE_FP32)) return LINMIN_EINVAL;
  const int code = lm::ipm_choice_code(N, stage == LINMIN_STAGE_FP32);
  if (code < 0) return LINMIN_EUNSUPPORTED;
  if (lanes) *lanes = code >> 8;
  return code & 0xff;
}

int linmin_extra_spectra(int L, int n_extra, const double* wavelengths, float* out) {
  if (!out || L < 2 || (n_extra != 4 && n_extra != 12)) return LINMIN_EINVAL;
  if (wavelengths) {
    for (int l = 0; l < L; ++l)
      if (!isfinite(wavelengths[l]) || (l > 0 && !(wavelengths[l] > wavelengths[l - 1]))) return LINMIN_EINVAL;
  }
  const double w0 = wavelengths ? wavelengths[0] : 0.0;
  const double span = wavelengths ? wavelengths[L - 1] - w0 : (double)(L - 1);
  const double pi = 3.14159265358979323846;
  for (int l = 0; l < L; ++l) {
    // position along the spectral domain, 0 at the first channel, 1 at the last
    const double t = ((wavelengths ? wavelengths[l] : (double)l) - w0) / span;
    double v[12];
    v[0] = 1.0;      // level near one
    v[1] = 1e-4;     // level near zero
    v[2] = t;        // increasing slope
    v[3] = 1.0 - t;  // decreasing slope
    for (int k = 0; k < 2; ++k) {
      // periods four and two times the domain: a quarter and a half cycle
      const double ph = 2.0 * pi * (k == 0 ? 0.25 : 0.5) * t;
      const double c = cos(ph), sn = sin(ph);
      v[4 + 4 * k] = c;
      v[5 + 4 * k] = sn;
      v[6 + 4 * k] = -c;
      v[7 + 4 * k] = -sn;
    }
    for (int i = 0; i < n_extra; ++i) out[(size_t)i * L + l] = (float)v[i];
  }
  return LINMIN_OK;
}

int linmin_create_library(const float* S, int L, int N, const double* noise_cov, linmin_lib* out) {
  if (!out) return LINMIN_EINVAL;
  *out = nullptr;
  if (!S || L < 1 || N < 1 || N > L || N > LINMIN_N_MAX) return LINMIN_EINVAL;
  const int NC = lm::ipm_shape_nc(N);
  if (NC < 0) return LINMIN_EUNSUPPORTED;
  if (noise_cov)
    for (int64_t i = 0; i < (int64_t)L * L; ++i)
      if (!isfinite(noise_cov[i])) return LINMIN_ENOTSPD;

  int rc = LINMIN_OK;
  linmin_lib lib = new (std::nothrow) linmin_lib_s();
  if (!lib) return LINMIN_ENOMEM;
  lib->L = L;
  lib->N = N;
  lib->NC = NC;
  lib->ldw = 16 * ((N + 15) / 16);
  float* dS = nullptr;
  double *dC = nullptr, *dW = nullptr, *dgam = nullptr;
  int* derr = nullptr;
  int herr = 0;
  hipStream_t st = nullptr;
  TRY(hip_ok(hipGetDevice(&lib->dev)));
  TRY(hip_ok(hipStreamCreate(&st)));
  {
    const size_t wbytes = sizeof(double) * (size_t)L * lib->ldw;
    if (hipMalloc(&dS, sizeof(float) * (size_t)N * L) != hipSuccess ||
        hipMalloc(&dW, wbytes) != hipSuccess || hipMalloc(&lib->Wh, wbytes) != hipSuccess ||
        hipMalloc(&lib->G, sizeof(double) * (size_t)N * N) != hipSuccess ||
        hipMalloc(&lib->Gh64, sizeof(double) * (size_t)NC * NC) != hipSuccess ||
        hipMalloc(&lib->Gh32, sizeof(float) * (size_t)NC * NC) != hipSuccess ||
        hipMalloc(&dgam, sizeof(double)) != hipSuccess || hipMalloc(&derr, sizeof(int)) != hipSuccess) {
      rc = LINMIN_ENOMEM;
      goto fail;
    }
    if (noise_cov) {
      if (hipMalloc(&dC, sizeof(double) * (size_t)L * L) != hipSuccess ||
          hipMalloc(&lib->Ci, sizeof(double) * (size_t)L * L) != hipSuccess) {
        rc = LINMIN_ENOMEM;
        goto fail;
      }
      TRY(hip_ok(hipMemcpyAsync(dC, noise_cov, sizeof(double) * (size_t)L * L, hipMemcpyHostToDevice, st)));
    }
    TRY(hip_ok(hipMemcpyAsync(dS, S, sizeof(float) * (size_t)N * L, hipMemcpyHostToDevice, st)));
    TRY(hip_ok(hipMemsetAsync(derr, 0, sizeof(int), st)));
    TRY(from_launch(lm::launch_setup(dS, L, N, dC, lib->Ci, dW, derr, st)));
    // Gram matrix G = S W on MFMA (library rows as pixels)
    TRY(from_launch(lm::launch_gemm_proj_f64(dS, N, L, dW, lib->ldw, N, lib->G, nullptr, st)));
    TRY(from_launch(lm::launch_gram_finish(lib->G, N, dW, L, NC, lib->Gh64, lib->Gh32, lib->Wh, lib->ldw,
                                           dgam, derr, st)));
    TRY(hip_ok(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st)));
    TRY(hip_ok(hipMemcpyAsync(&lib->gamma, dgam, sizeof(double), hipMemcpyDeviceToHost, st)));
    TRY(hip_ok(hipStreamSynchronize(st)));
    if (herr != 0) {
      rc = LINMIN_ENOTSPD;
      goto fail;
    }
    std::vector<double> Gh((size_t)N * N);
    TRY(hip_ok(hipMemcpy(Gh.data(), lib->G, sizeof(double) * Gh.size(), hipMemcpyDeviceToHost)));
    lib->stable = nearly_singular(Gh.data(), N, lib->gamma, kNearlySingular) ? 1 : 0;
  }
  lib->S = dS;  // kept for the RMS map
  (void)hipFree(dC);
  (void)hipFree(dW);
  (void)hipFree(dgam);
  (void)hipFree(derr);
  (void)hipStreamDestroy(st);
  *out = lib;
  return LINMIN_OK;
fail:
  if (st) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  (void)hipFree(dS);
  (void)hipFree(dC);
  (void)hipFree(dW);
  (void)hipFree(dgam);
  (void)hipFree(derr);
  free_lib(lib);
  return rc;
}

int linmin_destroy_library(linmin_lib lib) {
  if (!lib) return LINMIN_EINVAL;
  free_lib(lib);
  return LINMIN_OK;
}

int linmin_library_info(linmin_lib lib, int* L, int* N, double* gamma) {
  if (!lib) return LINMIN_EINVAL;
  if (L) *L = lib->L;
  if (N) *N = lib->N;
  if (gamma) *gamma = lib->gamma;
  return LINMIN_OK;
}

int linmin_library_gram(linmin_lib lib, double* G_host) {
  if (!lib || !G_host) return LINMIN_EINVAL;
  return hip_ok(hipMemcpy(G_host, lib->G, sizeof(double) * (size_t)lib->N * lib->N, hipMemcpyDeviceToHost));
}

size_t linmin_workspace_bytes(linmin_lib lib, int64_t P, const linmin_opts* opts) {
  if (!lib || P <= 0) return 0;
  linmin_opts o;
  if (opts) o = *opts;
  else linmin_default_opts(&o);
  return plan(lib, P, o, o.cov_layout != LINMIN_COV_NONE).total;
}

int linmin_unmix(linmin_lib lib, const float* cube, int64_t P, const float* sigma, double* out_coeffs,
                 double* out_cov, const linmin_opts* opts, void* stream) {
  linmin_opts o;
  size_t bytes = 0;
  {
    const int rc0 = lm::unmix_check(lib, cube, P, out_coeffs, out_cov, opts, &o, &bytes);
    if (rc0 != LINMIN_OK || P == 0) return rc0;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = nullptr;
  if (hipMallocAsync((void**)&ws, bytes, st) != hipSuccess) return LINMIN_ENOMEM;
  int rc = lm::unmix_ws(lib, cube, P, sigma, out_coeffs, out_cov, o, st, ws);
  if (hipFreeAsync(ws, st) != hipSuccess && rc == LINMIN_OK) rc = LINMIN_EHIP;
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many cubes, possibly of different libraries, in a few launches.
// The plan groups the cubes by compiled kernel (projection column blocks,
// interior-point shape) and uploads one job table per launch; a run only
// enqueues kernels.
// ---------------------------------------------------------------------------
struct linmin_batch_s {
  int dev = -1;
  linmin_opts o{};
  char* ws = nullptr;   // device: the cubes' work areas
  char* tab = nullptr;  // device: job tables and their block prefixes
  size_t ws_bytes = 0, tab_bytes = 0;
  struct Proj {
    int N;
    const lm::ProjJob* jobs;
    const int64_t* start;
    int njobs;
    int64_t blocks;
  };
  std::vector<Proj> proj;
  Proj quad{0, nullptr, nullptr, 0, 0};
  struct Ipm {
    int n, mode, stable;
    bool fp32;
    int code;  // kernel (family | group width << 8), fixed at planning
    lm::IpmBatch b;
    int lane = 0;  // 0: the caller's stream; k > 0: side stream k - 1
  };
  std::vector<Ipm> ipm;  // in launch order
  lm::CovBatch cov[3]{};
  // interior-point groups of different library sizes are independent: they
  // run on up to kLanes streams at once (forked from and joined back to the
  // caller's stream with events), so small groups fill the device beside
  // the largest one
  static constexpr int kLanes = 4;
  int lanes = 1;
  hipStream_t side[kLanes - 1] = {};
  hipEvent_t fork = nullptr, join[kLanes - 1] = {};
};

namespace {

// host image of the job tables: arrays appended at 256-byte boundaries
struct Image {
  std::vector<char> bytes;
  template <typename T>
  size_t put(const std::vector<T>& v) {
    const size_t at = align256(bytes.size());
    bytes.resize(at + sizeof(T) * v.size());
    if (!v.empty()) memcpy(bytes.data() + at, v.data(), sizeof(T) * v.size());
    return at;
  }
};

// a group's jobs and its prefix of work units (njobs + 1 values)
template <typename J>
struct Group {
  std::vector<J> jobs;
  std::vector<int64_t> start{0};
  size_t jobs_at = 0, start_at = 0;
  void add(const J& j, int64_t units) {
    jobs.push_back(j);
    start.push_back(start.back() + units);
  }
  void place(Image& im) {
    jobs_at = im.put(jobs);
    start_at = im.put(start);
  }
  int64_t units() const { return start.back(); }
};

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

extern "C" {

int linmin_batch_create(const linmin_job* jobs, int n_jobs, const linmin_opts* opts, linmin_batch* out) {
  if (!out || n_jobs < 0 || (n_jobs > 0 && !jobs)) return LINMIN_EINVAL;
  *out = nullptr;
  linmin_opts o;
  if (opts) o = *opts;
  else linmin_default_opts(&o);
  int rc = check_opts(o);
  if (rc != LINMIN_OK) return rc;
  if (o.keep) return LINMIN_EINVAL;  // per-pixel spectrum selection is for single calls
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LINMIN_EHIP;
  for (int j = 0; j < n_jobs; ++j) {
    const linmin_job& J = jobs[j];
    if (!J.lib || J.P < 0 || J.lib->dev != dev) return LINMIN_EINVAL;
    if (J.P > 0 && (!J.cube || !J.out_coeffs)) return LINMIN_EINVAL;
    if (lm::ipm_kernel_class(J.lib->N, false, false) < 0 || lm::ipm_kernel_class(J.lib->N, true, false) < 0)
      return LINMIN_EUNSUPPORTED;
  }
  const bool mixed = o.precision == LINMIN_MIXED;
  const bool any_cov = o.cov_layout != LINMIN_COV_NONE;

  // work areas, one after the other
  std::vector<Work> work(n_jobs);
  std::vector<size_t> base(n_jobs, 0);
  size_t total = 0;
  for (int j = 0; j < n_jobs; ++j) {
    if (jobs[j].P == 0) continue;
    linmin_opts oj = o;
    oj.status = jobs[j].status;
    work[j] = plan(jobs[j].lib, jobs[j].P, oj, any_cov && jobs[j].out_cov);
    base[j] = total;
    total += align256(work[j].total);
  }
  linmin_batch b = new (std::nothrow) linmin_batch_s;
  if (!b) return LINMIN_ENOMEM;
  b->dev = dev;
  b->o = o;
  b->ws_bytes = total;
  if (total && hipMalloc((void**)&b->ws, total) != hipSuccess) {
    delete b;
    return LINMIN_ENOMEM;
  }

  // job tables
  std::map<int, Group<lm::ProjJob>> proj;  // by column blocks
  Group<lm::ProjJob> quad;
  std::map<int, Group<lm::IpmParams>> ipm1, ipm2, ipm3;  // by kernel class: FP64 (or stage 2), FP32 stage 1, retry
  std::map<int, std::pair<int, int>> class_n1, class_n2, class_n3;  // a library size of each class, its kernel code
  std::map<int, int> code1, code2;                         // kernel code per library size
  Group<lm::CovJob> cov[3];
  int qcap = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const linmin_job& J = jobs[j];
    if (J.P == 0) continue;
    const linmin_lib_s* lib = J.lib;
    const Work& w = work[j];
    char* ws = b->ws + base[j];
    auto at = [&](size_t off) -> char* { return off == (size_t)-1 ? nullptr : ws + off; };
    const bool want_cov = any_cov && J.out_cov;
    uint8_t* status = J.status ? J.status : (uint8_t*)at(w.status);
    const int64_t P = J.P;

    lm::ProjJob pj{J.cube, P, lib->L, lib->Wh, lib->ldw, lib->N, (double*)at(w.bh), (double*)at(w.c), lib->Ci,
                   lib->L};
    proj[(lib->N + 15) / 16].add(pj, cdiv(P, lm::proj_pixels_per_block()));
    if (lib->Ci) quad.add(pj, cdiv(P, lm::proj_pixels_per_block()));

    lm::IpmParams prm = make_ipm(lib, P, J.sigma, J.out_coeffs, status, J.iters, J.objective, o, w, ws, want_cov);
    // the kernel of each stage is fixed here, once per job, so that block
    // counts and launches agree whatever linmin_set_kernel does later
    const int c2 = code2.count(lib->N) ? code2[lib->N] : (code2[lib->N] = lm::ipm_choice_code(lib->N, false));
    const int k2 = lm::ipm_kernel_class_of(lib->N, false, lib->stable != 0, c2);
    prm.Gh = lib->Gh64;
    ipm2[k2].add(prm, cdiv(P, lm::ipm_pixels_per_block_code(c2, lib->NC)));
    class_n2[k2] = {lib->N, c2};
    if (mixed) {
      const int c1 = code1.count(lib->N) ? code1[lib->N] : (code1[lib->N] = lm::ipm_choice_code(lib->N, true));
      const int k1 = lm::ipm_kernel_class_of(lib->N, true, lib->stable != 0, c1);
      prm.Gh = lib->Gh32;
      ipm1[k1].add(prm, cdiv(P, lm::ipm_pixels_per_block_code(c1, lib->NC)));
      class_n1[k1] = {lib->N, c1};
      const int c3 = lm::ipm_retry_code(lib->N);
      const int k3 = lm::ipm_kernel_class_of(lib->N, false, lib->stable != 0, c3);
      prm.Gh = lib->Gh64;
      ipm3[k3].add(prm, cdiv(P, lm::ipm_pixels_per_block_code(c3, lib->NC)));
      class_n3[k3] = {lib->N, c3};
    }
    if (want_cov) {
      const lm::CovJob cj{lib->N, P, lib->Gh64, lib->NC, (double*)at(w.dcov), (double*)at(w.dcorner), J.sigma,
                          lib->gamma, status, o.cov_layout, J.out_cov, (uint8_t*)at(w.big)};
      cov[0].add(cj, cdiv(P, 16));
      if (lib->N + 1 > 16) cov[1].add(cj, cdiv(P, 64));
      if (lib->N + 1 > 32) {
        cov[2].add(cj, cdiv(P, 64));
        if (lib->N + 1 > qcap) qcap = lib->N + 1;
      }
    }
  }
  Image im;
  for (auto& kv : proj) kv.second.place(im);
  quad.place(im);
  for (auto& kv : ipm1) kv.second.place(im);
  for (auto& kv : ipm2) kv.second.place(im);
  for (auto& kv : ipm3) kv.second.place(im);
  for (auto& g : cov) g.place(im);
  b->tab_bytes = im.bytes.size();
  if (b->tab_bytes) {
    if (hipMalloc((void**)&b->tab, b->tab_bytes) != hipSuccess) {
      linmin_batch_destroy(b);
      return LINMIN_ENOMEM;
    }
    if (hipMemcpy(b->tab, im.bytes.data(), b->tab_bytes, hipMemcpyHostToDevice) != hipSuccess) {
      linmin_batch_destroy(b);
      return LINMIN_EHIP;
    }
  }
  char* t = b->tab;
  for (auto& kv : proj) {
    const auto& g = kv.second;
    b->proj.push_back({g.jobs.front().N, (const lm::ProjJob*)(t + g.jobs_at), (const int64_t*)(t + g.start_at),
                       (int)g.jobs.size(), g.units()});
  }
  if (!quad.jobs.empty())
    b->quad = {0, (const lm::ProjJob*)(t + quad.jobs_at), (const int64_t*)(t + quad.start_at), (int)quad.jobs.size(),
               quad.units()};
  auto add_ipm = [&](std::map<int, Group<lm::IpmParams>>& m, std::map<int, std::pair<int, int>>& nmap, int mode,
                     bool fp32) {
    for (auto& kv : m) {
      const auto& g = kv.second;
      linmin_batch_s::Ipm e{nmap[kv.first].first, mode, g.jobs.front().stable, fp32, nmap[kv.first].second,
                            {(const lm::IpmParams*)(t + g.jobs_at), (const int64_t*)(t + g.start_at),
                             (int)g.jobs.size(), g.units()}};
      b->ipm.push_back(e);
    }
  };
  if (mixed) {
    add_ipm(ipm1, class_n1, lm::kStage1, true);
    add_ipm(ipm2, class_n2, lm::kStage2, false);
    add_ipm(ipm3, class_n3, lm::kRetry, false);
  } else {
    add_ipm(ipm2, class_n2, lm::kFull, false);
  }
  for (int k = 0; k < 3; ++k) {
    const auto& g = cov[k];
    if (!g.jobs.empty())
      b->cov[k] = {(const lm::CovJob*)(t + g.jobs_at), (const int64_t*)(t + g.start_at), (int)g.jobs.size(), g.units(),
                   qcap};
  }
  // Streams for the interior-point groups: the groups of one padded size
  // (both stages of the mixed form, both factorisations) stay on one stream
  // in launch order; sizes are placed largest first on the least loaded
  // stream, the load being pixels x NC^3 (the factorisation's work).
  {
    std::map<int, double> cost;  // by padded size
    for (const auto& g : b->ipm) {
      const double nc = lm::ipm_shape_nc(g.n);
      if (g.mode == lm::kRetry) {  // few pixels do any work
        cost[(int)nc] += 0.0;
        continue;
      }
      const double pixels = (double)g.b.blocks * lm::ipm_pixels_per_block_code(g.code, (int)nc);
      cost[(int)nc] += pixels * nc * nc * nc;
    }
    std::vector<std::pair<double, int>> order;
    for (const auto& kv : cost) order.push_back({kv.second, kv.first});
    std::sort(order.begin(), order.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    const int lanes = std::min<int>(linmin_batch_s::kLanes, (int)order.size());
    std::vector<double> load(lanes > 0 ? lanes : 1, 0.0);
    std::map<int, int> lane_of;
    for (const auto& [c, nc] : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[k] += c;
      lane_of[nc] = k;
    }
    for (auto& g : b->ipm) g.lane = lane_of[lm::ipm_shape_nc(g.n)];
    b->lanes = std::max(lanes, 1);
    bool ok = true;
    if (b->lanes > 1) ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k + 1 < b->lanes; ++k)
      ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      linmin_batch_destroy(b);
      return LINMIN_EHIP;
    }
  }
  *out = b;
  return LINMIN_OK;
}

int linmin_batch_run(linmin_batch b, void* stream) {
  if (!b) return LINMIN_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LINMIN_EHIP;
  if (dev != b->dev) return LINMIN_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(b->o.stage_events);
  auto mark = [&](int i) {
    if (ev && hipEventRecord(ev[i], st) != hipSuccess) return LINMIN_EHIP;
    return LINMIN_OK;
  };
  int rc = mark(0);
  for (size_t i = 0; rc == LINMIN_OK && i < b->proj.size(); ++i) {
    const auto& g = b->proj[i];
    rc = from_launch(lm::launch_gemm_proj_batch(g.N, g.jobs, g.start, g.njobs, g.blocks, st));
  }
  if (rc == LINMIN_OK && b->quad.njobs)
    rc = from_launch(lm::launch_quadform_batch(b->quad.jobs, b->quad.start, b->quad.njobs, b->quad.blocks, st));
  if (rc == LINMIN_OK) rc = mark(1);
  // fork the side streams off the caller's stream, launch every group on its
  // stream, join them back
  const int nside = b->lanes - 1;
  if (rc == LINMIN_OK && nside > 0) rc = hip_ok(hipEventRecord(b->fork, st));
  for (int k = 0; rc == LINMIN_OK && k < nside; ++k) rc = hip_ok(hipStreamWaitEvent(b->side[k], b->fork, 0));
  for (size_t i = 0; rc == LINMIN_OK && i < b->ipm.size(); ++i) {
    const auto& g = b->ipm[i];
    hipStream_t gs = g.lane == 0 ? st : b->side[g.lane - 1];
    rc = from_launch(lm::launch_ipm_batch(g.n, b->o.constraint, g.stable, g.b, g.mode, g.fp32, g.code, gs));
  }
  for (int k = 0; k < nside; ++k) {
    // join even after a failed launch, so that no side stream is left forked
    const int r1 = hip_ok(hipEventRecord(b->join[k], b->side[k]));
    const int r2 = hip_ok(hipStreamWaitEvent(st, b->join[k], 0));
    if (rc == LINMIN_OK) rc = r1 != LINMIN_OK ? r1 : r2;
  }
  if (rc == LINMIN_OK) rc = mark(2);
  if (rc == LINMIN_OK) rc = from_launch(lm::launch_cov_batch(b->cov[0], b->cov[1], b->cov[2], st));
  if (rc == LINMIN_OK) rc = mark(3);
  return rc;
}

size_t linmin_batch_device_bytes(linmin_batch b) { return b ? b->ws_bytes + b->tab_bytes : 0; }

int linmin_batch_destroy(linmin_batch b) {
  if (!b) return LINMIN_EINVAL;
  for (int k = 0; k + 1 < linmin_batch_s::kLanes; ++k) {
    if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  (void)hipFree(b->ws);
  (void)hipFree(b->tab);
  delete b;
  return LINMIN_OK;
}

}  // extern "C"

extern "C" {

int linmin_error_maps(linmin_lib lib, int64_t P, const float* cube, const double* coeffs, const double* cov,
                      int cov_layout, double* rms, double* sigma1, void* stream) {
  if (!lib || P < 0) return LINMIN_EINVAL;
  if (P == 0) return LINMIN_OK;
  if ((rms && (!cube || !coeffs)) || (sigma1 && !cov)) return LINMIN_EINVAL;
  if (sigma1 && (cov_layout < LINMIN_COV_FULL || cov_layout > LINMIN_COV_DIAG)) return LINMIN_EINVAL;
  return from_launch(lm::launch_error_maps(lib->N, P, lib->L, cube, coeffs, lib->S, cov, cov_layout, rms, sigma1,
                                           static_cast<hipStream_t>(stream)));
}

int linmin_thresholds(int N, int64_t P, const double* coeffs, const uint8_t* present, double* thresholds,
                      void* stream) {
  if (N < 1 || N > LINMIN_N_MAX || P < 0 || !thresholds || (P > 0 && (!coeffs || !present))) return LINMIN_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* ws = nullptr;
  if (hipMallocAsync((void**)&ws, lm::thresholds_workspace_bytes(N, P), st) != hipSuccess) return LINMIN_ENOMEM;
  int rc = from_launch(lm::launch_thresholds(N, P, coeffs, present, thresholds, ws, st));
  if (hipFreeAsync(ws, st) != hipSuccess && rc == LINMIN_OK) rc = LINMIN_EHIP;
  return rc;
}

int linmin_detect(int N, int64_t P, const double* coeffs, const double* sigma1, const double* rms,
                  const double* thresholds, double rms_max, uint8_t* detected, void* stream) {
  if (N < 1 || N > LINMIN_N_MAX || P < 0) return LINMIN_EINVAL;
  if (P == 0) return LINMIN_OK;
  if (!coeffs || !sigma1 || !rms || !thresholds || !detected) return LINMIN_EINVAL;
  return from_launch(lm::launch_detect(N, P, coeffs, sigma1, rms, thresholds, rms_max, detected,
                                       static_cast<hipStream_t>(stream)));
}

}  // extern "C"

