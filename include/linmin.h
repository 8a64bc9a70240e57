/*
 * linmin.h -- C ABI of lib_linmin, per-pixel constrained linear unmixing of
 * hyperspectral cubes on AMD Instinct MI355X (gfx950).
 *
 * Method (Schmidt, Legendre & Le Mouelic, "Minerals detection for
 * hyperspectral images using adapted linear unmixing: LinMin"):
 *   - linear mixing model X = A S + E (Sec. 2.1, eq. 1);
 *   - per pixel, the least-squares criterion (eq. 2), renormalised by the
 *     noise covariance C^{-1} = L L^T (Sec. 2.3, eqs. 5-6);
 *   - positivity a >= 0 (eq. 3) and sum-to-one 1^T a = 1 (eq. 4), solved by
 *     a primal-dual interior-point method (IPLS, Sec. 2.2) with an exact
 *     finishing step on the identified free set;
 *   - the coefficient covariance "provided by the Hessian" (end of Sec. 2.3).
 *
 * Conventions shared by every entry point:
 *   - Library S: N x L float32, row-major, one reference spectrum per row
 *     (the paper's S).  Cube X: P x L float32, row-major, one pixel spectrum
 *     per row (band-interleaved-by-pixel).  sigma: P float32 per-pixel noise
 *     scales s_p; the pixel's noise covariance is s_p^2 C.
 *   - Outputs are FP64.  Coefficients: P x N row-major.
 *   - Pointers documented as "device" must be device memory (hipMalloc, or a
 *     torch CUDA tensor's data_ptr) on the current HIP device; "host" means
 *     ordinary host memory.  The caller owns every buffer it passes.
 *   - Return codes are LINMIN_OK or a negative LINMIN_E* value; they report
 *     misuse or HIP failures, never per-pixel numerical trouble (that goes
 *     to the optional per-pixel status array).
 */
#ifndef LINMIN_H
#define LINMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct linmin_lib_s *linmin_lib;

/* return codes */
#define LINMIN_OK 0
#define LINMIN_EINVAL (-1)       /* bad argument (NULL, size out of range, N > L, ...) */
#define LINMIN_ENOMEM (-2)       /* device or host allocation failed */
#define LINMIN_EHIP (-3)         /* a HIP runtime call or kernel launch failed */
#define LINMIN_ENOTSPD (-4)      /* noise covariance not symmetric positive definite,
                                    or the library's Gram matrix is not positive */
#define LINMIN_EUNSUPPORTED (-5) /* option combination not built in */
#define LINMIN_ESCRATCH (-6)     /* linmin_unmix_noalloc: the call needs more work
                                    area than LINMIN_NOALLOC_SCRATCH_BYTES */

/* precision of the interior-point iterations */
#define LINMIN_FP64 0  /* every step in FP64 */
#define LINMIN_MIXED 1 /* FP32 Newton steps until mu <= mu_switch, then FP64
                          steps, finishing step and KKT check; a pixel that
                          the finishing step does not certify (or whose
                          steps stop at the cap or lose positive
                          definiteness) is solved again in FP64 from the
                          start, so its outputs and iteration count are
                          those of LINMIN_FP64 */

/* covariance output layouts (per pixel) */
#define LINMIN_COV_NONE 0   /* out_cov ignored */
#define LINMIN_COV_FULL 1   /* N x N row-major */
#define LINMIN_COV_PACKED 2 /* lower triangle row by row, N (N+1) / 2 values */
#define LINMIN_COV_DIAG 3   /* N variances */

/* per-pixel status bits (0 = solved and certified) */
#define LINMIN_PX_MAXIT 1u       /* interior-point iteration cap reached */
#define LINMIN_PX_NONFINITE 2u   /* spectrum has NaN/Inf; outputs are NaN */
#define LINMIN_PX_BAD_SIGMA 4u   /* s_p <= 0 or not finite; covariance and
                                    objective are NaN, coefficients valid */
#define LINMIN_PX_NOT_PD 8u      /* a Newton matrix lost positive definiteness */
#define LINMIN_PX_DEGENERATE 16u /* certified, but some index has both a_i and
                                    its multiplier below deg_tol (no strict
                                    complementarity): covariance is one of
                                    several valid choices */
#define LINMIN_PX_INEXACT 32u    /* the finishing step could not certify the
                                    free set; outputs are the last interior
                                    iterate */

#define LINMIN_N_MAX 128 /* largest library supported */

/* Constraint on the sum of the coefficients besides a >= 0 (eq. 3): the
 * options of IPLS named in the results (Sec. 3.1 and 3.3; the OMEGA run of
 * Sec. 4.1 uses LINMIN_SLO). */
#define LINMIN_STO 0 /* sum-to-one, 1^T a = 1 (eq. 4) */
#define LINMIN_SLO 1 /* sum-lower-than-one, 1^T a <= 1 */
#define LINMIN_POS 2 /* positivity only */

typedef struct {
    int precision;      /* LINMIN_FP64 or LINMIN_MIXED */
    int cov_layout;     /* LINMIN_COV_* */
    int maxit;          /* interior-point iteration cap (default 200) */
    int max_polish;     /* partition corrections in the finishing step (16) */
    int constraint;     /* LINMIN_STO (default), LINMIN_SLO or LINMIN_POS.  With
                           SLO the slack of 1^T a <= 1 and the sum multiplier
                           form one more complementarity pair; the covariance
                           has the sum row only where the constraint binds
                           (none for POS). */
    double tol_mu;      /* stop when mu <= tol_mu (1e-13) ...          */
    double tol_d;       /* ... ||r_d||_inf <= tol_d (1 + ||bh||_inf) (1e-12) */
    double tol_p;       /* ... and |1^T a (+ slack) - 1| <= tol_p (1e-13) */
    double eta;         /* fraction of the step to the boundary (0.99) */
    double lambda0;     /* starting multipliers (0.1) */
    double tau;         /* KKT sign tolerance of the finishing step (1e-11) */
    double deg_tol;     /* strict-complementarity threshold (1e-9) */
    double mu_switch;   /* MIXED: FP32 -> FP64 hand-over point (1e-10); the
                           FP32 stage also hands over after 60 steps or a
                           step below 1e-3 of the way to the boundary */
    uint8_t *status;    /* device, P entries or NULL: LINMIN_PX_* bits */
    int32_t *iters;     /* device, P entries or NULL: interior-point iterations */
    double *objective;  /* device, P entries or NULL: renormalised criterion
                           F_p = (x' - a S')(x' - a S')^T / s_p^2 (eq. 6) */
    void **stage_events; /* NULL, or 4 caller-created hipEvent_t recorded on the
                            stream before the projections, before the
                            interior-point solve, before the covariance pass
                            and after it (stage timing without a profiler) */
    const uint8_t *keep; /* device, P x N or NULL: the second pass of the
                            conclusion (unmix again with the detected spectra
                            only).  Nonzero keeps spectrum i for pixel p; the
                            others are held at a_i = 0 (their projection is
                            replaced by one large negative enough that the
                            result is the minimiser over the kept spectra).
                            A pixel that keeps none is reported
                            LINMIN_PX_NONFINITE.  Batches reject it. */
} linmin_opts;

/* Fill *opts with the defaults quoted above (pointer members NULL). */
void linmin_default_opts(linmin_opts *opts);

/*
 * Build a reference library (Sec. 2.1 S, renormalised per Sec. 2.3).
 *   S          host, N x L float32 row-major (copied).
 *   L, N       1 <= N <= min(L, LINMIN_N_MAX) (the paper limits the number of
 *              spectra to the number of wavelengths, Sec. 2.4).
 *   noise_cov  host, L x L FP64 row-major symmetric positive definite, or
 *              NULL for C = I (copied).
 *   out        receives the handle.
 * Runs synchronously on the current device: it computes W = C^{-1} S^T,
 * the Gram matrix G = S C^{-1} S^T (on MFMA), gamma = max_i G_ii and the
 * scaled copies used by unmix.  The handle is immutable afterwards and may be
 * used from several streams at once.  Errors: EINVAL, ENOMEM, EHIP, ENOTSPD.
 */
int linmin_create_library(const float *S, int L, int N, const double *noise_cov, linmin_lib *out);

/*
 * Unmix P pixels (Sec. 2.2 under eqs. 3-4, renormalised per eq. 6).
 *   cube        device, P x L float32 row-major.
 *   P           >= 0; P == 0 is a no-op.
 *   sigma       device, P float32 s_p, or NULL for s_p = 1.  Coefficients do
 *               not depend on s_p; covariance scales with s_p^2 and the
 *               objective with 1 / s_p^2.
 *   out_coeffs  device, P x N FP64: the mixing coefficients.
 *   out_cov     device, per-pixel covariance in opts->cov_layout (P x N x N,
 *               P x N(N+1)/2 or P x N FP64), or NULL (then no covariance is
 *               computed whatever the layout).
 *   opts        NULL for defaults (FP64, COV_FULL).
 *   stream      hipStream_t to enqueue on, NULL for the default stream.
 * Asynchronous like a kernel launch: returns once the work is enqueued.
 * Temporary device memory (about P (N + 2) doubles) is taken from the
 * stream-ordered allocator and released on the same stream.  Errors:
 * EINVAL (NULL handle/buffers, P < 0), EUNSUPPORTED, ENOMEM, EHIP.
 */
int linmin_unmix(linmin_lib lib, const float *cube, int64_t P, const float *sigma,
                 double *out_coeffs, double *out_cov, const linmin_opts *opts, void *stream);

/* Bytes of temporary device memory linmin_unmix takes for these arguments. */
size_t linmin_workspace_bytes(linmin_lib lib, int64_t P, const linmin_opts *opts);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * linmin_unmix with the same arguments, results and errors, except that its
 * temporary memory is a fixed array of LINMIN_NOALLOC_SCRATCH_BYTES inside
 * the library, one per GPU, held from the first call on that GPU until the
 * process ends.  The call allocates and frees nothing; the caller still
 * passes every input and output.
 *   Limit: linmin_workspace_bytes(lib, P, opts) (with the same out_cov
 *   presence) must not exceed LINMIN_NOALLOC_SCRATCH_BYTES, else the call
 *   returns LINMIN_ESCRATCH and enqueues nothing; split larger cubes into
 *   row ranges (pixels are independent).  For the FP64 path with FULL
 *   covariance that is about 113,000 pixels at N = 36.
 *   Concurrency: every call on one GPU uses that GPU's one array, so calls
 *   whose work overlaps in time on the same GPU (different streams, or
 *   different host threads) race and produce wrong results; order them on
 *   one stream or with events.  The array keeps the last call's contents;
 *   nothing in it needs to start at zero.
 */
#define LINMIN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int linmin_unmix_noalloc(linmin_lib lib, const float *cube, int64_t P, const float *sigma,
                         double *out_coeffs, double *out_cov, const linmin_opts *opts, void *stream);

/* Library shape and scale: any output pointer may be NULL.  gamma is
 * max_i G_ii of the renormalised Gram matrix.  Returns EINVAL for NULL lib. */
int linmin_library_info(linmin_lib lib, int *L, int *N, double *gamma);

/* Copy the renormalised Gram matrix G (N x N FP64) to host memory. */
int linmin_library_gram(linmin_lib lib, double *G_host);

/*
 * The additional spectra of Sec. 2.5 (listed by name after the references),
 * which a caller appends to its mineral library so that the fit can absorb
 * differences of level, slope and large-scale continuum shape between the
 * pixels and the library.  With t in [0, 1] the position along the spectral
 * domain (0 at the first channel, 1 at the last), the rows are
 *   n_extra = 4:  1, 1e-4, t, 1 - t  (flat near one, flat near zero,
 *                 increasing and decreasing slope);
 *   n_extra = 12: those four, then cos, sin, -cos, -sin of 2 pi f t for
 *                 f = 1/4 and then f = 1/2 (periods four and two times the
 *                 spectral domain; both signs because a >= 0).
 * The rows are linearly dependent (rank 2 of 4, 6 of 12): with them the
 * minimiser can be non-unique, and pixels whose free set holds a dependent
 * group are reported through the status bits.
 *   L            channels, >= 2.
 *   n_extra      4 or 12.
 *   wavelengths  host, L strictly increasing finite values, or NULL for
 *                equally spaced channels.
 *   out          host, n_extra x L float32 row-major, caller-owned.
 * Host only, no device work.  Errors: EINVAL (NULL out, L < 2, n_extra not 4
 * or 12, wavelengths not finite and increasing).
 */
int linmin_extra_spectra(int L, int n_extra, const double *wavelengths, float *out);

/*
 * Batches: many cubes, each with its own library (any sizes), unmixed by a
 * few fused launches instead of one sequence of launches per cube.  Pixels
 * are independent (eq. 2 is a sum over pixels), so a batch computes for
 * every cube exactly what linmin_unmix computes for it alone.
 *
 * One cube of a batch: the arguments of linmin_unmix, with the per-pixel
 * arrays that linmin_opts carries for a single call.  Every pointer is
 * device memory (NULL where linmin_unmix allows NULL); out_cov is filled in
 * the layout of the batch's opts->cov_layout.
 */
typedef struct {
    linmin_lib lib;
    const float *cube;   /* P x L */
    int64_t P;           /* >= 0; P == 0 makes the job a no-op */
    const float *sigma;  /* P, or NULL for s_p = 1 */
    double *out_coeffs;  /* P x N */
    double *out_cov;     /* per the batch's cov_layout, or NULL */
    uint8_t *status;     /* P, or NULL */
    int32_t *iters;      /* P, or NULL */
    double *objective;   /* P, or NULL */
} linmin_job;

typedef struct linmin_batch_s *linmin_batch;

/*
 * Plan a batch.  Synchronous on the current device: checks every job,
 * groups the cubes by compiled kernel (projection width, interior-point
 * kernel as linmin_set_kernel has chosen it at this moment), allocates the
 * work areas of all cubes in one device buffer, uploads one job table per
 * launch and creates up to three streams and four events of the batch's own
 * (default priority).  Afterwards linmin_batch_run enqueues
 * the fused launches only: no allocation, no host-to-device copy, so a run
 * may be captured in a HIP graph.
 *   jobs, n_jobs  host array of n_jobs >= 0 jobs (copied; the buffers they
 *                 point to are not, and must stay valid for every run).
 *   opts          NULL for defaults; its precision, layout, constraint and
 *                 tolerances apply to every job; its status / iters /
 *                 objective members are ignored (each job carries its own)
 *                 and its keep member must be NULL;
 *                 stage_events, if set, are recorded by every run.
 * The libraries must outlive the batch.  Errors: EINVAL (NULL out, a job
 * with a NULL library or a library of another device, P < 0, NULL cube or
 * out_coeffs with P > 0), EUNSUPPORTED, ENOMEM, EHIP.
 */
int linmin_batch_create(const linmin_job *jobs, int n_jobs, const linmin_opts *opts, linmin_batch *out);

/*
 * Enqueue every job of the batch on stream (NULL: the default stream):
 * projections, interior-point solves and covariance, each stage as one
 * launch per compiled shape over all cubes of that shape.  The
 * interior-point launches of different library sizes run concurrently on
 * the batch's streams, forked from stream after the projections and joined
 * back to it before the covariance (events only, so a run captured from
 * stream into a HIP graph captures the fork and the join).  Asynchronous
 * like a kernel launch.  Runs of one batch share its work areas and
 * streams: two runs in flight at once race.  Errors: EINVAL (NULL batch,
 * other device current), EHIP.
 */
int linmin_batch_run(linmin_batch batch, void *stream);

/* Device bytes the batch holds (work areas and job tables); 0 for NULL. */
size_t linmin_batch_device_bytes(linmin_batch batch);

/* Release a batch (after all its runs have completed). */
int linmin_batch_destroy(linmin_batch batch);

/*
 * Detection post-processing (Sec. 3.1 and 4).  All pointers are device
 * memory; every call is asynchronous on stream (NULL: default stream).
 *
 * linmin_error_maps: per pixel the RMS of the fit, the root mean square over
 * the L channels of the residual y - a S in reflectance units (Sec. 3.1;
 * not whitened by a noise covariance), from the cube (P x L float32) and
 * the coefficients (P x N) of linmin_unmix; and per coefficient the 1-sigma
 * error, the square root of the covariance diagonal (cov in cov_layout as
 * written by linmin_unmix).  rms (P) or sigma1 (P x N) may be NULL to skip
 * it; NaN inputs give NaN.  Errors: EINVAL.
 */
int linmin_error_maps(linmin_lib lib, int64_t P, const float *cube, const double *coeffs, const double *cov,
                      int cov_layout, double *rms, double *sigma1, void *stream);

/*
 * Detection threshold of eq. 8 for each of N endmembers, from coefficients
 * (P x N) of pixels where each endmember is known present (present: P x N,
 * nonzero) or absent: half the sum of (mean - 2 std) over present pixels and
 * (mean + 6 std) over absent ones, population standard deviations; NaN for
 * an endmember with no present or no absent pixel.  thresholds: N doubles.
 * Takes a small stream-ordered workspace.  Errors: EINVAL, ENOMEM, EHIP.
 */
int linmin_thresholds(int N, int64_t P, const double *coeffs, const uint8_t *present, double *thresholds,
                      void *stream);

/*
 * Detection rules of Sec. 4: detected[p][i] = 1 when coeffs[p][i] exceeds
 * thresholds[i], sigma1[p][i] < coeffs[p][i] (a significant coefficient) and
 * rms[p] < rms_max (a fit at the noise level), else 0.  P x N bytes.  The
 * result may serve as linmin_opts.keep of a second pass.  Errors: EINVAL.
 */
int linmin_detect(int N, int64_t P, const double *coeffs, const double *sigma1, const double *rms,
                  const double *thresholds, double rms_max, uint8_t *detected, void *stream);

/*
 * Interior-point kernel choice.  Every family below is a complete
 * implementation of the same solve (Sec. 2.2); they differ in how a pixel's
 * Newton matrix is mapped onto the GPU, and which is fastest depends on the
 * library size.  Without a choice, a library of N uses the first family
 * compiled for its padded size NC in the order ROWCYCLIC, TILE, GROUP (FP64
 * kernels: the FP64 path and the mixed form's second stage) or TILE32,
 * GROUP (the mixed form's FP32 stage).  A tuning table measured on the
 * device (paper_1402_2518_amd/autotune.py) installs its choices here.
 */
#define LINMIN_KERNEL_DEFAULT 0   /* the rule above */
#define LINMIN_KERNEL_ROWCYCLIC 1 /* FP64, one pixel per wavefront, 4x4x4 FP64 matrix cores */
#define LINMIN_KERNEL_TILE 2      /* FP64, four pixels per wavefront, 4x4x4 FP64 matrix cores */
#define LINMIN_KERNEL_GROUP 3     /* FP64 or FP32, a group of lanes per pixel, vector units */
#define LINMIN_KERNEL_TILE32 4    /* FP32, sixteen pixels per wavefront, 4x4x1 FP32 matrix cores */
#define LINMIN_STAGE_FP64 0       /* the FP64 interior-point kernels */
#define LINMIN_STAGE_FP32 1       /* the FP32 stage of LINMIN_MIXED */

/*
 * Use family for the interior-point solves of stage for every library whose
 * padded size equals that of a library of N (1 <= N <= LINMIN_N_MAX), in
 * this process, for unmix calls enqueued and batches created afterwards
 * (work already enqueued and batches already created keep their kernels;
 * safe to call from any thread).  lanes: for LINMIN_KERNEL_GROUP the lanes
 * per pixel (0 = the default width), else 0.  LINMIN_KERNEL_DEFAULT
 * restores the rule.  Errors: EINVAL (N, stage, family or lanes out of
 * range), EUNSUPPORTED (that kernel is not compiled for the size and stage).
 */
int linmin_set_kernel(int N, int stage, int family, int lanes);

/* The family a library of N uses for stage now (a LINMIN_KERNEL_* value
 * other than DEFAULT), with its group width in *lanes (0 for the other
 * families; lanes may be NULL), or EINVAL. */
int linmin_get_kernel(int N, int stage, int *lanes);

/* Release a library (after all work using it has completed). */
int linmin_destroy_library(linmin_lib lib);

/* Static text for a return code. */
const char *linmin_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* LINMIN_H */
