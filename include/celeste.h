/*
 * celeste.h — C ABI of the MI355X (gfx950) Celeste ELBO / trust-region Newton library.
 *
 * Celeste (Regier et al., "Learning an Astronomical Catalog of the Visible Universe
 * through Scalable Bayesian Inference", IPDPS 2017) infers a catalog of stars and
 * galaxies from multi-band images.  Section III-A defines the model (Poisson pixel
 * counts whose rates are a deterministic function of the catalog and each image's
 * metadata), section III-B the variational objective (the ELBO of Eq. 1 under a
 * mean-field q), its per-source decomposition with neighbours held fixed, and its
 * optimisation by trust-region Newton with a hand-derived gradient and dense Hessian.
 * Section III-C lists what one source needs: the images containing it, its initial
 * estimate and its neighbours' estimates.  This header exports exactly that work.
 *
 * Conventions (all entry points):
 *   - Return codes: CELESTE_OK (0) or a negative CELESTE_E_* code; the message of the
 *     last failing call on the calling host thread is returned by celeste_last_error().
 *     Non-convergence of a fit is a per-source status, not a call error.
 *   - Ownership: every buffer is owned by the caller.  The library keeps no pointer
 *     after a call returns.  Device scratch lives in the context and is reused.
 *   - Memory kinds: celeste_batch.mem_kind says where the pixel arrays (and the theta /
 *     output arrays passed with that batch) live: CELESTE_MEM_HOST or CELESTE_MEM_DEVICE
 *     (device pointers of the context's device).  The metadata structs themselves
 *     (images, offsets, prior, profiles, options, results) are always host memory.
 *   - Threading: a context is not thread-safe; use one context per host thread.
 *   - Precision: per-pixel arithmetic is FP32; pixel-sum accumulation, the ELBO, the
 *     gradient, the Hessian and the 27x27 trust-region subproblem are FP64.
 *
 * Parameter vector (27 natural coordinates per source; derivatives are reported in
 * these coordinates):
 *   0,1   u: source-frame position (px)            2   a = q(source is a star)
 *   3     e_dev: weight of the de Vaucouleurs profile   4 e_axis: minor/major ratio
 *   5     e_angle: major-axis angle (rad, CCW from +x)   6 e_scale: half-light radius (px)
 *   7,8   r1[star, galaxy]: mean of log reference-band (r) brightness (ln nMgy)
 *   9,10  r2[star, galaxy]: variance of log reference-band brightness
 *   11-14 c1[star][0..3], 15-18 c1[galaxy][0..3]: colour means (log ratios u/g.. of
 *         adjacent bands: c_j = log(l_{j+1} / l_j), bands u,g,r,i,z = 0..4)
 *   19-22 c2[star][0..3], 23-26 c2[galaxy][0..3]: colour variances (diagonal q)
 * Hessians are row-major 27x27.
 */
#ifndef CELESTE_H
#define CELESTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CELESTE_NP 27
#define CELESTE_MAX_PSF 4
#define CELESTE_MAX_PROTO 8

enum {
  CELESTE_OK = 0,
  CELESTE_E_INVALID = -1,      /* bad shape, range, NaN, band, or count */
  CELESTE_E_NOMEM = -2,        /* device or host allocation failed */
  CELESTE_E_DEVICE = -3,       /* a HIP runtime call failed */
  CELESTE_E_UNSUPPORTED = -4   /* valid request the library or the device does not support */
};

enum { CELESTE_MEM_HOST = 0, CELESTE_MEM_DEVICE = 1 };

enum {                          /* per-source fit status */
  CELESTE_CONVERGED = 0,        /* predicted gain below tolerance at a concave point */
  CELESTE_MAX_ITER = 1,         /* iteration cap reached */
  CELESTE_TR_COLLAPSED = 2,     /* trust radius fell below delta_min */
  CELESTE_NONFINITE = 3,        /* the starting point has a non-finite ELBO */
  CELESTE_LINE_SEARCH_FAILED = 4 /* L-BFGS: no sufficient decrease within max_backtracks halvings */
};

enum {                          /* start of a fit */
  CELESTE_INIT_AS_GIVEN = 0,    /* theta_inout as passed */
  CELESTE_INIT_PLAIN = 1,       /* plain start from the data around theta_inout's position */
  CELESTE_INIT_SURROGATE = 2    /* surrogate network's start, or the plain start where its ELBO is higher */
};

enum { CELESTE_FLAG_FALLBACK_USED = 1 };   /* per-source result flag: the plain start was kept */

enum {                          /* context options (celeste_ctx_set_option) */
  CELESTE_OPT_CHUNK_PX = 1,     /* pixels per work item (64 .. 2^24; default 4096) */
  CELESTE_OPT_BLOCK = 2,        /* threads per pixel-kernel block: 128 or 256 (default 256) */
  CELESTE_OPT_USE_GRAPH = 3,    /* batched fit replays a captured HIP graph per iteration (default 1) */
  CELESTE_OPT_PROFILE = 4,      /* 1: time every kernel phase with HIP events (fits run without a graph) */
  CELESTE_OPT_VARIANT = 5,      /* pixel-kernel variant 0..7 (default 3): bit 0 = register budget of
                                   three resident waves per SIMD for the value+gradient+Hessian
                                   kernel (two with bit 2; otherwise the kernel takes two), bit 1 =
                                   loops unrolled for 6 exp + 8 dev components (both kernels), bit 2
                                   (with bit 1) = the J^T W J part of the Hessian summed on the
                                   matrix cores; all variants compute the same quantities, to FP32
                                   rounding */
  CELESTE_OPT_TILE_W = 6,       /* width of the 64-pixel tile a wavefront of the value+gradient+Hessian
                                   kernel takes per step: 8, 16, 32 or 64 (default 8) */
  CELESTE_OPT_VALUE_BLOCK = 7,  /* threads per value-kernel block: 128 or 256 (default 256) */
  CELESTE_OPT_VALUE_TILE_W = 8, /* tile width of the value kernel: 8, 16, 32 or 64 (default 8) */
  CELESTE_OPT_EXACT_ZERO = 9,   /* skip threshold of the value+gradient+Hessian kernel: a mixture
                                   component whose density is below 2^-v on a whole tile is skipped.
                                   160 (always exact: below the smallest FP32 subnormal), 127 (exact
                                   where the device's exp2 flushes results below 2^-126 to zero, which
                                   the context checks at creation; E_UNSUPPORTED elsewhere), 0 for
                                   the context's choice (127 where exact, else 160; the default), or
                                   1 to skip nothing: every component, galaxy group and tile is
                                   evaluated (the reference the skips are tested against) */
  CELESTE_OPT_PERSISTENT = 10,  /* trust-region fits (celeste_newton_fit, celeste_batch_fit): before
                                   each value+gradient+Hessian pass the work items of the sources
                                   still being fitted are compacted into a device list, and a
                                   persistent grid of the pixel kernel draws them in turn (grids do
                                   not shrink otherwise: blocks of finished sources exit at once).
                                   n in 1..16 = n blocks per compute unit; -1 (default) = as many
                                   blocks per compute unit as the launched kernel instance keeps
                                   resident (its register budget, CELESTE_OPT_VARIANT bit 0);
                                   0 = one block per work item. Results are bitwise the same */
  CELESTE_OPT_TR_CHOLESKY = 11, /* trust-region subproblem (section III-B): 1 = where -H is positive
                                   definite, Cholesky factorisations of -H + lam I give the exact
                                   solution (lam = 0 for a Newton step inside the region, else
                                   Newton's method on lam for the step on the boundary); otherwise,
                                   and always with 0, the eigendecomposition and secular equation
                                   (default 1).  The two differ by rounding */
  CELESTE_OPT_FP64_SUMS = 12,   /* value+gradient+Hessian kernel: 1 = each tile step's FP32 gradient
                                   and Hessian pixel terms are summed across the wavefront in FP64,
                                   so every pixel sum is FP64 from the first addition (about 10%
                                   slower); 0 = FP32 sums per lane over up to 16 tile steps and an
                                   FP32 wavefront butterfly before FP64 (default).  The ELBO value is
                                   summed in FP64 per lane either way */
  CELESTE_OPT_TRIAL_DERIVATIVES = 13  /* trust-region fits (celeste_newton_fit, celeste_batch_fit;
                                   section III-B): 1 = each iteration evaluates the ELBO with its
                                   gradient and Hessian at the trial point, and an accepted step
                                   takes them over, so the next iteration needs no evaluation at
                                   its new point (one value+gradient+Hessian pass before the first
                                   iteration; default); 0 = the ELBO alone at the trial point and
                                   the gradient and Hessian at each newly accepted point.  Both run
                                   the same algorithm; they differ by the rounding of the summed
                                   ELBO values the ratio test compares.  n_full_evals counts every
                                   value+gradient+Hessian evaluation of a source (with 1: its
                                   iterations + 1) */
};

/* Cumulative work and time counters of a context (since creation or the last reset). */
typedef struct celeste_stats {
  int64_t full_px;              /* pixel evaluations by the value+gradient+Hessian kernel */
  int64_t value_px;             /* pixel evaluations by the value-only kernel */
  int64_t full_launches;        /* launches of the value+gradient+Hessian pixel kernel */
  int64_t value_launches;       /* launches of the value-only pixel kernel */
  int64_t iterations;           /* trust-region iterations enqueued (all sources together) */
  /* milliseconds per phase, measured with HIP events on the library's stream; only
   * accumulated while CELESTE_OPT_PROFILE is set */
  double ms_setup, ms_full, ms_reduce_full, ms_tr, ms_value, ms_reduce_value, ms_accept;
  /* host wall-clock milliseconds of the fits' other stages (CELESTE_OPT_PROFILE only): packing and
   * validating the batch on the host, uploading metadata and checking pixels, choosing the start
   * (start evaluations; the network in ms_net below), and the iterations' polling and result
   * download */
  double ms_host_pack, ms_prepare, ms_start, ms_loop, ms_results;
  /* linear-response covariance launches, and their kernel milliseconds (CELESTE_OPT_PROFILE only) */
  int64_t lr_launches;
  double ms_lr;
  /* value+gradient pixel kernel (celeste_elbo_eval without a Hessian, L-BFGS fits): pixel
   * evaluations, launches, and milliseconds of the kernel, its reduction and the L-BFGS direction
   * and line-search kernels (the milliseconds under CELESTE_OPT_PROFILE only) */
  int64_t grad_px, grad_launches;
  double ms_grad, ms_reduce_grad, ms_lbfgs;
  /* trust-region subproblems solved by the interior Newton step (one Cholesky factorisation),
   * by the boundary step from Cholesky factorisations of -H + lam I, and by the
   * eigendecomposition and secular equation (CELESTE_OPT_TR_CHOLESKY) */
  int64_t tr_interior, tr_boundary, tr_eigen;
  /* host wall-clock milliseconds of the surrogate network's inference (patches, forward pass and
   * the map to parameters) in a surrogate start (CELESTE_OPT_PROFILE only; ms_start then holds the
   * rest of the start: plain start and the evaluation of both starts) */
  double ms_net;
  /* Jacobi sweeps of the eigendecomposition solves, the solves that reached the 40-sweep cap, and
   * Newton steps on the multiplier of the boundary solves by Cholesky */
  int64_t tr_sweeps, tr_sweep_cap, tr_newton_steps;
  /* blocks of the last trust-region fit's persistent value+gradient+Hessian grid (0: one block per
   * work item; CELESTE_OPT_PERSISTENT) */
  int64_t fit_grid_blocks;
  /* with CELESTE_OPT_TRIAL_DERIVATIVES: pixel evaluations of the value+gradient+Hessian passes at
   * trial points (included in full_px), and the pixels of the sources at each accepted step (the
   * value+gradient+Hessian evaluations that iterations without trial derivatives make at the new
   * points); both 0 otherwise */
  int64_t trial_full_px, taken_px;
} celeste_stats;

typedef struct celeste_ctx celeste_ctx;
typedef struct celeste_net celeste_net;

/* One band image cut-out ("patch") seen by one source (section III-A: image n has
 * metadata Lambda_n and pixels x_nm ~ Poisson(F_nm)).  Pixel element (r, c) is centred
 * at image-frame coordinates origin + (c, r); the model density is sampled there. */
typedef struct celeste_image {
  int32_t band;                 /* 0..4 = u,g,r,i,z (reference band r = 2) */
  int32_t h, w;                 /* patch rows and columns, >= 1 */
  int32_t pitch;                /* elements between rows of pixels/nbr arrays, >= w */
  int32_t n_psf;                /* PSF mixture components, 1..CELESTE_MAX_PSF */
  int32_t nbr_pitch;            /* elements between rows of nbr_mean/nbr_var (>= w), or 0 = pitch */
  double origin[2];             /* image-frame (x, y) of element (0,0)'s centre */
  double wcs[6];                /* p = A u + b: A row-major 2x2 (wcs[0..3]), b (wcs[4..5]) */
  double sky;                   /* sky level epsilon_n, counts per pixel, > 0 */
  double calib;                 /* iota_n, counts per nMgy, > 0 */
  double psf[CELESTE_MAX_PSF][6]; /* weight, mean_x, mean_y, cov_xx, cov_xy, cov_yy (px) */
  const float* pixels;          /* counts x_nm, h rows of `pitch` floats */
  const float* nbr_mean;        /* optional fixed E[F] of other sources (counts/px), or NULL */
  const float* nbr_var;         /* optional fixed Var[F] of other sources, or NULL */
} celeste_image;

/* Prior parameters Phi (P(star)), Upsilon (lognormal brightness) and Xi (colours),
 * section III-A; index 0 = star, 1 = galaxy. */
typedef struct celeste_prior {
  double p_star;
  double r_mean[2], r_var[2];   /* normal prior on log r-band brightness */
  double c_mean[2][4];
  double c_cov[2][4][4];        /* full colour covariance, symmetric positive definite */
} celeste_prior;

/* Galaxy prototype profiles: exponential and de Vaucouleurs, each a mixture of
 * isotropic zero-mean Gaussians with amplitude amp[j] and variance var[j] in units
 * of the half-light radius squared.  Amplitudes of each mixture sum to 1. */
typedef struct celeste_profiles {
  int32_t n_exp, n_dev;         /* 1..CELESTE_MAX_PROTO each */
  double exp_amp[CELESTE_MAX_PROTO], exp_var[CELESTE_MAX_PROTO];
  double dev_amp[CELESTE_MAX_PROTO], dev_var[CELESTE_MAX_PROTO];
} celeste_profiles;

/* A batch of independent sources (section III-B: each source is optimised with the
 * others held fixed).  Source s owns images[image_offsets[s] .. image_offsets[s+1]). */
typedef struct celeste_batch {
  int32_t n_sources;            /* >= 1 */
  int32_t mem_kind;             /* CELESTE_MEM_HOST or CELESTE_MEM_DEVICE */
  const int64_t* image_offsets; /* host, n_sources + 1 entries, non-decreasing, [0] = 0 */
  const celeste_image* images;  /* host array of image_offsets[n_sources] entries */
  const celeste_prior* prior;   /* host */
  const celeste_profiles* profiles; /* host */
} celeste_batch;

typedef struct celeste_fit_opts {
  int32_t max_iter;             /* trust-region iterations, >= 1 (default 50) */
  int32_t init_mode;            /* CELESTE_INIT_AS_GIVEN or CELESTE_INIT_PLAIN */
  double pred_rtol;             /* converged when predicted gain <= pred_rtol * max(1,|L|) (1e-8) */
  double curv_tol;              /* ... and lambda_min(-H) >= -curv_tol * max(1, |lambda|max) (1e-8) */
  double delta0, delta_max, delta_min;  /* trust radius: start 1, cap 100, collapse 1e-10 */
  double eta;                   /* acceptance threshold on rho (0.1) */
  double u_box;                 /* half-width (px) of the position box around the start (3) */
  int32_t poll_every;           /* batched fit: iterations between host reads of the active count */
  int32_t reserved;
} celeste_fit_opts;

typedef struct celeste_fit_result {
  double elbo;                  /* ELBO at the returned parameters */
  double pred_gain;             /* last predicted gain of the trust-region model */
  double delta;                 /* final trust radius */
  int32_t iters;                /* trust-region iterations taken */
  int32_t status;               /* CELESTE_CONVERGED, ... */
  int32_t n_full_evals;         /* value+gradient+Hessian evaluations */
  int32_t flags;                /* CELESTE_FLAG_* bits */
  int32_t n_accepted;           /* steps accepted by the ratio test (L-BFGS: by the line search) */
  int32_t reserved;             /* 0 */
} celeste_fit_result;

/* Create a context on HIP device `hip_device` (makes it current).  *out receives the
 * context; destroy it with celeste_ctx_destroy.  Errors: E_INVALID (bad device),
 * E_DEVICE, E_NOMEM. */
int celeste_ctx_create(int hip_device, celeste_ctx** out);
void celeste_ctx_destroy(celeste_ctx* ctx);

/* Message for the last failing call on this host thread ("" if none). */
const char* celeste_last_error(void);

/* Set a tuning option of the context (CELESTE_OPT_*).  The options change only how the
 * pixel sums are grouped or how the trust-region subproblem is solved (results move by
 * rounding, far inside the stated tolerances);
 * CELESTE_OPT_EXACT_ZERO changes only which exactly-zero work is skipped (results are
 * bitwise the same).
 * Errors: E_INVALID (unknown option or value out of range). */
int celeste_ctx_set_option(celeste_ctx* ctx, int option, int64_t value);

/* Read (and optionally reset) the context's counters.  Errors: E_INVALID, E_DEVICE. */
int celeste_ctx_get_stats(celeste_ctx* ctx, celeste_stats* out, int reset);

/* sizeof of the ABI structs, for bindings to check their layouts: 0 celeste_image,
 * 1 celeste_prior, 2 celeste_profiles, 3 celeste_batch, 4 celeste_fit_opts,
 * 5 celeste_fit_result, 6 celeste_stats, 7 celeste_tune_result, 8 celeste_lbfgs_opts; 0 for any
 * other value. */
size_t celeste_struct_size(int which);

/* Defaults for celeste_fit_opts (values in the comments above). */
void celeste_fit_opts_default(celeste_fit_opts* opts);

/* ELBO, gradient and dense Hessian of every source of the batch at theta
 * (sections III-A/B: L = sum over the source's images and pixels of the expected
 * Poisson log-likelihood, with E[log F] by the second-order delta method, minus the
 * Kullback-Leibler terms of q(a), q(r|a), q(c|a) from their priors).
 *   theta : n_sources x 27 (natural coordinates)
 *   elbo  : n_sources
 *   grad  : n_sources x 27, or NULL
 *   hess  : n_sources x 27 x 27 row-major, or NULL (requires grad); with grad and no hess the
 *           value+gradient pixel kernel runs (no Hessian work), with neither the value kernel
 *   stream: hipStream_t to run on, or NULL for the context's stream.  The call
 *           returns after the results are written (host or device memory).
 * Pixel arrays are checked on the device first: any negative or non-finite pixel or
 * neighbour value makes the call fail with E_INVALID before any evaluation.
 * Errors: E_INVALID (validation; nothing is launched), E_DEVICE, E_NOMEM. */
int celeste_elbo_eval(celeste_ctx* ctx, const celeste_batch* batch, const double* theta,
                      double* elbo, double* grad, double* hess, void* stream);

/* Size of the device array that celeste_elbo_eval_noalloc works in (64 MiB on each GPU). */
#define CELESTE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* celeste_elbo_eval for callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same kernels and results
 * (bitwise equal to celeste_elbo_eval under the same context options), with no hipMalloc,
 * hipHostMalloc, hipFree or other allocating library call during the call.  Device memory
 * for the packed metadata, setup tables, partial sums and flags comes from one library-wide
 * array of CELESTE_NOALLOC_SCRATCH_BYTES per GPU, resident until the process ends; its
 * device address is taken once per GPU when a context is created there.  Host-side packing
 * uses the process heap.  Every call on a GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU (from several threads, or on streams that
 * run concurrently) race and must be serialised by the caller.
 *   batch: mem_kind must be CELESTE_MEM_DEVICE (host batches need staging memory);
 *   theta, elbo, grad, hess: device memory, as celeste_elbo_eval; stream as there.
 * The call returns after the results are written.  About 4.9 KB per image (3 PSF
 * components), 16 B per work item plus 624 B (value only: 8 B) per work item, 0.5 MB fixed:
 * a batch of about 11,000 images fits.
 * Errors: as celeste_elbo_eval; E_INVALID for a host batch; E_NOMEM (nothing launched) when
 * the batch needs more than CELESTE_NOALLOC_SCRATCH_BYTES, with the size in the message. */
int celeste_elbo_eval_noalloc(celeste_ctx* ctx, const celeste_batch* batch, const double* theta,
                              double* elbo, double* grad, double* hess, void* stream);

/* Pixel-subsampled estimate of the same quantities (the paper's closing section names
 * subsampling pixels, a second source of randomness in the stochastic optimisation, as a
 * further speed-up).  Each image is cut into 8-row blocks (the last one may be shorter);
 * a kept block's pixels weigh 1 / keep_prob, a dropped block's weigh 0, and the part of
 * every pixel's term that does not depend on theta (x log E_bg - E_bg - lgamma(x + 1),
 * E_bg = sky + neighbour mean) is summed over all pixels.  With blocks kept independently
 * with probability keep_prob the estimate is unbiased for celeste_elbo_eval's results;
 * an all-ones keep with keep_prob 1 gives them exactly.  Only kept blocks are evaluated.
 *   keep     : host array, keep_off[n_images] bytes; keep[keep_off[i] + j] != 0 keeps
 *              rows [8j, 8j + 8) of image i (image order of the batch)
 *   keep_off : host array of n_images + 1 offsets; keep_off[0] == 0 and
 *              keep_off[i + 1] - keep_off[i] == (h_i + 7) / 8
 *   keep_prob: in (0, 1]
 * Other arguments as celeste_elbo_eval.  Both host arrays are read before the call
 * returns and stay owned by the caller.  Errors: as celeste_elbo_eval; E_INVALID for a
 * NULL keep / keep_off, keep_prob outside (0, 1] or offsets that do not match the
 * image heights. */
int celeste_elbo_eval_sampled(celeste_ctx* ctx, const celeste_batch* batch, const double* theta,
                              const uint8_t* keep, const int64_t* keep_off, double keep_prob,
                              double* elbo, double* grad, double* hess, void* stream);

/* Linear-response covariance of fitted sources (the paper's closing section proposes linear
 * response methods, after Giordano et al. 2015, because a factorised q under-estimates the
 * posterior variance and point-estimated parameters get none).  At a fitted theta, tilting the
 * objective by t theta_i moves the optimum by d theta / dt = Sigma e_i with
 *   Sigma = D (-H_psi)^{-1} D,   H_psi = D H D + diag(D' g),
 * where psi are the fit's unconstrained coordinates (position box of half-width u_box around
 * u0, logistic boxes of a, e_dev, e_axis, e_scale, logs of the variances), D = d theta / d psi
 * (diagonal), and g, H the natural gradient and Hessian of the ELBO.  A coordinate held at a
 * box edge gets (near) zero variance; at an interior stationary point Sigma = -H^{-1}.
 * Entries of u, a, e_*, r1 and c1 are covariances of first moments of q or of point
 * estimates; rows of r2 and c2 are sensitivities of the variance parameters.  FP64 Cholesky
 * per source, one wavefront each.
 *   theta : n x 27 natural coordinates      u0 : n x 2 position-box centres of the fit
 *   grad  : n x 27, hess : n x 27 x 27 (row-major; symmetrised before use)
 *   cov   : n x 27 x 27 out, row-major, exactly symmetric; NaN where status != 0
 *   status: host array of n: 0, 1 (-H_psi not positive definite: no strict local maximum),
 *           2 (a non-finite input)
 * theta, u0, grad, hess and cov are in mem_kind memory (CELESTE_MEM_HOST or _DEVICE).
 * Errors: E_INVALID (NULL pointers, n out of range, u_box not > 0), E_DEVICE, E_NOMEM. */
int celeste_lr_covariance_from_hessian(celeste_ctx* ctx, int64_t n, int mem_kind, const double* theta,
                                       const double* u0, double u_box, const double* grad, const double* hess,
                                       double* cov, int32_t* status, void* stream);

/* The same for every source of a batch, with gradient and Hessian evaluated at theta by the
 * pixel sum (celeste_elbo_eval) first.  theta, u0 and cov in batch->mem_kind memory; status a
 * host array of n_sources.  Errors: as celeste_elbo_eval and celeste_lr_covariance_from_hessian. */
int celeste_lr_covariance(celeste_ctx* ctx, const celeste_batch* batch, const double* theta, const double* u0,
                          double u_box, double* cov, int32_t* status, void* stream);

/* Trust-region Newton fit of ONE source (batch->n_sources must be 1), host-driven:
 * one host/device round trip per iteration (section III-B).  theta_inout: 27 natural
 * coordinates in (start) and out (result), in batch->mem_kind memory.  Returns the
 * per-source status in *result.  Errors as for celeste_elbo_eval. */
int celeste_newton_fit(celeste_ctx* ctx, const celeste_batch* batch, double* theta_inout,
                       const celeste_fit_opts* opts, celeste_fit_result* result);

/* Trust-region Newton fit of all sources of the batch at once: every iteration is one
 * launch per step over all still-active sources (ragged images and patch sizes),
 * per-source trust-region state stays on the device, and iterations are replayed from
 * a captured HIP graph.  theta_inout: n_sources x 27 (batch->mem_kind memory);
 * results: host array of n_sources.  With init_mode CELESTE_INIT_PLAIN the start is
 * computed on the device from the data (theta_inout's u entries give the catalog
 * position).  Errors as for celeste_elbo_eval. */
int celeste_batch_fit(celeste_ctx* ctx, const celeste_batch* batch, double* theta_inout,
                      const celeste_fit_opts* opts, celeste_fit_result* results, void* stream);

/* celeste_batch_fit with a pixel-subsampled early phase (the paper's closing section proposes
 * subsampling pixels, a second source of randomness in stochastic optimisation, as a speed-up).
 * Every source first fits the unbiased subsampled estimate of its ELBO that
 * celeste_elbo_eval_sampled computes for the same keep / keep_off / keep_prob (kept 8-row blocks
 * weighted 1 / keep_prob, the theta-free part of every pixel summed whole): trust-region
 * iterations whose gradient, Hessian and trial values come from the kept blocks only.  When the
 * model's predicted gain there is at most switch_rtol max(1, |L|), the source re-evaluates its
 * current point on the full ELBO (that step is not an iteration) and continues with full
 * evaluations, the trust radius it reached and opts' stopping rule; max_iter counts both
 * phases.  Masks as in celeste_elbo_eval_sampled (host arrays, read before the call returns);
 * other arguments and results as celeste_batch_fit.  Errors as there; E_INVALID for NULL masks,
 * keep_prob outside (0, 1], switch_rtol <= 0 or offsets that do not match the image heights. */
int celeste_batch_fit_sampled(celeste_ctx* ctx, const celeste_batch* batch, double* theta_inout,
                              const celeste_fit_opts* opts, const uint8_t* keep, const int64_t* keep_off,
                              double keep_prob, double switch_rtol, celeste_fit_result* results, void* stream);

/* Options of the L-BFGS fit (celeste_lbfgs_fit). */
typedef struct celeste_lbfgs_opts {
  int32_t max_iter;             /* accepted steps (gradient evaluations - 1), >= 1 (default 1000) */
  int32_t memory;               /* curvature pairs kept, 1..32 (default 10) */
  int32_t max_backtracks;       /* halvings of the step per line search, 1..60 (default 30) */
  int32_t init_mode;            /* CELESTE_INIT_AS_GIVEN, _PLAIN or _SURROGATE (as celeste_fit_opts) */
  int32_t poll_every;           /* loop steps between host reads of the active count (default 4) */
  int32_t max_loops;            /* cap on loop steps (one gradient and/or one trial value pass per
                                   source each); 0 = 4 * max_iter + 64 (default 0) */
  double pred_rtol;             /* converged when -g'p/2 <= pred_rtol * max(1, |L|) (1e-8) */
  double armijo_c1;             /* sufficient-decrease constant, in (0, 1/2) (1e-4) */
  double u_box;                 /* half-width (px) of the position box around the start (3) */
} celeste_lbfgs_opts;

/* Defaults for celeste_lbfgs_opts (values in the comments above). */
void celeste_lbfgs_opts_default(celeste_lbfgs_opts* opts);

/* Limited-memory BFGS fit of all sources of the batch: the optimiser of the earlier Celeste,
 * which section III-B reports needed thousands of iterations on some sources before trust-
 * region Newton replaced it; built to compare the two on the same data and hardware.  The
 * same unconstrained coordinates, starts and pixel sums as celeste_batch_fit, without the
 * Hessian: every loop step evaluates the value and gradient (value+gradient pixel kernel) of
 * the sources that accepted a step, forms their L-BFGS directions by the two-loop recursion
 * (Nocedal & Wright, Algorithm 7.4; initial scaling s'y / y'y, unit-length first step), and
 * evaluates one trial point per source in a line search (backtracking by halving from step 1
 * until f(psi + a p) <= f(psi) + c1 a g'p for f = -ELBO; pairs with s'y <= 1e-10 |s||y| are not
 * stored; a non-descent direction restarts from the scaled negative gradient).  Converged when
 * the quasi-Newton model's predicted gain -g'p/2 is at most pred_rtol max(1, |L|).
 * theta_inout and results as celeste_batch_fit; results[i].iters = accepted steps,
 * n_full_evals = value+gradient evaluations, delta = the last accepted step length, pred_gain =
 * the last predicted gain.  State per source on the device: 2 memory x 27 + 40 FP64 values.
 * Errors as for celeste_batch_fit; E_INVALID for options out of range. */
int celeste_lbfgs_fit(celeste_ctx* ctx, const celeste_batch* batch, double* theta_inout,
                      const celeste_lbfgs_opts* opts, celeste_fit_result* results, void* stream);

/* ----------------------------------------------------------------------------------------
 * Surrogate initialiser network.  A convolutional network maps a source's 5-band 32x32
 * patch (each band's first image, centre-cropped or zero-padded around the source's
 * position, scaled (x - sky) / sqrt(sky)) to its 27 parameters in standardised
 * unconstrained coordinates: psi = psi_mean + psi_std * output, theta = T(psi) with the
 * position box centred on the catalog position.  Layers: 3x3 convolutions 5->32->64->64->128
 * (ReLU; 2x2 max-pool after the last three), dense 2048->256 (ReLU) and 256->27.  BF16
 * activations and matrix products with FP32 accumulation; FP32 master weights and Adam.
 * Parameter blob (float32): per convolution weights [out][in][3][3] then bias, then each
 * dense layer's weights [out][in] then bias.  x arrays are device BF16 (n x 5 x 32 x 32),
 * t / y device float32 (n x 27), orders device int32 (epochs x n, a permutation per epoch).
 * The network belongs to the context's device and runs on the context's stream.
 * ---------------------------------------------------------------------------------------- */
int64_t celeste_net_num_params(void);
int celeste_net_create(celeste_ctx* ctx, const float* params, int64_t n_params, const float* psi_mean,
                       const float* psi_std, celeste_net** out);
void celeste_net_destroy(celeste_net* net);
int celeste_net_get_params(celeste_net* net, float* params_out /* host */);
/* Mean squared error over batch x 27 outputs and its gradient (host, n_params; may be NULL).
 * x must be 16-byte aligned (E_INVALID otherwise), as for celeste_net_forward. */
int celeste_net_loss_grad(celeste_net* net, const void* x, const float* t, int batch, float* loss_out,
                          float* grad_out);
/* Forward pass of n inputs; x must be 16-byte aligned (the first layer reads its image rows in
 * 16-byte pieces); E_INVALID otherwise. */
int celeste_net_forward(celeste_net* net, const void* x, int64_t n, float* y);
/* Adam (lr, betas 0.9 / 0.999, eps 1e-8) over minibatches in the given orders; epoch_loss
 * (host, epochs entries, may be NULL) receives the mean minibatch loss of each epoch. */
int celeste_net_train(celeste_net* net, const void* x, const float* t, int64_t n, const int32_t* orders,
                      int epochs, int batch, float lr, float* epoch_loss);
/* Network inputs for every source of a batch around theta's positions (theta in mem_kind
 * memory, n_sources x 27; out: device BF16 n_sources x 5 x 32 x 32). */
int celeste_make_patches(celeste_ctx* ctx, const celeste_batch* batch, const double* theta, void* out);
/* Network used by CELESTE_INIT_SURROGATE (NULL to clear).  The context does not own it. */
int celeste_ctx_set_surrogate(celeste_ctx* ctx, celeste_net* net);

/* Unconstrained coordinates of the fits (host arrays, n x 27): position in a box of
 * half-width u_box around u0 (n x 2) by a scaled logistic, a and e_dev on [1e-4, 1-1e-4],
 * e_axis on [0.01, 0.99], e_scale on [0.2, 15] by scaled logistics, variances by exp,
 * the rest identity.  Values outside a box are clipped into it first. */
int celeste_theta_to_psi(const double* theta, const double* u0, int64_t n, double u_box, double* psi);
int celeste_psi_to_theta(const double* psi, const double* u0, int64_t n, double u_box, double* theta);

/* ----------------------------------------------------------------------------------------
 * Crowded fields (section III-B: each source is optimised with the other sources held fixed
 * at their current estimates; a pixel can receive photons from several sources).  Patches
 * are views into shared field images: image i of the batch belongs to field img_field[i],
 * its origin is the integer field-pixel position of its element (0,0) and it lies inside
 * the field.  Batches must use CELESTE_MEM_DEVICE.
 * ---------------------------------------------------------------------------------------- */
typedef struct celeste_fields {
  int32_t n_fields, height, width;   /* field images, each height x width, row-major */
  int32_t reserved;                  /* must be 0 */
  const int32_t* img_field;          /* host: field of every image of the batch */
  float* mean;                       /* device, n_fields x height x width */
  float* var;                        /* device, n_fields x height x width */
} celeste_fields;

/* Sum over all sources of calib * E[l G] (expected counts without sky) and of the variance
 * into fields->mean / fields->var, each source within its own patches, at theta (device,
 * n_sources x 27).  Deterministic (a gather per 32x32 tile in source order, FP64 sums). */
int celeste_render_fields(celeste_ctx* ctx, const celeste_batch* batch, const double* theta,
                          const celeste_fields* fields);

/* Per-patch neighbour arrays: rendered fields minus the source's own contribution at theta,
 * clamped at 0, written with pitch = w at nbr_mean/nbr_var + nbr_off[i] (device; nbr_off
 * host, one element offset per image).  Feed them back as celeste_image.nbr_mean/nbr_var. */
int celeste_neighbour_arrays(celeste_ctx* ctx, const celeste_batch* batch, const double* theta,
                             const celeste_fields* fields, const int64_t* nbr_off, float* nbr_mean,
                             float* nbr_var);

/* Colours for Gauss-Seidel block sweeps over a crowded field (host only, no device work).
 * Section III-B optimises one source with the others held fixed; sources that share no pixel
 * can take that step at the same time and the result is a block coordinate step on the joint
 * ELBO.  Sources whose bounding boxes (union of their images' rectangles [origin, origin +
 * (w, h)) in image-frame coordinates) intersect get different colours, so no two sources of
 * one colour touch a common pixel of any field image.  Greedy in source order, smallest free
 * colour.  colour: host, n_sources (out); n_colours: host (out).  Errors: E_INVALID. */
int celeste_colour_sources(const celeste_batch* batch, int32_t* colour, int32_t* n_colours);

/* Moves rendered fields (celeste_render_fields) of the batch's sources from theta_old to
 * theta_new (device, n_sources x 27 each): every pixel of every patch gets the difference of
 * its source's two contributions, clamped at 0.  The batch's patches must not overlap within a
 * field (one colour of celeste_colour_sources; checked, E_INVALID otherwise), so each field
 * pixel has one writer and the update is deterministic. */
int celeste_update_fields(celeste_ctx* ctx, const celeste_batch* batch, const double* theta_old,
                          const double* theta_new, const celeste_fields* fields);

/* Joint ELBO of a crowded field (the objective that section III-B's per-source steps
 * increase): the delta-method expected log-likelihood of every pixel of every field image, with
 * E = sky + fields->mean and Var = fields->var (rendered at theta), plus the prior terms (minus
 * KL) of all sources at theta (device, n_sources x 27).  field_pixels: device counts, n_fields x
 * height x width; field_sky: host, n_fields, > 0.  elbo_out: host.  FP64, fixed summation order. */
int celeste_field_elbo(celeste_ctx* ctx, const celeste_batch* batch, const double* theta,
                       const celeste_fields* fields, const float* field_pixels, const double* field_sky,
                       double* elbo_out);

/* The start a fit with these options would use (plain or surrogate-with-fallback, clipped
 * into the boxes), without fitting; elbo_out (n_sources, batch memory, may be NULL) gets its
 * ELBO.  opts->max_iter is ignored. */
int celeste_start(celeste_ctx* ctx, const celeste_batch* batch, double* theta_inout, const celeste_fit_opts* opts,
                  double* elbo_out);

/* ------------------------------------------------------------------ autotuner */

/* Options chosen by celeste_autotune and the kernel times behind the choice. */
typedef struct celeste_tune_result {
  int32_t chunk_px, block, variant, tile_w;   /* value+gradient+Hessian kernel (CELESTE_OPT_*) */
  int32_t value_block, value_tile_w;          /* value kernel */
  int32_t n_candidates;                       /* configurations timed (0 when read from the cache) */
  int32_t from_cache;                         /* 1: taken from the cache file without timing */
  int64_t sample_sources, sample_px;          /* tuning sample */
  double full_ms, value_ms;                   /* best time per launch over the sample */
  double default_full_ms, default_value_ms;   /* the default options' times on the same sample
                                                 (default_full_ms from the same pass as full_ms) */
  double vector_full_ms, matrix_full_ms;      /* best value+gradient+Hessian time with J^T W J on the
                                                 vector units / on the matrix cores */
} celeste_tune_result;

/* Tile shapes and launch shapes of the pixel kernels, chosen by timing (the batching of
 * the per-source pixel sums of section III-B on this device).  Takes a deterministic
 * sample of the batch (every k-th source, about sample_px pixels; sample_px <= 0 means
 * 6e7), evaluates it at theta (n_sources x 27, batch memory) with the value+gradient+
 * Hessian kernel under every candidate work-item size (4096..16384 px), block size,
 * register budget, J^T W J unit (vector or matrix cores) and tile width (minimum of three
 * timed launches each, HIP events on the library's stream), re-times the four fastest and
 * the default options together (minimum of nine launches each) and keeps the fastest of
 * that pass, so full_ms <= default_full_ms; then times the value kernel under every block
 * size and tile width on the chosen work items, and sets the choice on the context (on an
 * error the context keeps its earlier options).  cache_path (may be NULL) names a text
 * file of earlier choices, one per line, keyed by device, compute-unit count, component
 * counts and the batch's size class: a hit is applied without timing, a miss is appended.
 * out may be NULL.  Errors: as celeste_elbo_eval; E_INVALID for an unreadable or
 * unwritable cache file. */
int celeste_autotune(celeste_ctx* ctx, const celeste_batch* batch, const double* theta, int64_t sample_px,
                     const char* cache_path, celeste_tune_result* out);

#ifdef __cplusplus
}
#endif

#endif /* CELESTE_H */
