/*
 * appga.h — C ABI of the MI355X library for APPGA reconstruction of
 * SHOITV-regularised Poisson PET images (arXiv 2409.13344).
 *
 * The model (Section 2.1): data g in R+^m, system matrix A in R+^{m x d},
 * background gamma in R+^m, image f in R+^d with d = N^2, and
 *   Phi(f) = <Af, 1> - <ln(Af + gamma), g>
 *          + lambda1 sum_i s_eps((B1 f)_i, (B1 f)_{d+i})
 *          + lambda2 sum_i s_eps((B2 f)_i, ..., (B2 f)_{3d+i}) + iota_{>=0}(f)
 * (eq. model:SHOTV, smoothed norm eq. def:smoothL2).  The solver is APPGA
 * (Section 2.2, eq. APPGAiter): f~ = f^k + theta_k (f^k - f^{k-1}),
 * f^{k+1} = max(f~ - P (grad F(f~) + B^T grad phi~(B f~)), 0), with the GN
 * momentum weights theta_k = (t_{k-1} - 1)/t_k, t_k = a k^omega + b
 * (eq. GNtheta) and the EM preconditioner P = beta diag(f^k / Lambda),
 * Lambda = A^T 1 with zeros replaced by 1 (eq. EM, Section 4.1).
 *
 * Conventions
 *  - Every call returns appga_status (0 = success, < 0 = error); no C++
 *    exception crosses the ABI.  appga_last_error() gives a message for the
 *    calling thread's last failure.
 *  - Image layout: row-major, pixel (r, c) at r*N + c.  Sinogram layout:
 *    angle-major, bin (a, b) at a*n_bins + b.  Batched arrays are solve-major
 *    (solve s starts at s*m or s*d).
 *  - Host pointers: owned by the caller, read (or written) only during the
 *    call; inputs are copied before the call returns.
 *  - Device pointers (calls ending in _device): HIP device memory owned by
 *    the caller; work is queued on the given hipStream_t (passed as void*,
 *    NULL = the context's stream) and the pointers are not retained after
 *    that work completes.
 *  - Validation errors return before any work and leave outputs untouched.
 *  - A context is used by one thread at a time, except appga_submit and
 *    appga_wait on a server, which are thread-safe.
 */
#ifndef APPGA_H
#define APPGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    APPGA_OK = 0,
    APPGA_E_INVALID_ARG = -1, /* null pointer, unknown enum value, bad size */
    APPGA_E_SHAPE = -2,       /* m != n_angles*n_bins, column out of range, bad row_ptr */
    APPGA_E_DOMAIN = -3,      /* a parameter outside the range the method is defined on */
    APPGA_E_OOM = -4,         /* device or host allocation failed */
    APPGA_E_DEVICE = -5,      /* a HIP runtime call failed */
    APPGA_E_NONFINITE = -6,   /* NaN/Inf in the inputs or in the result */
    APPGA_E_BUSY = -7,        /* matrix still in use by in-flight server requests */
    APPGA_E_NOT_FOUND = -8,   /* unknown ticket */
    APPGA_E_TIMEOUT = -9      /* appga_wait timed out (the request keeps running) */
} appga_status;

/* Storage type of the system-matrix values; accumulation is always FP32. */
typedef enum {
    APPGA_F32 = 1,
    APPGA_BF16 = 2,
    APPGA_F16 = 3,
    APPGA_FP8_E4M3_ROWSCALE = 4 /* OCP e4m3 with one FP32 scale per matrix row */
} appga_dtype;

/* GN: theta_k from t_k = a k^omega + b (eq. GNtheta).  NONE: theta_k = 0.
 * NESTEROV (AFPPA only): t_0 = 1, t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2 (Section 4.3). */
enum { APPGA_MOMENTUM_GN = 0, APPGA_MOMENTUM_NONE = 1, APPGA_MOMENTUM_NESTEROV = 2 };
/* EM: P = beta f^k / Lambda every iteration (eq. EM).  EM_FROZEN: updated for
 * k <= precond_freeze_iter, then kept (allowed by Section 4.1).  FIXED: P = fixed_p I. */
enum { APPGA_PRECOND_EM = 0, APPGA_PRECOND_EM_FROZEN = 1, APPGA_PRECOND_FIXED = 2 };

typedef struct appga_ctx appga_ctx;
typedef struct appga_matrix appga_matrix;
typedef struct appga_server appga_server;

/* Image N x N (d = N^2), n_angles projection angles (NPA of Section 4.1),
 * n_bins radial bins; m = n_angles * n_bins rows of A. */
typedef struct {
    int32_t n, n_angles, n_bins;
} appga_geometry;

/* Model and algorithm parameters (Sections 2.1, 2.2, 4.1).
 * Domain (APPGA_E_DOMAIN otherwise): lambda1, lambda2 >= 0; eps > 0;
 * omega in (0, 1]; a > 0, and a < 1/2 when omega = 1 (Lemma 8); b not equal to
 * -a k^omega for any k >= 1; beta > 0; iterations >= 0; fixed_p > 0 in FIXED
 * mode; gamma_scalar >= 0.  monitor_every = M > 0 (solve sessions; the first
 * solve's value counts for a batch) computes the FP64 objective Phi(f^k) of
 * every solve at k = 1, M + 1, 2M + 1, ... (one extra forward projection and
 * a stream synchronisation each), read with appga_solve_history; 0 = only at
 * the start and the end. */
typedef struct {
    double lambda1, lambda2, eps, omega, a, b, beta;
    int32_t iterations, momentum, precond, precond_freeze_iter, monitor_every;
    double fixed_p;
    double gamma_scalar; /* background in every bin when the background pointer is NULL */
} appga_params;

/* Per-solve report.  objective0 = Phi(f^1), objective = Phi(f^{K+1}) (FP64 on
 * the device), re = ||f^{K+1} - f^K|| / ||f^{K+1}|| (FP64), guard_clamps = number
 * of bins where A f~ + gamma fell below the floor tau = 1e-6 gamma (1e-30 when
 * gamma = 0) and was replaced by tau before the ratio g / (A f~ + gamma). */
typedef struct {
    int32_t iterations_done;
    double objective0, objective, re;
    int64_t guard_clamps;
    double seconds;
} appga_stats;

/* Fills *p with the paper's defaults: a = 1/8, b = 1 (Section 4.1), beta = 1,
 * eps = 1e-3 (Table 1), omega = 1, GN momentum, EM preconditioner, no
 * regularisation (lambda1 = lambda2 = 0), 100 iterations, gamma_scalar = 0. */
appga_status appga_params_default(appga_params *p);

/* Checks *p against the domain rules above; touches no device. */
appga_status appga_validate_params(const appga_params *p);

/* Checks a system matrix against the rules of appga_load_system_matrix
 * (shape, row_ptr, column range, finite non-negative values); touches no device. */
appga_status appga_validate_system_matrix(const appga_geometry *geom, int64_t nnz,
                                          const int64_t *row_ptr, const int32_t *col_idx,
                                          const double *values);

/* Creates a context on HIP device `device` with its own stream (default priority). */
appga_status appga_create(appga_ctx **ctx, int device);
appga_status appga_destroy(appga_ctx *ctx);

/* Uploads A (CSR, FP64 values, rows ordered angle-major) and builds, on the
 * host, the stored transpose used for A^T, the per-row FP8 scales when asked,
 * Lambda = A^T 1 (eq. EM) from the stored values, and the launch plan.
 * row_ptr: m+1 entries, row_ptr[0] = 0, non-decreasing, row_ptr[m] = nnz.
 * col_idx: nnz entries in [0, d).  values: nnz finite entries >= 0.
 * nnz < 2^31.  The handle is owned by the library until appga_free_system_matrix. */
appga_status appga_load_system_matrix(appga_ctx *ctx, const appga_geometry *geom, int64_t nnz,
                                      const int64_t *row_ptr, const int32_t *col_idx,
                                      const double *values, appga_dtype storage,
                                      appga_matrix **out);
/* Factored forward model (the physics of Section 4.1's simulation): the system
 * is A = diag(row_factors) G H, where G is the matrix given as for
 * appga_load_system_matrix, row_factors (m doubles, finite, >= 0, or NULL for
 * 1) are per-ray factors such as the attenuation exp(-(G mu)_i), and H is a
 * space-invariant Gaussian PSF of full width at half maximum psf_fwhm_px
 * pixels (0 = none, at most 24).  H has taps w_t = exp(-t^2 / (2 sigma^2)) at
 * offsets |t| <= R = ceil(3 sigma), sigma = FWHM / (2 sqrt(2 ln 2)), normalised
 * to sum 1, applied along rows and columns with zero outside the image (so H
 * is symmetric).  The row factors are folded into the stored values; Lambda
 * = A^T 1 = H (G^T n).  Sessions of both models (appga_solve_*, appga_afppa_*,
 * appga_reconstruct*) then project H f~ and back-project H (A^T e);
 * appga_op_forward / appga_op_ratio / appga_op_back apply the whole A;
 * appga_op_step and the server (appga_submit) return APPGA_E_INVALID_ARG for
 * a matrix with a PSF.  Scatter and randoms enter as the background gamma. */
appga_status appga_load_system_matrix_factored(appga_ctx *ctx, const appga_geometry *geom, int64_t nnz,
                                               const int64_t *row_ptr, const int32_t *col_idx,
                                               const double *values, appga_dtype storage,
                                               const double *row_factors, double psf_fwhm_px,
                                               appga_matrix **out);
/* Quarter-turn symmetry of a loaded matrix: with an even number of angles on
 * the square grid, row (a + n_angles/2, b) is row (a, b) with pixel (r, c)
 * moved to (c, N-1-r).  When every such pair agrees to 1e-9 of its largest
 * entry (checked at load when the environment sets APPGA_SYMMETRY=1; FP32,
 * BF16 or FP16 storage, d <= 65536), the single-solve (B = 1) kernels read
 * only the first half of the rows and of the transpose and generate the rest
 * by the pixel map, halving their matrix bytes and memory (not their time:
 * they are bound by per-entry gathers of the image).  *folds = 2 then, else 1;
 * *stored_bytes (may be NULL) = the bytes those kernels read per forward +
 * back pair. */
appga_status appga_matrix_symmetry(const appga_matrix *mat, int32_t *folds, int64_t *stored_bytes);
/* The PSF of a loaded matrix: *fwhm_px (0 when none) and the tap radius *radius (-1 when none). */
appga_status appga_matrix_psf(const appga_matrix *mat, double *fwhm_px, int32_t *radius);
appga_status appga_free_system_matrix(appga_ctx *ctx, appga_matrix *mat);

/* Matrix facts: nnz, stored bytes of A and A^T (values + indices + row
 * pointers + scales), the storage type.  Any output pointer may be NULL. */
appga_status appga_matrix_info(const appga_matrix *mat, int64_t *nnz, int64_t *bytes_a,
                               int64_t *bytes_at, int32_t *storage);

/* Tile forms of a loaded matrix (Section 2.2: A x and A^T e of batches).  For
 * B > 1 the library projects over tiles of 64 outputs (rays for A x, 8 x 8
 * pixel blocks for A^T e) whose entries read their inputs from windows staged
 * in on-chip memory; appga_load_system_matrix builds them unless
 * APPGA_FWD_TILES=0 / APPGA_BACK_TILES=0, and falls back to the row kernels
 * for a direction whose tile form does not fit the kernel's limits.  Results
 * agree with the row kernels to FP32 rounding (the back projection with one
 * workgroup per tile, APPGA_BACK_SPLIT=1, bit for bit).  `which` is
 * APPGA_TILES_FORWARD or APPGA_TILES_BACK; *out receives the tile form's
 * counts (valid = 0: the row kernels serve that direction).
 * Errors: APPGA_E_INVALID_ARG (NULL pointer or unknown `which`). */
enum { APPGA_TILES_FORWARD = 0, APPGA_TILES_BACK = 1 };
typedef struct {
    int32_t valid;      /* 1: the tile kernel serves B > 1 in this direction */
    int32_t tiles;      /* tiles of 64 outputs */
    int32_t split;      /* workgroups per tile (partial sums; forward: 1) */
    int32_t pad0;
    int64_t windows;    /* windows staged over all tiles */
    int64_t records;    /* input records staged over all windows (256 bytes per 64 solves) */
    int64_t entries;    /* stored entries including the quad padding */
    int64_t bytes;      /* device bytes of the tile form */
} appga_tile_info;
appga_status appga_matrix_tiles(const appga_matrix *mat, int32_t which, appga_tile_info *out);

/* Host-only emulation of a tile form (Section 2.2 products): builds the tile
 * form that appga_load_system_matrix would build for the given CSR (F32, BF16
 * or F16 storage; no device is used) and applies it to one vector in FP32 as
 * the tile kernel sums it (each output's entries window by window in stored
 * order, partial sums added in order), before any epilogue:
 * out = A in (which = APPGA_TILES_FORWARD; in: d, out: m) or
 * out = A^T in (APPGA_TILES_BACK; in: m, out: d).  `split`: forward -- 0 whole
 * tiles (the default form), K > 0 runs of at most K windows, -1 the automatic
 * run length; back projection -- workgroups per tile (1 .. groups).  *info
 * (nullable) receives the counts; info->valid = 0 when the form does not fit
 * the kernel's limits (then out is untouched).  Host buffers, owned by the
 * caller.  Errors: APPGA_E_INVALID_ARG (NULL pointer, storage, which, split),
 * APPGA_E_SHAPE / APPGA_E_DOMAIN (matrix checks as appga_validate_system_matrix). */
appga_status appga_tiles_emulate(const appga_geometry *geom, int64_t nnz, const int64_t *row_ptr,
                                 const int32_t *col_idx, const double *values, appga_dtype storage,
                                 int32_t which, int32_t split, const float *in, float *out,
                                 appga_tile_info *info);

/* Launch-configuration autotuner.  Times the candidate launch configurations
 * of the projector kernels for `mat` on the device and keeps the fastest:
 * APPGA_TUNE_SINGLE -- lanes per matrix row (4..64) of the single-solve
 * forward and back projection kernels; APPGA_TUNE_BATCH -- workgroups of the
 * batched forward grid and the XCD tile order of the batched step kernel.
 * Parameters pinned by the environment (APPGA_GROUP_FWD, APPGA_GROUP_BACK,
 * APPGA_FWD_WGS, APPGA_XCD_REMAP) are not searched.  Results only change
 * speed, never values.  appga_load_system_matrix runs it (both flags) unless
 * APPGA_AUTOTUNE=0.  *out (nullable) receives the choice and the timings
 * (microseconds per launch; 0 = not searched).  Synchronises the context's
 * stream; APPGA_E_BUSY while server requests use the matrix. */
enum { APPGA_TUNE_SINGLE = 1, APPGA_TUNE_BATCH = 2 };
typedef struct {
    int32_t group_fwd, group_back, fwd_wgs, xcd_remap;
    double us_fwd_single, us_back_single, us_fwd_batch, us_step_batch;
} appga_tuning;
appga_status appga_tune(appga_ctx *ctx, appga_matrix *mat, int32_t flags, appga_tuning *out);

/* Writes the values A holds after storage rounding (dequantised, FP64) in
 * the caller's CSR order: nnz entries. */
appga_status appga_matrix_dequantized(const appga_matrix *mat, double *values_out);

/* One solve (Section 2.2, eq. APPGAiter).  sinogram: m counts >= 0.
 * background: m values >= 0, or NULL for params->gamma_scalar in every bin.
 * f_init: d values used as f^0 = f^1, or NULL for the initial image of
 * Section 4.1: TMC * 1_disk, TMC = ACTc / (NPFOV * NPA), ACTc = sum g - sum gamma
 * (> 0 required), disk of radius N/2.  f_out: d values f^{K+1}.  stats may be NULL. */
appga_status appga_reconstruct(appga_ctx *ctx, const appga_matrix *mat, const float *sinogram,
                               const float *background, const appga_params *params,
                               const float *f_init, float *f_out, appga_stats *stats);

/* appga_reconstruct with lambda1 = lambda2 = lambda and the remaining defaults. */
appga_status appga_reconstruct_simple(appga_ctx *ctx, const appga_matrix *mat, const float *g,
                                      const float *gamma, double lambda, double eps, double omega,
                                      int32_t iterations, float *f_out);

/* B independent solves sharing A, advanced together (one pass over the matrix
 * per iteration for all of them).  g: B*m, gamma: B*m or NULL (then each
 * params[s].gamma_scalar), params: B entries (all with the same iterations
 * and precond mode), f_init: B*d or NULL, f_out: B*d, stats: B or NULL.
 * Solve s equals appga_reconstruct of solve s alone up to FP32 rounding. */
appga_status appga_reconstruct_batch(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                     const float *g, const float *gamma, const appga_params *params,
                                     const float *f_init, float *f_out, appga_stats *stats);

/* Device-memory form of appga_reconstruct_batch (no host copies of the data):
 * d_g, d_gamma (or NULL), d_f_init (or NULL) and d_out are HIP device arrays,
 * solve-major; params is a host array of B entries; hip_stream as above.
 * Returns after queueing; the result is ready when the stream reaches it. */
appga_status appga_reconstruct_batch_device(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                            const float *d_g, const float *d_gamma,
                                            const appga_params *params, const float *d_f_init,
                                            float *d_out, void *hip_stream);

/* AFPPA on the nonsmooth HOITV model (Section 4.3, model HOTV: Phi without
 * smoothing, lambda1 sum ||(B1 f)_i|| + lambda2 sum ||(B2 f)_i||).  Per
 * iteration, with theta_k of params.momentum (GN = AFPPA-GN, NONE = FPPA,
 * NESTEROV = AFPPA-N) and P = beta f^k / Lambda (EM) or fixed_p (FIXED):
 *   f~, b~, c~ = extrapolations of f, b, c with theta_k;
 *   f^{k+1} = max(f~ - P (grad F(f~) + B1^T b~ + B2^T c~), 0);
 *   b^{k+1} = rho1 (I - prox_{(lambda1/rho1)||.||})(b~ / rho1 + B1 (2 f^{k+1} - f~)) per
 *   pixel (2 components), c^{k+1} likewise with rho2, lambda2 and B2 (4 components);
 *   rho1 = 1 / (2 * 8 * p_max), rho2 = 1 / (2 * 64 * p_max), p_max = max_j P_jj
 *   (floored at 1e-30).
 * The prox uses the plain group l2 norm, so every dual group stays in the
 * ball of radius lambda.  f^0 = f^1 = f_init (or the disk image of Section
 * 4.1), b^0 = b^1 = 0, c^0 = c^1 = 0.
 *
 * params: as for APPGA, except that eps is not used, momentum may be NESTEROV
 * and precond must be EM or FIXED (else APPGA_E_INVALID_ARG).  stats report
 * the nonsmooth objective.  g, gamma, f_init, f_out and stats are as for
 * appga_reconstruct_batch.  duals_out (B * 6 d floats, or NULL): per solve b^{K+1}
 * (2 d: the (I kron D) plane, then the (D kron I) plane), then c^{K+1} (4 d:
 * the four blocks of B2 in order).  B = 1 runs the single-solve kernels. */
appga_status appga_afppa_batch(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                               const float *g, const float *gamma, const appga_params *params,
                               const float *f_init, float *f_out, float *duals_out,
                               appga_stats *stats);
/* Device-memory form of appga_afppa_batch (d_duals_out may be NULL); queues
 * on hip_stream like appga_reconstruct_batch_device. */
appga_status appga_afppa_batch_device(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                                      const float *d_g, const float *d_gamma,
                                      const appga_params *params, const float *d_f_init,
                                      float *d_out, float *d_duals_out, void *hip_stream);

/* Solve sessions: the batched solver split into its phases, so a caller can
 * advance B solves a few iterations at a time (the serving loop and the
 * benchmark do).  appga_solve_begin validates like appga_reconstruct_batch_device,
 * uploads per-solve parameters, forms f^0 = f^1 and queues nothing else;
 * appga_solve_step queues n_iters iterations; appga_solve_end writes f^{k}
 * (solve-major, d_out device memory) and the stats (B entries, may be NULL),
 * synchronises the stream and frees the session.  params[s].iterations is
 * ignored by sessions (the caller decides how many steps to run). */
typedef struct appga_solve appga_solve;
appga_status appga_solve_begin(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                               const float *d_g, const float *d_gamma, const appga_params *params,
                               const float *d_f_init, void *hip_stream, appga_solve **out);
appga_status appga_solve_step(appga_solve *s, int32_t n_iters);
/* Objective history of solve `solve` (sessions with monitor_every > 0, before
 * appga_solve_end): *count = number of monitored iterations so far; the first
 * min(count, cap) pairs (k, Phi(f^k) in FP64), f^1 first, go to iters_out and
 * obj_out (host arrays of cap entries; may be NULL when cap = 0). */
appga_status appga_solve_history(const appga_solve *s, int32_t solve, int32_t cap, int32_t *iters_out,
                                 double *obj_out, int32_t *count);
appga_status appga_solve_end(appga_solve *s, float *d_out, appga_stats *stats);
/* The current image f^k of a session (either model) into d_out (device, B * d
 * floats, solve-major); synchronises the session's stream.  The session goes on. */
appga_status appga_solve_image(const appga_solve *s, float *d_out);
/* An AFPPA session (same phases; the AFPPA parameter rules above; monitors and
 * stats give the nonsmooth objective). */
appga_status appga_afppa_begin(appga_ctx *ctx, const appga_matrix *mat, int32_t B,
                               const float *d_g, const float *d_gamma, const appga_params *params,
                               const float *d_f_init, void *hip_stream, appga_solve **out);
/* The current duals (b^k, c^k) of an AFPPA session into d_duals (device, B * 6 d
 * floats, layout of duals_out above); synchronises the session's stream.
 * APPGA_E_INVALID_ARG for a session of the smoothed model. */
appga_status appga_solve_duals(const appga_solve *s, float *d_duals);

/* Device operators (each one kernel of the iteration, for tests and timing).
 * All arrays are HIP device memory, solve-major, FP32.
 *  appga_op_forward:   d_y = A d_x (+ d_gamma when non-NULL), B solves.
 *  appga_op_ratio:     d_e = 1 - d_g / max(A d_x + gamma, tau) (the floor above).
 *  appga_op_back:      d_out = A^T d_r (stored transpose).
 *  appga_op_grad_reg:  d_out = B1^T w1 B1 x + B2^T w2 B2 x with w = lambda/max(|.|, eps)
 *                      per pixel (Section 2.2, gradient of phi~); lambda1/lambda2/eps
 *                      are per solve (B entries, host).
 *  appga_op_step:      one APPGA iteration from (d_f = f^k, d_ft = f~^k): writes f^{k+1}
 *                      into d_f and f~^{k+1} (extrapolated with theta_next) into d_ft_next.
 *                      theta_next, beta, lambda1, lambda2, eps: B entries (host). */
appga_status appga_op_forward(appga_ctx *ctx, const appga_matrix *mat, int32_t B, const float *d_x,
                              const float *d_gamma, float *d_y, void *hip_stream);
appga_status appga_op_ratio(appga_ctx *ctx, const appga_matrix *mat, int32_t B, const float *d_x,
                            const float *d_g, const float *d_gamma, float *d_e, void *hip_stream);
appga_status appga_op_back(appga_ctx *ctx, const appga_matrix *mat, int32_t B, const float *d_r,
                           float *d_out, void *hip_stream);
appga_status appga_op_grad_reg(appga_ctx *ctx, int32_t n, int32_t B, const double *lambda1,
                               const double *lambda2, const double *eps, const float *d_x,
                               float *d_out, void *hip_stream);
appga_status appga_op_step(appga_ctx *ctx, const appga_matrix *mat, int32_t B, const float *d_g,
                           const float *d_gamma, const double *lambda1, const double *lambda2,
                           const double *eps, const double *beta, const double *theta_next,
                           float *d_f, const float *d_ft, float *d_ft_next, void *hip_stream);

/* Kernel timing: when enabled, the library records HIP events around each
 * kernel it launches (on the launch stream) and accumulates per-kernel
 * launch counts and durations.  appga_kernel_times returns, for up to `cap`
 * kernels, a NUL-separated list of names (names_out, names_cap bytes), the
 * launch counts and total milliseconds.  Reading synchronises the stream. */
appga_status appga_set_kernel_timing(appga_ctx *ctx, int32_t enable);
appga_status appga_kernel_times(appga_ctx *ctx, int32_t cap, char *names_out, int32_t names_cap,
                                int64_t *counts, double *total_ms, int32_t *n_kernels);

/* Serving: a continuous-batching request loop on one device (Algorithm 1 per
 * request; Section 4.1 initial image; EM preconditioner, eq. EM; momentum by
 * eq. GNtheta from each request's own iteration counter).
 *
 * One loop thread owns all device work.  Per loaded system matrix it keeps a
 * pool of 64 lanes in device memory (data, background, f, two f~ buffers, the
 * ratio residual and the back projection per lane; appga_server_footprint
 * gives its size) and
 * advances every occupied lane of a pool by one iteration per step, replayed
 * from captured hipGraphs on the pool's own stream.  A request is admitted as
 * soon as its pool has a free lane among the first slots_per_matrix (1..64)
 * and, for a pool not yet present, the pools' total footprint stays within
 * hbm_budget_bytes (idle pools of other matrices are freed to make room); it
 * leaves after exactly params->iterations iterations.  A served result equals
 * the result of the same request in appga_reconstruct_batch bit for bit (the
 * lanes never interact).  The system matrices are the caller's: they are not
 * counted in the budget and must stay loaded (appga_free_system_matrix returns
 * APPGA_E_BUSY while requests on them are in flight). */
typedef struct {
    int64_t hbm_budget_bytes;
    int32_t slots_per_matrix;
    int32_t reserved;
} appga_server_cfg;

/* Device bytes of one 64-lane pool of `mat` (what admission charges against
 * hbm_budget_bytes).  APPGA_E_INVALID_ARG for NULL arguments. */
appga_status appga_server_footprint(const appga_matrix *mat, int64_t *bytes);
/* Starts the loop thread.  APPGA_E_INVALID_ARG for NULL arguments or a
 * non-positive budget or slot count. */
appga_status appga_server_start(appga_ctx *ctx, const appga_server_cfg *cfg, appga_server **out);
/* Thread-safe.  Copies g (m host floats), gamma (m host floats, or NULL =
 * params->gamma_scalar in every bin) and *params; *ticket identifies the
 * request.  Errors (nothing queued): APPGA_E_INVALID_ARG (NULL argument, a
 * matrix of another context, a preconditioner other than EM, a stopping
 * server); APPGA_E_DOMAIN (parameters outside the method's domain, iterations
 * < 1, ACTc = sum(g) - sum(gamma) <= 0); APPGA_E_NONFINITE (NaN/Inf in g or
 * gamma); APPGA_E_OOM (this matrix's pool alone exceeds the budget). */
appga_status appga_submit(appga_server *srv, const appga_matrix *mat, const float *g,
                          const float *gamma, const appga_params *params, uint64_t *ticket);
/* Thread-safe.  Waits up to timeout_ms (< 0 = forever) for the ticket, then
 * copies f^{K+1} into f_out (host, n*n floats of the request's matrix, row
 * major) and the stats into *stats (either may be NULL), and forgets the
 * ticket.  stats->seconds is the latency from submission to completion and
 * guard_clamps the floored bins of the request; objective0, objective and re
 * are not monitored by the server (0).  Errors: APPGA_E_NOT_FOUND (unknown or
 * already collected ticket), APPGA_E_TIMEOUT (still running; wait again),
 * APPGA_E_NONFINITE (the result holds NaN/Inf; it is copied out), or the
 * device error that ended the request. */
appga_status appga_wait(appga_server *srv, uint64_t ticket, float *f_out, appga_stats *stats,
                        int32_t timeout_ms);
/* Stops admitting, finishes every queued and running request (their tickets
 * can no longer be collected), joins the loop and frees the server. */
appga_status appga_server_stop(appga_server *srv);

/* Message describing the calling thread's most recent failure ("" if none). */
const char *appga_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* APPGA_H */
