/*
 * msr.h -- C ABI of libmsr, the MI355X (gfx950) minor-cycle solver of the
 * two-step radio-interferometric reconstruction of Wang, Prunet, Mignot and
 * Ferrari, "Multi-Step Reconstruction of Radio-Interferometric Images".
 *
 * The library solves, with the dictionary W = I (msr_config.dictionary = 0;
 * the wavelet dictionary of msr_dictionary_synthesis takes x = W alpha and
 * penalises ||alpha||_1 instead),
 *   step 1 (Eq. 4):  min_x ||i_L - H_L x||^2 + lambda_L ||x||_1
 *   step 2 (Eq. 5):  min_x ||G_H (i_H - H_H x)||^2 + ||G_L (l - x)||^2 + lambda_H ||x||_1
 * with FISTA (Algorithm 1: momentum (k-1)/(k+2), soft threshold at mu*lambda),
 * the gradients of Eqs. 11-12, the filters of Eqs. 6-10 and the step size
 * mu = 1/theta, theta = 2 lambda_max of the normal operator (Sect. 3.4).
 *
 * Discretisation.  H x = E^T F^-1[h_hat . F(E x)]: E zero-embeds the N x N
 * image into a P x P grid, F is the P x P DFT, h_hat = F(ifftshift(PSF)).
 * With pad = 2 (P = 2N) this is the exact linear convolution of the image
 * with the PSF; with pad = 1 (P = N) it is circular.  G = C_g E: the filter
 * multiplies the spectrum of the zero-embedded image and its norm is taken
 * over the whole P x P grid.  The filter radius r of a DFT cell is its
 * distance from the origin in cells of the P grid (signed indices), and
 * ell, delta are given in the same unit.
 *
 * Conventions.
 *   - Every call returns msr_status; no C++ exception crosses the ABI.
 *     msr_last_error() returns a text for the last failed call on a context.
 *   - Images are row-major, contiguous device arrays of N x N reals (PSFs:
 *     P x P with the phase centre at (P/2, P/2)), float32 or float64 as the
 *     context's msr_config.precision says (passed as void*).  They stay owned
 *     by the caller; the library keeps no pointer to them after a call.
 *   - precision 32 runs the transforms, the prox and the momentum in float32
 *     with FP64 reductions (objectives, power iteration, sigma2_hat);
 *     precision 64 runs everything in float64 (N <= 4096 zero padded,
 *     N <= 8192 circular).
 *   - All device memory the library uses is one workspace the caller
 *     allocates (size from msr_workspace_bytes) and hands over with
 *     msr_set_workspace, or the library's static array of
 *     MSR_STATIC_WORKSPACE_BYTES per device (msr_set_workspace_static, for
 *     small images); the library itself never allocates device memory.
 *   - Work is ordered on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL is the default stream).  Calls that return scalars
 *     synchronise that stream before returning.
 *   - A context is not thread safe; separate contexts are independent.
 */
#ifndef MSR_H
#define MSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSR_ABI_VERSION 3  /* 2: msr_step2_full_res takes image_out; 3: msr_config.iterate_precision */

typedef enum msr_status {
    MSR_OK = 0,
    MSR_ERR_INVALID = 1,     /* bad argument, shape or PSF */
    MSR_ERR_OOM = 2,         /* workspace missing or too small */
    MSR_ERR_HIP = 3,         /* a HIP runtime call failed (text in msr_last_error) */
    MSR_ERR_STATE = 4,       /* calls out of order (e.g. step 2 before its PSF or filters) */
    MSR_ERR_NUMERIC = 5,     /* NaN/Inf in an objective; msr_result.iters says where */
    MSR_ERR_UNSUPPORTED = 6  /* a combination the library does not implement */
} msr_status;

typedef struct msr_ctx msr_ctx;

typedef struct msr_config {
    int32_t n;           /* image side N: a power of two, 8 <= N <= 8192 */
    int32_t pad;         /* 2: zero padding to P = 2N (linear convolution); 1: circular, P = N */
    int32_t positivity;  /* 0: l1 prox (the paper); 1: l1 plus the constraint x >= 0 */
    int32_t device;      /* HIP device ordinal */
    uint64_t seed;       /* power-iteration start vector seed (SplitMix64 counter) */
    double prune_tol;    /* spectral columns k_x whose |h_hat| stays below prune_tol * max|h_hat|
                            are treated as zero; 0 keeps every column */
    int32_t precision;   /* 32: float32 images and arithmetic; 64: float64 */
    int32_t dictionary;  /* 0: W = I (the image itself is sparse); 1: W = the concatenation of the
                            orthonormal Daubechies bases db1 .. db8 (Sect. 3, App. A.1): separable 2-D,
                            periodic, 4 levels, needs N >= 16; positivity is not available with it */
    int32_t iterate_precision; /* 0 (or = precision): the iterates beta_k are stored in the context's
                            precision; 64 with precision 32: float32 transforms and pointwise
                            spectral work, float64 iterates and update (prox, momentum), so that
                            the iterate is not rounded to float32 between iterations.  Single
                            contexts with dictionary 0 only (batches, msr_major_cycles and the
                            dictionary return MSR_ERR_UNSUPPORTED); msr_get_state / msr_set_state
                            then exchange float64 images. */
} msr_config;

typedef struct msr_solve {
    double lambda;       /* regularisation weight lambda of Eq. 4 / Eq. 5 */
    int32_t max_iters;   /* number of FISTA prox steps K */
    int32_t check_every; /* evaluate F(beta_k) exactly every m steps (0: only at the end) */
    double tol;          /* stop once (F(beta_k) - f_ref) / |f_ref| <= tol (needs f_ref != 0, check_every > 0) */
    double f_ref;        /* reference objective F* for the stopping rule (0: no rule) */
} msr_solve;

typedef struct msr_result {
    int32_t iters;       /* prox steps done */
    int32_t converged;   /* 1 if the tol rule stopped the loop */
    double objective;    /* F(beta) at the end (FP64 reductions) */
    double data_term;    /* the data term(s) of F */
    double l1_norm;      /* ||beta||_1 */
    double theta;        /* Lipschitz constant used (mu = 1/theta) */
    double elapsed_ms;   /* device time of the iteration loop, objective checks included */
    double time_to_tol_ms; /* device time until the tol rule held (-1 if never) */
} msr_result;

/* Returns MSR_ABI_VERSION. */
int msr_abi_version(void);

/* Validates cfg and creates a context on cfg->device.  Returns MSR_ERR_INVALID
 * for an unsupported n or pad.  *out is set to NULL on failure. */
msr_status msr_init(const msr_config* cfg, msr_ctx** out);

/* Destroys a context (NULL is allowed).  The workspace stays the caller's. */
void msr_destroy(msr_ctx* ctx);

/* Text of the last error on ctx (never NULL; "" when there was none). */
const char* msr_last_error(const msr_ctx* ctx);

/* Bytes of device workspace a context with this configuration needs (0 for an
 * invalid configuration). */
size_t msr_workspace_bytes(const msr_config* cfg);

/* Hands the library its workspace: dev must be device memory of at least
 * msr_workspace_bytes bytes, 256-byte aligned, and must outlive the context's
 * use of it.  Invalidates everything computed before. */
msr_status msr_set_workspace(msr_ctx* ctx, void* dev, size_t bytes);

/* Size of the static workspace of msr_set_workspace_static: 32 MiB, enough
 * for N <= 512 in single precision and N <= 256 in double precision (zero
 * padded, W = I; msr_workspace_bytes gives the exact need). */
#define MSR_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * msr_set_workspace, with the workspace taken from a static device array of
 * MSR_STATIC_WORKSPACE_BYTES that the library holds on each device from the
 * loading of its device code until the process ends.  Allocates nothing (no
 * hipMalloc, hipFree or allocating library call); the caller still passes
 * every input and output to the later calls, which run unchanged on that
 * array.  Returns MSR_ERR_OOM, with the two sizes in msr_last_error, if
 * msr_workspace_bytes for the context's configuration exceeds
 * MSR_STATIC_WORKSPACE_BYTES; MSR_ERR_HIP if the array's device address
 * cannot be looked up.
 * Sharing: all contexts on one device share its one array.  Binding a
 * context takes the array from the context bound before it, whose later
 * calls then fail with MSR_ERR_STATE until it is given a workspace again;
 * calls of contexts on one device that overlap in time race (do not bind a
 * second context while work of the first is still queued).  The array keeps
 * the last call's contents; nothing in it has to start at zero (every buffer
 * is written before it is read, as in a freshly allocated caller workspace).
 * Invalidates everything computed before, as msr_set_workspace does. */
msr_status msr_set_workspace_static(msr_ctx* ctx);

/* Sets the dirty image i_s and the PSF of step s (1 = short baselines, L;
 * 2 = long baselines, H) -- the inputs of Eq. 4 / Eq. 5.  Computes and caches
 * h_hat = Re F(ifftshift(PSF)) (Sect. 3.2-3.3, "the convolution by the PSF").
 * Fails with MSR_ERR_INVALID if PSF[P/2][P/2] differs from 1 by more than
 * 1e-5, or if max|Im h_hat| > 1e-4 max|h_hat| (a PSF that is not point
 * symmetric).  dirty: N x N; psf: P x P.  Invalidates that step's theta. */
msr_status msr_set_dirty_psf(msr_ctx* ctx, int step, const void* dirty, const void* psf, void* stream);

/* The filters of Eqs. 6-10 for step 2: centre ell and half-width delta of the
 * overlap band (grid cells), and the noise variances sigma^2 (of i_H) and
 * eta^2 (of the low-resolution image).  Requires delta > 0, sigma2 > 0,
 * eta2 > 0.  Invalidates step 2's theta. */
msr_status msr_set_filters(msr_ctx* ctx, double ell, double delta, double sigma2, double eta2);

/* theta_s = 2 lambda_max of the step's normal operator (Sect. 3.4) by the
 * Lanczos iteration (theta_j = 2 x the largest eigenvalue of the j x j
 * tridiagonal projection; no reorthogonalisation), started from
 * v0[n] = splitmix64_mix(seed + n) * 2^-64 - 1/2, stopped when
 * |theta_j - theta_{j-1}| <= rtol * theta_j, when the Krylov space is
 * invariant, or after max_iter applications.  Writes the estimate to *theta and the number of operator
 * applications to *iters (either may be NULL).  The solver then uses
 * margin * estimate as its Lipschitz constant (margin 1.01, see
 * msr_set_lipschitz to override). */
msr_status msr_lipschitz(msr_ctx* ctx, int step, int max_iter, double rtol, double* theta, int* iters, void* stream);

/* Overrides the Lipschitz constant theta used by step s (mu = 1/theta). */
msr_status msr_set_lipschitz(msr_ctx* ctx, int step, double theta);

/* Step 1: FISTA on Eq. 4 from x0 (NULL: zeros).  Writes beta_K to model_out
 * (N x N).  If image_out is not NULL it receives the low-resolution image
 * i_L = beta_K + (i_L~ - H_L beta_K) (Sect. 3.2, one major cycle).  Computes
 * theta by power iteration first if none is cached.  Fills *res (may be
 * NULL).  Blocks until the results are written. */
msr_status msr_step1_low_res(msr_ctx* ctx, const msr_solve* opt, const void* x0,
                             void* model_out, void* image_out, msr_result* res, void* stream);

/* Step 2: FISTA on Eq. 5 with the constraint image l = low_res (N x N), from
 * x0 (NULL: zeros; any warm start may be passed here).  Writes beta_K to
 * model_out; if image_out is not NULL it receives the reconstructed image
 * i^ = beta_K + (i_H~ - H_H beta_K) (Sect. 3.3: the model plus the residual
 * image left after it, one major cycle).  Requires msr_set_dirty_psf(step 2)
 * and msr_set_filters, else MSR_ERR_STATE.  Blocks until the results are
 * written. */
msr_status msr_step2_full_res(msr_ctx* ctx, const msr_solve* opt, const void* low_res, const void* x0,
                              void* model_out, void* image_out, msr_result* res, void* stream);

/* `cycles` major cycles of step s (Sect. 3.2 for step 1, Sect. 3.3 for step 2)
 * with the residual image formed in the image domain: cycle n solves its
 * problem (Eq. 4 or Eq. 5) on i~_n = i~_1 - H_s sum_{j<n} i_j -- the paper
 * recomputes i~_n from the visibilities, which this library does not hold --
 * with lambda_n = c ||i~_n||_2 2^(n-1) (Sect. 5) and, for step 2, the
 * constraint l_n = low_res - sum_{j<n} i_j; each cycle runs `iters` FISTA
 * iterations from zero and i_n is its result.  model_out (may be NULL)
 * receives sum_n i_n, image_out (may be NULL) the step's image
 * i~_{N+1} + sum_n i_n; res, if not NULL, holds one msr_result per cycle.
 * i~_1 is the dirty image set with msr_set_dirty_psf and is left unchanged.
 * Synchronises the stream. */
msr_status msr_major_cycles(msr_ctx* ctx, int step, int cycles, double c, int iters, const void* low_res,
                            void* model_out, void* image_out, msr_result* res, void* stream);

/* Checkpoint and resume of a solve (the FISTA state of Algorithm 1).
 * msr_get_state copies the last two iterates beta_K, beta_{K-1} of the latest
 * solve of step s on this context (N x N images in the iterate precision,
 * float64 with iterate_precision 64; with the wavelet dictionary the
 * coefficient arrays, 8 x N x N each) to beta_k / beta_km1 (device,
 * caller-owned) and writes K to *k (may be NULL).  The iterates stay
 * available until the next solve, msr_major_cycles, msr_time_pass or
 * msr_set_workspace on the context, else MSR_ERR_STATE.
 * msr_set_state loads such a state: the next msr_step1_low_res /
 * msr_step2_full_res of step s continues from iteration K + 1 (its x0 is
 * ignored; the momentum goes on with (k-1)/(k+2), alpha_K is formed from the
 * two iterates) and msr_result.iters counts the iterations of that call, so
 * that a solve of K1 iterations, get, set and a solve of K2 iterations reach
 * the iterate of one solve of K1 + K2 iterations (with the same theta: set
 * it with msr_set_lipschitz on a new context).  A loaded state is dropped by
 * msr_time_pass and msr_set_workspace and by loading one for the other step
 * (the steps share the buffers); msr_major_cycles and batched solves refuse
 * to run while one waits (MSR_ERR_STATE / MSR_ERR_UNSUPPORTED).  Both calls
 * synchronise the stream. */
msr_status msr_get_state(msr_ctx* ctx, int step, void* beta_k, void* beta_km1, int* k, void* stream);
msr_status msr_set_state(msr_ctx* ctx, int step, const void* beta_k, const void* beta_km1, int k, void* stream);

/* Exact objective of step s at x: out[0] = F(x), out[1] = data term(s),
 * out[2] = ||x||_1 (FP64 accumulation).  low_res is required for step 2. */
msr_status msr_objective(msr_ctx* ctx, int step, double lambda, const void* x, const void* low_res,
                         double out[3], void* stream);

/* Gradient of the smooth part of step s at x (Eq. 11 or Eq. 12), N x N. */
msr_status msr_gradient(msr_ctx* ctx, int step, const void* x, const void* low_res, void* grad_out,
                        void* stream);

/* H_s x (N x N in, N x N out): the PSF convolution of step s alone. */
msr_status msr_apply_psf(msr_ctx* ctx, int step, const void* x, void* out, void* stream);

/* The down-sampled low-resolution image (Sect. 6.1).  Step 1 may run on an
 * image of N_s = N / d pixels a side (a context of size N_s with the short
 * baselines' dirty image and PSF on the coarse grid, whose uv cells are those
 * of the full grid); step 2 then takes out = U small as its low_res, where U
 * zero-fills the DFT of the N_s x N_s image to N x N (the Nyquist cell split
 * in halves between +-N_s/2) and transforms back: flux per pixel is
 * conserved, and a flux-conserving decimation D of the DFT band undoes it
 * (D U = I).  In circular mode || G_L (U small - x) ||^2 equals
 * || G_L' (small - D x) ||^2 on the small grid with g_L' = g_L / d whenever
 * ell + delta < N_s / 2, so step 2 on U small is the paper's step 2 with the
 * decimation operator and the modified filter; zero padded, the library uses
 * the same full-grid form.  factor: d, a power of two with N / d >= 2;
 * small: N_s x N_s device image; out: N x N device image (not aliasing
 * small).  Computed as K small K^T with the N x N_s interpolation matrix;
 * uses workspace scratch and synchronises the stream. */
msr_status msr_upsample(msr_ctx* ctx, int factor, const void* small, void* out, void* stream);

/* The wavelet dictionary (msr_config.dictionary = 1; Sect. 3 and App. A.1):
 * x = W alpha = sum_{b=1..8} Psi_b alpha_b, where Psi_b is the orthonormal
 * 2-D transform of db_b (2b taps, minimum phase, low-pass sum sqrt(2),
 * high-pass g[k] = (-1)^k h[2b-1-k]), periodic, 4 levels; each level filters
 * the rows, then the columns, of the top-left s x s block and stores
 * [low | high] halves (the approximation of the coarsest level ends in the
 * top-left (N/16) x (N/16) corner).  coeffs: 8 x N x N reals, alpha_b at
 * offset b N^2.  W W^T = 8 I, so with the dictionary a solve runs FISTA on
 * alpha (the gradient is W^T of the image gradient, the prox is the soft
 * threshold of alpha, theta is 8 times the image operator's), x0 is an image
 * (alpha_0 = W^T x0 / 8, so W alpha_0 = x0), model_out receives W alpha_K
 * and msr_result.l1_norm is ||alpha_K||_1; msr_lipschitz returns the theta
 * of the problem in alpha, msr_objective and msr_gradient keep working on
 * images (W = I).  Both calls use workspace scratch and
 * synchronise the stream; MSR_ERR_STATE on a context without the dictionary. */
msr_status msr_dictionary_synthesis(msr_ctx* ctx, const void* coeffs, void* image, void* stream);
msr_status msr_dictionary_analysis(msr_ctx* ctx, const void* image, void* coeffs, void* stream);

/* Copies the cached h_hat of step s to host memory as P x (P/2 + 1) doubles
 * (rfft half plane, row = k_y, column = k_x), pruned columns as zeros, and
 * writes the number of kept columns to *kept (may be NULL). */
msr_status msr_get_spectrum(msr_ctx* ctx, int step, double* host_out, int* kept, void* stream);

/* sigma2_hat of Sect. 4.3 on an N x N device image: the mean over all 5 x 5
 * windows inside the image of the window's population variance (FP64). */
msr_status msr_estimate_sigma2(msr_ctx* ctx, const void* dirty, double* sigma2, void* stream);

/* Default regularisation weight: c * ||i_s~||_2 * 2^(cycle - 1) (Sect. 5 and
 * App. A.2), from the dirty image set for step s. */
msr_status msr_default_lambda(msr_ctx* ctx, int step, int cycle, double c, double* lambda, void* stream);

#define MSR_MAX_VARIANTS 4

/* Picks, by timing, the kernel variant (elements per thread, hence radix
 * schedule and LDS footprint) of the column PSF pass and of the fused row pass
 * of each step whose PSF is set with msr_set_dirty_psf, and, once the filters
 * are set, of the step-2 low-band filter pass: each built variant is run
 * `reps` times and the fastest kept.  Results of later solves differ from the
 * default variant's only by rounding.  Writes the step-1 choices (0 = default)
 * to *row_variant / *col_variant and, if times_ms is not NULL, the step-1 mean
 * times in ms to times_ms[2*v] (column pass) and times_ms[2*v + 1] (row pass)
 * for v < MSR_MAX_VARIANTS (-1: not built).  Any output pointer may be NULL.
 * The winners are cached for the process, keyed by image size, padding,
 * precision, dictionary, the kept spectral columns of both PSFs and of the
 * filters, and which passes were tuned: a later call on any context with the
 * same key applies them (and reports the cached times) without timing.
 * reps < 0 times again with -reps launches and replaces the cached entry;
 * reps = 0 means 10. */
msr_status msr_autotune(msr_ctx* ctx, int reps, int* row_variant, int* col_variant, double* times_ms,
                        void* stream);

/* Kernel variants of a step's passes, as msr_autotune chooses them (variant
 * v: v = 0 large E, whole column tiles; 1 small E, whole tiles; 2 small E,
 * single columns; 3 large E, single columns; E = complex values per thread of
 * a transform).  msr_set_variants selects them explicitly: row_variant for
 * the row passes, col_variant for the column PSF passes and filter_variant
 * for the step-2 low-band filter pass (-1: the column pass's variant; step 1
 * takes -1).  Results do not depend on the variant beyond rounding order.
 * MSR_ERR_UNSUPPORTED if a variant is not built for this image size (its
 * LDS footprint does not fit), MSR_ERR_INVALID for a bad step or number.
 * msr_get_variants reports the current choice (filter_variant -1 for
 * step 1). */
msr_status msr_set_variants(msr_ctx* ctx, int step, int row_variant, int col_variant, int filter_variant);
msr_status msr_get_variants(msr_ctx* ctx, int step, int* row_variant, int* col_variant, int* filter_variant);

/* Runs one kernel of an iteration of step s `reps` times back to back on
 * `stream` (on the context's current state, which it overwrites: call it
 * outside a solve) and returns its mean device time in milliseconds, plus the
 * algorithmic bytes and flops one launch moves / performs.  which: 0 = column
 * PSF pass, 1 = residual row pass, 2 = fused update row pass, 3 = step-2
 * low-band filter pass (C_w and C_{g_L^2}, Eq. 12; step 2 only, filters
 * set); with the wavelet dictionary also 4 = W alpha (all levels, 8 N^2 read
 * and N^2 written) and 5 = W^T of the gradient image with the fused FISTA
 * coefficient update (all levels; N^2 + 4 x 8 N^2 moved).  Flops count
 * 5 n log2 n per complex transform of length P and 4 L s^2 per 2-D wavelet
 * level of size s and L taps.  Any output may be NULL.  For measurement. */
msr_status msr_time_pass(msr_ctx* ctx, int step, int which, int reps, double* ms, double* bytes, double* flops,
                         void* stream);

/* ---------------------------------------------------------------------------
 * Batched solves.  A batch holds C channels: independent instances of the
 * two-step problem, e.g. the frequency channels of one observation (the
 * paper partitions visibilities per channel as well as by baseline length,
 * Sect. 3.1), of possibly different image sizes.  Channels of equal size are
 * solved by the same launches (one launch per pass for all of them), and the
 * iterations of all channels are captured once into a HIP graph and replayed.
 * Results equal those of msr_step1_low_res / msr_step2_full_res on each
 * channel alone (same kernels, same arithmetic order), apart from the
 * stopping rule: a batched solve runs a fixed number of iterations.
 * ------------------------------------------------------------------------- */
typedef struct msr_batch msr_batch;

/* Bytes of device workspace a batch of these channel configurations needs
 * (0 if the configurations are invalid: all channels must share pad,
 * precision, positivity and device). */
size_t msr_batch_workspace_bytes(int channels, const msr_config* cfgs);

/* Creates a batch of `channels` contexts configured by cfgs[0..channels-1]. */
msr_status msr_batch_init(int channels, const msr_config* cfgs, msr_batch** out);

/* Frees the batch, its contexts, streams and graph (not the workspace). */
void msr_batch_destroy(msr_batch* batch);

/* Text of the last failed batch call. */
const char* msr_batch_last_error(const msr_batch* batch);

/* Number of channels. */
int msr_batch_channels(const msr_batch* batch);

/* Channel c's context, owned by the batch: set its dirty images and PSFs
 * (msr_set_dirty_psf), filters (msr_set_filters) and, optionally, its
 * Lipschitz constants with the single-context calls.  Do not give it a
 * workspace or destroy it.  NULL if c is out of range. */
msr_ctx* msr_batch_channel(msr_batch* batch, int c);

/* Hands over the caller-allocated workspace (256-byte aligned, at least
 * msr_batch_workspace_bytes) and places every channel's context in it. */
msr_status msr_batch_set_workspace(msr_batch* batch, void* dev, size_t bytes);

/* msr_autotune on the first channel of each size and the choice copied to the
 * others of that size. */
msr_status msr_batch_autotune(msr_batch* batch, int reps, void* stream);

/* `iters` FISTA iterations of step s (1: Eq. 4, 2: Eq. 5) for every channel:
 * lambda[c] its regularisation weight, low_res[c] its constraint image (step 2),
 * x0 NULL or x0[c] its start (NULL entries: 0), model_out[c] its result
 * beta_iters (device, N_c x N_c); image_out (step 1 only, may be NULL) receives
 * each channel's low-resolution image beta + (i~_L - H_L beta) (Sect. 3.2, as
 * msr_step1_low_res).  res, if not NULL, receives per channel the
 * exact objective of the result (FP64), theta and the elapsed time of the whole
 * batched iteration loop.  Channels without a cached theta get one by power
 * iteration first.  The first call for a given (step, iters, kept columns,
 * variants, runs) captures the graph; later calls replay it.  Blocks until done. */
msr_status msr_batch_solve(msr_batch* batch, int step, const double* lambda, int iters, const void* const* low_res,
                           const void* const* x0, void* const* model_out, void* const* image_out, msr_result* res,
                           void* stream);

/* How msr_batch_solve runs the iterations.
 *  mode 0 (default): one launch per pass for each run of equal-sized
 *    channels with similar kept columns (groups of 2048^2 and larger images
 *    are cut into runs whose kept columns stay within 1.2x; smaller sizes
 *    form one run), all captured in one graph (runs spread over four streams).
 *  Mode 1 is switched off (msr_batch_set_mode returns MSR_ERR_UNSUPPORTED): its first
 *  solve did not return within minutes, in two designs of its memory
 *  ordering, and the cause has not been found.
 *  mode 1: one persistent launch for all channels and all iterations.  The
 *    passes of Algorithm 1 (four per step-1 iteration, six per step-2) of
 *    every channel become work items; each channel is assigned to one XCD,
 *    whose blocks take its items from that XCD's ticket counter in
 *    iteration-major, then pass-major, then channel order; an item waits until
 *    the pass it reads from has finished on its channel (counters in device
 *    memory).  Each channel runs with its own kept columns (no widening to the
 *    widest of its size, unlike mode 0), so mode-1 results equal
 *    msr_step*_ on that channel alone when the same kernel variants are in
 *    use.  Supported: single precision, pad 2, image sides 512, 1024, 2048
 *    and 4096 (MSR_ERR_UNSUPPORTED otherwise, at solve time).
 *  spin_limit: polls of a wait before the launch gives up (0: 2^22, about a
 *    second); a wait that gives up raises an abort flag every block sees,
 *    all blocks return, and msr_batch_solve fails with MSR_ERR_HIP and the
 *    models are undefined.  Returns MSR_ERR_INVALID for another mode. */
msr_status msr_batch_set_mode(msr_batch* batch, int mode, unsigned int spin_limit);

/* Sets (raise != 0) or clears the host's give-up flag of the persistent
 * launch: while it is set, a mode-1 solve's blocks return at their next
 * item or wait and the solve fails with MSR_ERR_HIP.  The flag is kept for
 * later solves until cleared.  Blocks until the flag is written. */
msr_status msr_batch_give_up(msr_batch* batch, int raise, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSR_H */
