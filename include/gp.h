/*
 * gp.h - C ABI of libmercergp, a decomposed-kernel (Mercer) Gaussian-process
 * library for AMD Instinct MI355X (gfx950).
 *
 * Method: D. Carminati, "Parallel Gaussian Process with Kernel Approximation
 * in CUDA" (arXiv 2403.12797), Sec. 2.  The squared-exponential kernel
 * (eq. 13, ARD form eq. 17) is replaced by its truncated Mercer expansion
 * k ~ Phi Lambda Phi^T (eq. 7) over all M = n^p tensor-product multi-indices
 * (eqs. 18-20), with 1-D eigenpairs of eqs. 14-16.  The FAGP posterior
 * (eqs. 10-12) is computed in the algebraically equal weight-space form
 *     A  = Phi^T Phi + sigma^2 Lambda^-1        (= sigma^2 Lambda_bar, eq. 10)
 *     w  = A^-1 Phi^T y
 *     mu_* = Phi_* w                             (eq. 11)
 *     v_*  = sigma^2 diag(Phi_* A^-1 Phi_*^T)    (diagonal of eq. 12)
 * (W of eq. 11 simplifies to Phi_* A^-1 Phi^T; I - A^-1 Phi^T Phi equals
 * sigma^2 A^-1 Lambda^-1.)  The prior mean is zero and v_* is the variance of
 * the latent f_* (no added sigma^2).
 *
 * Conventions for every entry point
 *  - Return value: gp_status; 0 is success, negative is an error.  No C++
 *    exception crosses the ABI.  gp_last_error() gives a message for the last
 *    failing call on the calling thread.
 *  - Arrays named "device" are device pointers in the memory of the context's
 *    GPU (for example torch tensors); arrays named "host" are host pointers.
 *    The caller owns every array it passes; the library never frees them.
 *  - x arrays are row-major float64 [count * p] (sample i, dimension j at
 *    i*p + j); y / mean / var are float64 [count].
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is ordered on that stream.
 *  - Multi-indices (eq. 18) are enumerated in C order: index
 *    m = sum_j k_j n^(p-1-j), the last input dimension varying fastest.  Only
 *    the layout of w (gp_model_get) depends on that order.
 */
#ifndef MERCERGP_GP_H
#define MERCERGP_GP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GP_OK = 0,
  GP_PENDING = 1,      /* gp_poll: request not finished yet                     */
  GP_EINVAL = -1,      /* invalid argument (checked before any device work)     */
  GP_ENOMEM = -2,      /* device allocation failed or request can never fit     */
  GP_ENOTSPD = -3,     /* Cholesky found a non-positive pivot (message: column) */
  GP_EDEVICE = -4,     /* HIP runtime error                                     */
  GP_ENOTFOUND = -5,   /* unknown request id                                    */
  GP_ECANCELED = -6    /* request dropped because the context is shutting down  */
} gp_status;

typedef enum {
  GP_PREC_FP64 = 0,      /* every contraction in FP64 (FP64 MFMA)               */
  GP_PREC_MIXED = 1,     /* Gram as split-BF16 MFMA products (three BF16 terms
                            per value, six products), predictive variance as
                            split-BF16 (two terms, three products), FP32
                            accumulation; FP64 factorisation, solves, one FP64
                            iterative-refinement step on w                     */
  GP_PREC_MIXED_F16 = 2  /* as GP_PREC_MIXED, but the Gram as split-FP16 MFMA
                            products (two FP16 terms per value, three
                            products) on Phi scaled by exact powers of two per
                            1-D table row.  The FP16 pair keeps about 22
                            significant bits per value (the BF16 triple keeps
                            all 24 of FP32) at half the matrix work; the
                            same tolerances hold for both                      */
} gp_precision;

typedef enum {
  GP_KERNEL_SE = 0,       /* squared exponential (Sec. 2.3, eqs. 13-20)          */
  GP_KERNEL_PERIODIC = 1  /* periodic (exp-sine-squared), per dimension
                             k = exp(-2 eps^2 sin^2(alpha (x - x') / 2)): one of
                             the other Mercer kernels Sec. 2.3 mentions.  Its
                             expansion on one period (Jacobi-Anger): features
                             1, sqrt2 cos(k alpha x), sqrt2 sin(k alpha x),
                             eigenvalues e^-a I_0(a), then e^-a I_k(a) for
                             both of harmonic k, a = eps^2                     */
} gp_kernel;

/* Limits enforced by validation. */
#define GP_MAX_P 8
#define GP_MAX_N 64
#define GP_MAX_M 16384
#define GP_MAX_PERIODIC_EPS 16.0   /* periodic kernel: eps_j <= this            */

/* Problem parameters (Sec. 2.1 problem statement; eqs. 13-20).
 *  p      input dimension, 1..GP_MAX_P
 *  n      eigenvalues per dimension, 1..GP_MAX_N; M = n^p <= GP_MAX_M
 *  sigma  noise standard deviation, > 0 (Sigma_n = sigma^2 I, Sec. 2.2)
 *  eps    host [p]: ARD length scales eps_j > 0 (eq. 17); periodic kernel:
 *         inverse length scales, 0 < eps_j <= GP_MAX_PERIODIC_EPS
 *  alpha  host [p]: global scale factors rho_j > 0 (eqs. 14-16, 19-20);
 *         periodic kernel: angular frequencies (period 2 pi / alpha_j) > 0
 *  precision  gp_precision
 *  kernel     gp_kernel (0, the SE kernel, when the field is zeroed)       */
typedef struct {
  int32_t p;
  int32_t n;
  double sigma;
  const double *eps;
  const double *alpha;
  int32_t precision;
  int32_t kernel;
} gp_params;

typedef struct gp_ctx gp_ctx;      /* one GPU: streams, workspace, scheduler   */
typedef struct gp_model gp_model;  /* device-resident fitted model             */

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory the served path (gp_submit) may hold at once; 0 means 90% of the
 * free memory at creation.  Errors: GP_EINVAL (bad device), GP_EDEVICE.     */
gp_status gp_ctx_create(int device, size_t hbm_budget_bytes, gp_ctx **out);

/* Destroy a context: stops its scheduler (pending requests end as
 * GP_ECANCELED) and frees its workspace.  Models created from it must be
 * freed first.  NULL is accepted.                                           */
gp_status gp_ctx_destroy(gp_ctx *ctx);

/* Fit: Lambda (eq. 20), A = Phi^T Phi + sigma^2 Lambda^-1 and b = Phi^T y with
 * Phi generated on the fly (eqs. 15, 19), Cholesky A = L L^T, w = A^-1 b
 * (mixed precision: plus one FP64 refinement step), and L^-1 for the
 * variance.  x: device [N*p], y: device [N], N >= 1.  The call returns once
 * the model is ready (it waits on `stream`); x and y may then be freed.
 * *out_model receives a new model owned by the caller (gp_model_free).
 * Errors: GP_EINVAL (parameters, N < 1, NULL pointers), GP_ENOMEM,
 * GP_ENOTSPD (numerically non-SPD A), GP_EDEVICE.                          */
gp_status gp_fit(gp_ctx *ctx, const gp_params *params, const double *x, const double *y,
                 int64_t N, void *stream, gp_model **out_model);

/* Predict: mean = Phi_* w (eq. 11) and var = sigma^2 diag(Phi_* A^-1 Phi_*^T)
 * (diagonal of eq. 12).  xs: device [Ns*p]; mean, var: device [Ns]; either
 * output may be NULL (not computed).  Ns = 0 is a no-op.  The work is
 * enqueued on `stream` and the call returns without waiting; outputs are
 * valid once the stream has reached this point.  Precision follows the
 * model.  Errors: GP_EINVAL, GP_ENOMEM, GP_EDEVICE.                          */
gp_status gp_predict(gp_ctx *ctx, const gp_model *model, const double *xs, int64_t Ns,
                     double *mean, double *var, void *stream);

/* Predict without allocating, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): as gp_predict, same kernels and results, but the
 * prediction's workspace (the variance partial sums) is a fixed device array
 * of GP_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; no hipMalloc / hipFree or other allocating call is
 * made.  The array is shared by every call on a GPU and keeps the last
 * call's contents (nothing in it needs to start at zero): calls that overlap
 * on one GPU, from any thread or stream, race and must be serialised by the
 * caller.  Profiling events are not recorded.  Errors: as gp_predict, and
 * GP_EINVAL when Ns is too large for the array (a mixed model needs
 * 8 * Ns * g + 256 bytes, g <= ceil(M / 256) partial-sum groups, g = 1 once
 * Ns >= 128 * 1024; the FP64 path g <= ceil(M / 64), g = 1 once Ns >=
 * 64 * 2048).                                                                */
#define GP_NOALLOC_SCRATCH_BYTES (32u << 20)
gp_status gp_predict_noalloc(gp_ctx *ctx, const gp_model *model, const double *xs, int64_t Ns,
                             double *mean, double *var, void *stream);

/* Free a model (waits for the device work that uses it).  NULL accepted.
 * A served model's bytes leave the context's admission budget here.        */
gp_status gp_model_free(gp_model *model);

/* Model shape: any output pointer may be NULL.                              */
gp_status gp_model_info(const gp_model *model, int32_t *p, int32_t *n, int64_t *M,
                        int32_t *precision, double *sigma);

/* Copy w (eq. 11 in weight-space form: mu_* = Phi_* w) to host memory,
 * w_host [M] in C-order multi-index (synchronous).  Errors: GP_EINVAL.      */
gp_status gp_model_weights(const gp_model *model, double *w_host);

/* Copy a model array to host memory (synchronous).  `count` is the capacity
 * of host_out in doubles and must be at least the array size:
 *   GP_MODEL_W        [M]    weights w, C-order multi-index
 *   GP_MODEL_LAMBDA   [M]    Lambda_m, eq. 20
 *   GP_MODEL_A        [M*M]  A = Phi^T Phi + sigma^2 Lambda^-1 (row-major,
 *                            both triangles), as accumulated on the GPU
 *   GP_MODEL_B        [M]    Phi^T y
 *   GP_MODEL_L        [M*M]  Cholesky factor L (row-major, upper part zero)
 *   GP_MODEL_LINV     [M*M]  L^-1 (row-major, upper part zero)
 * Models from gp_fit / gp_fit_batch keep every array.  Served models
 * (gp_submit) are lean: they keep w, Lambda, b and what the variance needs
 * (L^-1 for FP64; its BF16 terms for mixed precision), so GP_MODEL_A,
 * GP_MODEL_L and, for mixed precision, GP_MODEL_LINV are not available.
 * Errors: GP_EINVAL (unknown or absent array, count too small), GP_EDEVICE. */
enum { GP_MODEL_W = 0, GP_MODEL_LAMBDA = 1, GP_MODEL_A = 2, GP_MODEL_B = 3, GP_MODEL_L = 4,
       GP_MODEL_LINV = 5 };
gp_status gp_model_get(const gp_model *model, int32_t what, double *host_out, int64_t count);

/* Log marginal likelihood of the data a model was fitted to, log p(y) for
 * y ~ N(0, Phi Lambda Phi^T + sigma^2 I) (the truncated-kernel GP of eqs.
 * 7-8 with zero prior mean), formed at fit time from the M x M system:
 *   log p(y) = -(y^T y - b^T w) / (2 sigma^2)
 *              - ((N - M) log sigma^2 + sum_m log Lambda_m + log det A) / 2
 *              - N log(2 pi) / 2,
 * A = L L^T = Phi^T Phi + sigma^2 Lambda^-1, b = Phi^T y, w = A^-1 b (Woodbury
 * and the matrix determinant lemma).  Mixed-precision models use their
 * mixed A.  Synchronous.  Errors: GP_EINVAL, GP_EDEVICE.                    */
gp_status gp_model_lml(const gp_model *model, double *lml);

/* Full predictive covariance of the latent f_* at a block of Ns test points
 * (eq. 12): Sigma_* = sigma^2 Phi_* A^-1 Phi_*^T = sigma^2 Z Z^T with
 * Z = Phi_* L^-T, in FP64 on FP64 MFMA (Phi_* of the block is materialised,
 * Ns x M, in a workspace of 16 Ns M bytes).  xs: device [Ns*p]; cov: device,
 * row-major with row pitch ld >= Ns, both triangles written; its diagonal
 * equals gp_predict's variance up to rounding (the FP64 path bit for bit in
 * exact arithmetic).  Needs the model's FP64 L^-1: models from gp_fit and
 * gp_fit_batch (all precisions), not the lean served models.  Enqueued on
 * `stream`; returns without waiting.  Ns <= 2^20.
 * Errors: GP_EINVAL, GP_ENOMEM, GP_EDEVICE.                                 */
gp_status gp_predict_cov(gp_ctx *ctx, const gp_model *model, const double *xs, int64_t Ns,
                         double *cov, int64_t ld, void *stream);

/* Hyperparameter learning (the paper's Sec. 5 outlook): maximise the log
 * marginal likelihood (gp_model_lml) over log eps, optionally log alpha and
 * log sigma, by Nelder-Mead from `start` (initial simplex steps of 0.3 in
 * each log-parameter).  Every evaluation is a full gp_fit on the device at
 * start's precision, p and n; a fit that fails as not SPD counts as -inf.
 *  max_evals    fits at most (<= 0: 150)
 *  per_dim      0: one eps (and alpha) shared by all dimensions, starting
 *               from start->eps[0] (alpha[0]); 1: one per dimension (ARD)
 *  learn_alpha  nonzero: alpha is learnt, else kept at start's
 *  learn_sigma  nonzero: sigma is learnt, else kept at start's
 *  tol          stop once the simplex's log likelihoods span <= tol
 *               (<= 0: 1e-6)
 * Outputs (each may be NULL): eps_out[p], alpha_out[p], *sigma_out of the
 * best point, *lml_out its log likelihood, *evals_out the fits made.  x, y as
 * in gp_fit.  Synchronous.  Errors: GP_EINVAL, GP_ENOMEM, GP_EDEVICE,
 * GP_ENOTSPD (no evaluated point was SPD).                                  */
typedef struct {
  int32_t max_evals;
  int32_t per_dim;
  int32_t learn_alpha;
  int32_t learn_sigma;
  double tol;
} gp_learn_opts;
gp_status gp_learn(gp_ctx *ctx, const gp_params *start, const double *x, const double *y, int64_t N,
                   const gp_learn_opts *opts, void *stream, double *eps_out, double *alpha_out,
                   double *sigma_out, double *lml_out, int32_t *evals_out);

/* Batched fit of `count` independent problems (uneven N, p, n allowed):
 * params/x/y/N/out_models are arrays of length count (x[k], y[k] device
 * arrays as in gp_fit).  The mixed-precision problems of each Gram scheme
 * share one persistent Gram launch over all their tiles (work list, longest
 * first); the per-problem work runs on four forked streams (enqueued
 * directly; MGP_BATCH_GRAPH=1 captures the whole batch in one HIP graph
 * first, the same results).  Waits for completion.  Each
 * out_models[k] is a new model; on an error the failing problem's model is
 * NULL and the first error is returned (other models stay valid).
 * Errors: as gp_fit, with the problem index in the message.               */
gp_status gp_fit_batch(gp_ctx *ctx, int32_t count, const gp_params *params, const double *const *x,
                       const double *const *y, const int64_t *N, void *stream, gp_model **out_models);

/* Batched predict: as gp_predict for each k (mean/var may be NULL arrays or
 * hold NULL entries); enqueued on `stream`, returns without waiting.        */
gp_status gp_predict_batch(gp_ctx *ctx, int32_t count, const gp_model *const *models,
                           const double *const *xs, const int64_t *Ns, double *const *mean,
                           double *const *var, void *stream);

/* Autotuner: time the mixed Gram kernel (split-FP16 scheme; the chunk it
 * picks serves both mixed modes) for (p, n, N) on synthetic
 * inputs at several sample-chunk lengths and keep the fastest for later fits
 * of this context with the same p, n and floor(log2 N) (and in the file named
 * by the environment variable MGP_TUNE_CACHE, read at context creation).
 * *chunk_out (may be NULL) receives the chosen chunk.  Errors: GP_EINVAL,
 * GP_ENOMEM, GP_EDEVICE.                                                     */
gp_status gp_autotune(gp_ctx *ctx, int32_t p, int32_t n, int64_t N, int32_t *chunk_out);

/* Served path: asynchronous requests with continuous batching.
 *  kind   GP_REQ_FIT (x, y, N -> model), GP_REQ_PREDICT (model, xs, Ns ->
 *         mean/var), GP_REQ_FIT_PREDICT (both; the model is kept only if
 *         model_out is requested at poll time, else freed).
 * All arrays are device arrays as above and must stay valid until gp_poll
 * has returned a final (non-PENDING) status for the request.  Requests run
 * on the context's own streams, ordered after nothing of the caller's: the
 * work that writes x, y, xs (or that still touches mean, var) must be
 * complete when gp_submit is called (synchronise its stream first).  Requests are
 * admitted when their device footprint fits what the context's HBM budget
 * has left (the budget less the bytes of admitted requests and of served
 * models not yet freed); work of admitted requests overlaps on the device.
 * Admission takes the first queued request that fits; a request that does
 * not fit yet is passed over by later ones at most 32 times, after which
 * admission waits for it.  Fitted models are lean (see gp_model_get) and
 * stay charged to the budget until gp_model_free (or, when model_out is not
 * requested, until gp_poll frees them).
 * gp_submit errors: GP_EINVAL, GP_ENOMEM (footprint exceeds the whole budget).
 * gp_poll: waits up to wait_us microseconds (0 = just check, <0 = forever);
 * returns GP_PENDING, or the request's final status exactly once, after
 * which the id is retired (GP_ENOTFOUND afterwards).  For FIT kinds the
 * fitted model is stored to *model_out if model_out is not NULL.          */
enum { GP_REQ_FIT = 0, GP_REQ_PREDICT = 1, GP_REQ_FIT_PREDICT = 2 };
typedef struct {
  int32_t kind;
  gp_params params;           /* FIT kinds; eps/alpha copied at submit        */
  const double *x, *y;        /* device [N*p], [N]                            */
  int64_t N;
  const gp_model *model;      /* PREDICT                                      */
  const double *xs;           /* device [Ns*p]                                */
  int64_t Ns;
  double *mean, *var;         /* device [Ns], either may be NULL              */
} gp_request;
gp_status gp_submit(gp_ctx *ctx, const gp_request *req, int64_t *req_id);
gp_status gp_poll(gp_ctx *ctx, int64_t req_id, int32_t wait_us, gp_model **model_out);

/* Device bytes a request would hold if submitted now (validated as in
 * gp_submit, nothing enqueued): *model_bytes (may be NULL) is the lean model
 * of a FIT kind, which stays resident while the caller holds the model;
 * *transient_bytes (may be NULL) is the fit and predict workspace held while
 * the request runs.  Errors: as gp_submit's validation.                     */
gp_status gp_request_footprint(gp_ctx *ctx, const gp_request *req, size_t *model_bytes,
                               size_t *transient_bytes);

/* Admission state of the served path: the HBM budget, the bytes held by
 * admitted requests, and the bytes of served models not yet freed.  Any
 * output may be NULL.  Errors: GP_EINVAL.                                    */
gp_status gp_ctx_memory(gp_ctx *ctx, size_t *budget, size_t *in_flight, size_t *resident);

/* Profiling: device time per phase, measured with HIP events recorded on
 * the stream each phase runs on.  gp_profile_enable(ctx, 1) clears the totals
 * and starts recording for later gp_fit / gp_predict calls of this context
 * (one call at a time per context while enabled); gp_profile_read waits for
 * the recorded events and returns the total milliseconds and the number of
 * timed intervals of one phase.  Errors: GP_EINVAL (phase), GP_EDEVICE.     */
enum { GP_PH_GRAM = 0,          /* fused Phi + Gram kernels (a3)            */
       GP_PH_GRAM_REDUCE = 1,   /* split-K reduction into A                 */
       GP_PH_PHIT = 2,          /* b = Phi^T y                              */
       GP_PH_CHOL = 3,          /* Cholesky                                 */
       GP_PH_TRTRI = 4,         /* L^-1                                     */
       GP_PH_SOLVE = 5,         /* solves and the refinement step           */
       GP_PH_SPLIT = 6,         /* BF16 split of L^-1 (mixed)               */
       GP_PH_PREDICT = 7,       /* fused predict / variance kernels (a5)    */
       GP_PH_PREDICT_MEAN = 8,  /* FP64 mean kernel (FP64 path)             */
       GP_PH_PREDICT_REDUCE = 9,
       GP_PH_COUNT = 10 };
gp_status gp_profile_enable(gp_ctx *ctx, int32_t on);
gp_status gp_profile_read(gp_ctx *ctx, int32_t phase, double *total_ms, int64_t *count);

/* Message describing the last failing call on the calling thread ("" if
 * none).  Messages are kept per thread, not per context; ctx may be NULL.   */
const char *gp_last_error(const gp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MERCERGP_GP_H */
