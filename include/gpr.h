/*
 * gpr.h — C-ABI of the MI355X (gfx950) exact Gaussian-process regression library.
 *
 * The operations follow Section 4 of "GPRat: Gaussian Process Regression with
 * Asynchronous Tasks" (arXiv 2505.00136): the squared-exponential kernel
 * (Eq. 2), the Cholesky factor of the training covariance K (Section 4.2),
 * the posterior mean (Eq. 3), the posterior covariance (Eq. 4), the log
 * marginal likelihood (Eq. 5), its gradient and the Adam hyperparameter
 * optimisation (Section 4.1), computed with the tiled right-looking Cholesky
 * of Fig. 1 (POTRF / TRSM / SYRK / GEMM on T x T tiles).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All arrays are device pointers unless marked "host".  The caller allocates
 *    and frees every buffer; the library keeps no pointer after a call returns.
 *  - Matrices are row-major and contiguous: Z is n x d (row i = z_i), Zs is m x d.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it
 *    and calls return without waiting, except where a host output is documented;
 *    those calls synchronise `stream` before returning.  Calls that launch tile
 *    products (gpr_cholesky, gpr_predict_var, gpr_nlml_grad, gpr_optimize) copy their
 *    job tables through a ring of 8 pinned host slots per device; a call waits only when
 *    all 8 hold copies that the GPU has not reached yet.
 *  - Resources: the library allocates no device memory; the caller passes every buffer.
 *    Its own host-side resources (the staging ring, an auxiliary stream of default
 *    priority and events, per device) are created by gpr_init, or by the first call that
 *    needs them on a device gpr_init did not cover, and kept until the process ends.
 *  - `tile` is the tile edge b, any b >= 1: T = ceil(n / b) tiles per dimension (T = 1
 *    is the untiled, sequential case).  When b does not divide n the tiled matrix has
 *    T b rows, and rows and columns n..Tb-1 are an identity block with a zero border,
 *    so its factor is that of the n x n covariance bordered by the identity and every
 *    result (alpha, NLML, gradient, posterior) is the one of the n x n problem.  Vectors
 *    passed in and out (y, alpha) always have n entries.  n = 0 is accepted and does
 *    nothing.
 *  - Hyperparameters (Eq. 2): lengthscale l > 0, signal_var nu > 0, noise_var sigma^2 >= 0,
 *    all finite.  sigma^2 enters K only on equal indices (the Kronecker delta of Eq. 2);
 *    cross-covariances and the test prior carry no noise.
 *  - Status: every call returns GPR_OK or an error code and never throws; the
 *    message of the last error on the calling thread is gpr_last_error().
 *  - `prec` selects the arithmetic of the Cholesky's trailing updates (GPR_FP64
 *    everywhere, or a mixed mode: diagonal-tile POTRF, the log-determinant, the
 *    refinement residuals and the variance subtraction always stay float64).
 *
 * Tiled matrix ("K_tiles") layout, size from gpr_tiles_bytes()
 * ------------------------------------------------------------
 *  Region D: T diagonal tiles b x b, float64, row-major; tile k at element k*b*b.
 *  Region W: T diagonal-tile inverses L_kk^{-1} (float64, lower triangular, zero upper),
 *            written by gpr_cholesky and used by the solves, the variance and the gradient.
 *  Region O: the T(T-1)/2 strictly-lower tiles (i > j), row-major each, stored
 *            column by column: tile (i,j) has index j(T-1) - j(j-1)/2 + (i-j-1).
 *            Element type float64 for GPR_FP64, float32 for the mixed modes.
 *  Only the lower triangle of K is stored; strictly-upper parts of diagonal tiles
 *  are zero after gpr_cholesky.  Rows and columns n..Tb-1 (present when b does not
 *  divide n) are the identity padding, in K and in L alike.
 */
#ifndef GPR_H_
#define GPR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPR_API __attribute__((visibility("default")))

/* Covariance functions.  GPR_KERNEL_SE is the squared exponential of Eq. 2,
 * k(r) = nu exp(-r^2 / (2 l^2)).  The Matern kernels are the further kernel functions
 * that Section 6 names, with s = r / l:
 *   GPR_KERNEL_MATERN12: nu exp(-s)
 *   GPR_KERNEL_MATERN32: nu (1 + sqrt(3) s) exp(-sqrt(3) s)
 *   GPR_KERNEL_MATERN52: nu (1 + sqrt(5) s + 5 s^2 / 3) exp(-sqrt(5) s)
 * In every case sigma^2 is added on the diagonal of the training covariance. */
enum gpr_kernel {
  GPR_KERNEL_SE = 0,
  GPR_KERNEL_MATERN12 = 1,
  GPR_KERNEL_MATERN32 = 2,
  GPR_KERNEL_MATERN52 = 3
};

/* Hyperparameters of Eq. 2: l, nu, sigma^2, and the covariance function (a gpr_kernel;
 * 0, the squared exponential, when a caller zero-initialises the struct). */
typedef struct {
  double lengthscale;
  double signal_var;
  double noise_var;
  int32_t kernel;
} gpr_hyper_t;

enum gpr_status {
  GPR_OK = 0,
  GPR_ERR_ARG = 1,        /* null pointer, bad precision tag, non-finite or non-positive hyperparameter */
  GPR_ERR_SHAPE = 2,      /* tile < 1, negative size */
  GPR_ERR_NOT_SPD = 3,    /* a non-positive pivot in the Cholesky factorisation */
  GPR_ERR_OOM = 4,        /* a size whose byte count overflows */
  GPR_ERR_HIP = 5,        /* a HIP runtime error */
  GPR_ERR_WORKSPACE = 6   /* ws_bytes smaller than gpr_workspace_size() */
};

/* Precision of the trailing updates of the tiled Cholesky (TRSM / SYRK / GEMM tasks). */
enum gpr_precision {
  GPR_FP64 = 0,    /* float64 everywhere (the paper's double-precision BLAS, Section 5) */
  GPR_FP32 = 1,    /* float32 off-diagonal tiles, float32 matrix-core products */
  GPR_BF16X3 = 2,  /* float32 tiles; products from the hi/mid/lo bfloat16 split: hh+hm+mh */
  GPR_BF16X6 = 3   /* as GPR_BF16X3 plus hl+lh+mm (close to float32 accuracy) */
};

/* Library version, (major << 16) | (minor << 8) | patch. */
GPR_API int gpr_version(void);

/* Message of the last failing call on this thread (static storage, never NULL). */
GPR_API const char* gpr_last_error(void);

/* Set-up of the current device, outside any hot loop: creates the auxiliary stream and
 * the events of the factorisation's look-ahead and the pinned staging ring of the job
 * tables, sized for every call on problems up to n training points, m test points and
 * tile edge `tile` in precision `prec` (n = 0: the minimum sizes).  Later calls on larger
 * problems grow these resources when they first need them.  Optional: every call creates
 * what it lacks.  Host only; may be called again (it only grows the resources). */
GPR_API int gpr_init(int64_t n, int64_t m, int64_t tile, int prec);

/* Schedules of the tiled factorisation (gpr_set_schedule); all give the same bits.
 *  GPR_SCHEDULE_STREAM:    every launch on the caller's stream, in the order of Fig. 1.
 *  GPR_SCHEDULE_LOOKAHEAD: (the default) diagonal tile k+1 and its panel are factored on an
 *                          auxiliary stream while step k's remaining update runs on the
 *                          caller's stream, events ordering the two (in the mixed
 *                          precisions the diagonal tile starts as soon as step k has updated
 *                          it, beside the update of the rest of its block column).
 *  GPR_SCHEDULE_DEVICE:    the tasks of Fig. 1 (and the block steps inside the diagonal
 *                          tiles) form a graph whose edges are their tile dependencies
 *                          (Section 4.2's dataflow), executed by one persistent kernel: a
 *                          task whose predecessors have finished enters a ready queue (the
 *                          critical path first) and workgroups take its work items, the
 *                          dependencies being resolved by per-task counters on the device
 *                          (in place of the futures of Section 3.1).  GPR_FP64 only; the
 *                          other precisions use the look-ahead.  When no task finishes for
 *                          10 s the run gives up: gpr_cholesky then reports GPR_ERR_HIP when
 *                          `info` is requested. */
enum gpr_schedule { GPR_SCHEDULE_STREAM = 0, GPR_SCHEDULE_LOOKAHEAD = 1, GPR_SCHEDULE_DEVICE = 2 };

/* Schedule of gpr_cholesky (a gpr_schedule), process-wide, for factorisations issued
 * afterwards.  Host only.  Errors: GPR_ERR_ARG for an unknown schedule. */
GPR_API int gpr_set_schedule(int mode);

/* gpr_set_schedule(on ? GPR_SCHEDULE_LOOKAHEAD : GPR_SCHEDULE_STREAM). */
GPR_API int gpr_set_lookahead(int on);

/* Bytes of the tiled matrix of an n x n covariance with tile edge `tile` in precision `prec`
 * (layout above).  bytes: host out. */
GPR_API int gpr_tiles_bytes(int64_t n, int64_t tile, int prec, size_t* bytes);

/* Workspace bytes that suffice for every call below with these sizes (n training
 * points, m test points, d features).  bytes: host out. */
GPR_API int gpr_workspace_size(int64_t n, int64_t m, int64_t d, int64_t tile, int prec, size_t* bytes);

/* Covariance assembly, Eq. 2 (Section 4.1: all pairwise combinations of feature
 * vectors; Section 4.2: tile by tile).  Writes regions D and O of K_tiles with
 * K_ij = nu exp(-|z_i - z_j|^2 / (2 l^2)) + sigma^2 [i == j], lower tiles only
 * (diagonal tiles in full), and the identity padding for i or j >= n.  Z: n x d
 * float64 (read only; rows beyond n are never read).  K_tiles: out.
 * Accuracy: for the squared exponential the squared distances of a 128 x 128 block of
 * points come from |z_i|^2 + |z_j|^2 - 2 z_i . z_j on the matrix cores when
 * (max |z_i|^2 + max |z_j|^2) / (2 l^2) <= 16 over the block, from explicit differences
 * otherwise (and for the Matern kernels), so every kernel value is within a few dozen
 * ulp of nu; a point with itself is at distance 0, a NaN feature gives NaN values.  The
 * kernel-vector products of gpr_solve's residual and of gpr_predict follow the same rule. */
GPR_API int gpr_assemble(const double* Z, int64_t n, int64_t d, gpr_hyper_t h, int64_t tile, int prec,
                         void* K_tiles, void* stream);

/* Tiled right-looking Cholesky K = L L^T in place (Section 4.2, Fig. 1): for each
 * step k, POTRF of the diagonal tile (float64), TRSM of the tiles below it, SYRK
 * of the later diagonal tiles and GEMM of the other trailing tiles.  On return
 * regions D and O hold L (zero strictly-upper parts in D) and region W holds the
 * inverses of the diagonal tiles of L.  Diagonal tile k+1 and its panel are factored
 * on a second stream while the rest of step k's update runs on `stream` (events order
 * the two, and the call returns with all work ordered on `stream`).  After
 * gpr_set_lookahead(0) every launch goes to `stream` instead; both schedules give the
 * same bits.
 * info: host out, or NULL.  When non-NULL the call synchronises `stream` and stores
 * 0, or the 1-based global column of the first non-positive pivot (LAPACK
 * convention), in which case it returns GPR_ERR_NOT_SPD and the factor is unspecified.
 * ws: device workspace of at least ws_bytes (gpr_workspace_size). */
GPR_API int gpr_cholesky(void* K_tiles, int64_t n, int64_t tile, int prec, void* ws, size_t ws_bytes,
                         int64_t* info, void* stream);

/* alpha = K^{-1} y by forward (L z = y) then backward (L^T alpha = z) substitution
 * over the tiles (Section 4.2; alpha feeds Eq. 3 and Eq. 5).  With refine_sweeps > 0
 * each sweep computes the float64 residual r = y - K alpha with K regenerated from Z
 * and h (never stored), solves for the correction with the factor and adds it;
 * this lifts a mixed-precision factor to float64 accuracy.  refine_sweeps < 0 takes the
 * precision's default, which gpr_optimize uses too: 0 for GPR_FP64, 3 for GPR_FP32 and
 * GPR_BF16X6, 6 for GPR_BF16X3 (each sweep contracts the error by about kappa u of the
 * factor).  Z and h are read only when sweeps are run.  y: n (in), alpha: n (out; may
 * not alias y). */
GPR_API int gpr_solve(const void* L_tiles, const double* Z, int64_t n, int64_t d, gpr_hyper_t h, int64_t tile,
                      int prec, const double* y, double* alpha, int refine_sweeps, void* ws, size_t ws_bytes,
                      void* stream);

/* Posterior mean, Eq. 3: mean_j = sum_i k(zs_j, z_i) alpha_i for j < m, with the
 * cross-covariance regenerated from Z and Zs (never stored).  mean: m (out). */
GPR_API int gpr_predict(const double* Z, int64_t n, const double* Zs, int64_t m, int64_t d, gpr_hyper_t h,
                        const double* alpha, double* mean, void* ws, size_t ws_bytes, void* stream);

/* gpr_predict without a workspace, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same result, bit for bit, with the partial sums in a fixed device array of the library
 * (16 MiB per GPU, held until the process ends; its address is looked up by gpr_init or
 * by the first call on a device).  The call allocates nothing.  Sizes: ceil(n / 4096) * m
 * must not exceed 2^21 (e.g. m <= 131072 at n = 65536), else GPR_ERR_WORKSPACE.  Every
 * call on one GPU shares that array: calls that overlap on one GPU (different streams
 * without ordering between them) race and must not be issued.  n = 0 writes zeros. */
GPR_API int gpr_predict_noalloc(const double* Z, int64_t n, const double* Zs, int64_t m, int64_t d, gpr_hyper_t h,
                                const double* alpha, double* mean, void* stream);

/* Posterior uncertainty, Eq. 4, from the factor: V = L^{-1} K_{Z,Zs} by one tiled
 * forward substitution with m right-hand sides (the same substitution that serves
 * the mean; Section 5.1), then
 *   full_cov = 0: out[j] = nu - sum_i V_ij^2                  (m values, the diagonal of Eq. 4)
 *   full_cov = 1: out[j*m + k] = k(zs_j, zs_k) - (V^T V)_jk   (m x m, row-major)
 * add_noise = 1 adds sigma^2 to the variances (the diagonal).  Sums of squares and
 * the subtraction are float64 in every precision. */
GPR_API int gpr_predict_var(const double* Z, int64_t n, const double* Zs, int64_t m, int64_t d, gpr_hyper_t h,
                            const void* L_tiles, int64_t tile, int prec, int full_cov, int add_noise, double* out,
                            void* ws, size_t ws_bytes, void* stream);

/* Negative log marginal likelihood, the negative of Eq. 5:
 *   nlml = 1/2 y^T alpha + sum_i log L_ii + n/2 log(2 pi)   (log|K| = 2 sum log L_ii).
 * nlml: one float64 on the device (out). */
GPR_API int gpr_nlml(const void* L_tiles, int64_t n, int64_t tile, int prec, const double* y, const double* alpha,
                     double* nlml, void* stream);

/* Gradient of the NLML in log coordinates theta = log(l, nu, sigma^2) (Section 4.1):
 *   g_k = 1/2 sum_ij (K^{-1} - alpha alpha^T)_ij (dK/dtheta_k)_ij
 * with dK/dlog l = K_f o R^2 / l^2, dK/dlog nu = K_f, dK/dlog sigma^2 = sigma^2 I,
 * K_f the noise-free kernel and R^2 the squared distances, both regenerated from Z
 * (Matern kernels, s = r / l: dK/dlog l = nu s exp(-s), 3 nu s^2 exp(-sqrt(3) s) and
 * (5/3) nu s^2 (1 + sqrt(5) s) exp(-sqrt(5) s) for 1/2, 3/2 and 5/2).
 * K^{-1} = L^{-T} L^{-1} is formed tile by tile from the factor and consumed inside
 * the reduction.  The products run in float64 (GPR_FP64), float32 (GPR_FP32, and the
 * split modes when the tile is not a multiple of 256), or as the mode's split-bfloat16
 * products (GPR_BF16X3 / GPR_BF16X6, tiles a multiple of 256); the contraction with
 * the kernel weights is float64.  L_tiles is destroyed: region O is overwritten with the
 * strictly-lower tiles of L^{-1}.  trainable: host[3] (0 = that entry is returned as 0,
 * NULL = all trainable).  grad_log: device[3] (out). */
GPR_API int gpr_nlml_grad(const double* Z, int64_t n, int64_t d, gpr_hyper_t h, void* L_tiles, int64_t tile,
                          int prec, const double* alpha, const int* trainable, double* grad_log, void* ws,
                          size_t ws_bytes, void* stream);

/* Adam hyperparameter optimisation (Section 4.1) of theta = log(l, nu, sigma^2) for the
 * covariance function `kernel` (a gpr_kernel):
 * `steps` iterations of { assemble, Cholesky, alpha, NLML, gradient, Adam update }
 * with the optimiser state on the device, then one more NLML at the final theta.
 * theta_log: host[3] in/out.  adam_state: host[7] in/out = m[3], v[3], t (zeros to
 * start; passing the returned state resumes bit-exactly).  nlml_trace: host[steps+1]
 * out (NLML at theta_0..theta_steps) or NULL.  K_tiles: device scratch of
 * gpr_tiles_bytes().  Synchronises `stream`.  Adam: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, theta -= lr mhat / (sqrt(vhat) + eps) with bias correction;
 * entries with trainable[k] == 0 keep theta and state. */
GPR_API int gpr_optimize(const double* Z, const double* y, int64_t n, int64_t d, int64_t tile, int prec, int kernel,
                         double* theta_log, const int* trainable, int steps, double lr, double beta1, double beta2,
                         double eps, double* adam_state, double* nlml_trace, void* K_tiles, void* ws,
                         size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- learned warm start
 * A small network maps 32 summary statistics of a dataset to initial log-hyperparameters
 * for gpr_optimize; the default initialisation remains the fallback, chosen whenever its
 * NLML is lower.  These calls are additions to the paper's method. */

/* Workspace bytes of gpr_summary_stats for a subsample of nsub points. */
GPR_API int gpr_stats_workspace(int64_t nsub, size_t* bytes);

/* The 32 summary statistics of one dataset, in float64 (stats64[32]) and/or cast to
 * float32 (stats32[32]); either output may be NULL:
 *   [0:8]   quantiles at k/7, k = 0..7, of the d population variances of the raw feature columns;
 *   [8:31]  quantiles at k/24, k = 1..23, of log |zs_i - zs_j| over all pairs i < j of the
 *           subsample rows sub_idx[0..nsub) of the standardised features Z_std;
 *   [31]    log of the population variance of the raw targets.
 * Quantiles interpolate linearly between order statistics at position q (count - 1).
 * Z_raw, Z_std: n x d float64; y_raw: n; sub_idx: nsub distinct row indices (int64, device);
 * 1 <= d <= 256, 2 <= nsub <= min(n, 4096). */
GPR_API int gpr_summary_stats(const double* Z_raw, const double* Z_std, const double* y_raw, int64_t n, int64_t d,
                              const int64_t* sub_idx, int64_t nsub, double* stats64, float* stats32, void* ws,
                              size_t ws_bytes, void* stream);

/* Parameter count of the network 32 -> 128 -> 128 -> 3 (exact-erf GELU after the first two
 * layers): 21,123 float32 values in the order W1 (128x32, row-major [out][in]), b1, W2
 * (128x128), b2, W3 (3x128), b3. */
GPR_API int gpr_mlp_nparams(void);

/* Workspace bytes of the network calls for a batch of `batch` rows. */
GPR_API int gpr_mlp_workspace(int64_t batch, size_t* bytes);

/* out[batch x 3] = network(X[batch x 32]); float32, row-major. */
GPR_API int gpr_mlp_forward(const float* params, const float* X, int64_t batch, float* out, void* ws, size_t ws_bytes,
                            void* stream);

/* Mean-squared-error loss over the batch x 3 outputs against Y (loss: device scalar or NULL)
 * and its gradient w.r.t. the parameters (grad: 21,123 floats, out). */
GPR_API int gpr_mlp_loss_grad(const float* params, const float* X, const float* Y, int64_t batch, float* loss,
                              float* grad, void* ws, size_t ws_bytes, void* stream);

/* One training step: loss, gradient and an Adam update (bias correction with the
 * 1-based step t) of params, adam_m and adam_v (21,123 floats each, in/out). */
GPR_API int gpr_mlp_train_step(float* params, float* adam_m, float* adam_v, int t, const float* X, const float* Y,
                               int64_t batch, float lr, float beta1, float beta2, float eps, float* loss, void* ws,
                               size_t ws_bytes, void* stream);

/* The three-way bfloat16 split used by GPR_BF16X3 / GPR_BF16X6 after each panel solve:
 * hi = rne(x), mid = rne(x - hi), lo = rne(x - hi - mid), each a bfloat16 stored as
 * uint16 bits (rne = round to nearest, ties to even; the subtractions are exact in
 * float32, so hi + mid + lo == x for normal x).  x: count float32 (in); hi, mid, lo:
 * count uint16 each (out). */
GPR_API int gpr_split_bf16x3(const float* x, int64_t count, void* hi, void* mid, void* lo, void* stream);

/* Profiling hook: while enabled, every trailing-update launch of gpr_cholesky (the
 * batched SYRK + GEMM of one factorisation step) and every inversion and trace launch of
 * gpr_nlml_grad is bracketed by HIP events on the call's stream.  Host only; not needed
 * for computing anything. */
GPR_API int gpr_timing_enable(int on);

/* Waits for the recorded events of one kind of timed tile-GEMM launch and returns, since
 * the last read of that kind: the number of launches, their summed duration (ms) and
 * their algorithmic flops.  Kinds:
 *   0/1  float64/float32 trailing update of the Cholesky (per step with T' = T-k-1
 *        remaining tiles: T' b^2 (b+1) for the SYRKs plus T'(T'-1) b^3 for the GEMMs;
 *        the float32 kind covers the GEMM tiles only, the diagonal-tile SYRK of the mixed
 *        modes runs as a separate float64 launch);
 *   2/3  bf16x3/bf16x6 trailing update (GEMM tiles only, as kind 1);
 *   4/5  float64/float32 step of the triangular inversion of the gradient (b^2 (b+1) per
 *        triangular tile product, 2 b^3 per full one);
 *   6/7  float64/float32 K^{-1} product fused with the gradient reduction (as kind 4/5
 *        for tile pairs off the diagonal; a diagonal tile pair is symmetric and computed
 *        on and below its diagonal only: b^2 (b+1) from full tiles, b (b+1)(b+2)/3 from
 *        two triangular tiles; all launches of one gradient add up to about n^3 / 3);
 *   8/9  bf16x3/bf16x6 step of the triangular inversion (split modes with tiles a
 *        multiple of 256; the same algorithmic count as kind 4/5, although these launches
 *        multiply the triangular tiles in full);
 *   10/11 bf16x3/bf16x6 K^{-1} product fused with the gradient reduction (as 8/9, the
 *        count of kind 6/7).
 * Resets that kind's record.  All three are host outputs. */
GPR_API int gpr_timing_read(int kind, int64_t* launches, double* total_ms, double* algo_flops);

/* Host model of the device task-graph schedule (GPR_SCHEDULE_DEVICE), host only: builds the
 * graph that gpr_cholesky executes for (n, tile) in float64 (symbolic addresses) and runs
 * the executor's claim / wait / finish code with `threads` host threads in place of
 * workgroups, each item checking that every predecessor task has finished.  A task index
 * withhold >= 0 gets one predecessor more than it has, so its wait can never end: the
 * waits must then give up after limit_ms and every thread return.  withhold <= -2 drops
 * edge number -2 - withhold (in successor-list order) before the checks.  report[0..8] (host
 * array of 9): tasks, items, edges, items run, violations (items that started before a
 * predecessor finished, and items that did not run exactly once; 0 for a correct graph
 * and executor), abort flag, threads that gave up, threads that returned, and pairs of
 * tasks whose byte ranges overlap with one writing but that no path of edges orders (0 for
 * a correct graph; -1 when the graph has over 4096 tasks). */
GPR_API int gpr_dag_check(int64_t n, int64_t tile, int threads, int64_t withhold, double limit_ms, int64_t* report);

/* Task census of the tiled Cholesky with T tiles per dimension as scheduled by this
 * library (Fig. 1): counts[0..3] = POTRF, TRSM, SYRK, GEMM tile tasks.  Host only. */
GPR_API int gpr_cholesky_census(int64_t T, int64_t* counts);

/* Dependency check of the factorisation's two-stream schedule (the task dependencies of
 * Fig. 1 as ordering between launches), host only: runs the same description that
 * gpr_cholesky executes for (n, tile, prec) in a pass that launches nothing, recording the
 * byte ranges each launch reads and writes and the events between the caller's stream
 * and the auxiliary stream, and replays it with vector clocks.  report[0..7] (host array
 * of 8): launches, launches on the caller's stream, on the auxiliary stream, event waits,
 * pairs of launches on different streams ordered in neither direction, such pairs that
 * touch common bytes with at least one writing (a correct schedule has none), launches
 * without access ranges, waits issued before their event was recorded.  omit_event >= 0
 * analyses the schedule as if every wait on that event were missing (event 0: start,
 * 1 + 3k: diagonal tile k+1 updated by step k, 2 + 3k: the rest of block column k+1
 * updated by step k, 3 + 3k: panel k solved); -1 analyses it as issued.
 * Touches no device memory.  Errors: GPR_ERR_ARG (unknown precision tag or NULL report),
 * GPR_ERR_SHAPE. */
GPR_API int gpr_cholesky_schedule_check(int64_t n, int64_t tile, int prec, int64_t omit_event, int64_t* report);

#ifdef __cplusplus
}
#endif
#endif /* GPR_H_ */
