/*
 * adasap.h -- C ABI of the MI355X (gfx950) ADASAP hot path.
 *
 * Solves (K + lambda I) W = Y for a Gaussian-process kernel matrix K = k(X, X)
 * with ADASAP: approximate, accelerated sketch-and-project ("Turbocharging
 * Gaussian Process Inference with Approximate Sketch-and-Project", Sec. 4,
 * Alg. 2).  Every iteration samples a row block B, evaluates the kernel row
 * block K_{B,:} on the fly against the current iterate, builds a randomized
 * Nystrom preconditioner of K_BB + rho I (Appendix, Alg. NysApprox), picks the
 * step size by randomized powering (Appendix, Alg. GetStepsize) and takes the
 * Nesterov-accelerated projected step (Appendix, Alg. NestAcc).
 *
 * Conventions shared by every entry point:
 *  - Matrices are row-major and contiguous.  X is n x d, Y and W are n x k.
 *  - Pointers documented as "device" must point to memory of the current HIP
 *    device (for example torch tensors' data_ptr()); "host" pointers to host
 *    memory.  The caller owns every buffer it passes in.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls that return
 *    numbers to the host synchronise that stream before returning.
 *  - Errors are reported by status code only; no call aborts or throws.  The
 *    message of the last failure on the calling thread is returned by
 *    adasap_last_error().  Invalid arguments are rejected before any device
 *    work, and output buffers are then left untouched.
 *  - Results are deterministic: the same inputs, configuration and seed give
 *    bit-identical outputs on the same device (no floating-point atomics).
 */
#ifndef ADASAP_H
#define ADASAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADASAP_OK = 0,
  ADASAP_ERR_INVALID_ARG = 1,   /* argument out of range, null pointer, bad config */
  ADASAP_ERR_OOM = 2,           /* device or host allocation failed */
  ADASAP_ERR_DEVICE = 3,        /* a HIP runtime call failed */
  ADASAP_ERR_NOT_PD = 4,        /* Nystrom core not positive definite after shift retries */
  ADASAP_ERR_NONFINITE = 5,     /* NaN/Inf in inputs or iterates */
  ADASAP_ERR_UNSUPPORTED = 6,   /* valid request this build does not implement */
  ADASAP_ERR_NOT_CONVERGED = 7  /* tol > 0 and the last checked relative residual is above it;
                                   W holds the returned iterate and the report is filled */
} adasap_status_t;

/* Covariance functions (textbook forms; the paper names RBF and Matern kernels, Sec. 5):
 * RBF exp(-r^2/(2 ell^2)); Matern-1/2 exp(-r/ell); Matern-3/2 (1+a)e^{-a}, a = sqrt(3) r/ell;
 * Matern-5/2 (1+a+a^2/3)e^{-a}, a = sqrt(5) r/ell.  With one lengthscale per coordinate (the
 * fitted hyperparameters of the paper's regression experiments, appendix) the distance is
 * r^2 = sum_j ((x_j - x'_j)/ell_j)^2 and the forms are taken at ell = 1.  An output scale s
 * multiplies the kernel: K = s k(X, X). */
typedef enum { ADASAP_RBF = 0, ADASAP_MATERN12 = 1, ADASAP_MATERN32 = 2, ADASAP_MATERN52 = 3 } adasap_kernel_t;

/* Arithmetic of the kernel-block products.
 * FP64:  everything in float64.
 * FP32:  kernel values and their products in float32 (sketch eps = 2^-23); the
 *        Nystrom core, Woodbury applies, step size and residual norms in float64.
 * MIXED: squared distances from a three-term float16 split on matrix cores with
 *        float32 accumulation, kernel values rounded to float16 and multiplied
 *        with a float16 copy of the iterate on matrix cores (float32 accumulation);
 *        the rest as FP32; optional float64 refinement sweeps. */
typedef enum { ADASAP_FP64 = 0, ADASAP_FP32 = 1, ADASAP_MIXED = 2 } adasap_precision_t;

/* Preconditioner of the block step.  NYSTROM is ADASAP (P_B = U S U^T + rho I);
 * IDENTITY is ADASAP-I (Sec. 5, P_B = I, step size from powering on K_BB + lambda I);
 * EXACT is the exact block projection of SAP (Sec. 3, Alg. 1): P_B = K_BB + lambda I, formed
 * and Cholesky-factored in float64 (b <= 16384, b x b float64 of workspace), step size 1 (the
 * preconditioned block operator is the identity); with accel = 0 this is Alg. 1 itself, with
 * accel = 1 the Nesterov step of Alg. 2 around it.  EXACT takes FP64 or FP32 precision: the
 * unit step amplifies the float16 error of MIXED block gradients by up to 1/lambda, so MIXED
 * is rejected (ADASAP_ERR_INVALID_ARG). */
typedef enum { ADASAP_PRECOND_NYSTROM = 0, ADASAP_PRECOND_IDENTITY = 1,
               ADASAP_PRECOND_EXACT = 2 } adasap_precond_t;

/* Element type of X, Y, W, Xstar and prediction outputs. */
typedef enum { ADASAP_DTYPE_F32 = 0, ADASAP_DTYPE_F64 = 1 } adasap_dtype_t;

typedef struct {
  uint32_t struct_size;   /* sizeof(adasap_config_t) */
  int32_t kernel;         /* adasap_kernel_t */
  double lengthscale;     /* ell > 0 */
  double lambda;          /* likelihood variance lambda > 0 */
  int64_t block_size;     /* b, 0 < b <= n (Alg. 2 "blocksize") */
  int32_t rank;           /* r, 0 < r <= min(b, 128) (Nystrom rank) */
  int32_t rho_rule;       /* 0: rho = lambda + S_rr (Alg. 2); 1: rho = `rho` below */
  double rho;             /* damping for rho_rule 1, > 0 */
  double mu, nu;          /* acceleration parameters; <= 0 selects lambda and n/b (Sec. 4.2) */
  int32_t power_iters;    /* randomized powering applications (Alg. GetStepsize), default 10 */
  int64_t max_iters;      /* iterations of the solve (per refinement sweep) */
  double tol;             /* stop when the checked relative residual <= tol (0: never check) */
  int64_t check_every;    /* iterations between residual checks (0: only at the end) */
  int32_t refine_sweeps;  /* extra float64 iterative-refinement sweeps after the first solve */
  int32_t precond;        /* adasap_precond_t */
  int32_t precision;      /* adasap_precision_t */
  uint64_t seed;          /* key of every random draw (block, sketch, powering start) */
  int32_t accel;          /* 1: Nesterov step (Alg. NestAcc); 0: W <- W - eta I_B^T D */
  int32_t grad_at_z;      /* 1: block gradient at Z_t (reading of Alg. 2 Step IV); 0: at W_t */
  int32_t z_uses_v_next;  /* 1: Z_{t+1} = alpha V_{t+1} + (1-alpha) W_{t+1}; 0: uses V_t */
  int32_t tail_average;   /* 1: return the mean of W_j, j = floor(T/2) .. T-1 */
  int32_t n_lengthscale;  /* 0 or 1: the scalar `lengthscale`; d: per-coordinate lengthscales */
  const double* lengthscales; /* host, d entries > 0 when n_lengthscale == d (copied by
                                 adasap_create; unused otherwise, may be NULL) */
  double outputscale;     /* s > 0: K = s k(X, X) (default 1) */
  int64_t check_rows;     /* residual checks of a solve: 0 = all n rows; m > 0 = the
                             row-subsampled estimate of adasap_residual_rows on min(m, n) rows
                             (rows drawn with the configuration's seed) */
} adasap_config_t;

typedef struct {
  int64_t iters;           /* iterations run (all sweeps) */
  double relres;           /* last checked ||(K+lambda I)W - Y||_F / ||Y||_F (float64 accumulation), -1 if unchecked */
  double relres_maxcol;    /* same, maximum over the k columns */
  double solve_ms;         /* device time of the iterations (excludes residual checks) */
  double check_ms;         /* device time of the residual checks */
  double eta_last, rho_last, lambda_hat_last, delta_last;
  int32_t refine_done;     /* refinement sweeps performed */
  int32_t not_pd_events;   /* Nystrom cores that needed a shift increase */
  int32_t status;          /* adasap_status_t of the solve */
  double step1_kernel_ms;  /* device time of the step-I kernel-block product kernels (matrix-core path) */
  int64_t step1_launches;  /* number of those launches (batched solves: the rounds run eagerly) */
  int32_t jacobi_sweeps_max; /* most sweeps one Nystrom eigendecomposition needed */
  int32_t reserved;        /* batched solves: column tiles per work item chosen by the autotuner */
  int32_t tuned_rows_per_wg; /* batched solves: rows of X_B per workgroup (128 or 256) chosen by the autotuner */
  int32_t tuned_wg_per_cu;   /* batched solves: persistent workgroups per CU (2 or 4) chosen by the autotuner */
  int32_t tuned_from_cache;  /* batched solves: 1 if the choice came from this process's tuning cache */
} adasap_report_t;

typedef struct adasap_handle_s* adasap_handle_t;

/* Fills `cfg` with the paper's defaults (RBF, rho rule 0, mu = lambda, nu = n/b,
 * 10 power iterations, Nystrom preconditioner, Nesterov on, FP32). */
adasap_status_t adasap_config_default(adasap_config_t* cfg);

/* Creates a solver for (K + lambda I) W = Y (Sec. 2: the linear system behind the posterior
 * mean and pathwise samples), K = outputscale * k(X, X).  X (n x d) and Y (n x k) are device
 * pointers of element type `dtype`; the handle borrows them (they must stay alive
 * and unchanged until adasap_destroy) and allocates its own device workspace
 * (adasap_workspace_bytes); with per-coordinate lengthscales that includes a float64 copy
 * of X with coordinate j divided by ell_j, on which every kernel value is then computed.
 * Requires 1 <= d <= 64 (d <= 16 for MIXED), 1 <= k <= 128.
 * On success *out receives the handle. */
adasap_status_t adasap_create(const adasap_config_t* cfg, int64_t n, int32_t d, int32_t k,
                              const void* X, const void* Y, int32_t dtype, void* stream,
                              adasap_handle_t* out);

/* Device bytes adasap_create would allocate for this problem (0 on invalid input). */
int64_t adasap_workspace_bytes(const adasap_config_t* cfg, int64_t n, int32_t d, int32_t k);

/* Runs the solve: ADASAP (Sec. 4, Alg. 2) for max_iters iterations, each sampling B_t,
 * forming the block gradient at the extrapolated point Z_t, the Nystrom preconditioner of
 * K_BB + rho I (Alg. NysApprox), the step size by powering (Alg. GetStepsize) and the
 * Nesterov step (Alg. NestAcc); then `refine_sweeps` float64 refinement sweeps.  W (device,
 * n x k, handle dtype) holds W_0 on entry (zeros = cold start; V_0 = Z_0 = W_0) and the
 * returned iterate on exit.  With tol > 0 the relative residual is checked every
 * check_every iterations and at the end, and the solve stops at the first check <= tol;
 * if the last check is above tol the status is ADASAP_ERR_NOT_CONVERGED (W and the report
 * are still filled).  `report` (host, may be NULL) receives statistics.  Synchronises the
 * stream. */
adasap_status_t adasap_solve(adasap_handle_t h, void* W, adasap_report_t* report);

/* Continues the last adasap_solve of this handle for `iters` more iterations of the same
 * run: the iteration counter, the random streams (B_t, Omega_t, v_t for t = T, T + 1, ...)
 * and the Nesterov state (V_T, Z_T, kept by the handle) carry on, so a solve of T1
 * iterations continued by T2 equals one solve of T1 + T2 iterations bit for bit (residual
 * checks change nothing).  tol and check_every apply as in adasap_solve, counted from the
 * continuation.  W (device, n x k) receives W_{T + iters}.  Requires a preceding solve
 * without refinement sweeps and without tail averaging, and iters >= 1;
 * ADASAP_ERR_INVALID_ARG otherwise (nothing is run).  `report` covers the continuation;
 * its `iters` counts the iterations of this call.  Synchronises the stream. */
adasap_status_t adasap_solve_more(adasap_handle_t h, void* W, int64_t iters,
                                  adasap_report_t* report);

/* Posterior mean m(X*) = k(X*, X) W (Sec. 2, Eq. post_eqns, zero prior mean).
 * W (device, n x k), Xstar (device, m x d), out (device, m x k), all handle dtype. */
adasap_status_t adasap_predict(adasap_handle_t h, const void* W, int64_t m, const void* Xstar,
                               void* out);

/* Pathwise posterior samples (Sec. 2.1, pathwise conditioning): a posterior sample at X* is
 * f(X*) + k(X*, X)(K + lambda I)^{-1}(y - f(X) - zeta) for a prior function f and
 * zeta ~ N(0, lambda I).  W (device, n x k, handle dtype) must solve the handle's systems for
 * the right-hand sides Y = [y | f_1(X) + zeta_1 | ... | f_{k-1}(X) + zeta_{k-1}] (column 0
 * the observations, column s a prior function plus noise); prior_star (device, m x (k - 1),
 * handle dtype, may be NULL when k = 1) holds f_s(X*).  out (device, m x k, handle dtype)
 * receives the posterior mean k(X*, X) W_0 in column 0 and sample s,
 * f_s(X*) + k(X*, X)(W_0 - W_s), in column s; the products run as in adasap_predict.
 * Synchronises the stream. */
adasap_status_t adasap_posterior_samples(adasap_handle_t h, const void* W, int64_t m,
                                         const void* Xstar, const void* prior_star, void* out);

/* Predictive metrics on held-out data (Sec. 5.1: test RMSE and mean negative log-likelihood
 * from pathwise samples).  samples (device, m x k, dtype): posterior mean in column 0 and
 * k - 1 samples, as written by adasap_posterior_samples; ystar (device, m, dtype): the
 * held-out targets.  rmse = sqrt(mean_i (mu_i - y*_i)^2); nll = mean_i of the negative log
 * density of y*_i under N(mu_i, v_i + lambda), v_i the mean squared deviation of the samples
 * from mu_i (v_i = 0 when k = 1).  float64 accumulation, fixed order; host outputs, may be
 * NULL.  Synchronises the stream. */
adasap_status_t adasap_predictive_metrics(int64_t m, int32_t k, const void* samples,
                                          const void* ystar, double lambda, int32_t dtype,
                                          void* stream, double* rmse, double* nll);

/* Acquisition step of parallel Thompson sampling (Sec. 5.3 Bayesian optimisation: each
 * acquired point maximises one posterior sample over candidate points): for each of the k
 * columns of a (device, m x k with row stride ld >= k, dtype), the index of its largest entry
 * (the first such row on ties; NaN entries never win; -1 if a column has no comparable
 * entry).  out: device int64[k].  Synchronises the stream. */
adasap_status_t adasap_column_argmax(int64_t m, int32_t k, int64_t ld, const void* a,
                                     int32_t dtype, void* stream, int64_t* out);

/* Relative residual ||(K + lambda I) W - Y||_F / ||Y||_F with float64 accumulation
 * (relres) and its maximum over columns (relres_maxcol); host outputs, may be NULL. */
adasap_status_t adasap_residual(adasap_handle_t h, const void* W, double* relres,
                                double* relres_maxcol);

/* Row-subsampled estimate of the relative residual, for problems where the full product
 * (n^2 pairs) is too large: m rows S, a uniform m-subset of [0, n) (Floyd, Philox stream
 * (seed, 12, 0), ascending), give sqrt(sum_{i in S} |r_i|^2 / sum_{i in S} |y_i|^2) with
 * r = (K + lambda I) W - Y, each row computed against all n columns with the residual's
 * kernels (float16 hi/lo products or float64) and float64 sums.  relres, relres_maxcol
 * (host) may be NULL; rows_out (device int64[m]) may be NULL.  Synchronises the stream. */
adasap_status_t adasap_residual_rows(adasap_handle_t h, const void* W, int64_t m, uint64_t seed,
                                     double* relres, double* relres_maxcol, int64_t* rows_out);

/* Certificate of a reduced-precision solve (Sec. 2: the system whose solution gives the
 * posterior mean; residual in float64): the row-subsampled relative residual of
 * adasap_residual_rows (same rows for the same seed), with every kernel value and product
 * in float64 on the vector ALUs whatever the handle's precision (the coordinates are the
 * handle's X, in its dtype, converted exactly to float64).  rel_se (host, may be NULL)
 * receives the standard error of the estimate relative to it: the ratio estimator
 * sum_S a_i / sum_S c_i (a_i = |r_i|^2, c_i = |y_i|^2) has variance (1 - m/n) s^2 / (m cbar^2)
 * with s^2 the sample variance of a_i - Rhat c_i, and the square root halves the relative
 * error.  Synchronises the stream. */
adasap_status_t adasap_residual_rows_f64(adasap_handle_t h, const void* W, int64_t m,
                                         uint64_t seed, double* relres, double* relres_maxcol,
                                         double* rel_se, int64_t* rows_out);

/* The block gradient of Step I of Alg. 2 at a caller-given point:
 * G = K(X_B, X) Z + lambda Z[B] - Y[B], where B = B_t is the block adasap_solve samples at
 * iteration t (sorted, from the handle's seed), computed with the same kernels, precision
 * and launch as the solver's own Step I.  Z (device, n x k, handle dtype) is read only;
 * G_out (device, b x k, float64) and, if non-NULL, B_out (device, b int64) are written.
 * Returns after the stream completes. */
adasap_status_t adasap_block_gradient(adasap_handle_t h, int64_t t, const void* Z, int64_t* B_out,
                                      double* G_out);

/* Per-iteration step sizes eta_t, dampings rho_t and Rayleigh quotients of the last
 * solve, copied to host arrays of length `count` (entries beyond the run are left). */
adasap_status_t adasap_get_trace(adasap_handle_t h, double* eta, double* rho, double* lambda_hat,
                                 int64_t count);

void adasap_destroy(adasap_handle_t h);

/* One problem of a batch: X (device, n x d), Y (device, n x k), W (device, n x k: W_0 on
 * entry, the solution on exit), all of the batch's dtype, and the problem's lengthscale. */
typedef struct {
  int64_t n;
  int32_t d;
  int32_t k;
  const void* X;
  const void* Y;
  void* W;
  double lengthscale;
} adasap_problem_t;

/* Solves `count` independent systems (K_p + lambda I) W_p = Y_p of uneven size together:
 * every iteration advances all problems with batched launches (one persistent work-queue
 * launch for all step-I kernel-block products).  The configuration is shared (kernel,
 * lambda, block size b, rank, iterations, seed: problem p draws with seed + p); its
 * lengthscale is replaced by each problem's own.  Requirements: FP32 precision, Nystrom
 * preconditioner, accelerated steps with the gradient at Z, k = 1, 1 <= d <= 16 and n >= b
 * for every problem.  When tol > 0 or check_every > 0 each problem's final relative residual
 * is computed.  `reports` (host, count entries, may be NULL) receives per-problem statistics.
 * Execution: the host draws round t + 1's blocks while the device runs round t; the first
 * round times the step-I launch for every tile shape (128 or 256 rows per workgroup), 2 or 4
 * persistent workgroups per CU and work items of 16, 32, 64 or 128 column tiles, and keeps
 * the fastest (a process-wide cache keyed by device, kernel, b and the problems' tile counts
 * and dimensions skips the timing for a batch of the same shapes); every round but the first
 * and the last replays one captured hipGraph of the round's device work (the iteration
 * counter reaches it through device memory).
 * Synchronises the stream. */
adasap_status_t adasap_solve_batch(const adasap_problem_t* probs, int32_t count,
                                   const adasap_config_t* cfg, int32_t dtype, void* stream,
                                   adasap_report_t* reports);

/* ---- single steps of the iteration, for parity checks of each step --------------- */

/* Row block B_t of Alg. 2 Step I: a uniform b-subset of [0, n) without replacement,
 * ascending, drawn with Floyd's algorithm from the Philox4x64-10 stream
 * (seed, purpose, t) and Lemire bounded integers.  out: host int64[b]. */
adasap_status_t adasap_sample_block(uint64_t seed, uint64_t purpose, uint64_t t, int64_t n,
                                    int64_t b, int64_t* out);

/* Standard normals number 0 .. count-1 of stream (seed, purpose, t) (Box-Muller,
 * cosine branch; the Omega and powering draws of Alg. 2).  out: device double[count]. */
adasap_status_t adasap_normals(uint64_t seed, uint64_t purpose, uint64_t t, int64_t count,
                               double* out, void* stream);

/* Kernel block product OUT = k(Xr, Xc) R (Alg. 2 Step I/II column- and row-block
 * oracles).  Xr (m x d), Xc (n x d), R (n x k) and OUT (m x k) are device arrays of
 * element type `dtype`; `precision` selects the arithmetic as for the solver.
 * Synchronises the stream. */
adasap_status_t adasap_kblock_matmul(int32_t kernel, double lengthscale, int32_t precision,
                                     int64_t m, int64_t n, int32_t d, int32_t k, const void* Xr,
                                     const void* Xc, const void* R, void* out, int32_t dtype,
                                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): adasap_kblock_matmul in FP64 or FP32
 * precision with no allocation of any kind.  Arguments and results are those of
 * adasap_kblock_matmul (MIXED is rejected with ADASAP_ERR_INVALID_ARG).  The split partial
 * sums of the product live in a fixed 32 MiB device array of the library (each GPU the
 * library runs on holds its own copy until the process ends), so m * k * (8 for FP64, 4 for
 * FP32) must not exceed 32 MiB (ADASAP_ERR_INVALID_ARG otherwise, before any device work).
 * Every call on one GPU shares that array: calls that overlap in time on one GPU (on
 * different streams or host threads) race and must be serialised by the caller; calls in
 * order on one stream are safe.  Unlike adasap_kblock_matmul the call only enqueues the
 * work on `stream` and returns without synchronising. */
adasap_status_t adasap_kblock_matmul_noalloc(int32_t kernel, double lengthscale, int32_t precision,
                                             int64_t m, int64_t n, int32_t d, int32_t k,
                                             const void* Xr, const void* Xc, const void* R,
                                             void* out, int32_t dtype, void* stream);

/* Instruction rates of the current device, for the rooflines of a measurement (not a step
 * of the method): register-only loops of v_exp_f32, of v_fma_f32 and of float16 32x32x16
 * MFMAs (four independent accumulators per wave) over 2048 workgroups of 256 threads,
 * one warm-up and one timed launch each (about 30 ms in all).  out (host, 3 doubles):
 * [0] ns per v_exp_f32 wave instruction per SIMD, [1] ns per v_fma_f32 wave instruction
 * per SIMD, [2] TFLOP/s of the 32x32x16 MFMAs over the device.  Allocates a 2 MiB
 * scratch buffer; synchronises the stream. */
adasap_status_t adasap_probe_rates(void* stream, double* out);

/* Randomized Nystrom factors of a b x b PSD matrix from its sketch (Appendix,
 * Alg. NysApprox): Ysk = M Omega and Omega (device, b x r, float64).  Outputs
 * (device, float64): U (b x r, orthonormal columns), S (r, descending, >= 0) and
 * the shift actually used (delta, device double[1]).  eps is the machine epsilon
 * of the precision the sketch was computed in.  Synchronises the stream. */
adasap_status_t adasap_nystrom(int64_t b, int32_t r, const double* Ysk, const double* Omega,
                               double eps, double* U, double* S, double* delta, void* stream);

/* Woodbury applies with P = U diag(S) U^T + rho I (Eq. inv_nys_woodbury and
 * Eq. inv_sqrt_nys_woodbury): OUT = P^{-1} G (power = 0) or P^{-1/2} G (power = 1).
 * U (b x r), S (r), G and OUT (b x k): device float64.  Synchronises the stream. */
adasap_status_t adasap_precond_apply(int64_t b, int32_t r, int32_t k, const double* U,
                                     const double* S, double rho, int32_t power, const double* G,
                                     double* out, void* stream);

const char* adasap_last_error(void);
const char* adasap_status_string(adasap_status_t s);

#ifdef __cplusplus
}
#endif

#endif /* ADASAP_H */
