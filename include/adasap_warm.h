/* Learned warm start for ADASAP (libadasap.so, gfx950).
 *
 * Alg. 2 takes any initial iterate W_0; the posterior mean at the training points is
 * m = K (K + lambda I)^{-1} y = y - lambda W* (Sec. 2), so an estimate m^ of m gives
 * the initial iterate W_0 = (y - m^) / lambda.  This module learns m^ with a small
 * network and is an addition to the paper (which starts from W_0 = 0 in its analysis).
 *
 * Network input of a point x with target value y (a row of D + 2 floats):
 *   [cos(omega_1 . x + c_1), ..., cos(omega_D . x + c_D), y, m_rff(x)]
 * with random Fourier frequencies omega_j (D x d) and phases c_j (D) supplied by the
 * caller, and the ridge mean m_rff = phi^T theta, phi(x) = sqrt(2/D) cos(Omega x + c),
 * theta = (Phi^T Phi + lambda I)^{-1} Phi^T y computed over the problem's own points
 * (Sec. 2.1 uses the same features for pathwise conditioning).
 * Network: dense layers (D+2) -> H -> H -> H -> 1 with SiLU after the hidden layers,
 * trained by Adam on the mean squared error against m = y - lambda W of solved problems.
 * Parameters are one flat float32 vector, layer by layer: W_l (out x in, row-major), b_l.
 *
 * All arrays are device pointers, float32, row-major, owned by the caller unless stated.
 * Calls enqueue on the warm-start object's stream and return after it completes.
 * Errors are status codes (adasap_last_error() holds the message); invalid arguments are
 * rejected before any device work.
 */
#ifndef ADASAP_WARM_H
#define ADASAP_WARM_H

#include "adasap.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adasap_ws_s* adasap_ws_t;

typedef struct {
  uint32_t struct_size; /* sizeof(adasap_ws_config_t) */
  int32_t d;            /* point dimension, 1..64 */
  int32_t D;            /* Fourier features, 1..1024 */
  int32_t hidden;       /* hidden width H, 1..1024 */
  double lambda;        /* noise variance of the systems (K + lambda I) W = y, > 0 */
  double beta1;         /* Adam first-moment decay (0.9) */
  double beta2;         /* Adam second-moment decay (0.999) */
  double adam_eps;      /* Adam denominator offset (1e-8) */
} adasap_ws_config_t;

/* Defaults: d = 9, D = 512, hidden = 256, lambda = 1e-2, Adam (0.9, 0.999, 1e-8). */
adasap_status_t adasap_ws_config_default(adasap_ws_config_t* cfg);

/* Number of network parameters for cfg (0 if cfg is invalid). */
int64_t adasap_ws_param_count(const adasap_ws_config_t* cfg);

/* Creates a warm-start object.  freqs (D x d), phases (D) and params (param_count) are
 * copied; the object owns its copies and its training set.  stream: hipStream_t (may be
 * NULL for the default stream). */
adasap_status_t adasap_ws_create(const adasap_ws_config_t* cfg, const float* freqs,
                                 const float* phases, const float* params, void* stream,
                                 adasap_ws_t* out);

/* Appends a solved problem to the training set: its n points X (n x d), targets y (n) and
 * solution W (n) give n rows of network input (with the ridge mean of this problem) and
 * the labels m = y - lambda W. */
adasap_status_t adasap_ws_add_problem(adasap_ws_t ws, int64_t n, const float* X, const float* y,
                                      const float* W);

/* Rows in the training set. */
int64_t adasap_ws_train_rows(adasap_ws_t ws);

/* Minibatch Adam over the training set: epoch e visits the rows in the permutation drawn
 * by Fisher-Yates from the Philox stream (seed, 11, e), in batches of `batch` rows (the
 * last may be shorter); lr is Adam's step size.  epoch_loss (host, epochs entries, may be
 * NULL) receives each epoch's mean squared error averaged over its batches by row count.
 * Adam's moments persist across calls. */
adasap_status_t adasap_ws_train(adasap_ws_t ws, int32_t epochs, int32_t batch, double lr,
                                uint64_t seed, double* epoch_loss);

/* Network inputs of n points (out: n x (D + 2)) and, if theta != NULL, the ridge weights
 * theta (D, float64 device). */
adasap_status_t adasap_ws_features(adasap_ws_t ws, int64_t n, const float* X, const float* y,
                                   float* out, double* theta);

/* Loss (host double, may be NULL) and gradient (device, param_count) of the mean squared
 * error of the current network on m rows of inputs A (m x (D + 2)) with targets t (m). */
adasap_status_t adasap_ws_loss_grad(adasap_ws_t ws, int64_t m, const float* A, const float* t,
                                    double* loss, float* grad);

/* Network prediction m^ (n) for a problem's points X (n x d) and targets y (n); the ridge
 * mean is computed over these n points.  Streams the rows in chunks (no n x D array). */
adasap_status_t adasap_ws_predict_mean(adasap_ws_t ws, int64_t n, const float* X, const float* y,
                                       float* mhat);

/* The warm start W0 = (y - m^) / lambda (n) for a problem's points X and targets y. */
adasap_status_t adasap_ws_initial_iterate(adasap_ws_t ws, int64_t n, const float* X,
                                          const float* y, float* W0);

/* Copies the parameters out (device, param_count) or in (resets nothing else). */
adasap_status_t adasap_ws_get_params(adasap_ws_t ws, float* out);
adasap_status_t adasap_ws_set_params(adasap_ws_t ws, const float* in);

void adasap_ws_destroy(adasap_ws_t ws);

#ifdef __cplusplus
}
#endif

#endif /* ADASAP_WARM_H */
