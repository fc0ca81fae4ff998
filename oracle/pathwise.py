"""Pathwise posterior samples and predictive metrics (Sec. 2 and 2.1; Sec. 5.1).

Test infrastructure (see the package docstring).

Pathwise conditioning writes a posterior sample at test inputs X* as a prior sample plus a
data-driven correction: with f a prior function and zeta ~ N(0, lambda I),

    f_post(X*) = f(X*) + k(X*, X) (K + lambda I)^{-1} (y - f(X) - zeta)

(the printed formula writes k_n(X*, X) for the cross-covariance; the prior covariance k is
meant, reading A21 in the design notes).  Solving the k systems with right-hand sides
[y, f_1(X) + zeta_1, ..., f_S(X) + zeta_S] at once gives W = [W_0, W_1, .., W_S], and then
sample s is f_s(X*) + k(X*, X) (W_0 - W_s) while k(X*, X) W_0 is the posterior mean.

Predictive metrics on held-out (X*, y*) (Sec. 5.1 reports test RMSE and the mean negative
log-likelihood from 64 pathwise samples): RMSE of the posterior mean; for the NLL each test
point's predictive density is N(mu, v + lambda) with mu the posterior mean and v the mean
squared deviation of the S samples from mu (the samples are draws around the exact mean, so
this is an unbiased estimate of the posterior variance with S degrees of freedom).
"""
import math

import numpy as np

from . import kernels as kmod


def posterior_samples(X, W, Xstar, prior_star, kind, ell, outputscale=1.0):
    """[posterior mean | S pathwise samples] at Xstar (m x (S + 1)) from the solutions W
    (n x (S + 1)) of the systems with right-hand sides [y, f_s(X) + zeta_s]."""
    W = np.asarray(W, dtype=np.float64)
    Kx = kmod.kernel_matrix(Xstar, X, kind, ell, outputscale=outputscale)
    mean = Kx @ W[:, 0]
    out = np.empty((Kx.shape[0], W.shape[1]))
    out[:, 0] = mean
    for s in range(1, W.shape[1]):
        out[:, s] = np.asarray(prior_star)[:, s - 1] + Kx @ (W[:, 0] - W[:, s])
    return out


def predictive_metrics(samples, ystar, lam):
    """(RMSE of the posterior mean, mean Gaussian negative log-likelihood) on the test set."""
    samples = np.asarray(samples, dtype=np.float64)
    ystar = np.asarray(ystar, dtype=np.float64)
    mu = samples[:, 0]
    rmse = math.sqrt(float(np.mean((mu - ystar) ** 2)))
    S = samples.shape[1] - 1
    v = np.sum((samples[:, 1:] - mu[:, None]) ** 2, axis=1) / S if S > 0 else np.zeros_like(mu)
    var = v + lam
    nll = float(np.mean(0.5 * np.log(2.0 * math.pi * var) + (ystar - mu) ** 2 / (2.0 * var)))
    return rmse, nll
