"""Pins for the pathwise-conditioning oracle: with exact joint prior draws and exact solves,
pathwise samples have the closed-form GP posterior mean and covariance (Sec. 2, Eq. post_eqns);
the metrics against scipy's normal log-density."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import kernels as K
from oracle import linsys
from oracle import pathwise as PW


def test_pathwise_samples_have_the_posterior_mean_and_covariance():
    rs = np.random.default_rng(0)
    n, m, d, lam, ell, S = 40, 4, 2, 0.05, 0.8, 40000
    X = rs.standard_normal((n, d))
    Xs = rs.standard_normal((m, d))
    y = np.sin(X).sum(axis=1) + 0.2 * rs.standard_normal(n)
    # exact prior draws of f at X and X* jointly, plus zeta ~ N(0, lambda I)
    Xall = np.vstack([X, Xs])
    Kall = K.kernel_matrix(Xall, Xall, K.RBF, ell) + 1e-10 * np.eye(n + m)
    L = np.linalg.cholesky(Kall)
    F = L @ rs.standard_normal((n + m, S))
    zeta = math.sqrt(lam) * rs.standard_normal((n, S))
    Y = np.hstack([y[:, None], F[:n] + zeta])
    W = linsys.direct_solve(X, Y, K.RBF, ell, lam)
    out = PW.posterior_samples(X, W, Xs, F[n:], K.RBF, ell)
    # closed forms of Eq. post_eqns
    Kl = K.kernel_matrix(X, X, K.RBF, ell) + lam * np.eye(n)
    Ksx = K.kernel_matrix(Xs, X, K.RBF, ell)
    mean = Ksx @ np.linalg.solve(Kl, y)
    cov = K.kernel_matrix(Xs, Xs, K.RBF, ell) - Ksx @ np.linalg.solve(Kl, Ksx.T)
    assert np.allclose(out[:, 0], mean, rtol=1e-9, atol=1e-12)
    smp = out[:, 1:]
    se = np.sqrt(np.diag(cov) / S)
    assert np.all(np.abs(smp.mean(axis=1) - mean) <= 5 * se)
    emp = np.cov(smp)
    assert np.allclose(emp, cov, atol=0.05 * np.max(np.diag(cov)))
    # a plausible slip, the posterior covariance k_n in place of k in the correction, shows up
    bad_cov = np.cov(F[n:] + (Ksx - Ksx @ np.linalg.solve(Kl, K.kernel_matrix(X, X, K.RBF, ell)))
                     @ (W[:, :1] - W[:, 1:]))
    assert not np.allclose(bad_cov, cov, atol=0.05 * np.max(np.diag(cov)))


def test_predictive_metrics_match_scipy():
    rs = np.random.default_rng(1)
    m, S, lam = 300, 7, 0.03
    samples = rs.standard_normal((m, S + 1))
    ystar = rs.standard_normal(m)
    rmse, nll = PW.predictive_metrics(samples, ystar, lam)
    mu = samples[:, 0]
    v = np.mean((samples[:, 1:] - mu[:, None]) ** 2, axis=1) + lam
    assert rmse == pytest.approx(np.sqrt(np.mean((mu - ystar) ** 2)), rel=1e-14)
    assert nll == pytest.approx(-np.mean(norm.logpdf(ystar, loc=mu, scale=np.sqrt(v))), rel=1e-12)
