"""Random Fourier features and the RFF ridge mean, float64 (test infrastructure).

Random Fourier features approximate a stationary kernel by a finite cosine
expansion (the construction Sec. 2.1 uses for pathwise conditioning):
phi(x) = sqrt(2/D) cos(Omega x + c), with the rows of Omega drawn from the
kernel's spectral measure and c uniform on [0, 2 pi), so that
E[phi(x)^T phi(x')] = k(x, x').  The frequencies and phases are random draws
of the method and are passed in.

The warm-start network sees the unit-scale cosines cos(Omega x + c) (phi
without its sqrt(2/D) factor), the target y and the RFF ridge mean
m_rff = Phi theta, theta = (Phi^T Phi + lambda I)^{-1} Phi^T y: the posterior
mean of the finite-feature GP with noise variance lambda.
"""
import numpy as np


def cosines(X, freqs, phases):
    """cos(x_i . omega_j + c_j) as an (n x D) array."""
    X = np.asarray(X, dtype=np.float64)
    return np.cos(X @ np.asarray(freqs, dtype=np.float64).T + np.asarray(phases, dtype=np.float64))


def features(X, freqs, phases):
    """phi(x_i)_j = sqrt(2/D) cos(x_i . omega_j + c_j)."""
    D = np.asarray(phases).shape[0]
    return np.sqrt(2.0 / D) * cosines(X, freqs, phases)


def ridge_weights(X, y, freqs, phases, lam):
    """theta = (Phi^T Phi + lam I)^{-1} Phi^T y (normal equations, Cholesky)."""
    Phi = features(X, freqs, phases)
    D = Phi.shape[1]
    A = Phi.T @ Phi + lam * np.eye(D)
    L = np.linalg.cholesky(A)
    z = np.linalg.solve(L, Phi.T @ np.asarray(y, dtype=np.float64))
    return np.linalg.solve(L.T, z)


def ridge_mean(X, y, freqs, phases, lam):
    """m_rff(x_i) = phi(x_i)^T theta at the training points."""
    theta = ridge_weights(X, y, freqs, phases, lam)
    return features(X, freqs, phases) @ theta, theta


def network_inputs(X, y, freqs, phases, lam):
    """[cos(Omega x_i + c) | y_i | m_rff(x_i)], the (n x (D + 2)) input of the network."""
    m, _ = ridge_mean(X, y, freqs, phases, lam)
    return np.concatenate([cosines(X, freqs, phases), np.asarray(y, dtype=np.float64)[:, None],
                           m[:, None]], axis=1)
