"""Direct solve, residual and posterior mean for (K + lambda I) W = Y (Sec. 2, Eq. post_eqns).

Test infrastructure (see the package docstring).

* W* = (K + lambda I)^{-1} Y is the unique solution (K + lambda I is SPD).
* The posterior mean at the training inputs with zero prior mean is
  m_n(X) = k(X, X) W* = Y - lambda W* (Eq. post_eqns), and at new inputs
  m_n(X*) = k(X*, X) W.
* Relative residual ||(K + lambda I) W - Y||_F / ||Y||_F (the certificate;
  for several right-hand sides the Frobenius norm, and the per-column
  maximum is also reported).
"""
import numpy as np

from . import kernels as kmod


def cholesky_lower(A):
    """Lower factor L with A = L L^T by the textbook row recurrence (no library call)."""
    n = A.shape[0]
    L = np.zeros_like(A, dtype=np.float64)
    for i in range(n):
        s = A[i, i] - L[i, :i] @ L[i, :i]
        if not s > 0:
            raise np.linalg.LinAlgError("not positive definite at %d" % i)
        L[i, i] = np.sqrt(s)
        if i + 1 < n:
            L[i + 1:, i] = (A[i + 1:, i] - L[i + 1:, :i] @ L[i, :i]) / L[i, i]
    return L


def forward_subst(L, B):
    """Solve L X = B for lower-triangular L, row by row."""
    X = np.zeros_like(B, dtype=np.float64)
    for i in range(L.shape[0]):
        X[i] = (B[i] - L[i, :i] @ X[:i]) / L[i, i]
    return X


def backward_subst(U, B):
    """Solve U X = B for upper-triangular U, row by row from the bottom."""
    n = U.shape[0]
    X = np.zeros_like(B, dtype=np.float64)
    for i in range(n - 1, -1, -1):
        X[i] = (B[i] - U[i, i + 1:] @ X[i + 1:]) / U[i, i]
    return X


def direct_solve(X, Y, kind, ell, lam, outputscale=1.0):
    """W* = (K + lambda I)^{-1} Y with the oracle's own Cholesky and substitutions."""
    K = kmod.kernel_matrix(X, X, kind, ell, outputscale=outputscale)
    A = K + lam * np.eye(K.shape[0])
    L = cholesky_lower(A)
    return backward_subst(L.T, forward_subst(L, np.asarray(Y, dtype=np.float64)))


def residual(X, Y, W, kind, ell, lam, outputscale=1.0):
    """R = K W + lambda W - Y."""
    W = np.asarray(W, dtype=np.float64)
    return (kmod.kernel_matmul(X, X, W, kind, ell, outputscale=outputscale) + lam * W
            - np.asarray(Y, dtype=np.float64))


def relres(X, Y, W, kind, ell, lam, outputscale=1.0):
    """(||R||_F / ||Y||_F, max over columns of ||R_c|| / ||Y_c||)."""
    R = residual(X, Y, W, kind, ell, lam, outputscale)
    Y = np.asarray(Y, dtype=np.float64)
    fro = np.linalg.norm(R) / np.linalg.norm(Y)
    if R.ndim == 1:
        return fro, fro
    cols = np.linalg.norm(R, axis=0) / np.linalg.norm(Y, axis=0)
    return fro, float(cols.max())


def residual_rows(X, Y, W, kind, ell, lam, rows, outputscale=1.0):
    """Rows `rows` of the residual, computed one row at a time against all n columns."""
    W = np.asarray(W, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    rows = np.asarray(rows)
    return (kmod.kernel_matmul(X[rows], X, W, kind, ell, outputscale=outputscale) + lam * W[rows]
            - Y[rows])


def predict(Xstar, X, W, kind, ell, outputscale=1.0):
    """Posterior mean m(X*) = k(X*, X) W (zero prior mean)."""
    return kmod.kernel_matmul(Xstar, X, W, kind, ell, outputscale=outputscale)
