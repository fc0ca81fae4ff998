"""Randomized Nystrom approximation and Woodbury applies (Appendix, "Randomized Nystrom approximation").

Test infrastructure (see the package docstring).

What is computed (Alg. NysApprox, in the consistent form of Tropp et al. 2017, reading A5):
given a PSD matrix M seen only through its sketch M Omega with a Gaussian test matrix
Omega, the rank-r Nystrom approximation M_hat = (M Omega)(Omega^T M Omega)^+(M Omega)^T is
returned in eigen form U diag(S) U^T.  For numerical safety the sketch is first moved to
that of M + Delta I, with Delta a machine-epsilon multiple of tr(Omega^T M Omega) (epsilon of
the precision the sketch was formed in: 2**-52 for float64, 2**-23 for float32); the core
Omega^T (M + Delta I) Omega is factored by Cholesky, the shifted sketch is multiplied by the
inverse of that factor, and the squared singular values of the result, less Delta and
clipped at zero, are the eigenvalues S (the printed listing forms the triangular solve from
the unshifted sketch and writes S^2 where the squared singular values are meant).  When the
Cholesky factorisation fails, Delta grows tenfold and the step is repeated, at most 5 times
(a case the paper does not discuss).

The preconditioner P = U diag(S) U^T + rho I is inverted through the Woodbury identity
(Eq. inv_nys_woodbury and Eq. inv_sqrt_nys_woodbury): on range(U) P acts as S + rho, on its
orthogonal complement as rho, so P^{-1} and P^{-1/2} scale the two components by
(S + rho)^{-1} (or ^{-1/2}) and rho^{-1} (or ^{-1/2}).
"""
import numpy as np

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23


class NotPositiveDefinite(RuntimeError):
    pass


def _cholesky_upper(C):
    """Upper factor R with C = R^T R, by the textbook column recurrence (no library call)."""
    r = C.shape[0]
    R = np.zeros_like(C)
    for j in range(r):
        s = C[j, j] - np.dot(R[:j, j], R[:j, j])
        if not s > 0.0:
            raise NotPositiveDefinite("pivot %d = %r" % (j, s))
        R[j, j] = np.sqrt(s)
        if j + 1 < r:
            R[j, j + 1:] = (C[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / R[j, j]
    return R


def nystrom(Ysk, Omega, eps=EPS64, max_retries=5):
    """U (p x r, orthonormal columns), S (r, descending, >= 0), Delta used.

    Ysk = M @ Omega is the sketch, Omega the p x r test matrix.
    """
    Ysk = np.asarray(Ysk, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    delta = eps * np.trace(Omega.T @ Ysk)
    for _attempt in range(max_retries + 1):
        Ynu = Ysk + delta * Omega              # sketch of M + delta I
        C = Omega.T @ Ynu
        C = 0.5 * (C + C.T)
        try:
            R = _cholesky_upper(C)
        except NotPositiveDefinite:
            delta *= 10.0
            continue
        Bm = np.linalg.solve(R.T, Ynu.T).T     # Bm R = Y_nu
        U, sigma, _ = np.linalg.svd(Bm, full_matrices=False)
        S = np.maximum(0.0, sigma * sigma - delta)
        return U, S, delta
    raise NotPositiveDefinite("Nystrom core not positive definite after %d retries" % max_retries)


def precond_inv(U, S, rho, G):
    """P^{-1} G for P = U diag(S) U^T + rho I (Eq. inv_nys_woodbury)."""
    UtG = U.T @ G
    if G.ndim == 1:
        return U @ (UtG / (S + rho)) + (G - U @ UtG) / rho
    return U @ (UtG / (S + rho)[:, None]) + (G - U @ UtG) / rho


def precond_inv_sqrt(U, S, rho, v):
    """P^{-1/2} v for P = U diag(S) U^T + rho I (Eq. inv_sqrt_nys_woodbury)."""
    Utv = U.T @ v
    if v.ndim == 1:
        return U @ (Utv / np.sqrt(S + rho)) + (v - U @ Utv) / np.sqrt(rho)
    return U @ (Utv / np.sqrt(S + rho)[:, None]) + (v - U @ Utv) / np.sqrt(rho)
