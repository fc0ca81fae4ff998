"""Randomized Nystrom approximation and Woodbury applies (Appendix, "Randomized Nystrom approximation").

Test infrastructure (see the package docstring).

NysApprox (Appendix, Alg. NysApprox, after Tropp et al. 2017 Alg. 3) as read
consistently (the printed listing forms the triangular solve from the
unshifted sketch and writes S^2 for Sigma^2):

    Delta = eps * tr(Omega^T (M Omega))          shift for stability
    Y_nu  = M Omega + Delta * Omega              shifted sketch
    C     = Omega^T Y_nu  (symmetrised),  C = R^T R  (upper Cholesky factor R)
    B     = Y_nu R^{-1}                          triangular solve
    U, Sigma, _ = thin SVD of B
    S     = max(0, Sigma^2 - Delta)              remove the shift

so that Mhat = U diag(S) U^T.  eps is the machine epsilon of the precision the
sketch was computed in (2**-52 for a float64 sketch, 2**-23 for float32).  If
the Cholesky factorisation fails, Delta is multiplied by 10 and the step is
retried, at most 5 times (reading for a case the paper does not discuss).

Woodbury applies with P = U S U^T + rho I (Eq. inv_nys_woodbury and
Eq. inv_sqrt_nys_woodbury):

    P^{-1}   g = U (S + rho)^{-1}   U^T g + (g - U U^T g) / rho
    P^{-1/2} v = U (S + rho)^{-1/2} U^T v + (v - U U^T v) / sqrt(rho)
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
        Ynu = Ysk + delta * Omega
        C = Omega.T @ Ynu
        C = 0.5 * (C + C.T)
        try:
            R = _cholesky_upper(C)
        except NotPositiveDefinite:
            delta *= 10.0
            continue
        # B = Y_nu R^{-1}: solve B R = Y_nu row by row (R upper triangular)
        Bm = np.linalg.solve(R.T, Ynu.T).T
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
