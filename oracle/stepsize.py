"""Step size by randomized powering (Appendix, "Computing the stepsize", Alg. GetStepsize).

Test infrastructure (see the package docstring).

eta_B = 1 / lambda_1(P^{-1/2} H P^{-1/2}) with H = K_BB + lambda I.  Randomized
powering: v_0 Gaussian, normalised; each of the N = 10 applications maps
v -> P^{-1/2} H P^{-1/2} v and renormalises.  The estimate is the Rayleigh
quotient of the last application, lambda_hat = v_{N-1}^T (A v_{N-1}) with
v_{N-1} of unit length (reading: the printed listing takes the inner product
of two normalised vectors, which is a cosine and never exceeds 1).
"""
import numpy as np


def powering(apply_A, v0, iters=10):
    """lambda_hat for a symmetric PSD operator given as a callable; returns (lambda_hat, v_last)."""
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    lam_hat = None
    for _ in range(iters):
        u = apply_A(v)
        lam_hat = float(v @ u)
        v = u / np.linalg.norm(u)
    return lam_hat, v


def preconditioned_stepsize(apply_H, apply_Pinv_sqrt, v0, iters=10):
    """eta = 1 / lambda_hat(P^{-1/2} H P^{-1/2})."""
    lam_hat, _ = powering(lambda v: apply_Pinv_sqrt(apply_H(apply_Pinv_sqrt(v))), v0, iters)
    return 1.0 / lam_hat, lam_hat
