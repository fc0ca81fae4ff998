"""ADASAP (Alg. 2) with Nesterov acceleration (Appendix, Alg. NestAcc), SAP (Alg. 1), ADASAP-I.

Test infrastructure (see the package docstring).

Each iteration of Alg. 2 (Sec. 4) draws a uniform block B of b row indices, forms the block
of the gradient of the quadratic (K + lambda I) W - Y at the extrapolated point, builds the
randomized Nystrom preconditioner P_B of K_BB + rho I from a Gaussian sketch of K_BB
(Alg. NysApprox, nystrom.py), estimates the step size as the reciprocal of the largest
eigenvalue of P_B^{-1/2}(K_BB + lambda I)P_B^{-1/2} by randomized powering (Alg. GetStepsize,
stepsize.py), and moves the block rows along -P_B^{-1} G.  The accelerated form keeps three
sequences W, V, Z (Alg. NestAcc): W steps from Z, V mixes its previous value with Z and takes a
longer step, and Z is the convex combination of V and W that the next gradient is taken at.
The mixing weights come from mu and nu (defaults lambda and n/b, Sec. 4.2):
beta = 1 - sqrt(mu/nu), gamma = 1/sqrt(mu nu), alpha = 1/(1 + gamma nu); V_0 = Z_0 = W_0.

Readings of the printed listings (each switchable for the tests):
  * the gradient is taken at Z_t (grad_at_z=True), since the accelerated step moves from
    Z_t (the printed listing evaluates it at W_t);
  * Z_{t+1} mixes the updated V_{t+1} (z_uses_v_next=True), the accelerated
    sketch-and-project recurrence the constants come from;
  * tail averaging is off unless asked for; when on, the returned iterate is the mean of
    W_j for j = floor(T/2) .. T-1 (the form the theorems use).

Modes: precond='nystrom' (ADASAP), 'identity' (ADASAP-I, Sec. 5: P_B = I, the step size from
powering on K_BB + lambda I), 'exact' (P_B = K_BB + lambda I); accel=False replaces the
Nesterov step by W_{t+1} = W_t - eta I_B^T D_t with the gradient at W_t; 'sap' is Alg. 1
(exact block solve, unit step, no acceleration).
"""
import math

import numpy as np

from . import kernels as kmod
from . import nystrom as nys
from . import rng
from .stepsize import preconditioned_stepsize


def nesterov_constants(mu, nu):
    """(beta, gamma, alpha) of Alg. 2's initialisation."""
    if not (mu > 0 and nu > 0):
        raise ValueError("mu and nu must be positive")
    if mu > nu:
        raise ValueError("need mu <= nu so that beta >= 0")
    beta = 1.0 - math.sqrt(mu / nu)
    gamma = 1.0 / math.sqrt(mu * nu)
    alpha = 1.0 / (1.0 + gamma * nu)
    return beta, gamma, alpha


def adasap(X, Y, kind, ell, lam, b, r, iters, seed, *, W0=None, rho_rule=0, rho=None,
           mu=None, nu=None, power_iters=10, precond="nystrom", accel=True,
           grad_at_z=True, z_uses_v_next=True, tail_average=False, eps_sketch=nys.EPS64,
           sweep=0, callback=None, outputscale=1.0):
    """Run `iters` ADASAP iterations on (K + lam I) W = Y; returns (W, info).  K is
    outputscale * k(X, X); ell is a scalar or one lengthscale per coordinate."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    squeeze = Y.ndim == 1
    if squeeze:
        Y = Y[:, None]
    n, k = Y.shape
    if not (0 < b <= n):
        raise ValueError("need 0 < b <= n")
    if precond == "nystrom" and not (0 < r <= b):
        raise ValueError("need 0 < r <= b")
    mu = lam if mu is None else mu
    nu = n / b if nu is None else nu
    beta, gamma, alpha = nesterov_constants(mu, nu)
    W = np.zeros((n, k)) if W0 is None else np.array(W0, dtype=np.float64).reshape(n, k)
    V = W.copy()
    Z = W.copy()
    off = rng.PURPOSE_SWEEP_STRIDE * sweep
    etas, rhos, lam_hats = [], [], []
    tail_sum, tail_count = np.zeros_like(W), 0
    for t in range(iters):
        if tail_average and t >= iters // 2:
            tail_sum += W  # W_t, t = floor(T/2) .. T-1
            tail_count += 1
        # Step I: block and block gradient
        B = rng.sample_block(seed, t, n, b, purpose=rng.PURPOSE_B + off)
        XB = X[B]
        P_at = Z if (accel and grad_at_z) else W
        G = kmod.kernel_matmul(XB, X, P_at, kind, ell, outputscale=outputscale) + lam * P_at[B] - Y[B]
        KBB = kmod.kernel_matrix(XB, XB, kind, ell, outputscale=outputscale)
        v0 = rng.normals(seed, rng.PURPOSE_POW + off, t, b)
        if precond == "nystrom":
            # Step II: Gaussian test matrix, row i <-> B[i]
            Omega = rng.normals(seed, rng.PURPOSE_OMEGA + off, t, b * r).reshape(b, r)
            Ysk = KBB @ Omega
            # Step III: Nystrom factors, damping, step size
            U, S, _delta = nys.nystrom(Ysk, Omega, eps=eps_sketch)
            rho_t = lam + S[-1] if rho_rule == 0 else float(rho)
            eta, lam_hat = preconditioned_stepsize(
                lambda v: KBB @ v + lam * v,
                lambda v: nys.precond_inv_sqrt(U, S, rho_t, v), v0, power_iters)
            D = nys.precond_inv(U, S, rho_t, G)
        elif precond == "identity":
            rho_t = 0.0
            eta, lam_hat = preconditioned_stepsize(lambda v: KBB @ v + lam * v, lambda v: v,
                                                   v0, power_iters)
            D = G
        elif precond in ("exact", "sap"):
            rho_t = lam
            Hb = KBB + lam * np.eye(b)
            Lc = np.linalg.cholesky(Hb)
            D = np.linalg.solve(Lc.T, np.linalg.solve(Lc, G))
            if precond == "sap":
                eta, lam_hat = 1.0, 1.0
            else:
                evals, evecs = np.linalg.eigh(Hb)
                isq = (evecs / np.sqrt(evals)) @ evecs.T
                eta, lam_hat = preconditioned_stepsize(lambda v: Hb @ v, lambda v: isq @ v,
                                                       v0, power_iters)
        else:
            raise ValueError("unknown preconditioner %r" % (precond,))
        etas.append(eta)
        rhos.append(rho_t)
        lam_hats.append(lam_hat)
        # Step IV: update
        step = np.zeros_like(W)
        step[B] = eta * D
        if precond == "sap" or not accel:
            W = W - step
            V = W
            Z = W
        else:
            W_next = Z - step
            V_next = beta * V + (1.0 - beta) * Z - gamma * step
            Z = alpha * (V_next if z_uses_v_next else V) + (1.0 - alpha) * W_next
            V = V_next
            W = W_next
        if callback is not None:
            callback(t, W, V, Z)
    out = tail_sum / tail_count if (tail_average and tail_count) else W
    info = {"eta": np.array(etas), "rho": np.array(rhos), "lambda_hat": np.array(lam_hats),
            "beta": beta, "gamma": gamma, "alpha": alpha, "V": V, "Z": Z}
    return (out[:, 0] if squeeze else out), info


def adasap_from_zero(X, Y, kind, ell, lam, b, r, iters, seed, *, rho_rule=0, rho=None, mu=None,
                     nu=None, power_iters=10, eps_sketch=nys.EPS64, log=None, outputscale=1.0):
    """ADASAP (Alg. 2 with NestAcc, default readings) from W_0 = 0, on the touched rows only.

    Started from zero, an iterate row changes only when its index is sampled: the all-rows
    part of the Nesterov step maps a zero row of (V, Z) to zero, and the block part moves
    only the rows of B_t.  So W_t, V_t and Z_t vanish outside S_t = B_0 u ... u B_{t-1}, and
    Step I's product K(X_B, X) Z_t equals K(X_B, X_S) Z_t[S] exactly; it is evaluated that
    way, which makes the first iterations of problems with millions of points affordable.
    Every other step is that of adasap() with the same random streams.

    Returns (S, W_S, info): the ascending touched rows, W_T on them, and the per-iteration
    eta, rho and Rayleigh quotients.
    """
    X = np.asarray(X)
    Y = np.asarray(Y)
    if Y.ndim == 1:
        Y = Y[:, None]
    n, k = Y.shape
    mu = lam if mu is None else mu
    nu = n / b if nu is None else nu
    beta, gamma, alpha = nesterov_constants(mu, nu)
    S = np.zeros(0, dtype=np.int64)
    W = np.zeros((0, k))
    V = np.zeros((0, k))
    Z = np.zeros((0, k))
    etas, rhos, lam_hats = [], [], []
    for t in range(iters):
        B = rng.sample_block(seed, t, n, b, purpose=rng.PURPOSE_B)
        XB = np.asarray(X[B], dtype=np.float64)
        # Z_t on the block rows (zero where the row was never touched)
        ZB = np.zeros((b, k))
        if S.size:
            pos = np.minimum(np.searchsorted(S, B), S.size - 1)
            hit = S[pos] == B
            ZB[hit] = Z[pos[hit]]
        # Step I on the touched columns
        KZ = kmod.kernel_matmul(XB, np.asarray(X[S], dtype=np.float64), Z, kind, ell,
                                outputscale=outputscale) if S.size else np.zeros((b, k))
        G = KZ + lam * ZB - np.asarray(Y[B], dtype=np.float64)
        # Steps II and III
        KBB = kmod.kernel_matrix(XB, XB, kind, ell, outputscale=outputscale)
        Omega = rng.normals(seed, rng.PURPOSE_OMEGA, t, b * r).reshape(b, r)
        U, Sv, _delta = nys.nystrom(KBB @ Omega, Omega, eps=eps_sketch)
        rho_t = lam + Sv[-1] if rho_rule == 0 else float(rho)
        v0 = rng.normals(seed, rng.PURPOSE_POW, t, b)
        eta, lam_hat = preconditioned_stepsize(
            lambda v: KBB @ v + lam * v,
            lambda v: nys.precond_inv_sqrt(U, Sv, rho_t, v), v0, power_iters)
        D = nys.precond_inv(U, Sv, rho_t, G)
        etas.append(eta)
        rhos.append(rho_t)
        lam_hats.append(lam_hat)
        # Step IV on S_{t+1} = S_t u B_t (new rows enter as zeros)
        S_new = np.union1d(S, B)
        grow = lambda A: _scatter_rows(A, np.searchsorted(S_new, S), S_new.size)
        W, V, Z = grow(W), grow(V), grow(Z)
        step = np.zeros_like(W)
        step[np.searchsorted(S_new, B)] = eta * D
        W_next = Z - step
        V_next = beta * V + (1.0 - beta) * Z - gamma * step
        Z = alpha * V_next + (1.0 - alpha) * W_next
        V = V_next
        W = W_next
        S = S_new
        if log is not None:
            log("oracle iteration %d of %d: |S| = %d, eta = %.6e, rho = %.6e" % (t + 1, iters, S.size,
                                                                               eta, rho_t))
    info = {"eta": np.array(etas), "rho": np.array(rhos), "lambda_hat": np.array(lam_hats),
            "beta": beta, "gamma": gamma, "alpha": alpha}
    return S, W, info


def _scatter_rows(A, pos, m):
    out = np.zeros((m, A.shape[1]))
    out[pos] = A
    return out
