"""Pins for NysApprox, the Woodbury applies and randomized powering (Appendix)."""
import numpy as np
import pytest

from oracle import kernels as K
from oracle import nystrom as nys
from oracle import stepsize


def _psd_kernel(p, seed=0, ell=0.7):
    X = np.random.default_rng(seed).standard_normal((p, 3))
    return K.kernel_matrix(X, X, K.RBF, ell)


def test_cholesky_upper_matches_numpy():
    A = np.random.default_rng(3).standard_normal((9, 9))
    C = A @ A.T + 9 * np.eye(9)
    R = nys._cholesky_upper(C)
    assert np.allclose(R, np.linalg.cholesky(C).T, rtol=1e-13, atol=1e-13)
    with pytest.raises(nys.NotPositiveDefinite):
        nys._cholesky_upper(-np.eye(3))


def test_low_rank_is_recovered_exactly():
    r0 = np.random.default_rng(4)
    G = r0.standard_normal((60, 7))
    M = G @ G.T
    Om = r0.standard_normal((60, 10))
    U, S, delta = nys.nystrom(M @ Om, Om)
    Mhat = (U * S) @ U.T
    assert np.linalg.norm(Mhat - M) <= 1e-10 * np.linalg.norm(M)
    assert np.allclose(U.T @ U, np.eye(10), atol=1e-12)
    assert np.all(np.diff(S) <= 0) and np.all(S >= 0)
    assert delta == pytest.approx(2.0**-52 * np.trace(Om.T @ M @ Om))


def test_full_sketch_recovers_spd_matrix():
    M = _psd_kernel(40) + 1e-3 * np.eye(40)
    Om = np.random.default_rng(5).standard_normal((40, 40))
    U, S, _ = nys.nystrom(M @ Om, Om)
    assert np.linalg.norm((U * S) @ U.T - M) <= 1e-9 * np.linalg.norm(M)


def test_nystrom_is_dominated_and_range_invariant():
    M = _psd_kernel(80, seed=6)
    r0 = np.random.default_rng(7)
    Om = r0.standard_normal((80, 12))
    U, S, _ = nys.nystrom(M @ Om, Om)
    Mhat = (U * S) @ U.T
    # M - Mhat is PSD (the Nystrom approximation never overshoots)
    assert np.linalg.eigvalsh(M - Mhat).min() >= -1e-10 * np.linalg.eigvalsh(M).max()
    # Mhat depends on Omega only through its range (apart from the tiny shift)
    Q = r0.standard_normal((12, 12)) + 4 * np.eye(12)
    Om2 = Om @ Q
    U2, S2, _ = nys.nystrom(M @ Om2, Om2)
    assert np.linalg.norm((U2 * S2) @ U2.T - Mhat) <= 1e-8 * np.linalg.norm(Mhat)
    # and the brute-force formula Mhat = (M Om)(Om^T M Om)^+ (M Om)^T
    Y = M @ Om
    brute = Y @ np.linalg.pinv(Om.T @ Y) @ Y.T
    assert np.linalg.norm(brute - Mhat) <= 1e-8 * np.linalg.norm(Mhat)


def test_singular_core_raises_after_retries():
    M = _psd_kernel(30)
    Om = np.random.default_rng(8).standard_normal((30, 6))
    Om[:, 3] = 0.0  # zero column: Omega^T (M + Delta I) Omega is singular for every Delta
    with pytest.raises(nys.NotPositiveDefinite):
        nys.nystrom(M @ Om, Om)


def test_shift_retry_grows_delta():
    # slightly indefinite "kernel" matrix: the first Cholesky fails, a larger shift succeeds
    r0 = np.random.default_rng(9)
    Q, _ = np.linalg.qr(r0.standard_normal((20, 20)))
    ev = np.concatenate([np.linspace(1, 2, 19), [-1e-14]])
    M = (Q * ev) @ Q.T
    Om = Q[:, :20]
    U, S, delta = nys.nystrom(M @ Om, Om)
    assert delta > 2.0**-52 * np.trace(Om.T @ M @ Om)
    assert np.all(np.isfinite(U)) and np.all(S >= 0)


@pytest.mark.parametrize("rho", [1e-3, 0.5])
def test_woodbury_against_dense(rho):
    M = _psd_kernel(64, seed=10)
    Om = np.random.default_rng(11).standard_normal((64, 16))
    U, S, _ = nys.nystrom(M @ Om, Om)
    P = (U * S) @ U.T + rho * np.eye(64)
    G = np.random.default_rng(12).standard_normal((64, 3))
    assert np.allclose(nys.precond_inv(U, S, rho, G), np.linalg.solve(P, G), rtol=1e-9, atol=1e-9)
    w, V = np.linalg.eigh(P)
    Pis = (V / np.sqrt(w)) @ V.T
    assert np.allclose(nys.precond_inv_sqrt(U, S, rho, G), Pis @ G, rtol=1e-10, atol=1e-10)
    v = G[:, 0]
    assert np.allclose(nys.precond_inv_sqrt(U, S, rho, nys.precond_inv_sqrt(U, S, rho, v)),
                       nys.precond_inv(U, S, rho, v), rtol=1e-11, atol=1e-11)


def test_powering_diagonal_bound():
    lam = np.array([10.0, 5.0, 2.0, 1.0, 0.5, 0.1])
    v0 = np.random.default_rng(13).standard_normal(6)
    est, _ = stepsize.powering(lambda v: lam * v, v0, iters=10)
    assert est <= lam[0] * (1 + 1e-15)
    # Rayleigh quotient after N applications: lam1 - est <= lam1 * tan^2(theta0) * (lam2/lam1)^(2(N-1))
    c0 = abs(v0[0]) / np.linalg.norm(v0)
    tan2 = (1 - c0**2) / c0**2
    assert lam[0] - est <= lam[0] * tan2 * (lam[1] / lam[0]) ** 18 * (1 + 1e-9)


def test_powering_with_exact_preconditioner_gives_one():
    M = _psd_kernel(50, seed=14)
    Om = np.random.default_rng(15).standard_normal((50, 10))
    U, S, _ = nys.nystrom(M @ Om, Om)
    rho = 0.3
    H = (U * S) @ U.T + rho * np.eye(50)  # H equals P exactly
    eta, lam_hat = stepsize.preconditioned_stepsize(
        lambda v: H @ v, lambda v: nys.precond_inv_sqrt(U, S, rho, v),
        np.random.default_rng(16).standard_normal(50))
    assert abs(lam_hat - 1.0) < 1e-12 and abs(eta - 1.0) < 1e-12


def test_powering_carried_as_preconditioned_vector_matches_printed_form():
    """The GPU's powering keeps w = P^{-1/2} v: u = H w, y = P^{-1} u, v.(M v) = w.u,
    |M v|^2 = u.y and the next w = y / sqrt(u.y) for M = P^{-1/2} H P^{-1/2}.  In exact
    arithmetic these are the printed iterates; here both forms run on the same sketch and
    start, and the Rayleigh quotients agree to rounding at every step."""
    rs = np.random.default_rng(11)
    b, d, r, lam = 300, 4, 40, 1e-2
    X = rs.standard_normal((b, d))
    H = K.kernel_matrix(X, X, K.RBF, 0.8) + lam * np.eye(b)
    Om = rs.standard_normal((b, r))
    U, S, _ = nys.nystrom(H @ Om, Om)
    rho = lam + S[-1]
    v0 = rs.standard_normal(b)
    v = v0 / np.linalg.norm(v0)
    w = nys.precond_inv_sqrt(U, S, rho, v)
    for _ in range(10):
        # printed form
        z = nys.precond_inv_sqrt(U, S, rho, H @ nys.precond_inv_sqrt(U, S, rho, v))
        rq_printed = float(v @ z)
        v = z / np.linalg.norm(z)
        # carried form
        u = H @ w
        y = nys.precond_inv(U, S, rho, u)
        rq_carried = float(w @ u)
        w = y / np.sqrt(float(u @ y))
        assert rq_carried == pytest.approx(rq_printed, rel=1e-12)
    np.testing.assert_allclose(w, nys.precond_inv_sqrt(U, S, rho, v), rtol=0, atol=1e-12)
    eta, lam_hat = stepsize.preconditioned_stepsize(
        lambda x: H @ x, lambda x: nys.precond_inv_sqrt(U, S, rho, x), v0)
    assert rq_carried == pytest.approx(lam_hat, rel=1e-12)
