"""Parity of the matrix-core (MFMA) kernel-block products and the reduced-precision solves.

Error model of the float16 product (MIXED): kernel values and right-hand side are each
rounded once to float16 (relative 2^-11 each, a scale keeps R in range), so every term
of sum_j K_ij R_jc carries a relative error below 2^-10; the squared distances from the
three-term float16 split are accurate to about 2^-21 relative to |x~|^2.  The test bound
is 1.2e-3 * (|K| |R|)_ic.  The float16 hi/lo products (FP32 precision, residuals,
predictions) carry about 2^-21 per term: bound 2e-5 * (|K| |R|)_ic.
"""
import numpy as np
import pytest

from oracle import adasap as OA
from oracle import kernels as OK
from oracle import linsys as OL
from paper_2505_13723_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KINDS = {"rbf": OK.RBF, "matern12": OK.MATERN12, "matern32": OK.MATERN32, "matern52": OK.MATERN52}


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def abs_bound(Xr, Xc, R, kind, ell):
    return OK.kernel_matrix(Xr, Xc, kind, ell) @ np.abs(R)


@pytest.mark.parametrize("kind", list(KINDS))
# k = 17..64 runs on the 32x32x16 (wide) form: (5, 40) takes two distance K-slices, (9, 17),
# (11, 64) and (14, 33) three (3d + 6 = 48 at d = 14), (16, 64) four; the rest use the 16x16 form
@pytest.mark.parametrize("m,n,d,k", [(300, 1000, 3, 1), (257, 641, 8, 3), (64, 2000, 9, 17),
                                     (100, 333, 16, 64), (33, 77, 1, 100), (513, 4096, 11, 64),
                                     (130, 500, 5, 40), (200, 1000, 14, 33)])
def test_mixed_kblock_matches_oracle(lib, kind, m, n, d, k):
    r0 = np.random.default_rng(m + 3 * n + d + k)
    Xr, Xc = r0.standard_normal((m, d)), r0.standard_normal((n, d))
    R = r0.standard_normal((n, k)) * np.exp(r0.uniform(-3, 3, k))  # uneven column scales
    ell = 0.8 * np.sqrt(d)
    Xr32, Xc32, R32 = (a.astype(np.float32).astype(np.float64) for a in (Xr, Xc, R))
    got = lib.kblock_matmul(kind, ell, "mixed", dev(Xr), dev(Xc), dev(R)).cpu().double().numpy()
    ref = OK.kernel_matmul(Xr32, Xc32, R32, KINDS[kind], ell)
    bound = 1.2e-3 * abs_bound(Xr32, Xc32, R32, KINDS[kind], ell) + 1e-6
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


def _solve(lib, X, Y, **kw):
    Xd, Yd = dev(X), dev(Y)
    h = lib.create(lib.config(**kw), Xd, Yd)
    W = torch.zeros_like(Yd)
    rep = h.solve(W)
    return W.cpu().double().numpy(), rep, h


def knorm_diff(X, W1, W2, Y, kind, ell, lam):
    E = W1 - W2
    return np.linalg.norm(OK.kernel_matmul(X, X, E, kind, ell) + lam * E) / np.linalg.norm(Y)


@pytest.mark.parametrize("prec,kind,k,tol", [("mixed", "rbf", 4, 1e-3), ("mixed", "matern32", 1, 1e-3),
                                             ("fp32", "rbf", 20, 1e-3), ("fp32", "matern52", 2, 1e-3)])
def test_reduced_precision_solve_matches_oracle(lib, prec, kind, k, tol):
    n, d, lam, ell, b, r, T = 1500, 6, 0.05, 1.2, 300, 60, 25
    X, Y = inputs.make_small(31, n, d, k)
    X = X.astype(np.float32).astype(np.float64)
    Y = Y.astype(np.float32).astype(np.float64)
    Wo, info = OA.adasap(X, Y, KINDS[kind], ell, lam, b, r, T, 12, eps_sketch=2.0**-23)
    Wg, rep, h = _solve(lib, X, Y, kernel=kind, lengthscale=ell, lam=lam, block_size=b, rank=r,
                        max_iters=T, seed=12, precision=prec)
    delta = knorm_diff(X, Wg, Wo, Y, KINDS[kind], ell, lam)
    assert delta <= tol, delta
    # both are real solves: the residual fell well below its starting value of 1
    assert OL.relres(X, Y, Wg, KINDS[kind], ell, lam)[0] < 0.2


def test_residual_and_predict_through_matrix_cores(lib):
    n, d, k, lam, ell = 3000, 5, 3, 0.03, 1.0
    X, Y = inputs.make_small(41, n, d, k)
    X = X.astype(np.float32).astype(np.float64)
    Y = Y.astype(np.float32).astype(np.float64)
    W = np.random.default_rng(2).standard_normal((n, k)).astype(np.float32).astype(np.float64)
    h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=100, rank=10,
                              precision="fp32"), dev(X), dev(Y))
    rr, rm = h.residual(dev(W))
    ro, rmo = OL.relres(X, Y, W, OK.RBF, ell, lam)
    assert rr == pytest.approx(ro, rel=1e-4) and rm == pytest.approx(rmo, rel=1e-4)
    Xs = np.random.default_rng(5).standard_normal((123, d)).astype(np.float32).astype(np.float64)
    got = h.predict(dev(W), dev(Xs)).cpu().double().numpy()
    ref = OL.predict(Xs, X, W, OK.RBF, ell)
    bound = 2e-5 * abs_bound(Xs, X, W, OK.RBF, ell) + 1e-6
    assert np.all(np.abs(got - ref) <= bound)


def test_refinement_sweep_reduces_residual(lib):
    # a well-conditioned problem, so the float16 solve reaches its rounding floor quickly;
    # float64 refinement sweeps (residual from the hi/lo products, correction solved again in
    # float16) must then push the residual far below that floor
    n, d, k, lam, ell = 2000, 4, 2, 0.5, 1.0
    X, Y = inputs.make_small(51, n, d, k)
    X = X.astype(np.float32).astype(np.float64)
    Y = Y.astype(np.float32).astype(np.float64)
    kw = dict(kernel="rbf", lengthscale=ell, lam=lam, block_size=500, rank=100, max_iters=60,
              seed=3, precision="mixed", tol=1e-14)
    W0, rep0, _ = _solve(lib, X, Y, **kw)
    W1, rep1, h1 = _solve(lib, X, Y, refine_sweeps=2, **kw)
    assert rep1["refine_done"] == 2
    r0 = OL.relres(X, Y, W0, OK.RBF, ell, lam)[0]
    r1 = OL.relres(X, Y, W1, OK.RBF, ell, lam)[0]
    assert r0 > 1e-6, r0          # the float16 floor
    assert r1 < 1e-2 * r0, (r1, r0)
    assert rep1["relres"] == pytest.approx(r1, rel=1e-2, abs=1e-9)


def test_probe_rates_are_plausible(lib):
    # the instruction-rate probe behind the bench line's second roofline: a transcendental
    # costs at least as much as a full-rate vector instruction, and the matrix cores reach a
    # sizeable share of the part's published float16 rate (2.5 PFLOP/s at 2.4 GHz)
    r = lib.probe_rates()
    assert 0.5 < r["valu_ns"] < 20 and r["valu_ns"] <= r["exp_ns"] < 40, r
    assert 500 < r["mfma32_f16_tflops"] < 2600, r
