"""Parity of the HIP path (through the C ABI) with the float64 CPU oracle.

Each step of the iteration is compared on the same seeded inputs: the random draws,
the kernel-block products, the Nystrom factors, the Woodbury applies, and whole
solves (trajectory parity with identical random streams).  Tolerances:
float64 paths 1e-10 relative (steps) and relative residual difference
||(K + lambda I)(W_gpu - W_oracle)|| / ||Y|| <= 1e-6 (solves); float32 paths 1e-5 (steps)
and 1e-3 (solves).
"""
import ctypes

import numpy as np
import pytest

from oracle import adasap as OA
from oracle import kernels as OK
from oracle import linsys as OL
from oracle import nystrom as ON
from oracle import rng as OR
from paper_2505_13723_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
KINDS = {"rbf": OK.RBF, "matern12": OK.MATERN12, "matern32": OK.MATERN32, "matern52": OK.MATERN52}


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def knorm_diff(X, W1, W2, Y, kind, ell, lam):
    """||(K + lambda I)(W1 - W2)||_F / ||Y||_F in float64 on the CPU."""
    E = np.asarray(W1, dtype=np.float64) - np.asarray(W2, dtype=np.float64)
    R = OK.kernel_matmul(X, X, E, kind, ell) + lam * E
    return np.linalg.norm(R) / np.linalg.norm(Y)


def test_device_normals_match_oracle(lib):
    for seed, purpose, t, count in [(1, 6, 0, 1001), (3, 7, 122, 64), (2**40, 6, 5, 2)]:
        got = lib.normals(seed, purpose, t, count).cpu().numpy()
        ref = OR.normals(seed, purpose, t, count)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("m,n,d,k", [(300, 1000, 3, 1), (257, 641, 8, 3), (64, 2000, 11, 17),
                                     (5, 130, 1, 2), (100, 333, 16, 64), (33, 77, 40, 5)])
def test_kblock_fp64(lib, kind, m, n, d, k):
    r0 = np.random.default_rng(m * 7 + n + d + k)
    Xr, Xc, R = r0.standard_normal((m, d)), r0.standard_normal((n, d)), r0.standard_normal((n, k))
    ell = 0.9 * np.sqrt(d)
    got = lib.kblock_matmul(kind, ell, "fp64", dev(Xr), dev(Xc), dev(R)).cpu().numpy()
    ref = OK.kernel_matmul(Xr, Xc, R, KINDS[kind], ell)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max() + 1e-14


@pytest.mark.parametrize("kind", ["rbf", "matern32"])
@pytest.mark.parametrize("m,n,d,k", [(300, 1000, 3, 1), (257, 641, 11, 4), (64, 2000, 9, 17)])
def test_kblock_fp32(lib, kind, m, n, d, k):
    r0 = np.random.default_rng(m + n + d + k)
    Xr, Xc, R = r0.standard_normal((m, d)), r0.standard_normal((n, d)), r0.standard_normal((n, k))
    ell = 0.7 * np.sqrt(d)
    got = lib.kblock_matmul(kind, ell, "fp32", dev(Xr, torch.float32), dev(Xc, torch.float32),
                            dev(R, torch.float32)).cpu().double().numpy()
    ref = OK.kernel_matmul(Xr.astype(np.float32), Xc.astype(np.float32), R.astype(np.float32),
                           KINDS[kind], ell)
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()


def test_kblock_empty_columns(lib):
    Xr = dev(np.zeros((4, 3)))
    out = lib.kblock_matmul("rbf", 1.0, "fp64", Xr, dev(np.zeros((0, 3))), dev(np.zeros((0, 2))))
    assert out.shape == (4, 2) and torch.all(out == 0)


@pytest.mark.parametrize("b,r", [(200, 30), (257, 64), (128, 128), (64, 1), (64, 2), (64, 3), (300, 101)])
def test_nystrom_matches_oracle(lib, b, r):
    X = np.random.default_rng(b + r).standard_normal((b, 4))
    M = OK.kernel_matrix(X, X, OK.RBF, 1.2)
    Om = OR.normals(5, OR.PURPOSE_OMEGA, b, b * r).reshape(b, r)
    Ysk = M @ Om
    U, S, delta = lib.nystrom(dev(Ysk), dev(Om), 2.0**-52)
    U, S = U.cpu().numpy(), S.cpu().numpy()
    Ur, Sr, dr = ON.nystrom(Ysk, Om)
    assert delta == pytest.approx(dr, rel=1e-12)
    assert np.allclose(S, Sr, rtol=1e-9, atol=1e-12 * Sr[0])
    assert np.allclose(U.T @ U, np.eye(r), atol=1e-8)
    Mh, Mr = (U * S) @ U.T, (Ur * Sr) @ Ur.T
    assert np.linalg.norm(Mh - Mr) <= 1e-9 * np.linalg.norm(Mr)


@pytest.mark.parametrize("power,k", [(0, 1), (0, 5), (1, 1), (1, 3)])
def test_precond_apply_matches_oracle(lib, power, k):
    b, r, rho = 300, 40, 0.05
    X = np.random.default_rng(k).standard_normal((b, 3))
    M = OK.kernel_matrix(X, X, OK.MATERN32, 1.0)
    Om = np.random.default_rng(1).standard_normal((b, r))
    U, S, _ = ON.nystrom(M @ Om, Om)
    G = np.random.default_rng(2).standard_normal((b, k))
    got = lib.precond_apply(dev(U), dev(S), rho, dev(G), power).cpu().numpy()
    ref = ON.precond_inv(U, S, rho, G) if power == 0 else ON.precond_inv_sqrt(U, S, rho, G)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def _gpu_solve(lib, X, Y, dtype=torch.float64, W0=None, **cfgkw):
    Xd, Yd = dev(X, dtype), dev(Y, dtype)
    cfg = lib.config(**cfgkw)
    h = lib.create(cfg, Xd, Yd)
    W = torch.zeros_like(Yd) if W0 is None else dev(W0, dtype)
    rep = h.solve(W)
    tr = h.trace(rep["iters"])
    return W.cpu().double().numpy(), rep, tr, h


SOLVE_CASES = [
    dict(name="rbf_default", n=600, d=3, k=1, kind="rbf", ell=1.0, lam=0.02, b=100, r=30, T=25),
    dict(name="matern32_k3", n=517, d=5, k=3, kind="matern32", ell=1.5, lam=0.05, b=97, r=20, T=20),
    dict(name="matern52_rho_fixed", n=400, d=2, k=2, kind="matern52", ell=0.7, lam=0.01, b=64,
         r=64, T=15, rho_rule=1, rho=0.01),
    dict(name="matern12_noaccel", n=300, d=4, k=1, kind="matern12", ell=2.0, lam=0.05, b=50, r=10,
         T=20, accel=0),
    dict(name="identity_precond", n=350, d=3, k=2, kind="rbf", ell=0.8, lam=0.05, b=70, r=1, T=20,
         precond="identity"),
    dict(name="z_uses_v_old", n=300, d=3, k=1, kind="rbf", ell=1.0, lam=0.05, b=60, r=15, T=20,
         z_uses_v_next=0),
    dict(name="grad_at_w_printed", n=300, d=3, k=1, kind="rbf", ell=1.0, lam=0.05, b=60, r=15,
         T=15, grad_at_z=0),
    dict(name="tail_average", n=256, d=3, k=1, kind="rbf", ell=1.0, lam=0.05, b=64, r=16, T=11,
         tail_average=1),
    dict(name="block_is_all_rows", n=128, d=3, k=2, kind="rbf", ell=1.0, lam=0.05, b=128, r=128,
         T=1, rho_rule=1, rho=0.05),
]


@pytest.mark.parametrize("case", SOLVE_CASES, ids=[c["name"] for c in SOLVE_CASES])
def test_solve_fp64_trajectory_parity(lib, case):
    c = dict(case)
    X, Y = inputs.make_small(11, c["n"], c["d"], c["k"])
    kind = KINDS[c["kind"]]
    okw = dict(rho_rule=c.get("rho_rule", 0), rho=c.get("rho"), accel=bool(c.get("accel", 1)),
               z_uses_v_next=bool(c.get("z_uses_v_next", 1)), tail_average=bool(c.get("tail_average", 0)),
               precond=c.get("precond", "nystrom"), grad_at_z=bool(c.get("grad_at_z", 1)))
    Wo, info = OA.adasap(X, Y, kind, c["ell"], c["lam"], c["b"], c["r"], c["T"], 3, **okw)
    gkw = dict(kernel=c["kind"], lengthscale=c["ell"], lam=c["lam"], block_size=c["b"], rank=c["r"],
               rho_rule=c.get("rho_rule", 0), rho=c.get("rho") or 0.0, max_iters=c["T"], seed=3,
               precision="fp64", accel=c.get("accel", 1), z_uses_v_next=c.get("z_uses_v_next", 1),
               tail_average=c.get("tail_average", 0), grad_at_z=c.get("grad_at_z", 1),
               precond=1 if c.get("precond") == "identity" else 0)
    Wg, rep, tr, _h = _gpu_solve(lib, X, Y, **gkw)
    assert rep["iters"] == c["T"]
    assert np.allclose(tr["eta"], info["eta"], rtol=1e-8)
    if okw["precond"] == "nystrom":
        assert np.allclose(tr["rho"], info["rho"], rtol=1e-8)
    delta = knorm_diff(X, Wg, Wo, Y, kind, c["ell"], c["lam"])
    assert delta <= 1e-6, delta
    if c["name"] == "block_is_all_rows":
        assert OL.relres(X, Y, Wg, kind, c["ell"], c["lam"])[0] < 1e-9


def test_solve_small_fp64_workload(lib):
    # the whole 200-iteration run of the small float64 workload
    cfg = inputs.WORKLOADS["c1_fp64_n4096"]
    X, y = inputs.make_c1(seed=cfg["seed"])
    T = cfg["iters"]
    Wo, info = OA.adasap(X, y, OK.RBF, cfg["ell"], cfg["lam"], cfg["b"], cfg["r"], T, cfg["seed"],
                         rho_rule=1, rho=cfg["rho"])
    Wg, rep, tr, h = _gpu_solve(lib, X, y[:, None], kernel="rbf", lengthscale=cfg["ell"],
                                lam=cfg["lam"], block_size=cfg["b"], rank=cfg["r"], rho_rule=1,
                                rho=cfg["rho"], max_iters=T, seed=cfg["seed"], precision="fp64")
    assert np.allclose(tr["eta"], info["eta"], rtol=1e-8)
    delta = knorm_diff(X, Wg[:, 0], Wo, y, OK.RBF, cfg["ell"], cfg["lam"])
    assert delta <= 1e-6, delta
    # the residual the library reports equals the oracle's
    rr, rm = h.residual(dev(Wg))
    ro = OL.relres(X, y[:, None], Wg, OK.RBF, cfg["ell"], cfg["lam"])[0]
    assert rr == pytest.approx(ro, rel=1e-9)


def test_solve_fp32_matches_oracle(lib):
    n, d, k = 800, 4, 2
    X, Y = inputs.make_small(21, n, d, k)
    X32 = X.astype(np.float32).astype(np.float64)
    Y32 = Y.astype(np.float32).astype(np.float64)
    T, b, r, lam, ell = 30, 160, 40, 0.05, 1.0
    Wo, info = OA.adasap(X32, Y32, OK.RBF, ell, lam, b, r, T, 4, eps_sketch=2.0**-23)
    Wg, rep, tr, _ = _gpu_solve(lib, X, Y, dtype=torch.float32, kernel="rbf", lengthscale=ell, lam=lam,
                                block_size=b, rank=r, max_iters=T, seed=4, precision="fp32")
    delta = knorm_diff(X32, Wg, Wo, Y32, OK.RBF, ell, lam)
    assert delta <= 1e-3, delta
    assert np.allclose(tr["eta"], info["eta"], rtol=1e-3)


def test_solve_is_deterministic(lib):
    X, Y = inputs.make_small(5, 700, 3, 2)
    kw = dict(kernel="rbf", lengthscale=1.0, lam=0.03, block_size=128, rank=32, max_iters=8, seed=9,
              precision="fp64")
    W1 = _gpu_solve(lib, X, Y, **kw)[0]
    W2 = _gpu_solve(lib, X, Y, **kw)[0]
    assert np.array_equal(W1, W2)


def test_separable_right_hand_sides(lib):
    X, Y = inputs.make_small(6, 400, 3, 3)
    kw = dict(kernel="matern32", lengthscale=1.0, lam=0.03, block_size=80, rank=20, max_iters=10,
              seed=2, precision="fp64")
    Wj = _gpu_solve(lib, X, Y, **kw)[0]
    for c in range(3):
        Wc = _gpu_solve(lib, X, Y[:, c:c + 1], **kw)[0]
        assert np.allclose(Wj[:, c], Wc[:, 0], rtol=1e-11, atol=1e-11 * np.abs(Wc).max())


def test_predict_and_posterior_mean_identity(lib):
    n, d, k, lam, ell = 500, 3, 2, 0.05, 1.1
    X, Y = inputs.make_small(8, n, d, k)
    Wstar = OL.direct_solve(X, Y, OK.RBF, ell, lam)
    Xd, Yd = dev(X), dev(Y)
    h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=50, rank=10,
                              precision="fp64"), Xd, Yd)
    Xs = np.random.default_rng(3).standard_normal((77, d))
    got = h.predict(dev(Wstar), dev(Xs)).cpu().numpy()
    assert np.allclose(got, OL.predict(Xs, X, Wstar, OK.RBF, ell), rtol=1e-11, atol=1e-12)
    m = h.predict(dev(Wstar), Xd).cpu().numpy()
    assert np.linalg.norm(m - (Y - lam * Wstar)) <= 1e-10 * np.linalg.norm(Y)
    rr, rm = h.residual(dev(Wstar))
    assert rr < 1e-10 and rm < 1e-10


def test_nonfinite_inputs_are_rejected(lib):
    X, Y = inputs.make_small(9, 200, 3, 1)
    Y[5, 0] = np.nan
    h = lib.create(lib.config(block_size=50, rank=10, precision="fp64", max_iters=2), dev(X), dev(Y))
    W = torch.zeros_like(dev(Y))
    from paper_2505_13723_amd.binding import AdasapError
    with pytest.raises(AdasapError) as e:
        h.solve(W)
    assert e.value.status == 5



@pytest.mark.parametrize("precision", ["mixed", "fp32"])
def test_solve_after_early_exit_matches_fresh_handle(lib, precision):
    """Each iteration enqueues the next one's block and sketch ahead of time, so a solve that
    stops on its tolerance leaves such a head behind.  A second solve on the same handle must
    not use it: it repeats the first bit for bit and equals the solve on a fresh handle."""
    X, Y = inputs.make_small(61, 900, 4, 20)
    Xd, Yd = dev(X, torch.float32), dev(Y, torch.float32)
    cfg = lib.config(kernel="rbf", lengthscale=1.0, lam=0.05, block_size=128, rank=32, seed=5,
                     precision=precision, max_iters=40, tol=0.5, check_every=3)
    h = lib.create(cfg, Xd, Yd)
    W1 = torch.zeros_like(Yd)
    rep1 = h.solve(W1)
    W2 = torch.zeros_like(Yd)
    rep2 = h.solve(W2)
    h.close()
    g = lib.create(cfg, Xd, Yd)
    W3 = torch.zeros_like(Yd)
    g.solve(W3)
    g.close()
    assert 0 < rep1["iters"] < 40, rep1["iters"]  # stopped early, the next head queued
    assert rep2["iters"] == rep1["iters"]
    assert torch.equal(W1, W2) and torch.equal(W1, W3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_continued_equals_one_long_solve(lib, precision):
    # a solve of T1 iterations continued by T2 (adasap_solve_more) is the solve of T1 + T2
    # iterations: same random streams, same Nesterov state, bit for bit
    X, Y = inputs.make_small(71, 900, 4, 3)
    dt = torch.float64 if precision == "fp64" else torch.float32
    Xd, Yd = dev(X, dt), dev(Y, dt)
    kw = dict(kernel="rbf", lengthscale=1.0, lam=0.05, block_size=128, rank=32, seed=8,
              precision=precision)
    h = lib.create(lib.config(max_iters=12, **kw), Xd, Yd)
    W1 = torch.zeros_like(Yd)
    h.solve(W1)
    h.close()
    g = lib.create(lib.config(max_iters=5, **kw), Xd, Yd)
    W2 = torch.zeros_like(Yd)
    g.solve(W2)
    rep = g.solve_more(W2, 4)
    assert rep["iters"] == 4
    rep = g.solve_more(W2, 3)
    eta = g.trace(3)["eta"]
    g.close()
    assert torch.equal(W1, W2)
    tr = _gpu_solve(lib, X, Y, dtype=dt, max_iters=12, **kw)[2]
    assert np.array_equal(eta, tr["eta"][9:12])


def test_not_converged_status_and_continuation_rules(lib):
    from paper_2505_13723_amd.binding import AdasapError
    X, Y = inputs.make_small(72, 500, 3, 1)
    Xd, Yd = dev(X), dev(Y)
    h = lib.create(lib.config(kernel="rbf", lengthscale=1.0, lam=0.05, block_size=100, rank=20,
                              seed=2, precision="fp64", max_iters=3, tol=1e-12), Xd, Yd)
    W = torch.zeros_like(Yd)
    rep = h.solve(W)
    assert rep["status"] == 7 and 0 < rep["relres"] < 1 and rep["iters"] == 3
    assert lib.cdll.adasap_solve(h.h, ctypes.c_void_p(W.data_ptr()), None) == 7
    with pytest.raises(AdasapError):
        h.solve_more(W, 0)
    h.close()
    # refinement sweeps leave nothing to continue
    g = lib.create(lib.config(kernel="rbf", lengthscale=1.0, lam=0.05, block_size=100, rank=20,
                              seed=2, precision="fp64", max_iters=3, refine_sweeps=1), Xd, Yd)
    g.solve(W)
    with pytest.raises(AdasapError) as e:
        g.solve_more(W, 2)
    assert e.value.status == 1
    g.close()


ARD_ELL = [0.6, 1.3, 2.2, 0.9]


@pytest.mark.parametrize("kind", ["rbf", "matern32"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-3), ("mixed", 1e-3)])
def test_solve_per_dimension_lengthscales_and_outputscale(lib, kind, precision, tol):
    # the kernel of the paper's regression experiments: one lengthscale per coordinate and an
    # output scale (appendix, hyperparameters); trajectory parity with the oracle
    n, d, k, lam, s, b, r, T = 700, 4, 2, 0.04, 2.3, 140, 30, 15
    X, Y = inputs.make_small(81, n, d, k)
    reduced = precision != "fp64"
    if reduced:
        X, Y = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    ell = np.array(ARD_ELL)
    Wo, info = OA.adasap(X, Y, KINDS[kind], ell, lam, b, r, T, 6, outputscale=s,
                         eps_sketch=2.0 ** -23 if reduced else 2.0 ** -52)
    Wg, rep, tr, h = _gpu_solve(lib, X, Y, dtype=torch.float32 if reduced else torch.float64,
                                kernel=kind, lengthscales=ARD_ELL, outputscale=s, lam=lam,
                                block_size=b, rank=r, max_iters=T, seed=6, precision=precision)
    E = Wg - Wo
    delta = np.linalg.norm(OK.kernel_matmul(X, X, E, KINDS[kind], ell, outputscale=s) + lam * E) / \
        np.linalg.norm(Y)
    assert delta <= tol, delta
    assert np.allclose(tr["eta"], info["eta"], rtol=1e-8 if not reduced else 1e-3)
    assert np.allclose(tr["rho"], info["rho"], rtol=1e-8 if not reduced else 1e-3)
    # residual and prediction of the same handle
    dt = torch.float32 if reduced else torch.float64
    rr, _ = h.residual(dev(Wg, dt))
    ro = OL.relres(X, Y, Wg, KINDS[kind], ell, lam, outputscale=s)[0]
    assert rr == pytest.approx(ro, rel=1e-9 if not reduced else 1e-3)
    Xs = np.random.default_rng(9).standard_normal((55, d))
    if reduced:
        Xs = Xs.astype(np.float32).astype(np.float64)
    got = h.predict(dev(Wg, dt), dev(Xs, dt)).cpu().double().numpy()
    ref = OL.predict(Xs, X, Wg, KINDS[kind], ell, outputscale=s)
    bound = (1e-11 if not reduced else 2e-5) * (OK.kernel_matrix(Xs, X, KINDS[kind], ell, outputscale=s)
                                                @ np.abs(Wg)) + 1e-9
    assert np.all(np.abs(got - ref) <= bound)
    h.close()


def test_bad_lengthscales_are_rejected(lib):
    from paper_2505_13723_amd.binding import AdasapError
    X, Y = inputs.make_small(82, 100, 3, 1)
    for kw in (dict(lengthscales=[1.0, 0.0, 1.0]), dict(lengthscales=[1.0, 2.0]),
               dict(outputscale=0.0), dict(lengthscales=[1.0, float("nan"), 1.0])):
        with pytest.raises(AdasapError) as e:
            lib.create(lib.config(block_size=50, rank=10, precision="fp64", **kw), dev(X), dev(Y))
        assert e.value.status == 1


@pytest.mark.parametrize("b,accel", [(100, 0), (200, 0), (130, 1), (64, 0)])
def test_exact_block_projection_matches_oracle(lib, b, accel):
    # precond EXACT: P_B = K_BB + lambda I factored in float64 (blocked Cholesky, panels of 64
    # columns: b = 100, 130 and 200 have ragged last panels), unit step.  accel = 0 is SAP
    # (Alg. 1), accel = 1 the accelerated step around the exact projection
    n, d, k, lam, ell, T = 700, 3, 2, 0.03, 0.9, 12
    X, Y = inputs.make_small(91, n, d, k)
    Wo, info = OA.adasap(X, Y, OK.MATERN32, ell, lam, b, 1, T, 5,
                         precond="sap" if not accel else "exact")
    Wg, rep, tr, h = _gpu_solve(lib, X, Y, kernel="matern32", lengthscale=ell, lam=lam, block_size=b,
                                rank=1, max_iters=T, seed=5, precision="fp64", precond="exact",
                                accel=accel)
    h.close()
    assert np.all(tr["eta"] == 1.0) and np.allclose(info["eta"], 1.0, rtol=1e-12)
    delta = knorm_diff(X, Wg, Wo, Y, OK.MATERN32, ell, lam)
    assert delta <= 1e-6, delta


def test_exact_projection_with_full_block_solves_in_one_step(lib):
    n, k, lam = 160, 3, 0.02
    X, Y = inputs.make_small(92, n, 4, k)
    Wg, rep, tr, h = _gpu_solve(lib, X, Y, kernel="rbf", lengthscale=1.1, lam=lam, block_size=n,
                                rank=1, max_iters=1, seed=1, precision="fp64", precond="exact",
                                accel=0)
    rr, _ = h.residual(dev(Wg))
    h.close()
    assert rr < 1e-11, rr
    assert OL.relres(X, Y, Wg, OK.RBF, 1.1, lam)[0] < 1e-11


@pytest.mark.parametrize("precision", ["fp32"])
def test_exact_projection_reduced_precision(lib, precision):
    # the factor is float64 from the float32 coordinates; Step I runs at the handle's precision
    # (MIXED is rejected for this preconditioner: measured delta 1.1e-3 after 10 SAP steps)
    n, d, k, lam, ell, b, T = 900, 5, 2, 0.05, 1.2, 150, 10
    X, Y = inputs.make_small(93, n, d, k)
    X, Y = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    Wo, _ = OA.adasap(X, Y, OK.RBF, ell, lam, b, 1, T, 2, precond="sap")
    Wg, rep, tr, h = _gpu_solve(lib, X, Y, dtype=torch.float32, kernel="rbf", lengthscale=ell,
                                lam=lam, block_size=b, rank=1, max_iters=T, seed=2,
                                precision=precision, precond="exact", accel=0)
    h.close()
    assert knorm_diff(X, Wg, Wo, Y, OK.RBF, ell, lam) <= 1e-3
