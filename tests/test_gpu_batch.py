"""Batched uneven solves: each problem of a batch must match the float64 oracle's solve of
that problem alone (same seed + p streams, float32 sketch epsilon) to relative residual
difference 1e-3, and the batch result must equal the library's own single-problem solves to
the same bound (a batch is a set of independent solves)."""
import numpy as np
import pytest

from oracle import adasap as OA
from oracle import kernels as OK
from oracle import linsys as OL
from paper_2505_13723_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [(1000, 3, 0.9), (1537, 8, 1.6), (2300, 9, 0.4), (700, 16, 2.0), (999, 4, 1.1), (1290, 11, 0.7)]


def _problems():
    Xs, Ys = [], []
    for p, (n, d, ell) in enumerate(SIZES):
        X, y = inputs.make_c4_problem(p, n, d, seed=7)
        Xs.append(X.astype(np.float32).astype(np.float64))
        Ys.append(y.astype(np.float32).astype(np.float64))
    return Xs, Ys


def _knorm_diff(X, W1, W2, y, ell, lam):
    E = W1 - W2
    return np.linalg.norm(OK.kernel_matmul(X, X, E, OK.RBF, ell) + lam * E) / np.linalg.norm(y)


@pytest.mark.parametrize("r", [32, 37, 80])
def test_batch_matches_oracle_and_single_solves(lib, r):
    # r = 37: an odd rank (the eigensolver's padded index); r = 80: more than 64 rows of
    # eigenvectors per problem (two workgroups of the batched accumulation)
    Xs, Ys = _problems()
    lam, b, T, seed = 2e-2, 256, 12, 40
    cfg = lib.config(kernel="rbf", lam=lam, block_size=b, rank=r, max_iters=T, seed=seed,
                     precision="fp32", tol=1e-9)
    Xd = [torch.as_tensor(X, dtype=torch.float32).cuda() for X in Xs]
    Yd = [torch.as_tensor(y, dtype=torch.float32).cuda() for y in Ys]
    Wd = [torch.zeros_like(y) for y in Yd]
    reps = lib.solve_batch(cfg, Xd, Yd, Wd, [s[2] for s in SIZES])
    for p, (n, d, ell) in enumerate(SIZES):
        Wb = Wd[p].cpu().double().numpy()
        Wo, info = OA.adasap(Xs[p], Ys[p], OK.RBF, ell, lam, b, r, T, seed + p, eps_sketch=2.0**-23)
        delta = _knorm_diff(Xs[p], Wb, Wo, Ys[p], ell, lam)
        assert delta <= 1e-3, (p, delta)
        assert reps[p]["eta_last"] == pytest.approx(info["eta"][-1], rel=1e-3)
        ro = OL.relres(Xs[p], Ys[p], Wb, OK.RBF, ell, lam)[0]
        assert reps[p]["relres"] == pytest.approx(ro, rel=1e-3)
        # the same problem alone through the single-problem entry point
        h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=b, rank=r,
                                  max_iters=T, seed=seed + p, precision="fp32"), Xd[p], Yd[p])
        Ws = torch.zeros_like(Yd[p])
        h.solve(Ws)
        assert _knorm_diff(Xs[p], Wb, Ws.cpu().double().numpy(), Ys[p], ell, lam) <= 1e-3


def test_batch_with_fewer_work_items_than_xcds(lib):
    # one problem of 300 points: a single Step-I work item, so seven of the eight per-XCD
    # ranges of the persistent queue are empty; six rounds take the captured-graph path and
    # the Gaussian test matrices drawn one round ahead
    n, d, ell = 300, 5, 0.8
    X, y = inputs.make_c4_problem(3, n, d, seed=11)
    X = X.astype(np.float32).astype(np.float64)
    y = y.astype(np.float32).astype(np.float64)
    lam, b, r, T, seed = 2e-2, 64, 16, 6, 9
    cfg = lib.config(kernel="rbf", lam=lam, block_size=b, rank=r, max_iters=T, seed=seed,
                     precision="fp32", tol=1e-9)
    Xd = [torch.as_tensor(X, dtype=torch.float32).cuda()]
    Yd = [torch.as_tensor(y, dtype=torch.float32).cuda()]
    Wd = [torch.zeros_like(Yd[0])]
    reps = lib.solve_batch(cfg, Xd, Yd, Wd, [ell])
    Wb = Wd[0].cpu().double().numpy()
    Wo, info = OA.adasap(X, y, OK.RBF, ell, lam, b, r, T, seed, eps_sketch=2.0**-23)
    assert _knorm_diff(X, Wb, Wo, y, ell, lam) <= 1e-3
    assert reps[0]["eta_last"] == pytest.approx(info["eta"][-1], rel=1e-3)


@pytest.mark.parametrize("kind", ["matern12", "matern32", "matern52"])
def test_batch_matern_kernels_match_oracle(lib, kind):
    # the batched Step-I queue, sketches and powering products with each Matern kernel
    # (square root and exponential per pair), three uneven problems
    sizes = [(900, 4, 0.9), (1300, 10, 1.4), (700, 15, 2.0)]
    okind = {"matern12": OK.MATERN12, "matern32": OK.MATERN32, "matern52": OK.MATERN52}[kind]
    lam, b, r, T, seed = 2e-2, 128, 24, 5, 21
    Xs, Ys = [], []
    for p, (n, d, ell) in enumerate(sizes):
        X, y = inputs.make_c4_problem(10 + p, n, d, seed=13)
        Xs.append(X.astype(np.float32).astype(np.float64))
        Ys.append(y.astype(np.float32).astype(np.float64))
    cfg = lib.config(kernel=kind, lam=lam, block_size=b, rank=r, max_iters=T, seed=seed,
                     precision="fp32", tol=1e-9)
    Xd = [torch.as_tensor(X, dtype=torch.float32).cuda() for X in Xs]
    Yd = [torch.as_tensor(y, dtype=torch.float32).cuda() for y in Ys]
    Wd = [torch.zeros_like(y) for y in Yd]
    reps = lib.solve_batch(cfg, Xd, Yd, Wd, [s[2] for s in sizes])
    for p, (n, d, ell) in enumerate(sizes):
        Wb = Wd[p].cpu().double().numpy()
        Wo, info = OA.adasap(Xs[p], Ys[p], okind, ell, lam, b, r, T, seed + p, eps_sketch=2.0**-23)
        E = Wb - Wo
        delta = np.linalg.norm(OK.kernel_matmul(Xs[p], Xs[p], E, okind, ell) + lam * E) / np.linalg.norm(Ys[p])
        assert delta <= 1e-3, (kind, p, delta)
        assert reps[p]["eta_last"] == pytest.approx(info["eta"][-1], rel=1e-3)


def test_batch_rejects_bad_problems(lib):
    Xs, Ys = _problems()
    from paper_2505_13723_amd.binding import AdasapError
    Xd = [torch.as_tensor(Xs[0], dtype=torch.float32).cuda()]
    Yd = [torch.as_tensor(Ys[0], dtype=torch.float32).cuda()]
    Wd = [torch.zeros_like(Yd[0])]
    with pytest.raises(AdasapError):  # n < b
        lib.solve_batch(lib.config(block_size=5000, rank=16, precision="fp32"), Xd, Yd, Wd, [1.0])
    with pytest.raises(AdasapError):  # float64 precision is not batched
        lib.solve_batch(lib.config(block_size=100, rank=16, precision="fp64"), Xd, Yd, Wd, [1.0])


@pytest.mark.timeout(600)
def test_batch_of_32_benchmark_problems_matches_oracle(lib):
    # 32 problems of the 256-problem benchmark batch spanning its sizes (n from ~2,000 to
    # ~65,000, d from 4 to 16, lengthscales 0.2 to 2), three rounds from W_0 = 0 with the
    # benchmark's b = 1024, r = 64; each problem against the touched-rows oracle
    from oracle import adasap as OA2
    from support_delta import delta_support
    w = inputs.WORKLOADS["c4_batched_256"]
    ns, ds, ells = inputs.c4_problem_sizes(seed=w["seed"], count=w["count"], nmin=w["nmin"],
                                           nmax=w["nmax"], dmin=w["dmin"], dmax=w["dmax"],
                                           ellmin=w["ellmin"], ellmax=w["ellmax"])
    pick = np.argsort(ns)[::8]
    assert ns[pick].min() < 2500 and ns[pick].max() > 50000 and len(pick) == 32
    lam, b, r, T, seed = w["lam"], w["b"], w["r"], 3, 17
    Xs, Ys = [], []
    for p in pick:
        X, y = inputs.make_c4_problem(int(p), int(ns[p]), int(ds[p]), seed=w["seed"])
        Xs.append(X.astype(np.float32).astype(np.float64))
        Ys.append(y.astype(np.float32).astype(np.float64)[:, None])
    Xd = [torch.as_tensor(X, dtype=torch.float32).cuda() for X in Xs]
    Yd = [torch.as_tensor(y, dtype=torch.float32).cuda() for y in Ys]
    Wd = [torch.zeros_like(y) for y in Yd]
    cfg = lib.config(kernel="rbf", lam=lam, block_size=b, rank=r, max_iters=T, seed=seed,
                     precision="fp32")
    lib.solve_batch(cfg, Xd, Yd, Wd, [float(ells[p]) for p in pick])
    worst = 0.0
    for j, p in enumerate(pick):
        S, WS, info = OA2.adasap_from_zero(Xs[j], Ys[j], OK.RBF, float(ells[p]), lam, b, r, T,
                                           seed + j, eps_sketch=2.0 ** -23)
        Wg = Wd[j].cpu().double().numpy()
        outside = np.ones(Xs[j].shape[0], dtype=bool)
        outside[S] = False
        assert not np.any(Wg[outside])
        d = delta_support(Xs[j], Ys[j], S, Wg[S] - WS, OK.RBF, float(ells[p]), lam, 4096, j)
        worst = max(worst, d)
        assert d <= 1e-3, (int(p), int(ns[p]), int(ds[p]), d)
    print("32 batched problems: worst delta %.3e" % worst, flush=True)


def test_autotuner_choice_is_cached_and_reproducible(lib):
    # the first batch of these shapes times every tile shape; a second batch of the same shapes
    # takes the cached choice and, with the same seed, reproduces the first result bit for bit
    Xs, Ys = _problems()
    cfg = lib.config(kernel="rbf", lam=2e-2, block_size=256, rank=32, max_iters=6, seed=91,
                     precision="fp32")
    Xd = [torch.as_tensor(X, dtype=torch.float32).cuda() for X in Xs]
    Yd = [torch.as_tensor(y, dtype=torch.float32).cuda() for y in Ys]
    ells = [s[2] for s in SIZES]
    runs = []
    for _ in range(2):
        Wd = [torch.zeros_like(y) for y in Yd]
        reps = lib.solve_batch(cfg, Xd, Yd, Wd, ells)
        runs.append(([W.cpu() for W in Wd], reps[0]))
    (W1, r1), (W2, r2) = runs
    assert r1["tuned_rows_per_wg"] in (128, 256) and r1["tuned_wg_per_cu"] in (2, 4)
    assert r1["reserved"] in (16, 32, 64, 128)
    assert r2["tuned_from_cache"] == 1
    assert (r2["tuned_rows_per_wg"], r2["tuned_wg_per_cu"], r2["reserved"]) == \
        (r1["tuned_rows_per_wg"], r1["tuned_wg_per_cu"], r1["reserved"])
    for a, b in zip(W1, W2):
        assert torch.equal(a, b)
