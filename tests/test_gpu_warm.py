"""Parity of the learned warm start (features, ridge mean, gradients, Adam training,
prediction) against the float64 oracle, and the gain of the trained network over a cold
start on a problem drawn from the same field as its training windows.

Tolerances.  The GPU computes in float32 (cosine arguments, network layers) with float64
Gram accumulation and Cholesky for the ridge weights.  Cosines of arguments of size ~40
carry ~2e-5 absolute error; the ridge mean inherits that through a well-posed solve
(lambda = 1); network outputs and gradients are float32 sums of a few hundred terms
(relative ~1e-6 per layer).  The bounds below leave an order of magnitude of margin.
"""
import math

import numpy as np
import pytest

from oracle import mlp as OM
from oracle import rff as OF
from paper_2505_13723_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


def make_ws(lib, d, D, H, lam, seed=1):
    cfg = lib.ws_config(d=d, D=D, hidden=H, lam=lam)
    Wf, c = inputs.ws_rff(seed, d, 0.3, D)
    p0 = inputs.ws_init_params(seed + 1, [D + 2, H, H, H, 1])
    return lib.warm_start(cfg, Wf, c, p0), f32(Wf), f32(c), f32(p0)


@pytest.mark.parametrize("n,D", [(1000, 64), (40000, 512)])
def test_features_and_ridge_mean_match_oracle(lib, n, D):
    d, lam = 9, 1.0
    ws, Wf, c, _ = make_ws(lib, d, D, 32, lam)
    rs = np.random.default_rng(n)
    X = f32(rs.uniform(0, 0.5, (n, d)))
    y = f32(rs.standard_normal(n))
    A, theta = ws.features(dev(X), dev(y))
    A = A.cpu().double().numpy()
    ref = OF.network_inputs(X, y, Wf, c, lam)
    assert np.max(np.abs(A[:, :D] - ref[:, :D])) < 1e-4
    assert np.array_equal(A[:, D], y)
    m, mo = A[:, D + 1], ref[:, D + 1]
    assert np.linalg.norm(m - mo) <= 2e-3 * np.linalg.norm(mo)
    assert np.max(np.abs(m - mo)) <= 2e-3 * np.max(np.abs(mo)) + 1e-5
    ws.close()


@pytest.mark.parametrize("D,H,m", [(30, 20, 257), (512, 256, 1024), (100, 200, 65)])
def test_loss_gradient_matches_oracle(lib, D, H, m):
    ws, _, _, p0 = make_ws(lib, 4, D, H, 0.5, seed=D + H)
    rs = np.random.default_rng(m)
    A = f32(rs.standard_normal((m, D + 2)))
    t = f32(rs.standard_normal(m))
    loss, g = ws.loss_grad(dev(A), dev(t))
    g = g.cpu().double().numpy()
    lo, go = OM.loss_and_grad(p0, [D + 2, H, H, H, 1], A, t)
    assert loss == pytest.approx(lo, rel=1e-5)
    off = 0
    for o, i in OM.layer_shapes([D + 2, H, H, H, 1]):
        for size in (o * i, o):  # weights, then biases
            seg, ref = g[off:off + size], go[off:off + size]
            off += size
            assert np.linalg.norm(seg - ref) <= 1e-4 * np.linalg.norm(ref) + 1e-9, (o, i, size)
            assert np.max(np.abs(seg - ref)) <= 1e-4 * np.max(np.abs(ref)) + 1e-9
    ws.close()


def test_training_matches_oracle(lib):
    D, H, d = 16, 12, 3
    ws, Wf, c, p0 = make_ws(lib, d, D, H, 0.5, seed=3)
    rs = np.random.default_rng(4)
    n = 300  # batches of 64: four full ones and a ragged one of 44
    X = f32(rs.uniform(0, 1, (n, d)))
    y = f32(np.sin(3 * X).sum(axis=1) + 0.1 * rs.standard_normal(n))
    W = f32(rs.standard_normal(n) * 0.3)
    ws.add_problem(dev(X), dev(y), dev(W))
    assert ws.train_rows() == n
    losses = ws.train(epochs=3, batch=64, lr=1e-2, seed=9)
    A = OF.network_inputs(X, y, Wf, c, 0.5)
    t = y - 0.5 * W
    po, lo = OM.train(p0, [D + 2, H, H, H, 1], A, t, epochs=3, batch=64, lr=1e-2, seed=9)
    assert np.allclose(losses, lo, rtol=1e-3)
    p = ws.params().cpu().double().numpy()
    assert np.max(np.abs(p - po)) < 2e-3
    ws.close()


def test_predict_and_initial_iterate_match_oracle(lib):
    D, H, d, lam, n = 512, 256, 9, 1.0, 40000
    ws, Wf, c, p0 = make_ws(lib, d, D, H, lam, seed=5)
    rs = np.random.default_rng(6)
    X = f32(rs.uniform(0, 0.5, (n, d)))
    y = f32(rs.standard_normal(n))
    mh = ws.predict_mean(dev(X), dev(y)).cpu().double().numpy()
    ref, _ = OM.forward(p0, [D + 2, H, H, H, 1], OF.network_inputs(X, y, Wf, c, lam))
    assert np.max(np.abs(mh - ref)) <= 2e-3 * np.max(np.abs(ref)) + 1e-5
    W0 = ws.initial_iterate(dev(X), dev(y)).cpu().double().numpy()
    assert np.allclose(W0, (y - mh) / lam, rtol=1e-5, atol=1e-5)
    ws.close()


def test_rejects_bad_arguments(lib):
    from paper_2505_13723_amd.binding import AdasapError

    ws, _, _, _ = make_ws(lib, 3, 8, 4, 1.0)
    with pytest.raises(AdasapError):
        ws.train(epochs=1, batch=16, lr=1e-3, seed=0)  # empty training set
    with pytest.raises(AdasapError):
        ws.train(epochs=1, batch=0, lr=1e-3, seed=0)
    ws.close()


@pytest.mark.slow
def test_trained_network_beats_cold_start(lib):
    """Windows of one GP field (at the density of 1e8 points in the unit cube) are solved by
    the batched solver; the network trained on them warm-starts a larger problem of the same
    field.  Noise variance lambda = 1 (the regime where m^ can be accurate enough: the
    initial error is (m - m^) / lambda)."""
    w = inputs.WORKLOADS["ws_rbf_d9"]
    d, ell, lam, D, H = w["d"], w["ell"], 1.0, w["D"], w["H"]
    field = inputs.ws_field(w["seed"], d, ell, w["field_features"])
    outer = inputs.box_side(w["n_target"], w["density"], d)
    side = inputs.box_side(w["n_window"], w["density"], d)
    corners = inputs.ws_window_corners(w["seed"] + 1, w["windows"], d, outer, side)
    Xs, ys, Ws = [], [], []
    for p in range(w["windows"]):
        X, y = inputs.ws_points(field, w["n_window"], corners[p], side, lam, 100 + p, device="cuda")
        Xs.append(X.float().contiguous())
        ys.append(y.float().contiguous())
        Ws.append(torch.zeros(w["n_window"], dtype=torch.float32, device="cuda"))
    cfgb = lib.config(kernel="rbf", lam=lam, block_size=1024, rank=128, max_iters=480, seed=7,
                      precision="fp32", tol=1e-12)
    reps = lib.solve_batch(cfgb, Xs, [y.view(-1, 1) for y in ys], [W.view(-1, 1) for W in Ws],
                           [ell] * w["windows"])
    worst = max(r["relres"] for r in reps)
    print("training windows solved, worst relres %.2e" % worst, flush=True)
    assert worst < 1e-2
    cfg = lib.ws_config(d=d, D=D, hidden=H, lam=lam)
    Wf, c = inputs.ws_rff(w["seed"] + 2, d, ell, D)
    ws = lib.warm_start(cfg, Wf, c, inputs.ws_init_params(w["seed"] + 3, [D + 2, H, H, H, 1]))
    for p in range(w["windows"]):
        ws.add_problem(Xs[p], ys[p], Ws[p])
    losses = ws.train(epochs=12, batch=512, lr=1e-3, seed=11)
    print("training losses", np.round(losses, 5), flush=True)
    assert losses[-1] < 0.5 * losses[0]
    # the target problem: the whole box, fresh points of the same field
    X, y = inputs.ws_points(field, w["n_target"], np.zeros(d), outer, lam, 999, device="cuda")
    X, y = X.float().contiguous(), y.float().contiguous()
    W0 = ws.initial_iterate(X, y).view(-1, 1)
    Y = y.view(-1, 1)
    iters = 2 * w["n_target"] // w["b"]
    res = {}
    for name, start in (("cold", torch.zeros_like(Y)), ("warm", W0.clone())):
        h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=w["b"], rank=w["r"],
                                  max_iters=iters, seed=13, precision="fp32"), X, Y)
        r0 = h.residual(start)[0]
        h.solve(start)
        res[name] = (r0, h.residual(start)[0])
        h.close()
    print("relres (start, after %d iterations): %s" % (iters, res), flush=True)
    assert res["warm"][1] < 0.7 * res["cold"][1]
    ws.close()
