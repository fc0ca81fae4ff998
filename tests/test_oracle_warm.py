"""Pins of the warm-start oracle: random Fourier features, ridge mean, the MLP and Adam.

Each check compares against something other than the code under test: the kernel the
features approximate (Monte Carlo limit), the dual (kernel) form of the ridge mean,
library activations and autograd, central differences of the loss, closed-form
properties of Adam's first step, and uniformity of the minibatch permutation.
"""
import math

import numpy as np
import pytest
from scipy.special import expit

from oracle import kernels as OK
from oracle import mlp
from oracle import rff
from oracle import rng
from paper_2505_13723_amd import inputs


def test_features_approximate_the_rbf_kernel():
    d, ell, D = 5, 0.7, 200_000
    Wf, c = inputs.ws_rff(1, d, ell, D)
    X = np.random.default_rng(2).standard_normal((6, d)) * 0.5
    Phi = rff.features(X, Wf, c)
    approx = Phi @ Phi.T
    exact = OK.kernel_matrix(X, X, OK.RBF, ell)
    # each entry is a mean of D bounded terms of variance <= 2
    assert np.max(np.abs(approx - exact)) < 5 * math.sqrt(2.0 / D)
    assert np.max(np.abs(approx - exact)) > 0  # a finite sample, not the kernel itself


def test_ridge_mean_equals_dual_form():
    n, d, D, lam = 300, 4, 64, 0.3
    rs = np.random.default_rng(3)
    X = rs.uniform(size=(n, d))
    y = rs.standard_normal(n)
    Wf, c = inputs.ws_rff(4, d, 0.5, D)
    m, theta = rff.ridge_mean(X, y, Wf, c, lam)
    Phi = rff.features(X, Wf, c)
    # Phi (Phi^T Phi + lam I)^-1 Phi^T y = Phi Phi^T (Phi Phi^T + lam I)^-1 y
    Kf = Phi @ Phi.T
    dual = Kf @ np.linalg.solve(Kf + lam * np.eye(n), y)
    assert np.allclose(m, dual, rtol=1e-9, atol=1e-11)
    # and theta solves the regularised normal equations
    assert np.allclose(Phi.T @ (Phi @ theta - y) + lam * theta, 0, atol=1e-10)


def test_network_inputs_layout():
    n, d, D, lam = 50, 3, 16, 0.1
    rs = np.random.default_rng(5)
    X, y = rs.uniform(size=(n, d)), rs.standard_normal(n)
    Wf, c = inputs.ws_rff(6, d, 0.4, D)
    A = rff.network_inputs(X, y, Wf, c, lam)
    assert A.shape == (n, D + 2)
    assert np.allclose(A[:, :D], np.cos(X @ Wf.T + c))
    assert np.array_equal(A[:, D], y)
    assert np.allclose(A[:, D + 1], rff.ridge_mean(X, y, Wf, c, lam)[0])


def test_silu_and_its_derivative():
    z = np.linspace(-30, 30, 2001)
    assert np.allclose(mlp.silu(z), z * expit(z), rtol=1e-14, atol=1e-300)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.allclose(mlp.silu_grad(z), fd, atol=1e-8)


SIZES = [7, 6, 5, 4, 1]


def _problem(seed, m=9):
    rs = np.random.default_rng(seed)
    p = inputs.ws_init_params(seed, SIZES) + 0.1 * rs.standard_normal(mlp.param_count(SIZES))
    return p, rs.standard_normal((m, SIZES[0])), rs.standard_normal(m)


def test_forward_matches_torch_modules():
    torch = pytest.importorskip("torch")
    p, A, _ = _problem(7)
    mods = []
    for li, (W, b) in enumerate(mlp.unpack(p, SIZES)):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.as_tensor(W))
            lin.bias.copy_(torch.as_tensor(b))
        mods.append(lin)
        if li < len(SIZES) - 2:
            mods.append(torch.nn.SiLU())
    net = torch.nn.Sequential(*mods)
    ref = net(torch.as_tensor(A)).detach().numpy()[:, 0]
    out, _ = mlp.forward(p, SIZES, A)
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-14)


def _fd_grad(p, A, t, h=1e-6):
    g = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        g[i] = (mlp.mse(mlp.forward(p + e, SIZES, A)[0], t) - mlp.mse(mlp.forward(p - e, SIZES, A)[0], t)) / (2 * h)
    return g


def test_gradient_matches_central_differences():
    p, A, t = _problem(8)
    loss, g = mlp.loss_and_grad(p, SIZES, A, t)
    assert loss == pytest.approx(mlp.mse(mlp.forward(p, SIZES, A)[0], t))
    fd = _fd_grad(p, A, t)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_gradient_matches_autograd():
    torch = pytest.importorskip("torch")
    p, A, t = _problem(9)
    pt = torch.as_tensor(p).requires_grad_(True)
    act = torch.as_tensor(A)
    off = 0
    shapes = mlp.layer_shapes(SIZES)
    for li, (o, i) in enumerate(shapes):
        W = pt[off:off + o * i].view(o, i)
        off += o * i
        b = pt[off:off + o]
        off += o
        act = act @ W.T + b
        if li < len(shapes) - 1:
            act = torch.nn.functional.silu(act)
    loss = ((act[:, 0] - torch.as_tensor(t)) ** 2).mean()
    loss.backward()
    _, g = mlp.loss_and_grad(p, SIZES, A, t)
    assert np.allclose(g, pt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_planted_activation_derivative_error_is_caught(monkeypatch):
    p, A, t = _problem(10)
    monkeypatch.setattr(mlp, "silu_grad", lambda z: mlp.sigmoid(z))  # drops the z s (1 - s) term
    _, g = mlp.loss_and_grad(p, SIZES, A, t)
    monkeypatch.undo()
    assert not np.allclose(g, _fd_grad(p, A, t), rtol=1e-4, atol=1e-6)


def test_adam_first_step_is_a_signed_lr_step():
    g = np.array([3.0, -1e-3, 0.5, -20.0])
    opt = mlp.Adam(4, lr=0.01, eps=1e-12)
    p1 = opt.step(np.zeros(4), g)
    # bias correction makes the first moments exactly g and g^2
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=1e-9)


def test_adam_minimises_a_quadratic():
    rs = np.random.default_rng(11)
    c = rs.standard_normal(5)
    opt = mlp.Adam(5, lr=0.05)
    p = np.zeros(5)
    for _ in range(2000):
        p = opt.step(p, 2 * (p - c))
    assert np.allclose(p, c, atol=1e-3)


def test_permutation_is_uniform():
    seen = {}
    draws = 2400
    for t in range(draws):
        perm = rng.permutation(12, rng.PURPOSE_MINIBATCH, t, 4)
        assert sorted(perm.tolist()) == [0, 1, 2, 3]
        seen[tuple(perm)] = seen.get(tuple(perm), 0) + 1
    assert len(seen) == 24
    expected = draws / 24
    chi2 = sum((v - expected) ** 2 / expected for v in seen.values())
    assert chi2 < 49.7  # 23 degrees of freedom, p = 0.001


def test_training_fits_a_smooth_target():
    rs = np.random.default_rng(13)
    sizes = [3, 16, 16, 16, 1]
    A = rs.uniform(-1, 1, (256, 3))
    t = np.sin(A[:, 0]) + 0.5 * A[:, 1] * A[:, 2]
    p0 = inputs.ws_init_params(14, sizes)
    p, losses = mlp.train(p0, sizes, A, t, epochs=60, batch=32, lr=3e-3, seed=15)
    assert losses[-1] < 0.05 * losses[0]
    assert mlp.mse(mlp.forward(p, sizes, A)[0], t) < 0.05 * np.var(t)
