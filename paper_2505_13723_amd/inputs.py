"""Seeded synthetic inputs shaped like the paper's workloads (no solver arithmetic here).

This module only draws data: the feature matrix X and the right-hand sides Y
of (K + lambda I) W = Y, plus the hyperparameters of each workload.  It is the
one module that both the HIP path's tests/benchmark and the CPU oracle's
tests use, so it holds none of the method's arithmetic.  The paper's
datasets (UCI/OpenML/sGDML benchmarks, NYC taxi) are not available; these
synthetic stand-ins take their shapes (n, d, kernel, lambda, b, r).

Targets are GP prior draws f(X) plus Gaussian noise of variance lambda,
with f approximated by random Fourier features (the construction Sec. 2.1
uses for pathwise conditioning): phi(x) = sqrt(2/D) cos(W x + c), f = phi^T
theta, theta ~ N(0, I); for RBF the frequencies are N(0, ell^-2 I), for
Matern-nu they are multivariate Student-t with 2 nu degrees of freedom
scaled by 1/ell.
"""
import math

import numpy as np

WORKLOADS = {
    # small FP64 case the oracle finishes in seconds
    "c1_fp64_n4096": dict(n=4096, d=8, kernel="rbf", ell=1.0, lam=1e-2, b=256, r=64,
                          rho_rule=1, rho=1e-2, iters=200, k=1, precision="fp64", seed=1),
    # ill-conditioned Matern-3/2, FP32 kernel tiles
    "c2_matern32_n1m": dict(n=1_000_000, d=11, kernel="matern32", ell=0.3, lam=1e-3, b=8192,
                            r=100, rho_rule=0, k=1, precision="fp32", seed=2),
    # 64 right-hand sides, reduced-precision kernel blocks + FP64 refinement
    "c3_rbf_n2m_k64": dict(n=2_000_000, d=11, kernel="rbf", ell=0.5, lam=1e-2, b=16384,
                           r=128, rho_rule=0, k=64, precision="mixed", seed=3),
    # 256 batched uneven problems
    "c4_batched_256": dict(count=256, nmin=2000, nmax=65536, dmin=4, dmax=16, ellmin=0.2,
                           ellmax=2.0, kernel="rbf", lam=1e-2, b=1024, r=64, rho_rule=0,
                           k=1, precision="fp32", seed=4),
    # learned warm start target problem
    "c5_rbf_n100m": dict(n=100_000_000, d=9, kernel="rbf", ell=0.1, lam=1e-2, b=32768, r=128,
                         rho_rule=0, k=1, precision="fp32", seed=5),
    # warm-start training windows and target drawn from one field at the point density of
    # 1e8 points in the unit cube (d = 9, RBF ell = 0.1); network D = 512 cosines,
    # three hidden layers of 256
    "ws_rbf_d9": dict(d=9, ell=0.1, density=1e8, field_features=5000, D=512, H=256,
                      windows=32, n_window=8192, n_target=65536, b=4096, r=128, seed=6),
}


def _torch():
    import torch
    return torch


def rff_frequencies(rs, kernel, ell, d, D):
    """(D x d) frequencies and (D,) phases of the kernel's spectral measure."""
    Z = rs.standard_normal((D, d))
    if kernel == "rbf":
        Wf = Z / ell
    elif kernel.startswith("matern"):
        nu = {"matern12": 0.5, "matern32": 1.5, "matern52": 2.5}[kernel]
        chi = rs.chisquare(2.0 * nu, size=(D, 1))
        Wf = Z * np.sqrt(2.0 * nu / chi) / ell
    else:
        raise ValueError(kernel)
    c = rs.uniform(0.0, 2.0 * math.pi, size=D)
    return Wf, c


def rff_prior_params(kernel, ell, d, D, nsamples, rs):
    """Frequencies, phases and weights of nsamples random-feature prior functions."""
    Wf, c = rff_frequencies(rs, kernel, ell, d, D)
    theta = rs.standard_normal((D, nsamples))
    return Wf, c, theta


def rff_eval(X, params, chunk=1 << 16):
    """The prior functions of rff_prior_params at the rows of X (torch, any device), float64."""
    torch = _torch()
    Wf, c, theta = params
    n = X.shape[0]
    dev = X.device
    Wt = torch.as_tensor(Wf, dtype=torch.float64, device=dev)
    ct = torch.as_tensor(c, dtype=torch.float64, device=dev)
    th = torch.as_tensor(theta, dtype=torch.float64, device=dev)
    out = torch.empty((n, theta.shape[1]), dtype=torch.float64, device=dev)
    scale = math.sqrt(2.0 / Wf.shape[0])
    for i0 in range(0, n, chunk):
        xb = X[i0:i0 + chunk].to(torch.float64)
        out[i0:i0 + chunk] = (torch.cos(xb @ Wt.T + ct) * scale) @ th
    return out


def rff_prior_draws(X, kernel, ell, D, nsamples, rs, chunk=1 << 16):
    """nsamples prior function draws at the rows of X (torch tensor, any device), float64."""
    params = rff_prior_params(kernel, ell, X.shape[1], D, nsamples, rs)
    return rff_eval(X, params, chunk)


def make_c1(seed=1, n=4096, d=8):
    """X ~ N(0, I_d); y = sum_j sin(x_j) + 0.1 xi (float64 numpy)."""
    rs = np.random.default_rng(seed)
    X = rs.standard_normal((n, d))
    y = np.sin(X).sum(axis=1) + 0.1 * rs.standard_normal(n)
    return X, y


def make_c2(seed=2, n=1_000_000, d=11, ell=0.3, lam=1e-3, n_dup_centres=500, copies=100,
            device="cpu", dtype=None):
    """Uniform [0,1]^d with 5% clustered near-duplicates; Matern-3/2 prior target."""
    torch = _torch()
    rs = np.random.default_rng(seed)
    n_dup = n_dup_centres * copies
    n_base = n - n_dup
    Xb = rs.uniform(0.0, 1.0, (n_base, d))
    centres = Xb[rs.choice(n_base, n_dup_centres, replace=False)]
    Xd = np.repeat(centres, copies, axis=0) + 1e-6 * rs.standard_normal((n_dup, d))
    X = np.concatenate([Xb, Xd])[rs.permutation(n)]
    Xt = torch.as_tensor(X, dtype=torch.float64, device=device)
    f = rff_prior_draws(Xt, "matern32", ell, 2048, 1, rs)[:, 0]
    y = f + math.sqrt(lam) * torch.as_tensor(rs.standard_normal(n), device=device)
    dt = dtype or torch.float32
    return Xt.to(dt), y.to(dt)


def make_c3(seed=3, n=2_000_000, d=11, k=64, ell=0.5, lam=1e-2, device="cpu", dtype=None,
            n_test=0):
    """X ~ N(0, I_d); column 0 standardised y = f*(X) + eps, columns 1.. are
    pathwise right-hand sides f_s(X) + eps_s (RBF prior, 2048 features).

    With n_test > 0 also returns a held-out split drawn from the same functions:
    (X, Y, Xtest, ytest, prior_test) with ytest = f*(Xtest) + eps standardised like y and
    prior_test = f_s(Xtest) for s = 1 .. k-1 (the prior functions of the pathwise columns)."""
    torch = _torch()
    rs = np.random.default_rng(seed)
    X = torch.as_tensor(rs.standard_normal((n, d)), device=device)
    params = rff_prior_params("rbf", ell, d, 2048, k, rs)
    F = rff_eval(X, params)
    eps = torch.as_tensor(rs.standard_normal((n, k)), device=device) * math.sqrt(lam)
    Y = F + eps
    y0 = Y[:, 0]
    mu, sd = y0.mean(), y0.std()
    Y[:, 0] = (y0 - mu) / sd
    dt = dtype or torch.float32
    if n_test <= 0:
        return X.to(dt), Y.to(dt)
    rt = np.random.default_rng(seed + 7777)
    Xt = torch.as_tensor(rt.standard_normal((n_test, d)), device=device)
    Ft = rff_eval(Xt, params)
    yt = (Ft[:, 0] + math.sqrt(lam) * torch.as_tensor(rt.standard_normal(n_test), device=device)
          - mu) / sd
    return X.to(dt), Y.to(dt), Xt.to(dt), yt.to(dt), Ft[:, 1:].contiguous().to(dt)


def c4_problem_sizes(seed=4, count=256, nmin=2000, nmax=65536, dmin=4, dmax=16,
                     ellmin=0.2, ellmax=2.0):
    """(n_p, d_p, ell_p) for each batched problem."""
    rs = np.random.default_rng(seed)
    ns = np.rint(np.exp(rs.uniform(math.log(nmin), math.log(nmax), count))).astype(np.int64)
    ds = rs.integers(dmin, dmax + 1, count)
    ells = rs.uniform(ellmin, ellmax, count)
    return ns, ds, ells


def make_c4_problem(p, n, d, seed=4):
    """Problem p of the batch: X ~ N(0, I_d), y = sum_j sin(x_j) + 0.1 xi."""
    rs = np.random.default_rng(1000 * seed + p)
    X = rs.standard_normal((n, d))
    y = np.sin(X).sum(axis=1) + 0.1 * rs.standard_normal(n)
    return X, y


def make_c5(seed=5, n=100_000_000, d=9, ell=0.1, lam=1e-2, device="cpu", chunk=1 << 22):
    """X ~ U[0,1]^d (float32), y = f(X) + eps with a 5000-feature RBF prior draw."""
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    X = torch.rand((n, d), generator=g, device=device, dtype=torch.float32)
    rs = np.random.default_rng(seed)
    y = torch.empty(n, dtype=torch.float32, device=device)
    Wf, c = rff_frequencies(rs, "rbf", ell, d, 5000)
    theta = rs.standard_normal(5000)
    Wt = torch.as_tensor(Wf, dtype=torch.float32, device=device)
    ct = torch.as_tensor(c, dtype=torch.float32, device=device)
    th = torch.as_tensor(theta, dtype=torch.float32, device=device)
    scale = math.sqrt(2.0 / 5000)
    for i0 in range(0, n, chunk):
        phi = torch.cos(X[i0:i0 + chunk] @ Wt.T + ct) * scale
        y[i0:i0 + chunk] = phi @ th
    y += math.sqrt(lam) * torch.randn(n, generator=g, device=device, dtype=torch.float32)
    return X, y


def make_small(seed, n, d, k=1, dist="normal", noise=0.1):
    """Small generic problem for parity tests: X (n x d), Y (n x k), float64 numpy."""
    rs = np.random.default_rng(seed)
    X = rs.standard_normal((n, d)) if dist == "normal" else rs.uniform(0, 1, (n, d))
    Y = np.sin(X).sum(axis=1, keepdims=True) + noise * rs.standard_normal((n, k))
    return X, Y


def box_side(n, density, d):
    """Side of the cube that holds n points at the given density."""
    return (n / density) ** (1.0 / d)


def ws_field(seed, d, ell, features=5000):
    """One RBF prior draw f(x) = sqrt(2/F) sum_j theta_j cos(omega_j . x + c_j), as
    (frequencies F x d, phases F, theta F)."""
    rs = np.random.default_rng(seed)
    Wf, c = rff_frequencies(rs, "rbf", ell, d, features)
    return Wf, c, rs.standard_normal(features)


def ws_points(field, n, lo, side, noise_var, seed, device="cpu", chunk=1 << 15):
    """n points uniform in the cube [lo, lo + side]^d and y = f(x) + N(0, noise_var),
    as float64 torch tensors on `device`."""
    torch = _torch()
    Wf, c, theta = field
    rs = np.random.default_rng(seed)
    d = Wf.shape[1]
    X = torch.as_tensor(np.asarray(lo) + side * rs.uniform(0.0, 1.0, (n, d)), device=device)
    Wt = torch.as_tensor(Wf, device=device)
    ct = torch.as_tensor(c, device=device)
    th = torch.as_tensor(theta, device=device)
    y = torch.empty(n, dtype=torch.float64, device=device)
    for i0 in range(0, n, chunk):
        y[i0:i0 + chunk] = torch.cos(X[i0:i0 + chunk] @ Wt.T + ct) @ th
    y *= math.sqrt(2.0 / Wf.shape[0])
    y += math.sqrt(noise_var) * torch.as_tensor(rs.standard_normal(n), device=device)
    return X, y


def ws_window_corners(seed, count, d, outer, side):
    """Lower corners of `count` windows of the given side inside [0, outer]^d."""
    rs = np.random.default_rng(seed)
    return rs.uniform(0.0, max(0.0, outer - side), (count, d))


def ws_rff(seed, d, ell, D):
    """The network's D cosine frequencies (N(0, ell^-2 I)) and phases (U[0, 2 pi))."""
    return rff_frequencies(np.random.default_rng(seed), "rbf", ell, d, D)


def ws_init_params(seed, sizes):
    """Flat initial parameters of the dense layers sizes[0] -> ... -> sizes[-1]: weights
    uniform with variance 1/fan_in, biases zero; layer order W_l (out x in), b_l."""
    rs = np.random.default_rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        fan_in, fan_out = sizes[i], sizes[i + 1]
        a = math.sqrt(3.0 / fan_in)
        parts.append(rs.uniform(-a, a, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def bo_target(seed, d=8, ell=2.0, features=5000):
    """Black-box objective of the Bayesian-optimisation workload: one Matern-3/2 prior function
    on [0, 1]^d from `features` random features (evaluate with rff_eval)."""
    return rff_prior_params("matern32", ell, d, features, 1, np.random.default_rng(seed))


def bo_initial(seed, n0, d=8, noise=1e-6, target=None, device="cpu"):
    """n0 points uniform on [0, 1]^d and their noisy objective values (float64 torch)."""
    torch = _torch()
    rs = np.random.default_rng(seed)
    X = torch.as_tensor(rs.uniform(0.0, 1.0, (n0, d)), device=device)
    y = rff_eval(X, target)[:, 0] + math.sqrt(noise) * torch.as_tensor(rs.standard_normal(n0),
                                                                     device=device)
    return X, y
