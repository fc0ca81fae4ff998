"""Large-scale Bayesian optimisation with parallel Thompson sampling (Sec. 5.3).

The black box is a Matern-3/2 prior function on [0, 1]^d (random features); the model's
kernel matches it.  Each step acquires `acq` points: every acquired point maximises one
pathwise posterior sample over a candidate set, and the samples come from ADASAP solves with
the right-hand sides [y | f_s(X) + zeta_s] (the library's solve, posterior samples and
column argmax).  Random search with the same number of evaluations is the baseline; the
reported figure is the percentage improvement of the best objective value found over it.

Candidate points per batch: uniform draws on the cube plus Gaussian perturbations of the best
observed points, clipped to the cube (the paper maximises each sample by multi-start gradient
ascent from such points; a dense candidate set stands in for that maximiser here).
"""
import math
import time

import numpy as np

from . import inputs


def thompson_bo(lib, *, d=8, ell=2.0, noise=1e-6, n0=250_000, steps=10, acq=1000, batch=127,
                n_cand=50_000, n_local=10_000, passes=10, rank=100, precision="mixed", seed=0,
                log=None):
    """Run `steps` rounds of parallel Thompson sampling and the random-search baseline.

    Returns a dict with the best objective values per step of both methods, the improvement
    over random search (percent of |best random|) and the time spent in solves and sampling."""
    import torch

    dev = "cuda"
    target = inputs.bo_target(seed, d=d, ell=ell)
    X, y = inputs.bo_initial(seed + 1, n0, d=d, noise=noise, target=target, device=dev)
    fX = inputs.rff_eval(X, target)[:, 0]
    rs = np.random.default_rng(seed + 2)
    best_init = float(fX.max())
    best_ts, best_rs = [best_init], [best_init]
    best_rand = best_init
    t_solve = t_sample = 0.0
    iters_total = 0
    for step in range(steps):
        n = X.shape[0]
        b = max(1, n // 5)
        per_pass = int(math.ceil(n / b))
        new_pts = []
        for j0 in range(0, acq, batch):
            S = min(batch, acq - j0)
            prior = inputs.rff_prior_params("matern32", ell, d, 2048, S, rs)
            F = inputs.rff_eval(X, prior)
            zeta = math.sqrt(noise) * torch.as_tensor(rs.standard_normal((n, S)), device=dev)
            Y = torch.cat([y[:, None], F + zeta], dim=1).float().contiguous()
            Xf = X.float().contiguous()
            cfg = lib.config(kernel="matern32", lengthscale=ell, lam=noise, block_size=b,
                             rank=min(rank, b), max_iters=passes * per_pass,
                             seed=seed * 1000 + step * 16 + j0 // batch, precision=precision)
            h = lib.create(cfg, Xf, Y)
            W = torch.zeros_like(Y)
            t0 = time.perf_counter()
            rep = h.solve(W)
            torch.cuda.synchronize()
            t_solve += time.perf_counter() - t0
            iters_total += rep["iters"]
            # candidates: uniform points and perturbations of the best observed points
            top = torch.topk(y, min(10, n)).indices
            loc = X[top][torch.as_tensor(rs.integers(0, top.numel(), n_local), device=dev)]
            loc = (loc + 0.05 * torch.as_tensor(rs.standard_normal((n_local, d)), device=dev)).clamp(0, 1)
            cand = torch.cat([torch.as_tensor(rs.uniform(0, 1, (n_cand, d)), device=dev), loc])
            t0 = time.perf_counter()
            smp = h.posterior_samples(W, cand.float().contiguous(),
                                      inputs.rff_eval(cand, prior).float().contiguous())
            idx = lib.column_argmax(smp[:, 1:])
            torch.cuda.synchronize()
            t_sample += time.perf_counter() - t0
            h.close()
            new_pts.append(cand[idx])
        Xn = torch.cat(new_pts)
        fn = inputs.rff_eval(Xn, target)[:, 0]
        yn = fn + math.sqrt(noise) * torch.as_tensor(rs.standard_normal(Xn.shape[0]), device=dev)
        X = torch.cat([X, Xn])
        y = torch.cat([y, yn])
        best_ts.append(max(best_ts[-1], float(fn.max())))
        # random search: the same number of evaluations, uniform on the cube
        Xr = torch.as_tensor(rs.uniform(0, 1, (Xn.shape[0], d)), device=dev)
        best_rand = max(best_rand, float(inputs.rff_eval(Xr, target)[:, 0].max()))
        best_rs.append(best_rand)
        if log:
            log("BO step %d: n = %d, best Thompson %.5f, best random %.5f (solve %.1f s, sampling "
                "%.1f s so far)" % (step + 1, n, best_ts[-1], best_rs[-1], t_solve, t_sample))
    improvement = 100.0 * (best_ts[-1] - best_rs[-1]) / abs(best_rs[-1])
    return {"best_thompson": best_ts, "best_random": best_rs, "improvement_percent": improvement,
            "solve_seconds": t_solve, "sampling_seconds": t_sample, "iterations": iters_total,
            "n_final": int(X.shape[0])}
