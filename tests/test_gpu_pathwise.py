"""Pathwise posterior samples and predictive metrics through the C ABI, against the oracle.

adasap_posterior_samples forms k(X*, X) W in one product (float64 on the FP64 path, float16
hi/lo on the reduced paths) and combines the columns into the posterior mean and the samples
f_s(X*) + k(X*, X)(W_0 - W_s) (Sec. 2.1).  Bounds: 1e-11 relative on the FP64 path; on the
hi/lo path each product entry carries at most 2e-5 (|K| |W|) (the error model of the hi/lo
products), so sample s is within 2e-5 (|K| |W_0| + |K| |W_s|).  The metrics reduce in
float64 and agree with the oracle's to 1e-12.
"""
import numpy as np
import pytest

from oracle import kernels as OK
from oracle import linsys as OL
from oracle import pathwise as PW
from paper_2505_13723_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _split(n, m, k, seed=5):
    X, Y, Xt, yt, Pt = inputs.make_c3(seed=seed, n=n, d=6, k=k, ell=1.5, lam=0.05, device="cpu",
                                      dtype=torch.float64, n_test=m)
    return X.numpy(), Y.numpy(), Xt.numpy(), yt.numpy(), Pt.numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_posterior_samples_and_metrics_match_oracle(lib, precision):
    n, m, k, lam, ell = 1500, 300, 9, 0.05, 1.5
    X, Y, Xt, yt, Pt = _split(n, m, k)
    reduced = precision != "fp64"
    if reduced:
        X, Y, Xt, yt, Pt = (a.astype(np.float32).astype(np.float64) for a in (X, Y, Xt, yt, Pt))
    W = OL.direct_solve(X, Y, OK.RBF, ell, lam)
    if reduced:
        W = W.astype(np.float32).astype(np.float64)
    dt = torch.float32 if reduced else torch.float64
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dt).cuda()
    h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=100, rank=20,
                              precision=precision), d(X), d(Y))
    got = h.posterior_samples(d(W), d(Xt), d(Pt)).cpu().double().numpy()
    ref = PW.posterior_samples(X, W, Xt, Pt, OK.RBF, ell)
    if reduced:
        KA = OK.kernel_matrix(Xt, X, OK.RBF, ell) @ np.abs(W)
        bound = 2e-5 * (KA[:, :1] + np.where(np.arange(k) > 0, KA, 0.0)) + 1e-6
        assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)
    else:
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    rmse, nll = lib.predictive_metrics(d(got), d(yt), lam)
    r_ref, n_ref = PW.predictive_metrics(got if reduced else got, yt, lam)
    assert rmse == pytest.approx(r_ref, rel=1e-6 if reduced else 1e-12)
    assert nll == pytest.approx(n_ref, rel=1e-6 if reduced else 1e-12, abs=1e-9)
    h.close()


def test_solve_then_sample_end_to_end(lib):
    # an FP32 solve of y and eight pathwise right-hand sides, then samples and metrics at held-out
    # points: the test RMSE and NLL are those of the exact posterior within the solve's residual
    n, m, k, lam, ell = 4000, 500, 9, 0.05, 1.5
    X, Y, Xt, yt, Pt = _split(n, m, k, seed=8)
    X, Y, Xt, yt, Pt = (a.astype(np.float32).astype(np.float64) for a in (X, Y, Xt, yt, Pt))
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).float().cuda()
    h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=1000, rank=128,
                              precision="fp32", max_iters=3000, tol=1e-4, check_every=40, seed=4),
                   d(X), d(Y))
    W = torch.zeros((n, k), dtype=torch.float32, device="cuda")
    rep = h.solve(W)
    assert rep["relres"] <= 1e-4, rep["relres"]
    smp = h.posterior_samples(W, d(Xt), d(Pt))
    rmse, nll = lib.predictive_metrics(smp, d(yt), lam)
    h.close()
    Wstar = OL.direct_solve(X, Y, OK.RBF, ell, lam)
    r_ref, n_ref = PW.predictive_metrics(PW.posterior_samples(X, Wstar, Xt, Pt, OK.RBF, ell), yt, lam)
    print("end to end: rmse %.6f (exact %.6f), nll %.6f (exact %.6f)" % (rmse, r_ref, nll, n_ref),
          flush=True)
    assert rmse == pytest.approx(r_ref, rel=1e-3)
    assert nll == pytest.approx(n_ref, abs=2e-3)
