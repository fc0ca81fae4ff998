"""Parity of the row-subsampled residual estimate with the float64 oracle.

The rows are a Floyd draw on the Philox stream (seed, 12, 0) and must match the oracle's
draw bit for bit.  The estimate sqrt(sum_S |r_i|^2 / sum_S |y_i|^2) uses float64 products on
the FP64 path (relative agreement 1e-10) and the float16 hi/lo products on the reduced
paths, whose per-entry error is below 2e-5 (|K| |W|)_i: with W of unit scale the residual
rows are of the size of (K W)_i, so the estimate agrees to 1e-3 relative.
"""
import numpy as np
import pytest

from oracle import kernels as OK
from oracle import linsys as OL
from oracle import rng as OR
from paper_2505_13723_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision,dtype,tol", [("fp64", torch.float64, 1e-10), ("fp32", torch.float32, 1e-3),
                                                 ("mixed", torch.float32, 1e-3)])
@pytest.mark.parametrize("m", [1, 333, 2500])
def test_residual_rows_matches_oracle(lib, precision, dtype, tol, m):
    n, d, k, lam, ell = 2500, 5, 3, 0.05, 1.1
    X, Y = inputs.make_small(61, n, d, k)
    W = np.random.default_rng(3).standard_normal((n, k))
    if dtype == torch.float32:
        X, Y, W = (a.astype(np.float32).astype(np.float64) for a in (X, Y, W))
    Xd, Yd, Wd = (torch.as_tensor(a, dtype=dtype).cuda() for a in (X, Y, W))
    h = lib.create(lib.config(kernel="rbf", lengthscale=ell, lam=lam, block_size=200, rank=20,
                              precision=precision), Xd, Yd)
    est, worst, rows = h.residual_rows(Wd, m, 9, rows=True)
    ref_rows = OR.sample_block(9, 0, n, m, purpose=OR.PURPOSE_RESROWS)
    assert np.array_equal(rows.cpu().numpy(), ref_rows)
    R = OL.residual_rows(X, Y, W, OK.RBF, ell, lam, ref_rows)
    ref = np.sqrt((R ** 2).sum() / (Y[ref_rows] ** 2).sum())
    ref_worst = np.max(np.sqrt((R ** 2).sum(axis=0) / (Y[ref_rows] ** 2).sum(axis=0)))
    assert est == pytest.approx(ref, rel=tol) and worst == pytest.approx(ref_worst, rel=tol)
    if m == n:
        assert est == pytest.approx(h.residual(Wd)[0], rel=1e-9)
    h.close()
