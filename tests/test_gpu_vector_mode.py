"""The float32 vector-mode product (k <= 4 right-hand sides at FP32) through the solver's own
Step-I launch, against the float64 oracle.

adasap_block_gradient returns B_t and G = K(X_B, X) Z + lambda Z_B - Y_B from the launch that
adasap_solve runs.  At FP32 with k <= 4 that launch takes the distances on 32x32x16 MFMAs in
2 (d <= 8, one K-step of packed slots), 3 (3d + 6 <= 48) or 4 K-slices of 16, and the kernel
values and K Z in float32; these cases cover every slice count and the one-, two- and
four-column right-hand-side widths (k = 3 runs as four with a zero column).  The bound is the
error model of the float16 hi/lo distances: each kernel value moves by at most about
2e-5 relative, so |G - G_oracle| <= 3e-5 (|K| |Z|) + a float32 rounding floor.
"""
import numpy as np
import pytest

from oracle import kernels as OK
from paper_2505_13723_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KINDS = {"rbf": OK.RBF, "matern32": OK.MATERN32, "matern52": OK.MATERN52}


@pytest.mark.parametrize("kind", ["rbf", "matern32", "matern52"])
@pytest.mark.parametrize("d,k", [(3, 1), (8, 2), (11, 3), (14, 4), (16, 1)])
def test_vector_mode_block_gradient_matches_oracle(lib, kind, d, k):
    n, b, lam = 3000, 300, 0.05
    ell = 0.5 * np.sqrt(d)
    X, Y = inputs.make_small(40 + d, n, d, k)
    X = X.astype(np.float32).astype(np.float64)
    Y = Y.astype(np.float32).astype(np.float64)
    rs = np.random.default_rng(d * 7 + k)
    Z = rs.standard_normal((n, k)).astype(np.float32)
    Xd = torch.as_tensor(X, dtype=torch.float32).cuda()
    Yd = torch.as_tensor(Y, dtype=torch.float32).cuda()
    h = lib.create(lib.config(kernel=kind, lengthscale=ell, lam=lam, block_size=b, rank=32,
                              precision="fp32", max_iters=1, seed=5), Xd, Yd)
    B, G = h.block_gradient(3, torch.as_tensor(Z).cuda())
    h.close()
    B = B.cpu().numpy()
    G = G.cpu().numpy()
    Z64 = Z.astype(np.float64)
    Kb = OK.kernel_matrix(X[B], X, KINDS[kind], ell)
    ref = Kb @ Z64 + lam * Z64[B] - Y[B]
    bound = 3e-5 * (Kb @ np.abs(Z64)) + 1e-5 * (np.abs(lam * Z64[B]) + np.abs(Y[B])) + 1e-6
    err = np.abs(G - ref)
    assert np.all(err <= bound), (float(np.max(err / bound)), d, k)
