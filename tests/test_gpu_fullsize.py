"""Parity of the Step-I block gradient at the full workload sizes, on sampled rows.

The solver's own Step-I launch (adasap_block_gradient: same block B_t, kernels, precision
and grid as adasap_solve) is run on the full problems

* rbf, n = 2,000,000, d = 11, k = 64, b = 16384, MIXED (float16 matrix-core products);
* matern32, n = 1,000,000, d = 11 with 5% clustered near-duplicates, k = 1, b = 8192, FP32;
* rbf, n = 100,000,000, d = 9, k = 1, b = 32768, FP32;

and a handful of block rows (first, last and spread between) are recomputed by the float64
oracle against all n columns.  The block itself must equal the oracle's draw bit for bit.

Error model (the per-entry bound used below).  Squared distances come from the three-term
float16 split of the centred coordinates x~; the kernel value is then that of points moved
by about 2^-22 |x~|, so |d r^2| <= 2^-21 (|x~_i|^2 + |x~_j|^2) up to small constants, and
the kernel's relative error is at most L |d r^2| with L = max |d ln k / d r^2| (1 / (2 ell^2)
for RBF, 3 / (2 ell^2) for Matern-3/2).  MIXED rounds kernel values and the iterate to
float16 once each (relative 2^-10 per term, 1.2e-3 with margin); FP32 keeps float32
values (2^-20 with margin).  So |G - G_oracle|_ic <= (e_prod + L 2^-19 (|x~_i|^2 +
max_j |x~_j|^2)) (K |Z|)_ic + 1e-6 (lambda |Z_ic| + |Y_ic|), with a factor 4 of margin on
the distance term.
"""
import numpy as np
import pytest

from oracle import kernels as OK
from oracle import rng as OR
from paper_2505_13723_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


def _sample_rows(b, count, seed):
    rs = np.random.default_rng(seed)
    mid = rs.choice(np.arange(1, b - 1), count - 2, replace=False)
    return np.concatenate([[0], np.sort(mid), [b - 1]])


def _check(lib, X, Y, Z, kind, kname, ell, lam, b, r, precision, seed, rows, e_prod, t=3):
    n, k = Y.shape
    cfg = lib.config(kernel=kname, lengthscale=ell, lam=lam, block_size=b, rank=r, seed=seed,
                     precision=precision, max_iters=1)
    h = lib.create(cfg, X, Y)
    B, G = h.block_gradient(t, Z)
    torch.cuda.synchronize()
    B = B.cpu().numpy()
    print("block gradient n=%d b=%d k=%d done" % (n, b, k), flush=True)
    assert np.array_equal(B, OR.sample_block(seed, t, n, b))
    G = G[torch.as_tensor(rows, device=G.device)].cpu().numpy()
    h.close()
    Bi = B[rows]
    Xh = X.double().cpu().numpy()
    Zh = Z.double().cpu().numpy()
    Yh = Y.double().cpu().numpy()
    xt2 = ((Xh - Xh.mean(axis=0)) ** 2).sum(axis=1)
    # one pass of the oracle gives K Z and K |Z| together
    KZ = OK.kernel_matmul(Xh[Bi], Xh, np.concatenate([Zh, np.abs(Zh)], axis=1), kind, ell,
                          col_chunk=1 << 16)
    ref = KZ[:, :k] + lam * Zh[Bi] - Yh[Bi]
    L = {OK.RBF: 0.5, OK.MATERN32: 1.5}[kind] / ell ** 2
    rel = e_prod + L * 2.0 ** -19 * (xt2[Bi] + xt2.max())
    bound = rel[:, None] * KZ[:, k:] + 1e-6 * (lam * np.abs(Zh[Bi]) + np.abs(Yh[Bi])) + 1e-9
    err = np.abs(G - ref)
    assert np.all(err <= bound), (np.max(err / bound), np.unravel_index(np.argmax(err / bound), err.shape))


def test_block_gradient_rbf_n2m_k64_mixed(lib):
    w = inputs.WORKLOADS["c3_rbf_n2m_k64"]
    X, Y = inputs.make_c3(seed=w["seed"], n=w["n"], d=w["d"], k=w["k"], ell=w["ell"], lam=w["lam"],
                          device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    Z = torch.randn(Y.shape, generator=g, device="cuda", dtype=torch.float32) * 10.0
    _check(lib, X, Y, Z, OK.RBF, "rbf", w["ell"], w["lam"], w["b"], w["r"], "mixed", w["seed"],
           _sample_rows(w["b"], 12, 1), 1.2e-3)


def test_block_gradient_matern32_n1m_fp32(lib):
    w = inputs.WORKLOADS["c2_matern32_n1m"]
    X, y = inputs.make_c2(seed=w["seed"], n=w["n"], d=w["d"], ell=w["ell"], lam=w["lam"],
                          device="cuda")
    Y = y[:, None].contiguous()
    g = torch.Generator(device="cuda")
    g.manual_seed(12)
    Z = torch.randn(Y.shape, generator=g, device="cuda", dtype=torch.float32) * 30.0
    _check(lib, X, Y, Z, OK.MATERN32, "matern32", w["ell"], w["lam"], w["b"], w["r"], "fp32",
           w["seed"], _sample_rows(w["b"], 12, 2), 2.0 ** -20)


def test_block_gradient_rbf_n100m_fp32(lib):
    w = inputs.WORKLOADS["c5_rbf_n100m"]
    X, y = inputs.make_c5(seed=w["seed"], n=w["n"], d=w["d"], ell=w["ell"], lam=w["lam"],
                          device="cuda", chunk=1 << 18)
    Y = y[:, None].contiguous()
    del y
    g = torch.Generator(device="cuda")
    g.manual_seed(13)
    Z = torch.randn(Y.shape, generator=g, device="cuda", dtype=torch.float32)
    _check(lib, X, Y, Z, OK.RBF, "rbf", w["ell"], w["lam"], w["b"], w["r"], "fp32", w["seed"],
           _sample_rows(w["b"], 4, 3), 2.0 ** -20)
