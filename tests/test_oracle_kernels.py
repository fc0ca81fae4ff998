"""Pins for the oracle's covariance functions: library routines, the general Matern form, PSD."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist
from scipy.special import gamma as gamma_fn, kv
from sklearn.gaussian_process.kernels import RBF as SkRBF, Matern as SkMatern

from oracle import kernels as K


@pytest.fixture(scope="module")
def pts():
    r = np.random.default_rng(0)
    return r.standard_normal((37, 5)), r.standard_normal((23, 5)) * 1.5


def test_sqdist_matches_cdist(pts):
    A, B = pts
    assert np.allclose(K.sqdist(A, B), cdist(A, B, "sqeuclidean"), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("ell", [0.3, 1.0, 2.5])
def test_rbf_matches_sklearn(pts, ell):
    A, B = pts
    assert np.allclose(K.kernel_matrix(A, B, K.RBF, ell), SkRBF(length_scale=ell)(A, B),
                       rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("kind,nu", [(K.MATERN12, 0.5), (K.MATERN32, 1.5), (K.MATERN52, 2.5)])
@pytest.mark.parametrize("ell", [0.3, 1.0])
def test_matern_matches_sklearn_and_bessel(pts, kind, nu, ell):
    A, B = pts
    mine = K.kernel_matrix(A, B, kind, ell)
    assert np.allclose(mine, SkMatern(length_scale=ell, nu=nu)(A, B), rtol=1e-12, atol=1e-300)
    # the general Matern form with the modified Bessel function of the second kind
    r = np.sqrt(cdist(A, B, "sqeuclidean"))
    z = np.sqrt(2 * nu) * r / ell
    general = 2 ** (1 - nu) / gamma_fn(nu) * z ** nu * kv(nu, z)
    assert np.allclose(mine, general, rtol=1e-10, atol=1e-300)


def test_matern_zero_distance_is_one():
    x = np.zeros((1, 3))
    for kind in (K.RBF, K.MATERN12, K.MATERN32, K.MATERN52):
        assert K.kernel_matrix(x, x, kind, 0.7)[0, 0] == 1.0


@pytest.mark.parametrize("kind", [K.RBF, K.MATERN12, K.MATERN32, K.MATERN52])
def test_kernel_symmetric_psd(kind):
    X = np.random.default_rng(1).standard_normal((300, 4))
    Km = K.kernel_matrix(X, X, kind, 0.8)
    assert np.array_equal(Km, Km.T)
    assert np.all(np.diag(Km) == 1.0)
    ev = np.linalg.eigvalsh(Km)
    assert ev.min() >= -300 * 2.0**-52 * ev.max()


def test_kernel_matmul_chunked(pts):
    A, B = pts
    R = np.random.default_rng(2).standard_normal((23, 3))
    full = K.kernel_matrix(A, B, K.MATERN32, 0.9) @ R
    assert np.allclose(K.kernel_matmul(A, B, R, K.MATERN32, 0.9, col_chunk=5), full, rtol=1e-13)
    assert np.allclose(K.kernel_matmul(A, B, R[:, 0], K.MATERN32, 0.9, col_chunk=7), full[:, 0],
                       rtol=1e-13)


@pytest.mark.parametrize("kind,nu", [(K.RBF, None), (K.MATERN12, 0.5), (K.MATERN32, 1.5),
                                     (K.MATERN52, 2.5)])
def test_per_dimension_lengthscales_and_outputscale_match_sklearn(pts, kind, nu):
    from sklearn.gaussian_process.kernels import ConstantKernel
    A, B = pts
    ell = np.array([0.4, 1.7, 0.9, 3.0, 1.1])
    sk = SkRBF(length_scale=ell) if kind == K.RBF else SkMatern(length_scale=ell, nu=nu)
    assert np.allclose(K.kernel_matrix(A, B, kind, ell), sk(A, B), rtol=1e-12, atol=1e-300)
    scaled = ConstantKernel(2.7, constant_value_bounds="fixed") * sk
    assert np.allclose(K.kernel_matrix(A, B, kind, ell, outputscale=2.7), scaled(A, B),
                       rtol=1e-12, atol=1e-300)
    # equal per-dimension lengthscales reduce to the scalar form
    assert np.array_equal(K.sqdist(A, B, np.full(5, 1.0)), K.sqdist(A, B))
    R = np.random.default_rng(3).standard_normal((23, 2))
    assert np.allclose(K.kernel_matmul(A, B, R, kind, ell, col_chunk=4, outputscale=2.7),
                       scaled(A, B) @ R, rtol=1e-12)
