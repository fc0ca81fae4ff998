"""Covariance functions k(x, x') of the GP prior (Sec. 2), float64, direct differences.

Test infrastructure (see the package docstring).

The paper names RBF, Matern-3/2 and Matern-5/2 kernels (Sec. 5, Table 1) but
prints no formulas; these are the textbook forms with a scalar lengthscale
ell and unit output scale (reading recorded in the design notes):

* RBF          exp(-r^2 / (2 ell^2))
* Matern-1/2   exp(-r / ell)
* Matern-3/2   (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell)
* Matern-5/2   (1 + sqrt(5) r / ell + 5 r^2 / (3 ell^2)) exp(-sqrt(5) r / ell)

r = ||x - x'||_2 is formed from coordinate differences (no norm expansion),
so the oracle carries none of the cancellation the fast path must manage.

The paper's experiments fit one lengthscale per input dimension and an output
scale (appendix, hyperparameters for regression).  With a vector ell the
distance becomes r^2 = sum_j ((x_j - x'_j) / ell_j)^2 and the forms above are
taken at ell = 1; `outputscale` s multiplies the kernel, k -> s k.
"""
import numpy as np

RBF = 0
MATERN12 = 1
MATERN32 = 2
MATERN52 = 3
KERNEL_NAMES = {RBF: "rbf", MATERN12: "matern12", MATERN32: "matern32", MATERN52: "matern52"}


def sqdist(X1, X2, ell=None):
    """Squared distances sum_j ((x1_ij - x2_kj) / ell_j)^2 by explicit differences
    (plain Euclidean distances when ell is None)."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    diff = X1[:, None, :] - X2[None, :, :]
    if ell is not None:
        diff = diff / np.asarray(ell, dtype=np.float64)
    return np.einsum("ijk,ijk->ij", diff, diff)


def kernel_from_sqdist(r2, kind, ell):
    """Apply the covariance function to squared distances."""
    r2 = np.asarray(r2, dtype=np.float64)
    if kind == RBF:
        return np.exp(-r2 / (2.0 * ell * ell))
    r = np.sqrt(r2)
    if kind == MATERN12:
        return np.exp(-r / ell)
    if kind == MATERN32:
        a = np.sqrt(3.0) * r / ell
        return (1.0 + a) * np.exp(-a)
    if kind == MATERN52:
        a = np.sqrt(5.0) * r / ell
        return (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError("unknown kernel %r" % (kind,))


def kernel_matrix(X1, X2, kind, ell, col_chunk=8192, outputscale=1.0):
    """outputscale * k(X1, X2) as a dense float64 matrix, built in column chunks; ell is a
    scalar or one lengthscale per coordinate."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    ard = np.ndim(ell) > 0
    out = np.empty((X1.shape[0], X2.shape[0]), dtype=np.float64)
    step = max(1, min(col_chunk, (1 << 24) // max(1, X1.shape[0] * X1.shape[1])))
    for j0 in range(0, X2.shape[0], step):
        if ard:
            Kc = kernel_from_sqdist(sqdist(X1, X2[j0:j0 + step], ell), kind, 1.0)
        else:
            Kc = kernel_from_sqdist(sqdist(X1, X2[j0:j0 + step]), kind, ell)
        out[:, j0:j0 + step] = Kc if outputscale == 1.0 else outputscale * Kc
    return out


def kernel_matmul(X1, X2, R, kind, ell, col_chunk=4096, outputscale=1.0):
    """outputscale * k(X1, X2) @ R without holding the whole block (column chunks)."""
    R = np.asarray(R, dtype=np.float64)
    squeeze = R.ndim == 1
    if squeeze:
        R = R[:, None]
    out = np.zeros((np.asarray(X1).shape[0], R.shape[1]), dtype=np.float64)
    for j0 in range(0, np.asarray(X2).shape[0], col_chunk):
        Kc = kernel_matrix(X1, X2[j0:j0 + col_chunk], kind, ell, outputscale=outputscale)
        out += Kc @ R[j0:j0 + col_chunk]
    return out[:, 0] if squeeze else out
