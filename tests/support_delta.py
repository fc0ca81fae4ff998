"""Relative residual difference of two iterates that differ only on a known set of rows.

delta = ||(K + lambda I) E||_F / ||Y||_F for E = W_gpu - W_oracle supported on the ascending
rows S: exact over the rows of S, plus an unbiased estimate over the other rows from uniform
samples (used by the parity tests at sizes where the full n x n product is out of reach).
"""
import math

import numpy as np
import torch

from oracle import kernels as OK


def _kmat(A, B, kind, ell):
    """k(A, B) in float64 on the CPU (torch threads); squared distances by the norm
    expansion, which is ample for measuring a difference of iterates."""
    r2 = (A * A).sum(1)[:, None] + (B * B).sum(1)[None, :] - 2.0 * (A @ B.T)
    r2.clamp_(min=0.0)
    if kind == OK.RBF:
        return torch.exp(r2 * (-0.5 / (ell * ell)))
    a = torch.sqrt(r2) * (math.sqrt(3.0) / ell)
    return (1.0 + a) * torch.exp(-a)


def _klam_norm2(Xrows, XS, E, Erows, kind, ell, lam, chunk=2048):
    """sum over the given rows of |(K E)_i + lambda E_i|^2, with E supported on XS's rows."""
    tot = 0.0
    for i0 in range(0, Xrows.shape[0], chunk):
        R = _kmat(Xrows[i0:i0 + chunk], XS, kind, ell) @ E
        if Erows is not None:
            R += lam * Erows[i0:i0 + chunk]
        tot += float((R * R).sum())
    return tot


def delta_support(X, Y, S, E_S, kind, ell, lam, m_out, seed):
    """delta for an iterate difference supported on the ascending rows S: exact over S,
    plus an unbiased estimate over the other rows from m_out uniform samples."""
    Xt = torch.as_tensor(X, dtype=torch.float64)
    XS = Xt[torch.as_tensor(S)]
    E = torch.as_tensor(E_S, dtype=torch.float64)
    num = _klam_norm2(XS, XS, E, E, kind, ell, lam)
    n = X.shape[0]
    rest = n - S.size
    if rest > 0 and m_out > 0:
        mask = np.ones(n, dtype=bool)
        mask[S] = False
        others = np.flatnonzero(mask)
        pick = np.random.default_rng(seed).choice(others, min(m_out, rest), replace=False)
        num += _klam_norm2(Xt[torch.as_tensor(pick)], XS, E, None, kind, ell, lam) * rest / pick.size
    return math.sqrt(num) / float(np.linalg.norm(Y))
