"""Bayesian-optimisation pieces on the GPU: the acquisition argmax and a short Thompson run.

The column argmax is an index problem, so it must equal the first maximum exactly (torch's
argmax on the host copy as the reference, ties broken towards the first row).  The short BO
run (2,000 initial points, two steps of 40 acquisitions) checks the loop end to end: best
values never decrease, the acquisitions are evaluated points of the cube, and both methods
spend the same number of evaluations.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("m,k,dt", [(1, 1, torch.float32), (5000, 7, torch.float32),
                                    (300000, 3, torch.float64), (1025, 128, torch.float32)])
def test_column_argmax_is_the_first_maximum(lib, m, k, dt):
    g = torch.Generator(device="cuda")
    g.manual_seed(m + k)
    a = torch.randn((m, k + 2), generator=g, device="cuda", dtype=dt)[:, 1:k + 1]  # row stride k + 2
    if m > 10:
        a[m // 3, 0] = a[:, 0].max() + 1.0
        a[m // 2, 0] = a[m // 3, 0]          # tie: the first row wins
        a[7, k - 1] = float("nan")           # NaN never wins
    got = lib.column_argmax(a).cpu().numpy()
    h = a.cpu().double().numpy()
    ref = np.array([np.flatnonzero(h[:, c] == np.nanmax(h[:, c]))[0] for c in range(k)])
    assert np.array_equal(got, ref)


def test_short_thompson_run(lib):
    from paper_2505_13723_amd import bo
    out = bo.thompson_bo(lib, d=8, ell=2.0, noise=1e-6, n0=2000, steps=2, acq=40, batch=20,
                         n_cand=2000, n_local=500, passes=5, rank=64, seed=3)
    ts, rs = out["best_thompson"], out["best_random"]
    assert len(ts) == 3 and len(rs) == 3 and ts[0] == rs[0]
    assert all(a <= b for a, b in zip(ts, ts[1:])) and all(a <= b for a, b in zip(rs, rs[1:]))
    assert out["n_final"] == 2000 + 80 and np.isfinite(out["improvement_percent"])
    print("short BO run: %s" % out, flush=True)
