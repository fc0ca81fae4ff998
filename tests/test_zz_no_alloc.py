"""The no-allocation kernel-block product against the allocating one.

adasap_kblock_matmul_noalloc runs the kernels of adasap_kblock_matmul with the split partial
sums in the library's fixed device array instead of an allocation.  When both take the same
column splits the outputs agree bit for bit; when the fixed array forces fewer splits only
the order of the float64 (or float32) partial additions differs, so they agree to rounding:
1e-12 of (|K| |R|) in float64, 2e-6 in float32.  Every case makes two calls in a row on the
same stream, the second with a smaller input, so the shared array carries nothing from one
call into the next; sizes beyond the array are rejected before any device work.
"""
import ctypes

import numpy as np
import pytest

from oracle import kernels as OK

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KINDS = {"rbf": OK.RBF, "matern32": OK.MATERN32, "matern52": OK.MATERN52}


def _inputs(seed, m, n, d, k, dt):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    Xr = torch.randn((m, d), generator=g, device="cuda", dtype=dt)
    Xc = torch.randn((n, d), generator=g, device="cuda", dtype=dt)
    R = torch.randn((n, k), generator=g, device="cuda", dtype=dt)
    return Xr, Xc, R


# (kernel, precision, first call (m, n, d, k), second call, same splits in the first call)
CASES = [
    ("rbf", "fp64", (3000, 20000, 7, 5), (500, 3000, 7, 2), True),
    ("matern32", "fp32", (4000, 50000, 11, 3), (1000, 7000, 11, 1), True),
    ("matern52", "fp64", (40000, 30000, 6, 16), (9000, 2000, 6, 16), False),
    ("rbf", "fp32", (2500, 100000, 16, 20), (300, 100, 16, 20), True),
]


@pytest.mark.parametrize("kind,precision,first,second,same_splits", CASES)
def test_noalloc_product_matches_allocating_entry_point(lib, kind, precision, first, second,
                                                        same_splits):
    dt = torch.float64 if precision == "fp64" else torch.float32
    rel = 1e-12 if precision == "fp64" else 2e-6
    ell = 1.3
    for call, (m, n, d, k) in enumerate((first, second)):
        print("no-alloc product %s %s m=%d n=%d d=%d k=%d" % (kind, precision, m, n, d, k), flush=True)
        Xr, Xc, R = _inputs(100 + call, m, n, d, k, dt)
        ref = lib.kblock_matmul(kind, ell, precision, Xr, Xc, R)
        out = torch.full((m, k), float("nan"), dtype=dt, device="cuda")
        lib.kblock_matmul_noalloc(kind, ell, precision, Xr, Xc, R, out)
        torch.cuda.synchronize()
        if call == 0 and same_splits:
            assert torch.equal(out, ref)
        else:
            absref = lib.kblock_matmul(kind, ell, precision, Xr, Xc, R.abs())
            err = (out.double() - ref.double()).abs()
            assert bool(torch.all(err <= rel * absref.double() + 1e-300)), float((err / absref).max())
        assert bool(torch.isfinite(out).all())


def test_noalloc_rejects_what_does_not_fit(lib):
    from paper_2505_13723_amd.binding import AdasapError
    Xr, Xc, R = _inputs(1, 8, 16, 3, 1, torch.float64)
    fake = ctypes.c_void_p(0x1000)
    # 32 MiB / (128 columns x 8 bytes) = 32768 rows at most in float64
    st = lib.cdll.adasap_kblock_matmul_noalloc(0, 1.0, 0, 32769, 16, 3, 128, fake, fake, fake, fake,
                                               1, None)
    assert st == 1 and "scratch" in lib.last_error()
    with pytest.raises(AdasapError):
        lib.kblock_matmul_noalloc("rbf", 1.0, "mixed", Xr, Xc, R,
                                  torch.empty((8, 1), dtype=torch.float64, device="cuda"))
    # the largest float64 output that fits runs
    m, k = 32768, 128
    Xr, Xc, R = _inputs(2, m, 64, 2, k, torch.float64)
    out = torch.empty((m, k), dtype=torch.float64, device="cuda")
    lib.kblock_matmul_noalloc("rbf", 1.0, "fp64", Xr, Xc, R, out)
    torch.cuda.synchronize()
    ref = lib.kblock_matmul("rbf", 1.0, "fp64", Xr, Xc, R)
    absref = lib.kblock_matmul("rbf", 1.0, "fp64", Xr, Xc, R.abs())
    assert bool(torch.all((out - ref).abs() <= 1e-12 * absref))
