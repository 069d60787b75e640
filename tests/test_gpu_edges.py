"""Edge cases on the GPU: empty and oversized batches (rejected at the
boundary, no device work), and the largest FFT size in 3D under an exact
property (p = 2: the preconditioner is Ahat^{-1}, Sections 4 and 7)."""

import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402


def test_empty_and_oversized_batches_rejected():
    pl = I.Plan(3, 16, 3, precision="f32", max_rhs=2)
    r = torch.zeros((2,) + pl.shape, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    ws = pl._ws
    for nrhs in (0, -1, 3):
        rc = I.lib.iffd_precond_apply(pl._h, ctypes.c_void_p(r.data_ptr()),
                                      ctypes.c_void_p(z.data_ptr()), nrhs,
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
        assert rc == I.E_INVAL
    empty = torch.zeros((0,) + pl.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(I.IffdError):
        pl.apply(empty)
    with pytest.raises(ValueError):
        pl.apply(torch.zeros((3,) + pl.shape, dtype=torch.float64, device="cuda"))


def test_largest_size_p2_exact():
    """3D n = 512 (the largest FFT length, 134M unknowns), p = 2: Ahat P^{-1} r
    = r in FP64; the gate carries the (n/256)^2 growth of the eigenvalue
    tables' conditioning (see tol_apply in test_gpu_parity)."""
    d, n, p = 3, 512, 2
    print("n=512 p=2: right-hand side", flush=True)
    r = workloads.smooth_rhs(d, n, p, seed=3)
    pl = I.Plan(d, n, p, precision="f64")
    rd = torch.from_numpy(r).cuda()
    del r
    print("apply", flush=True)
    z = pl.apply(rd)
    back = pl.matvec(z)
    del z
    err = float((back - rd).norm() / rd.norm())
    print("rel", err, flush=True)
    assert err <= 1e-11 * (n / 256) ** 2
