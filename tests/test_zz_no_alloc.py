"""The allocation-free apply (iffd_precond_apply_noalloc) against the
workspace form (iffd_precond_apply), called through the C ABI: the same
kernels, so the same bits, on two calls in a row (the second with a smaller
input, reusing the scratch the first one left), for the IFFD apply in FP32
and FP64 and for dense FD; and a call that needs more than the scratch is
rejected before any launch."""

import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2512_20269_amd as I  # noqa: E402


def ws_apply(pl, r):
    z = torch.empty_like(r)
    nrhs = 1 if r.dim() == pl.d else r.shape[0]
    ws = pl._ws
    rc = I.lib.iffd_precond_apply(pl._h, ctypes.c_void_p(r.data_ptr()),
                                  ctypes.c_void_p(z.data_ptr()), nrhs,
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert rc == 0, I.lib.iffd_last_error()
    return z


def noalloc_apply(pl, r):
    z = torch.full_like(r, float("nan"))
    nrhs = 1 if r.dim() == pl.d else r.shape[0]
    rc = I.lib.iffd_precond_apply_noalloc(pl._h, ctypes.c_void_p(r.data_ptr()),
                                          ctypes.c_void_p(z.data_ptr()), nrhs, None)
    assert rc == 0, I.lib.iffd_last_error()
    return z


@pytest.mark.parametrize("method,prec", [("fft", "f32"), ("fft", "f64"), ("dense", "f32")])
def test_noalloc_equals_workspace_apply(method, prec):
    d, n, p = 3, 48, 4
    pl = I.Plan(d, n, p, method=method, precision=prec, max_rhs=3)
    big = torch.from_numpy(workloads.batched_uniform_rhs(d, n, p, [61, 62, 63])).cuda()
    small = torch.from_numpy(workloads.uniform_rhs(d, n, p, seed=64)).cuda()
    for r in (big, small):          # the second call is smaller
        za = noalloc_apply(pl, r)
        zb = ws_apply(pl, r)
        torch.cuda.synchronize()
        assert torch.equal(za, zb)
        assert bool(torch.isfinite(za).all())


def test_noalloc_largest_workload_then_small():
    """The 3D n = 256, p = 3 workload (68 MB of FP32 workspace) and then a
    2D n = 64 problem on the same scratch."""
    for d, n, p in ((3, 256, 3), (2, 64, 3)):
        pl = I.Plan(d, n, p, precision="f32")
        r = torch.from_numpy(workloads.uniform_rhs(d, n, p, seed=5)).cuda()
        za = noalloc_apply(pl, r)
        zb = ws_apply(pl, r)
        torch.cuda.synchronize()
        assert torch.equal(za, zb)
        del pl, r, za, zb


def test_noalloc_rejects_oversized_workspace():
    d, n, p = 3, 256, 8   # 4 N = 72 MB per right-hand side in FP32
    pl = I.Plan(d, n, p, precision="f32", max_rhs=2)
    need = 2 * 4 * pl.N
    assert need > I.NOALLOC_SCRATCH_BYTES
    r = torch.zeros((2,) + pl.shape, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    rc = I.lib.iffd_precond_apply_noalloc(pl._h, ctypes.c_void_p(r.data_ptr()),
                                          ctypes.c_void_p(z.data_ptr()), 2, None)
    assert rc == I.E_WORKSPACE
    assert b"scratch" in I.lib.iffd_last_error()
    torch.cuda.synchronize()
    assert bool((z == 0).all())
