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
    = r in FP64 (the residual of the FP64 operator on the FP64 apply)."""
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
    assert err <= 1e-11


def test_stepped_state_must_match_its_init():
    """The stepped PCG calls refuse a state buffer used with another slot
    count or another plan than at iffd_pcg_state_init (the buffer's offsets
    follow from both), and one that was never initialised."""
    pl = I.Plan(2, 16, 3, precision="f64", max_rhs=4)
    other = I.Plan(2, 16, 3, precision="f64", max_rhs=4)
    st = I.PcgState(pl, 2)
    f = torch.from_numpy(workloads.uniform_rhs(2, 16, 3, seed=3)).cuda()
    buf = ctypes.c_void_p(st.buf.data_ptr())
    slots = (ctypes.c_int * 1)(0)
    fp = ctypes.c_void_p(f.data_ptr())
    assert I.lib.iffd_pcg_begin(pl._h, buf, 3, slots, 1, fp, 1e-8, 50, None) == I.E_STATE
    assert I.lib.iffd_pcg_begin(other._h, buf, 2, slots, 1, fp, 1e-8, 50, None) == I.E_STATE
    assert I.lib.iffd_pcg_iterate(pl._h, buf, 3, 1, None) == I.E_STATE
    out = np.zeros(16)
    assert I.lib.iffd_pcg_poll(pl._h, buf, 1, out.ctypes.data_as(ctypes.c_void_p), None) == I.E_STATE
    u = torch.empty_like(f)
    assert I.lib.iffd_pcg_take(pl._h, buf, 4, 0, ctypes.c_void_p(u.data_ptr()), None) == I.E_STATE
    raw = torch.empty_like(st.buf)
    assert I.lib.iffd_pcg_iterate(pl._h, ctypes.c_void_p(raw.data_ptr()), 2, 1, None) == I.E_STATE
    # the matching calls work
    st.begin([0], f)
    st.iterate(20)
    assert st.poll()[0, 1] == 0
