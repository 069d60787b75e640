"""CPU-only checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments, and its host-side plan tables (built by
its own C++ code) agree with the oracle.  No device work is launched here."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2512_20269_amd as I
from oracle import bspline
from oracle import iffd as O

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "iffd.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(iffd_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    syms = declared_symbols()
    assert len(syms) >= 16
    lib = ctypes.CDLL(I.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(I.SIGNATURES), "binding and header disagree"


def host_plan(d, n, p, method=I.METHOD_FFT, prec=I.PREC_F32, max_rhs=1, coef_a=0.0):
    h = ctypes.c_void_p()
    opts = I._Opts(method, prec, max_rhs, coef_a)
    rc = I.lib.iffd_plan_create(ctypes.byref(h), d, n, p, ctypes.byref(opts))
    return rc, h


def read(h, what, count):
    buf = np.zeros(count)
    rc = I.lib.iffd_plan_read(h, what, buf.ctypes.data_as(ctypes.c_void_p), count, None)
    assert rc == 0, I.lib.iffd_last_error()
    return buf


@pytest.mark.parametrize("prec", [I.PREC_F16S, I.PREC_BF16S])
def test_fp16_scaled_option_is_dense_fd_only(prec):
    opts = I._Opts(I.METHOD_FFT, prec, 1)
    h = ctypes.c_void_p()
    assert I.lib.iffd_plan_create(ctypes.byref(h), 3, 16, 3, ctypes.byref(opts)) == I.E_INVAL
    rc, h = host_plan(3, 16, 3, I.METHOD_DENSE_FD, prec)
    assert rc == 0, I.lib.iffd_last_error()
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    m = O.dims(16, 3)[0]
    # workspace: two FP32 tensors, an FP16 copy and one FP32 scale per line
    assert info.apply_ws_bytes >= 8 * m ** 3 + 2 * m ** 3 + 4 * m ** 2
    I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("n,p", [(256, 3), (512, 3), (128, 1), (64, 6)])
def test_eigenvalue_tables_agree_with_oracle(n, p):
    """The plan's regular eigenvalues (Lemma 4's closed form, extended
    precision) against the oracle's seminorm quotients |F_j|^2_H1 /
    ||F_j||^2_L2 (eq:Lambda reg2, integrated from F_j'): two independent
    routes, neither with the eps * n^2 cancellation of x^T K x / x^T M x, so
    they agree to 1e-13 at every n (the FP64 x^T K x quotient of the
    smoothest mode is 1.8e-12 off at n = 512)."""
    rc, h = host_plan(2, n, p)
    assert rc == 0, I.lib.iffd_last_error()
    m, n_reg, _ = O.dims(n, p)
    lam = read(h, I.TABLE_LAM, m)[:n_reg]
    ref = O.factors_route_b(n, p)["lam_reg"]
    d = np.abs(lam - ref) / np.abs(ref)
    assert d.max() <= 1e-13
    assert d[:8].max() <= 2e-15 * n / 16   # the smooth modes that dominate P^{-1} r
    I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("n,p", [(8, 2), (16, 3), (12, 4), (32, 5), (24, 6), (16, 7), (32, 8),
                                 (96, 4), (128, 3)])
def test_host_tables_match_oracle(n, p):
    rc, h = host_plan(3, n, p)
    assert rc == 0, I.lib.iffd_last_error()
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    m, n_reg, n_out = O.dims(n, p)
    # the sine transforms run through length-n FFTs where that length is built
    # (n >= 16), else through length-2n ones; FP32 plans of odd degree >= 5
    # through the length-2n odd extension where 2n is built
    built = (16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512)
    L = n if n in built else 2 * n
    if p % 2 and p >= 5 and 2 * n in built:
        L = 2 * n
    assert (info.m, info.n_reg, info.n_out, info.N, info.fft_len) == (m, n_reg, n_out, m ** 3, L)
    fb = O.factors_route_b(n, p)
    lam = read(h, I.TABLE_LAM, m)[:n_reg]
    np.testing.assert_allclose(lam, fb["lam_reg"], rtol=1e-12)
    np.testing.assert_allclose(read(h, I.TABLE_DT, n_reg), fb["Dt"], rtol=1e-12)
    K, M = bspline.assemble_dirichlet(n, p)
    bw = 2 * p + 1
    for what, ref in ((I.TABLE_KBAND, K), (I.TABLE_MBAND, M)):
        band = read(h, what, m * bw).reshape(m, bw)
        dense = np.zeros((m, m))
        for i in range(m):
            for o in range(bw):
                j = i + o - p
                if 0 <= j < m:
                    dense[i, j] = band[i, o]
        np.testing.assert_allclose(dense, ref, atol=1e-13 * np.abs(ref).max())
    # the special-basis boundary block spans the same space as the oracle's
    half = p // 2
    V0 = read(h, I.TABLE_V0, (p - 1) * half).reshape(p - 1, half)
    np.testing.assert_allclose(V0, fb["V_reg"][:p - 1, :half], atol=1e-12)
    # Vt needs the device setup
    buf = np.zeros(max(1, n_out * m))
    assert I.lib.iffd_plan_read(h, I.TABLE_VT, buf.ctypes.data_as(ctypes.c_void_p), len(buf),
                                None) == I.E_STATE
    I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("n,p", [(9, 3), (17, 3)])
def test_dense_fd_host_eigenvalues(n, p):
    rc, h = host_plan(2, n, p, method=I.METHOD_DENSE_FD)
    assert rc == 0
    m = n + p - 2
    lam_fd = read(h, I.TABLE_LAM, m)
    lam_or, *_ = O.factors_fd(n, p)
    np.testing.assert_allclose(lam_fd, lam_or, rtol=1e-11)
    I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("d,n,p,code", [
    (1, 16, 3, I.E_INVAL), (4, 16, 3, I.E_INVAL), (3, 16, 0, I.E_INVAL), (3, 16, 9, I.E_INVAL),
    (3, 3, 3, I.E_INVAL), (3, 100, 3, I.E_UNSUPPORTED),
    (3, 1024, 3, I.E_UNSUPPORTED), (2, 640, 2, I.E_UNSUPPORTED), (2, 768, 4, I.E_UNSUPPORTED)])
def test_invalid_plans_rejected(d, n, p, code):
    rc, h = host_plan(d, n, p)
    assert rc == code
    assert h.value is None
    assert len(I.lib.iffd_last_error()) > 0


def test_dense_plan_above_two_gib_per_rhs_rejected():
    """3D dense FD at n = 700 (m^3 = 344M, 2.75 GB in FP64) passes the 2^31
    element bound but not the 2 GiB per right-hand side of buffer addressing;
    n = 512 (the largest IFFD size) stays inside it."""
    rc, h = host_plan(3, 700, 3, method=I.METHOD_DENSE_FD)
    assert rc == I.E_UNSUPPORTED and h.value is None
    assert "2 GiB" in I.lib.iffd_last_error().decode()


def test_null_and_state_errors():
    assert I.lib.iffd_plan_create(None, 3, 16, 3, None) == I.E_INVAL
    rc, h = host_plan(2, 16, 3)
    assert rc == 0
    info = I._Info()
    I.lib.iffd_plan_query(h, ctypes.byref(info))
    # compute entry points refuse a plan that has not been set up
    fake = ctypes.c_void_p(256)
    assert I.lib.iffd_precond_apply(h, fake, ctypes.c_void_p(512), 1, fake, 1 << 20, None) == I.E_STATE
    assert I.lib.iffd_kron_matvec(h, fake, ctypes.c_void_p(512), 1, fake, 1 << 20, None) == I.E_STATE
    # the default options are FFT / F32 / 1 RHS
    rc, h2 = host_plan(2, 16, 3)
    h3 = ctypes.c_void_p()
    assert I.lib.iffd_plan_create(ctypes.byref(h3), 2, 16, 3, None) == 0
    i3 = I._Info()
    I.lib.iffd_plan_query(h3, ctypes.byref(i3))
    assert (i3.method, i3.apply_prec, i3.max_rhs) == (I.METHOD_FFT, I.PREC_F32, 1)
    for x in (h, h2, h3):
        I.lib.iffd_plan_destroy(x)
    assert I.lib.iffd_status_string(I.E_BREAKDOWN) == b"PCG breakdown"


def band_to_dense(band, m, p):
    A = np.zeros((m, m))
    bw = 2 * p + 1
    for i in range(m):
        for o in range(bw):
            j = i + o - p
            if 0 <= j < m:
                A[i, j] = band[i * bw + o]
    return A


@pytest.mark.parametrize("n,p,a,method", [(16, 3, 1.0, I.METHOD_FFT), (24, 4, -0.5, I.METHOD_FFT),
                                          (20, 5, 3.0, I.METHOD_DENSE_FD)])
def test_system_matrix_stiffness_with_coefficient(n, p, a, method):
    """The plan's K_c (iffd_opts.coef_a, table 7) equals the oracle's
    variable-coefficient stiffness; the preconditioner's K (table 2) stays the
    Laplacian's."""
    from oracle import bspline
    from oracle import operator as OP
    rc, h = host_plan(3, n, p, method=method, coef_a=a)
    assert rc == 0, I.lib.iffd_last_error()
    m = n + p - 2
    Kc = band_to_dense(read(h, 7, m * (2 * p + 1)), m, p)
    K = band_to_dense(read(h, 2, m * (2 * p + 1)), m, p)
    Ko = OP.Operator(3, n, p, a).K
    K0 = bspline.assemble_dirichlet(n, p)[0]
    assert np.max(np.abs(Kc - Ko)) <= 1e-12 * np.max(np.abs(Ko))
    assert np.max(np.abs(K - K0)) <= 1e-12 * np.max(np.abs(K0))
    I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("a", [-1.0, -2.0, 1001.0, float("nan"), float("inf")])
def test_coefficient_out_of_range_rejected(a):
    rc, h = host_plan(3, 16, 3, coef_a=a)
    assert rc == I.E_INVAL and h.value is None


def test_p1_is_a_valid_iffd_plan():
    """p = 1: S = S^reg, no outliers, no boundary fold (Section 4)."""
    rc, h = host_plan(3, 32, 1)
    assert rc == 0, I.lib.iffd_last_error()
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert (info.m, info.n_reg, info.n_out, info.fft_len) == (31, 31, 0, 32)
    I.lib.iffd_plan_destroy(h)


def test_stepped_pcg_slot_counts_checked_on_the_host():
    """The stepped PCG calls reject a slot count outside 1..max_rhs before
    touching the state (no device work); with a valid count they refuse a
    plan that is not set up."""
    rc, h = host_plan(2, 16, 3, max_rhs=4)
    assert rc == 0
    fake = ctypes.c_void_p(256)
    out = np.zeros(64)
    optr = out.ctypes.data_as(ctypes.c_void_p)
    for ns in (0, -3, 5):
        assert I.lib.iffd_pcg_poll(h, fake, ns, optr, None) == I.E_INVAL
        assert I.lib.iffd_pcg_status(h, fake, ns, fake, None) == I.E_INVAL
        assert I.lib.iffd_pcg_take(h, fake, ns, 0, fake, None) == I.E_INVAL
        assert I.lib.iffd_pcg_iterate(h, fake, ns, 1, None) in (I.E_INVAL, I.E_STATE)
    assert I.lib.iffd_pcg_take(h, fake, 4, 4, fake, None) == I.E_INVAL
    assert I.lib.iffd_pcg_take(h, fake, 4, 0, fake, None) == I.E_STATE
    assert I.lib.iffd_pcg_status(h, fake, 4, fake, None) == I.E_STATE
    assert I.lib.iffd_pcg_poll(h, fake, 4, optr, None) == I.E_STATE
    I.lib.iffd_plan_destroy(h)


def test_noalloc_scratch_limit_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define IFFD_NOALLOC_SCRATCH_BYTES \((\d+)u \* 1024u \* 1024u\)", text)
    assert m and int(m.group(1)) * 1024 * 1024 == I.NOALLOC_SCRATCH_BYTES


def test_noalloc_validates_before_any_launch():
    rc, h = host_plan(2, 16, 3)
    fake = ctypes.c_void_p(256)
    assert I.lib.iffd_precond_apply_noalloc(None, fake, fake, 1, None) == I.E_INVAL
    assert I.lib.iffd_precond_apply_noalloc(h, fake, ctypes.c_void_p(512), 1, None) == I.E_STATE
    I.lib.iffd_plan_destroy(h)


# ---- general plans: per-direction n, p and Dirichlet / natural ends -------

GEN_ENDS = [(1, 1), (1, 0), (0, 1), (0, 0)]


def read_dir(h, k, what, count):
    buf = np.zeros(max(count, 1))
    rc = I.lib.iffd_plan_read_dir(h, k, what, buf.ctypes.data_as(ctypes.c_void_p), len(buf), None)
    assert rc == 0, I.lib.iffd_last_error()
    return buf[:count]


def band_dense(band, m, p):
    A = np.zeros((m, m))
    for i in range(m):
        for o in range(2 * p + 1):
            j = i + o - p
            if 0 <= j < m:
                A[i, j] = band[i * (2 * p + 1) + o]
    return A


@pytest.mark.parametrize("n", [16, 24, 64])
@pytest.mark.parametrize("ends", GEN_ENDS)
def test_general_host_tables_match_oracle(n, ends):
    """Every table the general plan builds on the host for one direction
    against the oracle's general route: dimensions (eq:reg_space_dim), K and
    M (Section 3), the special-basis end blocks AL and AR of V_reg
    (eq:special_basis, the oracle by least-squares collocation, the plan by
    Greville collocation and reflection), Dt (end of Section 6) and the
    regular eigenvalues (Lemma 4's closed form at alpha_j / n vs the
    oracle's seminorm quotients)."""
    from oracle import general as G
    D = {e for e, f in zip((0, 1), ends) if f}
    for p in range(1, 9):
        if n <= p:
            continue
        rc, h = I.create_general(2, [n, 16], [p, 2], [ends, (1, 1)])
        assert rc == 0, I.lib.iffd_last_error()
        di = I.query_dirs(h, 2)[0]
        m, nr, no = G.dims(n, p, D)
        assert (di["m"], di["n_reg"], di["n_out"], di["fft_len"]) == (m, nr, no, 2 * n)
        f = G.factors_route_b(n, p, D)
        lam = read_dir(h, 1, I.TABLE_LAM, m)[:nr]
        ref = f["lam_reg"]
        big = np.abs(ref) > 1e-12
        assert np.all(np.abs(lam[big] - ref[big]) <= 1e-13 * np.abs(ref[big])), p
        assert np.all(np.abs(lam[~big]) <= 1e-12)          # the constant mode of D = {}
        assert np.allclose(read_dir(h, 1, I.TABLE_DT, nr), f["Dt"], rtol=1e-12, atol=0)
        V = f["V_reg"]
        rl, rr = p - ends[0], p - ends[1]
        cl = p // 2 if (ends[0] or p % 2 == 0) else (p + 1) // 2
        cr = p // 2 if (ends[1] or p % 2 == 0) else (p + 1) // 2
        AL = read_dir(h, 1, I.TABLE_V0, rl * cl).reshape(rl, cl)
        AR = read_dir(h, 1, I.TABLE_V1, rr * cr).reshape(rr, cr)
        assert np.abs(V[:rl, :cl] - AL).max(initial=0) <= 1e-13
        assert np.abs(V[m - rr:, nr - cr:] - AR).max(initial=0) <= 1e-13
        # the rest of V_reg is the identity on the interior block
        Vi = V[rl:m - rr, cl:nr - cr]
        assert np.abs(Vi - np.eye(m - rl - rr)).max(initial=0) <= 1e-12
        K = band_dense(read_dir(h, 1, I.TABLE_KBAND, m * (2 * p + 1)), m, p)
        M = band_dense(read_dir(h, 1, I.TABLE_MBAND, m * (2 * p + 1)), m, p)
        assert np.abs(K - f["K"]).max() <= 1e-12 * np.abs(f["K"]).max()
        assert np.abs(M - f["M"]).max() <= 1e-12 * np.abs(f["M"]).max()
        I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("n,p,dl,opts,code", [
    ([16, 16], [3, 3], [(0, 0), (0, 0)], None, I.E_UNSUPPORTED),       # singular
    ([512, 16], [3, 3], [(1, 0), (0, 1)], None, I.E_UNSUPPORTED),      # L = 1024
    ([20, 16], [3, 3], [(1, 0), (0, 1)], None, I.E_UNSUPPORTED),       # n not 2^a, 3 2^a
    ([16, 16], [9, 3], [(1, 0), (0, 1)], None, I.E_INVAL),
    ([16, 8], [3, 8], [(1, 0), (0, 1)], None, I.E_INVAL),              # n <= p
    ([16, 16], [3, 3], [(2, 0), (0, 1)], None, I.E_INVAL),
    ([16, 16], [3, 3], [(1, 0), (0, 1)], (I.METHOD_DENSE_FD, I.PREC_F16S), I.E_INVAL),
    ([16, 16], [3, 3], [(1, 0), (0, 1)], (I.METHOD_FFT, I.PREC_F16S), I.E_INVAL),
])
def test_invalid_general_plans_rejected(n, p, dl, opts, code):
    o = I._Opts(opts[0], opts[1], 1, 0.0) if opts else None
    rc, h = I.create_general(2, n, p, dl, o)
    assert rc == code, (rc, I.lib.iffd_last_error())
    assert not h.value


def test_general_plan_sizes_and_errors():
    rc, h = I.create_general(3, [16, 24, 32], [3, 2, 4], [(1, 0), (0, 1), (0, 0)],
                             I._Opts(I.METHOD_FFT, I.PREC_F32, 2, 0.0))
    assert rc == 0
    dirs = I.query_dirs(h, 3)
    ms = [d["m"] for d in dirs]
    assert ms == [16 + 3 - 1, 24 + 2 - 1, 32 + 4]
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    N = ms[0] * ms[1] * ms[2]
    assert info.N == N and info.m == ms[0]
    assert info.apply_ws_bytes >= 4 * N * 2            # one FP32 tensor per RHS
    assert info.matvec_ws_bytes == 0                   # the operator runs in one pass
    # a single FFT shape: variants cannot be forced; tuning is a no-op
    assert I.lib.iffd_plan_set_variant(h, 0, 0) == I.E_UNSUPPORTED
    buf = np.zeros(8)
    assert I.lib.iffd_plan_read_dir(h, 4, 0, buf.ctypes.data_as(ctypes.c_void_p), 8, None) == I.E_INVAL
    assert I.lib.iffd_plan_read_dir(h, 1, 0, buf.ctypes.data_as(ctypes.c_void_p), 8, None) == I.E_WORKSPACE
    # compute entry points before setup
    assert I.lib.iffd_precond_apply(h, ctypes.c_void_p(256), ctypes.c_void_p(512), 1,
                                    ctypes.c_void_p(1024), 1 << 30, None) == I.E_STATE
    I.lib.iffd_plan_destroy(h)


def geo_ls(nel):
    """The operator workspace's stride per local index: the element count
    padded to an odd multiple of 32 doubles."""
    return (nel + 63) // 64 * 64 + 32


def test_geometry_host_rules():
    """iffd_plan_set_geometry: the kinds and their parameter ranges, d = 3,
    coef_a = 0, the operator workspace 8 ls (p+1)^3 bytes per RHS (ls: the
    element count padded to an odd multiple of 32), and
    IFFD_GEOMETRY_NONE restoring the table size."""
    par = lambda *v: (ctypes.c_double * len(v))(*v)
    rc, h = host_plan(3, 8, 3, max_rhs=2)
    assert rc == 0
    info0 = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info0)) == 0
    assert I.lib.iffd_plan_set_geometry(h, 7, par(0.0), 1) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_BUMP, par(0.2), 1) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_BUMP, None, 0) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_ANNULUS, par(2.0, 1.0, 1.0), 3) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_ANNULUS, par(1.0, 2.0, 0.0), 3) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_ANNULUS, par(1.0, 2.0), 2) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_ANNULUS, par(1.0, 2.0, 1.0), 3) == 0
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.matvec_ws_bytes == 8 * geo_ls(8 ** 3) * 4 ** 3 * 2
    assert info.table_bytes > info0.table_bytes
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_NONE, None, 0) == 0
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.table_bytes == info0.table_bytes
    assert info.matvec_ws_bytes == info0.matvec_ws_bytes
    I.lib.iffd_plan_destroy(h)
    # 2D: the cross sections, two parameters for the annulus and the plate
    _, h2 = host_plan(2, 8, 3)
    assert I.lib.iffd_plan_set_geometry(h2, I.GEOMETRY_BUMP, par(0.01), 1) == 0
    assert I.lib.iffd_plan_set_geometry(h2, I.GEOMETRY_ANNULUS, par(2.0, 1.0), 2) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h2, I.GEOMETRY_ANNULUS, par(1.0), 1) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h2, I.GEOMETRY_PLATE, par(1.0, 2.0), 2) == 0
    info2 = I._Info()
    assert I.lib.iffd_plan_query(h2, ctypes.byref(info2)) == 0
    assert info2.matvec_ws_bytes == 8 * geo_ls(8 ** 2) * 4 ** 2
    I.lib.iffd_plan_destroy(h2)
    _, h3 = host_plan(3, 8, 3, coef_a=0.5)
    assert I.lib.iffd_plan_set_geometry(h3, I.GEOMETRY_BUMP, par(0.01), 1) == I.E_INVAL
    I.lib.iffd_plan_destroy(h3)
    # the plate: 0 < R < L, H > 0, and its corner plane xi_1 = 1/2 on a breakpoint
    _, h4 = host_plan(3, 8, 3)
    assert I.lib.iffd_plan_set_geometry(h4, I.GEOMETRY_PLATE, par(2.0, 1.0, 1.0), 3) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h4, I.GEOMETRY_PLATE, par(1.0, 2.0), 2) == I.E_INVAL
    assert I.lib.iffd_plan_set_geometry(h4, I.GEOMETRY_PLATE, par(1.0, 2.0, 1.0), 3) == 0
    I.lib.iffd_plan_destroy(h4)
    rc, h5 = host_plan(3, 9, 2, method=I.METHOD_DENSE_FD)   # dense FD takes any n > p
    assert rc == 0, I.lib.iffd_last_error()
    assert I.lib.iffd_plan_set_geometry(h5, I.GEOMETRY_PLATE, par(1.0, 2.0, 1.0), 3) == I.E_INVAL
    assert b"even" in I.lib.iffd_last_error()
    I.lib.iffd_plan_destroy(h5)


@pytest.mark.parametrize("n", [16, 24])
@pytest.mark.parametrize("ends", GEN_ENDS)
def test_generic_basis_host_tables_match_oracle(n, ends):
    """iffd_plan_set_basis(IFFD_BASIS_GENERIC) against the oracle's generic
    route (eq:reg_eigenvectors): the orthonormalized end blocks of V_reg and
    D_jj = ||F_j||_L2 of the interpolants (eq:Dreg2); the eigenvalues are the
    special basis's (basis-independent)."""
    from oracle import general as G
    D = {e for e, f in zip((0, 1), ends) if f}
    for p in range(1, 9):
        if n <= p:
            continue
        rc, h = I.create_general(2, [n, 16], [p, 2], [ends, (1, 1)])
        assert rc == 0
        lam_special = read_dir(h, 1, 0, n + p)
        assert I.lib.iffd_plan_set_basis(h, I.BASIS_GENERIC) == 0, I.lib.iffd_last_error()
        di = I.query_dirs(h, 2)[0]
        m, nr = di["m"], di["n_reg"]
        f = G.factors_generic(n, p, D)
        _, cl, _, cr = f["sizes"]
        rl, rr = p - (1 if ends[0] else 0), p - (1 if ends[1] else 0)
        Vg = f["V_reg"]
        if cl:
            AL = read_dir(h, 1, 4, rl * cl).reshape(rl, cl)
            assert np.abs(AL - Vg[:rl, :cl]).max() < 1e-12, (p, ends)
        if cr:
            AR = read_dir(h, 1, 5, rr * cr).reshape(rr, cr)
            assert np.abs(AR - Vg[m - rr:, nr - cr:]).max() < 1e-12, (p, ends)
        Dg = read_dir(h, 1, 1, nr)
        assert np.abs(Dg - f["D"]).max() <= 1e-12 * f["D"].max(), (p, ends)
        lam = read_dir(h, 1, 0, m)
        assert np.array_equal(lam[:nr], lam_special[:nr])
        I.lib.iffd_plan_destroy(h)


def test_basis_rules():
    rc, h = host_plan(3, 16, 3)
    assert rc == 0
    assert I.lib.iffd_plan_set_basis(h, I.BASIS_GENERIC) == I.E_UNSUPPORTED   # uniform plan
    I.lib.iffd_plan_destroy(h)
    rc, h = I.create_general(3, [16, 24, 32], [3, 2, 4], [(1, 0), (0, 1), (0, 0)])
    assert rc == 0
    info0 = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info0)) == 0
    AL0 = read_dir(h, 1, 4, 2)
    assert I.lib.iffd_plan_set_basis(h, 5) == I.E_INVAL
    assert I.lib.iffd_plan_set_basis(h, I.BASIS_GENERIC) == 0
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.table_bytes >= info0.table_bytes          # the interpolation bands
    assert np.linalg.norm(read_dir(h, 1, 4, 2)) == pytest.approx(1.0)   # orthonormal column
    assert I.lib.iffd_plan_set_basis(h, I.BASIS_SPECIAL) == 0
    assert np.array_equal(read_dir(h, 1, 4, 2), AL0)
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.table_bytes == info0.table_bytes
    # a mapped domain keeps its map through a change of basis
    par = (ctypes.c_double * 3)(1.0, 2.0, 1.0)
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_ANNULUS, par, 3) == 0
    assert I.lib.iffd_plan_set_basis(h, I.BASIS_GENERIC) == 0
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.matvec_ws_bytes == 8 * geo_ls(16 * 24 * 32) * (4 * 3 * 5)
    I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("ends", GEN_ENDS)
@pytest.mark.parametrize("p,mult", [(2, 2), (3, 2), (3, 3), (4, 4), (5, 3), (6, 3)])
def test_repeated_knot_host_tables_match_oracle(p, mult, ends):
    """iffd_plan_set_knot (reduced regularity, eq:reg_space2) against
    oracle.reduced: m and n_out grow by mult - 1 (the remark's count), K and M
    of the reduced space, the regular eigenvalues and Dt unchanged (S^reg and
    its functions do not change)."""
    from oracle import reduced as R
    n = 32
    k = 13
    D = {e for e, f in zip((0, 1), ends) if f}
    rc, h = I.create_general(2, [n, 16], [p, 2], [ends, (1, 1)])
    assert rc == 0
    lam0 = read_dir(h, 1, 0, n + p)
    nr0 = I.query_dirs(h, 2)[0]["n_reg"]
    Dt0 = read_dir(h, 1, 1, nr0)
    assert I.lib.iffd_plan_set_knot(h, 1, k, mult) == 0, I.lib.iffd_last_error()
    di = I.query_dirs(h, 2)[0]
    m, nr, no = R.dims(n, p, D, mult)
    assert (di["m"], di["n_reg"], di["n_out"]) == (m, nr, no)
    K, M = R.assemble(n, p, D, k, mult)
    bw = 2 * p + 1
    assert np.abs(band_dense(read_dir(h, 1, 2, m * bw), m, p) - K).max() < 1e-10 * np.abs(K).max()
    assert np.abs(band_dense(read_dir(h, 1, 3, m * bw), m, p) - M).max() < 1e-13
    assert np.abs(read_dir(h, 1, 0, m)[:nr] - lam0[:nr]).max() <= 1e-14 * lam0[:nr].max()
    assert np.abs(read_dir(h, 1, 1, nr) - Dt0).max() <= 1e-12 * Dt0.max()
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.N == m * I.query_dirs(h, 2)[1]["m"]
    I.lib.iffd_plan_destroy(h)


def test_repeated_knot_rules():
    rc, h = host_plan(3, 32, 3)
    assert rc == 0
    assert I.lib.iffd_plan_set_knot(h, 1, 16, 2) == I.E_UNSUPPORTED   # uniform plan
    I.lib.iffd_plan_destroy(h)
    rc, h = I.create_general(3, [32, 24, 32], [3, 2, 4], [(1, 0), (0, 1), (0, 0)])
    assert rc == 0
    assert I.lib.iffd_plan_set_knot(h, 4, 16, 2) == I.E_INVAL        # direction
    assert I.lib.iffd_plan_set_knot(h, 1, 16, 4) == I.E_INVAL        # mult > p
    assert I.lib.iffd_plan_set_knot(h, 1, 32, 2) == I.E_INVAL        # not interior
    assert I.lib.iffd_plan_set_knot(h, 1, 3, 3) == I.E_INVAL         # too close to an end
    assert I.lib.iffd_plan_set_knot(h, 1, 16, 3) == 0
    assert I.query_dirs(h, 3)[0]["m"] == 32 + 3 - 1 + 2
    assert I.lib.iffd_plan_set_basis(h, I.BASIS_GENERIC) == I.E_UNSUPPORTED
    # a mapped domain takes the knot, before or after it is set
    info0, info = I._Info(), I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info0)) == 0
    par = (ctypes.c_double * 3)(1.0, 2.0, 1.0)
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_ANNULUS, par, 3) == 0
    assert I.lib.iffd_plan_set_knot(h, 1, 16, 1) == 0                # back to maximal smoothness
    assert I.query_dirs(h, 3)[0]["m"] == 32 + 3 - 1
    assert I.lib.iffd_plan_set_knot(h, 1, 16, 3) == 0
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.matvec_ws_bytes == 8 * geo_ls(32 * 24 * 32) * (4 * 3 * 5)   # the elements stay
    assert info.table_bytes > info0.table_bytes
    assert I.lib.iffd_plan_set_geometry(h, I.GEOMETRY_NONE, None, 0) == 0
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert info.table_bytes == info0.table_bytes
    I.lib.iffd_plan_destroy(h)


@pytest.mark.parametrize("ends", GEN_ENDS)
def test_general_dense_fd_eigenvalues_match_oracle(ends):
    """Dense FD on a general plan: every direction's eigenvalues of (K_k, M_k)
    (its own size and ends) against the oracle's Jacobi eigensolver."""
    from oracle import eig
    from oracle import general as G
    D = {e for e, f in zip((0, 1), ends) if f}
    for p in (2, 3, 5):
        n = 24
        rc, h = I.create_general(2, [n, 16], [p, 2], [ends, (1, 1)],
                                 I._Opts(I.METHOD_DENSE_FD, I.PREC_F32, 1, 0.0))
        assert rc == 0, I.lib.iffd_last_error()
        di = I.query_dirs(h, 2)[0]
        m = di["m"]
        assert (di["n_reg"], di["n_out"], di["fft_len"]) == (m, 0, 0)
        K, M = G.assemble(n, p, D)
        lam_o, _ = eig.gen_eigh(K, M)
        lam = read_dir(h, 1, 0, m)
        scale = max(abs(lam_o).max(), 1.0)
        assert np.abs(np.sort(lam) - np.sort(lam_o)).max() <= 1e-9 * scale, (p, ends)
        I.lib.iffd_plan_destroy(h)


def _route(h, nrhs):
    return I.lib.iffd_plan_get_route(h, nrhs)


def test_dense2d_route_rules():
    """The small 2-D route: which plans hold the dense Qt tables, the automatic
    choice by batch size, the setter's errors, and the table bytes it adds
    (one FP32 m x m array and m eigenvalues per direction)."""
    rc, h = host_plan(2, 64, 3)
    assert rc == 0, I.lib.iffd_last_error()
    m = O.dims(64, 3)[0]
    assert _route(h, 1) == I.ROUTE_DENSE2D and _route(h, 4096) == I.ROUTE_DENSE2D
    # the automatic choice looks at the plan's batch capacity only
    for max_rhs, want in ((30, I.ROUTE_DENSE2D), (31, I.ROUTE_PASSES)):
        rc, hb = host_plan(2, 64, 3, max_rhs=max_rhs)
        assert rc == 0 and m * m * 2 * m * 30 <= 2 ** 24 < m * m * 2 * m * 31
        assert _route(hb, 1) == want and _route(hb, max_rhs) == want
        assert I.lib.iffd_plan_set_route(hb, I.ROUTE_DENSE2D) == 0
        assert _route(hb, 1) == I.ROUTE_DENSE2D
        I.lib.iffd_plan_destroy(hb)
    assert I.lib.iffd_plan_set_route(h, I.ROUTE_PASSES) == 0
    assert _route(h, 1) == I.ROUTE_PASSES
    assert I.lib.iffd_plan_set_route(h, I.ROUTE_DENSE2D) == 0
    assert _route(h, 7) == I.ROUTE_DENSE2D
    assert I.lib.iffd_plan_set_route(h, 3) == I.E_INVAL
    assert I.lib.iffd_plan_set_route(h, -1) == I.E_INVAL
    assert _route(h, 0) == I.E_INVAL
    info = I._Info()
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    dense_bytes = info.table_bytes
    I.lib.iffd_plan_destroy(h)
    # the same plan with the passes only (FP64 apply) has no dense tables
    rc, h = host_plan(2, 64, 3, prec=I.PREC_F64)
    assert rc == 0
    assert _route(h, 1) == I.ROUTE_PASSES
    assert I.lib.iffd_plan_set_route(h, I.ROUTE_DENSE2D) == I.E_UNSUPPORTED
    assert I.lib.iffd_plan_set_route(h, I.ROUTE_AUTO) == 0
    I.lib.iffd_plan_destroy(h)
    rc, h = host_plan(2, 64, 3)
    assert I.lib.iffd_plan_query(h, ctypes.byref(info)) == 0
    assert dense_bytes == info.table_bytes
    I.lib.iffd_plan_destroy(h)
    # not eligible: 3-D, m > 128, p >= 5 in FP32, dense FD
    for d, n, p, method in [(3, 16, 3, I.METHOD_FFT), (2, 128, 3, I.METHOD_FFT),
                            (2, 64, 5, I.METHOD_FFT), (2, 64, 3, I.METHOD_DENSE_FD)]:
        rc, h = host_plan(d, n, p, method)
        assert rc == 0, (d, n, p)
        assert _route(h, 1) == I.ROUTE_PASSES, (d, n, p, method)
        assert I.lib.iffd_plan_set_route(h, I.ROUTE_DENSE2D) == I.E_UNSUPPORTED
        I.lib.iffd_plan_destroy(h)
    # the largest FFT size below the limit: n = 96, m = 98 at p = 4
    rc, h = host_plan(2, 96, 4)
    assert rc == 0 and O.dims(96, 4)[0] == 98 and _route(h, 1) == I.ROUTE_DENSE2D
    I.lib.iffd_plan_destroy(h)
    # general 2-D plans: per-direction sizes and ends, a repeated knot
    rc, h = I.create_general(2, [48, 32], [3, 4], [(1, 0), (0, 1)])
    assert rc == 0, I.lib.iffd_last_error()
    assert _route(h, 1) == I.ROUTE_DENSE2D
    assert I.lib.iffd_plan_set_knot(h, 1, 24, 2) == 0, I.lib.iffd_last_error()
    assert _route(h, 1) == I.ROUTE_DENSE2D
    I.lib.iffd_plan_destroy(h)
    rc, h = I.create_general(2, [48, 128], [3, 3], [(1, 1), (1, 1)])
    assert rc == 0 and _route(h, 1) == I.ROUTE_PASSES
    I.lib.iffd_plan_destroy(h)
