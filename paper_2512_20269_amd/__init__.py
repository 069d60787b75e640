"""Python binding of libiffd (include/iffd.h): the IFFD preconditioner of
Montardini, Takacs and Tani (arXiv 2512.20269) on MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libiffd.so.  PyTorch supplies device memory (tensors) and streams.
The library must have been built (``python -m paper_2512_20269_amd.build``);
importing this package without it raises immediately.

    import torch, paper_2512_20269_amd as iffd
    plan = iffd.Plan(d=3, n=128, p=3, precision="f32")
    z = plan.apply(r)                    # z = P^{-1} r, r: float64 [m]^d on cuda
    mixed = iffd.Plan(d=3, n=64, p=3,    # per-direction conditions (and n, p)
                      dirichlet=[(1, 0), (0, 1), (0, 0)])
    y = plan.matvec(x)                   # y = A x (Ahat, or A_c with coef_a)
    u, stats = plan.solve(f, rtol=1e-8)  # PCG
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiffd.so")

OK, W_NOT_CONVERGED = 0, 1
E_INVAL, E_UNSUPPORTED, E_HIP, E_BREAKDOWN, E_WORKSPACE, E_STATE = -1, -2, -3, -4, -5, -6
METHOD_FFT, METHOD_DENSE_FD = 0, 1
PREC_F64, PREC_F32, PREC_F16S, PREC_BF16S = 0, 1, 2, 3
GEOMETRY_NONE, GEOMETRY_BUMP, GEOMETRY_ANNULUS, GEOMETRY_PLATE = 0, 1, 2, 3
BASIS_SPECIAL, BASIS_GENERIC = 0, 1
ROUTE_AUTO, ROUTE_PASSES, ROUTE_DENSE2D = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024   # IFFD_NOALLOC_SCRATCH_BYTES

TABLE_LAM, TABLE_DT, TABLE_KBAND, TABLE_MBAND, TABLE_V0, TABLE_V1, TABLE_VT = range(7)


class IffdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"iffd error {code}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("apply_prec", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("coef_a", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int), ("p", ctypes.c_int), ("m", ctypes.c_int),
                ("n_reg", ctypes.c_int), ("n_out", ctypes.c_int), ("fft_len", ctypes.c_int),
                ("method", ctypes.c_int), ("apply_prec", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("N", ctypes.c_int64), ("table_bytes", ctypes.c_size_t),
                ("apply_ws_bytes", ctypes.c_size_t), ("pcg_ws_bytes", ctypes.c_size_t),
                ("matvec_ws_bytes", ctypes.c_size_t),
                ("state_bytes_per_slot", ctypes.c_size_t), ("state_bytes_fixed", ctypes.c_size_t)]


class _DirInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("dirichlet_lo", ctypes.c_int),
                ("dirichlet_hi", ctypes.c_int), ("m", ctypes.c_int), ("n_reg", ctypes.c_int),
                ("n_out", ctypes.c_int), ("fft_len", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("status", ctypes.c_int),
                ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("lanczos_lmin", ctypes.c_double), ("lanczos_lmax", ctypes.c_double),
                ("kappa_est", ctypes.c_double)]


# name -> (restype, argtypes), exactly the declarations of include/iffd.h
_P, _I, _D, _Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "iffd_plan_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, ctypes.POINTER(_Opts)]),
    "iffd_plan_create_general": (_I, [ctypes.POINTER(_P), _I, _P, _P, _P, ctypes.POINTER(_Opts)]),
    "iffd_plan_query": (_I, [_P, ctypes.POINTER(_Info)]),
    "iffd_plan_query_dirs": (_I, [_P, ctypes.POINTER(_DirInfo), _I]),
    "iffd_plan_read_dir": (_I, [_P, _I, _I, _P, _Z, _P]),
    "iffd_plan_set_geometry": (_I, [_P, _I, _P, _I]),
    "iffd_plan_set_basis": (_I, [_P, _I]),
    "iffd_plan_set_knot": (_I, [_P, _I, _I, _I]),
    "iffd_plan_setup": (_I, [_P, _P, _Z, _P]),
    "iffd_plan_read": (_I, [_P, _I, _P, _Z, _P]),
    "iffd_plan_destroy": (None, [_P]),
    "iffd_precond_apply": (_I, [_P, _P, _P, _I, _P, _Z, _P]),
    "iffd_precond_apply_noalloc": (_I, [_P, _P, _P, _I, _P]),
    "iffd_kron_matvec": (_I, [_P, _P, _P, _I, _P, _Z, _P]),
    "iffd_apply_pass_count": (_I, [_P]),
    "iffd_plan_set_variant": (_I, [_P, _I, _I]),
    "iffd_plan_get_variant": (_I, [_P, _I]),
    "iffd_plan_tune": (_I, [_P, _P, _Z, _I, _P]),
    "iffd_plan_set_route": (_I, [_P, _I]),
    "iffd_plan_get_route": (_I, [_P, _I]),
    "iffd_apply_pass": (_I, [_P, _I, _P, _P, _I, _P, _Z, _P]),
    "iffd_pcg_solve": (_I, [_P, _P, _P, _I, _D, _I, _I, ctypes.POINTER(_Stats), _P, _Z, _P]),
    "iffd_pcg_state_init": (_I, [_P, _P, _Z, _I, _P]),
    "iffd_pcg_begin": (_I, [_P, _P, _I, ctypes.POINTER(_I), _I, _P, _D, _I, _P]),
    "iffd_pcg_iterate": (_I, [_P, _P, _I, _I, _P]),
    "iffd_pcg_poll": (_I, [_P, _P, _I, _P, _P]),
    "iffd_pcg_status": (_I, [_P, _P, _I, _P, _P]),
    "iffd_pcg_take": (_I, [_P, _P, _I, _I, _P, _P]),
    "iffd_status_string": (ctypes.c_char_p, [_I]),
    "iffd_last_error": (ctypes.c_char_p, []),
    "iffd_device_ok": (_I, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2512_20269_amd.build` (there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(rc: int, what: str = "") -> int:
    if rc < 0:
        raise IffdError(rc, f"{what}: {lib.iffd_last_error().decode()}")
    return rc


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _need(t, shape, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if tuple(t.shape[-len(shape):]) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (..., {shape})")


def _ints(v, d, name):
    v = [int(x) for x in (v if hasattr(v, "__len__") else [v] * d)]
    if len(v) != d:
        raise ValueError(f"{name} needs {d} entries (direction 1 first)")
    return v


def create_general(d: int, n, p, dirichlet, opts=None):
    """iffd_plan_create_general: a host-side plan handle (no device work);
    n, p: one value or d values, dirichlet: d pairs (end 0, end 1) of 0/1,
    direction 1 first.  Returns (status, handle)."""
    nv, pv = _ints(n, d, "n"), _ints(p, d, "p")
    dv = []
    for pair in dirichlet:
        a, b = pair
        dv += [int(a), int(b)]
    if len(dv) != 2 * d:
        raise ValueError(f"dirichlet needs {d} (end 0, end 1) pairs")
    arr = lambda v: (ctypes.c_int * len(v))(*v)
    h = ctypes.c_void_p()
    o = opts if opts is not None else _Opts(METHOD_FFT, PREC_F32, 1, 0.0)
    rc = lib.iffd_plan_create_general(ctypes.byref(h), d, arr(nv), arr(pv), arr(dv), ctypes.byref(o))
    return rc, h


def query_dirs(h, d: int):
    info = (_DirInfo * d)()
    _check(lib.iffd_plan_query_dirs(h, info, d), "plan_query_dirs")
    return [{f: getattr(x, f) for f, _ in _DirInfo._fields_} for x in info]


class Plan:
    """One (d, n, p) problem with its device tables, workspace and PCG state.

    method: "fft" (IFFD) or "dense" (classical FD); precision: "f32" or "f64"
    for the preconditioner arithmetic (vectors and Krylov work are FP64), or
    "f16s" / "bf16s" (dense FD only: FP16 / BF16 matrix cores with per-line
    scaling).
    coef_a: the system matrix of matvec() and solve() (iffd_opts.coef_a): 0
    for A-hat, else the variable-coefficient A_c with c(x) = 1 + coef_a x in
    every direction; the preconditioner is built from A-hat either way.
    dirichlet: d pairs (end x_k = 0, end x_k = 1), 1 = Dirichlet, 0 = natural
    (Neumann), direction 1 first; given (or n, p given per direction as
    sequences) it makes a general plan (iffd_plan_create_general) whose
    tensors have shape (m_d, .., m_1).
    geometry: None, or (kind, params) with kind "bump" ({eps}), "annulus"
    ({r_in, r_out, H}) or "plate" ({R, L, H}): the system matrix becomes the Galerkin matrix of the
    mapped domain (iffd_plan_set_geometry, d = 3); the preconditioner stays
    that of A-hat.
    basis: "special" (eq:special_basis) or "generic" (general plans: Q_reg =
    C^{-1} U D^{-1} with a banded interpolation solve per line,
    iffd_plan_set_basis).
    knots: general plans, {direction (1-based): (k, mult)}: the breakpoint
    k / n of that direction repeated mult times (reduced regularity,
    iffd_plan_set_knot; one knot per direction)."""

    def __init__(self, d: int, n, p, method: str = "fft", precision: str = "f32",
                 max_rhs: int = 1, device=None, coef_a: float = 0.0, dirichlet=None,
                 geometry=None, basis: str = "special", knots=None):
        torch = _torch()
        self.device = torch.device(device if device is not None else "cuda")
        opts = _Opts(METHOD_FFT if method == "fft" else METHOD_DENSE_FD,
                     {"f32": PREC_F32, "f64": PREC_F64, "f16s": PREC_F16S,
                      "bf16s": PREC_BF16S}[precision], max_rhs,
                     float(coef_a))
        self.coef_a = float(coef_a)
        self.general = (dirichlet is not None or hasattr(n, "__len__") or hasattr(p, "__len__")
                        or bool(knots))
        h = ctypes.c_void_p()
        if self.general:
            dl = dirichlet if dirichlet is not None else [(1, 1)] * d
            rc, h = create_general(d, n, p, dl, opts)
            _check(rc, "plan_create_general")
        else:
            _check(lib.iffd_plan_create(ctypes.byref(h), d, n, p, ctypes.byref(opts)), "plan_create")
        self._h = h
        for direction, (kn, mult) in sorted((knots or {}).items()):
            _check(lib.iffd_plan_set_knot(h, int(direction), int(kn), int(mult)), "plan_set_knot")
        self.basis = basis
        if basis != "special":
            code = {"generic": BASIS_GENERIC}[basis]
            _check(lib.iffd_plan_set_basis(h, code), "plan_set_basis")
        self.geometry = None
        if geometry is not None:
            kind, params = geometry
            code = {"none": GEOMETRY_NONE, "bump": GEOMETRY_BUMP,
                    "annulus": GEOMETRY_ANNULUS, "plate": GEOMETRY_PLATE}[kind]
            par = (ctypes.c_double * max(len(params), 1))(*[float(v) for v in params])
            _check(lib.iffd_plan_set_geometry(h, code, par, len(params)), "plan_set_geometry")
            self.geometry = (kind, tuple(float(v) for v in params))
        info = _Info()
        _check(lib.iffd_plan_query(h, ctypes.byref(info)), "plan_query")
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        self.dirs = query_dirs(h, d)
        self.d, self.n, self.p, self.m = d, n, p, info.m
        self.N, self.max_rhs = info.N, max_rhs
        self.method, self.precision = method, precision
        self.shape = tuple(x["m"] for x in reversed(self.dirs))
        with torch.cuda.device(self.device):
            self.tables = torch.empty(info.table_bytes, dtype=torch.uint8, device=self.device)
            assert self.tables.data_ptr() % 256 == 0
            _check(lib.iffd_plan_setup(h, _ptr(self.tables), info.table_bytes, _stream()),
                   "plan_setup")
        # workspaces of apply() / matvec() / solve(), allocated on first use
        self._ws_t = self._mvws_t = self._pcg_ws = None

    @property
    def _ws(self):
        if self._ws_t is None:
            self._ws_t = _torch().empty(max(self.info["apply_ws_bytes"], 256),
                                        dtype=_torch().uint8, device=self.device)
        return self._ws_t

    @property
    def _mvws(self):
        if self._mvws_t is None:
            self._mvws_t = _torch().empty(max(self.info["matvec_ws_bytes"], 256),
                                          dtype=_torch().uint8, device=self.device)
        return self._mvws_t

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:   # lib is None at interpreter exit
            lib.iffd_plan_destroy(h)
            self._h = None

    # ---- tables ----------------------------------------------------------
    def read_table(self, what: int, direction: int = 1) -> np.ndarray:
        """A host table of direction `direction` (iffd_plan_read_dir)."""
        di = self.dirs[direction - 1]
        m, p = di["m"], di["p"]
        cap = 4 * m * (2 * p + 1) + 8 * m + 64
        buf = np.zeros(cap)
        _check(lib.iffd_plan_read_dir(self._h, direction, what,
                                      buf.ctypes.data_as(ctypes.c_void_p), cap, _stream()),
               "plan_read_dir")
        if self.general:
            rows = lambda dch: p - dch
            cols = lambda dch: p // 2 if (dch or p % 2 == 0) else (p + 1) // 2
            v0 = rows(di["dirichlet_lo"]) * cols(di["dirichlet_lo"])
            v1 = rows(di["dirichlet_hi"]) * cols(di["dirichlet_hi"])
        else:
            v0 = v1 = (p - 1) * (p // 2)
        sizes = {TABLE_LAM: m, TABLE_DT: di["n_reg"], TABLE_KBAND: m * (2 * p + 1),
                 TABLE_MBAND: m * (2 * p + 1), TABLE_V0: v0, TABLE_V1: v1,
                 TABLE_VT: di["n_out"] * m}
        return buf[:sizes[what]].copy()

    # ---- compute ----------------------------------------------------------
    def _batch(self, x, name):
        torch = _torch()
        _need(x, self.shape, torch.float64, name)
        nrhs = 1 if x.dim() == self.d else int(np.prod(x.shape[:-self.d]))
        if nrhs > self.max_rhs:
            raise ValueError(f"{name}: {nrhs} right-hand sides exceed max_rhs={self.max_rhs}")
        return nrhs

    def apply(self, r, out=None, stream=None):
        """z = P^{-1} r (FP64 in/out, batch = leading dims)."""
        torch = _torch()
        nrhs = self._batch(r, "r")
        z = out if out is not None else torch.empty_like(r)
        _need(z, self.shape, torch.float64, "out")
        _check(lib.iffd_precond_apply(self._h, _ptr(r), _ptr(z), nrhs, _ptr(self._ws),
                                      self._ws.numel(), _stream(stream)), "precond_apply")
        return z

    def apply_noalloc(self, r, out=None, stream=None):
        """z = P^{-1} r through iffd_precond_apply_noalloc: no workspace
        argument, the library's per-device scratch array serves instead."""
        torch = _torch()
        nrhs = self._batch(r, "r")
        z = out if out is not None else torch.empty_like(r)
        _need(z, self.shape, torch.float64, "out")
        _check(lib.iffd_precond_apply_noalloc(self._h, _ptr(r), _ptr(z), nrhs, _stream(stream)),
               "precond_apply_noalloc")
        return z

    def set_variant(self, k: int, v: int):
        _check(lib.iffd_plan_set_variant(self._h, k, v), "plan_set_variant")

    def variants(self):
        return [lib.iffd_plan_get_variant(self._h, k) for k in range(self.n_passes())]

    def set_route(self, route):
        """ROUTE_AUTO, ROUTE_PASSES or ROUTE_DENSE2D (or "auto", "passes",
        "dense2d"): how iffd_precond_apply runs a 2-D plan's apply."""
        if isinstance(route, str):
            route = {"auto": ROUTE_AUTO, "passes": ROUTE_PASSES, "dense2d": ROUTE_DENSE2D}[route]
        _check(lib.iffd_plan_set_route(self._h, int(route)), "plan_set_route")

    def route(self, nrhs: int = 1) -> str:
        """The route an apply of nrhs right-hand sides takes: "passes" or "dense2d"."""
        rc = lib.iffd_plan_get_route(self._h, int(nrhs))
        _check(rc if rc < 0 else 0, "plan_get_route")
        return "dense2d" if rc == ROUTE_DENSE2D else "passes"

    def tune(self, reps: int = 20, stream=None):
        """Time both FFT shapes of every pass on the device and keep the faster."""
        torch = _torch()
        if self.method != "fft":
            return []
        nbytes = 16 * self.N + self.info["apply_ws_bytes"] // max(self.max_rhs, 1) + 4096
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _check(lib.iffd_plan_tune(self._h, _ptr(scratch), nbytes, reps, _stream(stream)),
               "plan_tune")
        return self.variants()

    def n_passes(self) -> int:
        return lib.iffd_apply_pass_count(self._h)

    def apply_pass(self, k: int, r, z, stream=None):
        """One pass of apply() (see iffd_apply_pass); z must be preallocated."""
        nrhs = self._batch(r, "r")
        _check(lib.iffd_apply_pass(self._h, k, _ptr(r), _ptr(z), nrhs, _ptr(self._ws),
                                   self._ws.numel(), _stream(stream)), "apply_pass")

    def matvec(self, x, out=None, stream=None):
        """y = A x, the plan's system matrix (Ahat, or A_c for coef_a != 0)."""
        torch = _torch()
        nrhs = self._batch(x, "x")
        y = out if out is not None else torch.empty_like(x)
        _need(y, self.shape, torch.float64, "out")
        _check(lib.iffd_kron_matvec(self._h, _ptr(x), _ptr(y), nrhs, _ptr(self._mvws),
                                    self._mvws.numel(), _stream(stream)), "kron_matvec")
        return y

    def solve(self, f, rtol: float = 1e-8, maxit: int = 500, check_every: int = 1, out=None,
              stream=None):
        """PCG for A u = f (the plan's system matrix, preconditioner built from
        Ahat); returns (u, [stats dict per right-hand side])."""
        torch = _torch()
        nrhs = self._batch(f, "f")
        u = out if out is not None else torch.empty_like(f)
        if self._pcg_ws is None:
            self._pcg_ws = torch.empty(self.info["pcg_ws_bytes"], dtype=torch.uint8,
                                       device=self.device)
        st = (_Stats * nrhs)()
        rc = lib.iffd_pcg_solve(self._h, _ptr(f), _ptr(u), nrhs, rtol, maxit, check_every, st,
                                _ptr(self._pcg_ws), self._pcg_ws.numel(), _stream(stream))
        if rc < 0 and rc != E_BREAKDOWN:
            _check(rc, "pcg_solve")
        stats = [{f_: getattr(s, f_) for f_, _ in _Stats._fields_} for s in st]
        return u, stats


class PcgState:
    """Resident Krylov state for `nslots` solves of one plan (stepped PCG).

    Slots are independent: begin() starts solves in free slots, iterate()
    advances every active slot, poll() reports per-slot progress, take()
    copies a solution out and frees its slot."""

    def __init__(self, plan: Plan, nslots: int, stream=None):
        torch = _torch()
        if nslots > plan.max_rhs:
            raise ValueError("nslots exceeds the plan's max_rhs")
        self.plan, self.nslots = plan, nslots
        nbytes = plan.info["state_bytes_fixed"] + nslots * plan.info["state_bytes_per_slot"]
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=plan.device)
        _check(lib.iffd_pcg_state_init(plan._h, _ptr(self.buf), nbytes, nslots, _stream(stream)),
               "pcg_state_init")

    def begin(self, slots, f, rtol: float = 1e-8, maxit: int = 500, stream=None):
        torch = _torch()
        slots = list(slots)
        _need(f, self.plan.shape, torch.float64, "f")
        arr = (ctypes.c_int * len(slots))(*slots)
        _check(lib.iffd_pcg_begin(self.plan._h, _ptr(self.buf), self.nslots, arr, len(slots),
                                  _ptr(f), rtol, maxit, _stream(stream)), "pcg_begin")

    def iterate(self, k: int = 1, stream=None):
        _check(lib.iffd_pcg_iterate(self.plan._h, _ptr(self.buf), self.nslots, k,
                                    _stream(stream)), "pcg_iterate")

    def poll(self, stream=None) -> np.ndarray:
        """(nslots, 4): active, status (-100 = free slot), iterations, relres."""
        out = np.zeros((self.nslots, 4))
        _check(lib.iffd_pcg_poll(self.plan._h, _ptr(self.buf), self.nslots,
                                 out.ctypes.data_as(ctypes.c_void_p), _stream(stream)), "pcg_poll")
        return out

    def status_async(self, out, stream=None):
        """Enqueue the poll() records into the device tensor `out`
        (nslots x 4 FP64) without waiting."""
        _check(lib.iffd_pcg_status(self.plan._h, _ptr(self.buf), self.nslots, _ptr(out),
                                   _stream(stream)), "pcg_status")

    def take(self, slot: int, out=None, stream=None):
        """Copy slot `slot`'s iterate out and free the slot; slot = -1 copies
        every slot into a (nslots, m, ..) tensor and frees them all."""
        torch = _torch()
        shape = self.plan.shape if slot >= 0 else (self.nslots,) + self.plan.shape
        u = out if out is not None else torch.empty(shape, dtype=torch.float64,
                                                    device=self.plan.device)
        _need(u, self.plan.shape, torch.float64, "out")
        if u.numel() != int(np.prod(shape)):
            raise ValueError(f"out must hold {shape}")
        _check(lib.iffd_pcg_take(self.plan._h, _ptr(self.buf), self.nslots, slot, _ptr(u),
                                 _stream(stream)), "pcg_take")
        return u


class GraphSolver:
    """PCG for a batch of right-hand sides of one plan, with the iteration
    loop replayed from a HIP graph.

    The graph holds `k` PCG iterations over every slot of a resident state
    (iffd_pcg_iterate is asynchronous and allocation-free, and converged
    slots are skipped on the device), captured once per solver.  A solve
    starts the slots eagerly, replays the graph until poll() reports no
    active slot, and copies the solutions out."""

    def __init__(self, plan: Plan, nrhs: int, k: int = 2):
        torch = _torch()
        self.plan, self.nrhs, self.k = plan, nrhs, k
        self.state = PcgState(plan, nrhs)
        self.graph = None
        self._cap = torch.cuda.Stream(device=plan.device)

    def _capture(self):
        torch = _torch()
        g = torch.cuda.CUDAGraph()
        self._cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self._cap):
            with torch.cuda.graph(g, stream=self._cap):
                self.state.iterate(self.k)
        torch.cuda.current_stream().wait_stream(self._cap)
        self.graph = g

    def solve(self, f, rtol: float = 1e-8, maxit: int = 500, out=None):
        """f: (nrhs, m, ..) FP64.  Returns (u, [per-RHS dict: iterations,
        converged, status, relres])."""
        torch = _torch()
        _need(f, self.plan.shape, torch.float64, "f")
        if f.numel() != self.nrhs * self.plan.N:
            raise ValueError(f"f must hold {self.nrhs} right-hand sides")
        self.state.begin(range(self.nrhs), f, rtol, maxit)
        if self.graph is None:
            # capture with every slot inactive would record the same launches;
            # the slots just begun stay untouched until the first replay
            self._capture()
        done = 0
        while True:
            st = self.state.poll()
            if not st[:, 0].any() or done >= maxit:
                break
            self.graph.replay()
            done += self.k
        u = self.state.take(-1, out=out)
        stats = [{"iterations": int(r[2]), "converged": int(r[1]) == 0 and r[0] == 0,
                  "status": int(r[1]), "relres": float(r[3])} for r in st]
        return u, stats


def device_ok() -> bool:
    return bool(lib.iffd_device_ok())
