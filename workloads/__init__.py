"""Seeded synthetic inputs for the IFFD preconditioner workloads.

This module only draws random numbers and lays them out; it contains none of
the method's arithmetic.  Both the CPU oracle (through the tests) and the GPU
path (through the tests and the benchmark) take their inputs from here, so the
two sides always see the same bytes.

Layout convention (Section 2, lexicographic tensor basis): a d-dimensional
coefficient tensor is stored C-contiguous with direction 1 fastest, i.e. as a
NumPy array of shape ``(m_d, ..., m_1)``.  A batch of right-hand sides adds a
leading axis.

The paper's experiments use "random vectors" as right-hand sides
(Section 7); the distribution is not stated, so the reading used here is
i.i.d. uniform on [-1, 1] for the coefficient vector itself.
"""

from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Problem sizes
# ---------------------------------------------------------------------------


def dim_m(n: int, p: int) -> int:
    """Dimension of the Dirichlet-reduced univariate spline space, n + p - 2."""
    return n + p - 2


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_rhs(d: int, n: int, p: int, seed: int) -> np.ndarray:
    """f ~ U[-1, 1]^N, shape (m,)*d, direction 1 fastest."""
    m = dim_m(n, p)
    return rng(seed).uniform(-1.0, 1.0, size=(m,) * d)


def smooth_rhs(d: int, n: int, p: int, seed: int, modes: int = 8,
               noise: float = 1e-3) -> np.ndarray:
    """Sum of `modes` separable random-phase sine modes plus uniform noise.

    f[i_d, ..., i_1] = sum_q prod_k sin(pi * w_{q,k} * t_{i_k} + phi_{q,k})
                       + noise * xi,
    with t_i = i / (m + 1) (i = 1..m), w ~ U{1..8}, phi ~ U[0, 2 pi),
    xi ~ U[-1, 1], drawn in the order w (modes x d), phi (modes x d), xi (N).
    """
    m = dim_m(n, p)
    g = rng(seed)
    w = g.integers(1, 9, size=(modes, d))
    phi = g.uniform(0.0, 2.0 * np.pi, size=(modes, d))
    xi = g.uniform(-1.0, 1.0, size=(m,) * d)
    t = np.arange(1, m + 1, dtype=np.float64) / (m + 1)
    f = np.zeros((m,) * d)
    for q in range(modes):
        term = np.ones((1,) * d)
        for k in range(d):
            # direction k+1 lives on array axis d-1-k
            shape = [1] * d
            shape[d - 1 - k] = m
            term = term * np.sin(np.pi * w[q, k] * t + phi[q, k]).reshape(shape)
        f = f + term
    return f + noise * xi


def uniform_tensor(shape, seed: int) -> np.ndarray:
    """f ~ U[-1, 1] of a given shape (m_d, .., m_1): right-hand sides of
    problems whose directions differ in size (mixed boundary conditions,
    per-direction n and p)."""
    return rng(seed).uniform(-1.0, 1.0, size=tuple(shape))


def batched_uniform_rhs(d: int, n: int, p: int, seeds) -> np.ndarray:
    """One independent generator per right-hand side, so a RHS is the same
    whether it is drawn alone or inside a batch."""
    return np.stack([uniform_rhs(d, n, p, s) for s in seeds])


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper's experiments, Section 7, and the
# single-GPU measurement configurations)
# ---------------------------------------------------------------------------

WORKLOADS = {
    # 2D unit square, n = 64, p = 3 (the Table 2 setting at a small n)
    "square_n64_p3": dict(d=2, n=64, p=3, seed=1, rhs="uniform"),
    # 3D unit cube, n = 128, p = 3 (~2.1M DoFs)
    "cube_n128_p3": dict(d=3, n=128, p=3, seed=2, rhs="uniform"),
    # 3D unit cube, n = 256, p in {2,3,4,6,8}, smooth RHS
    "cube_n256": dict(d=3, n=256, ps=(2, 3, 4, 6, 8), seed=3, rhs="smooth"),
    # 64 right-hand sides on the 3D cube, n = 96, p = 4
    "cube_n96_p4_b64": dict(d=3, n=96, p=4, nrhs=64, seed0=4000, rhs="uniform"),
}

# Section 7's cube with mixed boundary conditions (Table 3): Dirichlet on the
# faces x = 0 and y = 1, natural conditions elsewhere, i.e. per direction
# (Dirichlet at 0, Dirichlet at 1) = (1, 0), (0, 1), (0, 0).
MIXED_CUBE_DIRICHLET = ((1, 0), (0, 1), (0, 0))
# the thick quarter of annulus: Dirichlet on the bottom face xi_3 = 0 only, and
# the map's (r_in, r_out, H)
ANNULUS_DIRICHLET = ((0, 0), (0, 0), (1, 0))
ANNULUS_PARAMS = (1.0, 2.0, 1.0)
# the plate with a hole (the stand-in for Section 7's plate with a C^0 line):
# the map's (R, L, H), the same bottom-face Dirichlet condition as the
# annulus, and the C^0 plane xi_1 = 1/2 as the knot (n_1 / 2, p) of direction 1
PLATE_PARAMS = (1.0, 2.0, 1.0)
PLATE_DIRICHLET = ANNULUS_DIRICHLET


def workload_rhs(name: str, p: int | None = None) -> np.ndarray:
    w = WORKLOADS[name]
    if w["rhs"] == "uniform" and "nrhs" in w:
        return batched_uniform_rhs(w["d"], w["n"], w["p"],
                                   [w["seed0"] + b for b in range(w["nrhs"])])
    if w["rhs"] == "uniform":
        return uniform_rhs(w["d"], w["n"], w["p"], w["seed"])
    assert p is not None
    return smooth_rhs(w["d"], w["n"], p, w["seed"])


# ---------------------------------------------------------------------------
# Serving stream: Poisson arrivals of mixed (d, n, p) solves
# ---------------------------------------------------------------------------

SERVE_NS = (32, 48, 64, 96, 128, 192, 256)
SERVE_PS = (2, 3, 4, 5, 6)


def serving_requests(count: int, qps: float, seed: int = 5, ds=(2, 3),
                     ns=SERVE_NS, ps=SERVE_PS):
    """Request list [(arrival_s, d, n, p, rhs_seed)], inter-arrival Exp(1/qps).

    The right-hand side of request k is uniform_rhs(d, n, p, 5_000_000 + k)."""
    g = rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += g.exponential(1.0 / qps)
        d = int(g.choice(ds))
        n = int(g.choice(ns))
        p = int(g.choice(ps))
        out.append((t, d, n, p, 5_000_000 + k))
    return out
