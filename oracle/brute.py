"""Dense d-dimensional operators for tiny sizes (brute force).

Test infrastructure only (see the package docstring).

For N = m^d up to a few hundred the Kronecker sums of Section 3
(eq:system_matrix) and Proposition 1 (eq:preconditioner2) are assembled as
dense N x N matrices, in the lexicographic order of eq:tp-B-basis (direction
1 fastest).  With that order, the d-fold Kronecker product of 1-D matrices
A_d (x) ... (x) A_1 acts with A_1 on the fastest index.
"""

from __future__ import annotations

import numpy as np


def kron_sum(stiff, mass, d: int) -> np.ndarray:
    """sum_k A_d (x) .. (x) A_1 with A_k = stiff, A_j = mass (j != k)."""
    m = stiff.shape[0]
    N = m ** d
    out = np.zeros((N, N))
    for k in range(1, d + 1):
        T = np.ones((1, 1))
        for j in range(d, 0, -1):
            T = np.kron(T, stiff if j == k else mass)
        out += T
    return out


def dense_system(K, M, d: int) -> np.ndarray:
    """Ahat (eq:system_matrix and its 3-D analogue)."""
    return kron_sum(K, M, d)


def dense_preconditioner(Kt, M, d: int) -> np.ndarray:
    """P = sum_k M (x) .. (x) Ktilde (slot k) (x) .. (x) M (eq:preconditioner2)."""
    return kron_sum(Kt, M, d)
