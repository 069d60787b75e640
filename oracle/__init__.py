"""FP64 CPU oracle for the Isogeometric Fast Fourier-based Diagonalization
(IFFD) preconditioner of Montardini, Takacs and Tani (arXiv 2512.20269).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP implementation.

The oracle is deliberately plain and slow: dense matrices, explicit
O(m^2)-per-line mode products, a textbook Jacobi eigensolver, no FFT.  Each
function cites the passage of the paper it follows.

Modules
    bspline   knots, Cox-de Boor recursion, Gauss assembly of 1-D K and M,
              symmetric cardinal B-splines (Sections 2, 3, 5)
    eig       Cholesky, cyclic Jacobi (round-robin order), generalized pencil
    iffd      splitting of the spline space, the IFFD factors built from the
              definition (route A) and from the special basis (route B),
              Kronecker applications, dense FD (Sections 3, 4, 5, 6)
    krylov    PCG with the paper's stopping rule, CG-Lanczos condition
              estimate (Sections 3, 7)
    brute     dense assembly of the d-dimensional operators for tiny sizes
"""

from . import bspline, eig, iffd, krylov, brute  # noqa: F401
