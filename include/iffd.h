/*
 * iffd.h -- C ABI of the MI355X (gfx950) implementation of the Isogeometric
 * Fast Fourier-based Diagonalization (IFFD) preconditioner of Montardini,
 * Takacs and Tani (arXiv 2512.20269), with the matrix-free Kronecker-sum
 * Galerkin operator, preconditioned conjugate gradients, and the classical
 * dense Fast Diagonalization (FD) as a baseline.
 *
 * Problem (Sections 2 and 3 of the paper): Poisson on [0,1]^d, d in {2,3},
 * homogeneous Dirichlet conditions on every face, tensor-product B-splines
 * of degree p and maximal smoothness C^{p-1} on a uniform grid of n elements
 * per direction.  Per direction the reduced spline space has dimension
 * m = n + p - 2; a coefficient vector has N = m^d entries.  General plans
 * (iffd_plan_create_general) give every direction its own n_k, p_k and a
 * Dirichlet or natural (Neumann) condition at each of its two ends (Section 4,
 * "other boundary conditions", Table 1): m_k = n_k + p_k - (number of
 * Dirichlet ends of direction k) and N = m_1 .. m_d.
 *
 * Conventions that hold for every entry point
 *   Layout     a d-dimensional coefficient tensor is stored C-contiguous with
 *              direction 1 fastest: entry (i_1, .., i_d), 0-based, sits at
 *              i_1 + m i_2 + m^2 i_3 (the lexicographic order of the tensor
 *              basis, Section 2).  A batch of nrhs vectors is nrhs such
 *              tensors back to back ([nrhs][m]^d).
 *   Memory     pointers named d_* are device pointers (hipMalloc'd memory of
 *              the current device, e.g. a torch CUDA tensor's data_ptr()),
 *              h_* are host pointers.  The library never allocates device
 *              memory: table, workspace and state sizes are queried from the
 *              plan and the caller owns every buffer.  The plan owns only its
 *              host-side struct and records the table pointer given to
 *              iffd_plan_setup; the table buffer must outlive the plan's use.
 *   Streams    `stream` is a hipStream_t passed as void* (NULL = the null
 *              stream).  Work is enqueued asynchronously unless stated.
 *   Errors     0 = success, > 0 = warning, < 0 = error (codes below).  All
 *              arguments are validated before anything is launched; an error
 *              leaves device buffers untouched.  iffd_last_error() returns a
 *              thread-local message describing the last failure.
 *   Threads    a plan is immutable after iffd_plan_setup and may be used from
 *              several host threads / streams at once, each with its own
 *              workspace or state buffer.
 */
#ifndef IFFD_H
#define IFFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define IFFD_OK               0
#define IFFD_W_NOT_CONVERGED  1   /* PCG stopped at maxit above the tolerance */
#define IFFD_E_INVAL         -1   /* bad argument: null pointer, d, n, p, nrhs  */
#define IFFD_E_UNSUPPORTED   -2   /* valid problem outside the built kernels   */
#define IFFD_E_HIP           -3   /* a HIP runtime call failed                 */
#define IFFD_E_BREAKDOWN     -4   /* PCG breakdown: p.Ap <= 0, r.z <= 0, NaN   */
#define IFFD_E_WORKSPACE     -5   /* workspace / table / state buffer too small */
#define IFFD_E_STATE         -6   /* plan not set up, or used with wrong method */

/* ---- options ----------------------------------------------------------- */
#define IFFD_METHOD_FFT       0   /* IFFD: sine transforms + O(p) outlier block */
#define IFFD_METHOD_DENSE_FD  1   /* classical FD: dense m x m eigenvectors     */

#define IFFD_PREC_F64         0   /* preconditioner arithmetic in FP64          */
#define IFFD_PREC_F32         1   /* preconditioner arithmetic in FP32; inputs,
                                     outputs and all Krylov work stay FP64.  For
                                     p >= 5 the IFFD forward pass along
                                     direction 1, which reads the FP64 input,
                                     computes in FP64 and stores FP32: the
                                     small eigenvalues of the high-degree mass
                                     matrices would otherwise amplify the
                                     rounding of the input itself (Section 3's
                                     mass matrix M in every Kronecker factor) */
#define IFFD_PREC_F16S        2   /* dense FD only: mode products on FP16 matrix
                                     cores (FP32 accumulation), every line along
                                     the transformed direction scaled by its own
                                     max |value| before rounding to FP16, Q by
                                     its max |entry|; FP32 in between          */
#define IFFD_PREC_BF16S       3   /* dense FD only: as IFFD_PREC_F16S with BF16
                                     operands (8-bit significand: larger error,
                                     no overflow concern)                      */

/* system matrix of a mapped domain (iffd_plan_set_geometry) */
#define IFFD_GEOMETRY_NONE     0  /* A-hat (or A_c of iffd_opts.coef_a)          */
#define IFFD_GEOMETRY_BUMP     1  /* the unit cube with an interior bump map      */
#define IFFD_GEOMETRY_ANNULUS  2  /* the thick quarter of annulus                 */
#define IFFD_GEOMETRY_PLATE    3  /* a plate with a hole, C^0 across one plane    */

typedef struct iffd_plan iffd_plan;

typedef struct {
  int method;       /* IFFD_METHOD_*                                           */
  int apply_prec;   /* IFFD_PREC_*                                             */
  int max_rhs;      /* largest batch (nrhs) the workspaces are sized for, >= 1 */
  double coef_a;    /* system matrix of iffd_kron_matvec and iffd_pcg_*: 0 gives
                       A-hat (the Laplacian's Galerkin matrix, Section 3); a != 0
                       gives A_c = sum_k M x .. x K_c (slot k) x .. x M with
                       [K_c]_ij = int (1 + a x) B_j' B_i', the matrix of the
                       weighted form int grad u . D grad v with the diagonal
                       coefficient D = diag(1 + a x_k) (a reading of Section 1's
                       coefficient-weighted form), -1 < a <= 1000.  The
                       preconditioners (IFFD and FD) are always built from
                       A-hat, so for a != 0 neither is exact and
                       kappa(A-hat^{-1} A_c) <= max c / min c (Section 3).   */
} iffd_opts;        /* NULL opts = {IFFD_METHOD_FFT, IFFD_PREC_F32, 1, 0.0}    */

typedef struct {
  int d, n, p;
  int m;            /* n + p - 2                                               */
  int n_reg;        /* dim of the regular subspace: n-1 (p odd), n (p even)    */
  int n_out;        /* dim of the outlier subspace: p-1 (p odd), p-2 (p even)  */
  int fft_len;      /* complex FFT length per pair of lines: n, or 2n for
                       n = 8, 12; 0 for FD                                    */
  int method, apply_prec, max_rhs;
  int64_t N;        /* m^d                                                     */
  size_t table_bytes;      /* device buffer for iffd_plan_setup               */
  size_t apply_ws_bytes;   /* workspace for iffd_precond_apply(nrhs=max_rhs)  */
  size_t pcg_ws_bytes;     /* workspace for iffd_pcg_solve(nrhs=max_rhs)      */
  size_t matvec_ws_bytes;  /* workspace for iffd_kron_matvec(nrhs=max_rhs)    */
  size_t state_bytes_per_slot; /* device state per slot of the stepped PCG    */
  size_t state_bytes_fixed;    /* plus this once per state buffer             */
} iffd_plan_info;

typedef struct {
  int iterations;          /* solution updates until ||r_k|| <= rtol ||f||    */
  int converged;           /* 1 if the tolerance was reached                  */
  int status;              /* IFFD_OK, IFFD_W_NOT_CONVERGED or IFFD_E_BREAKDOWN */
  double relres;           /* ||r_k||_2 / ||f||_2, recursively updated residual */
  double relres_true;      /* ||f - A u_k||_2 / ||f||_2 recomputed at exit     */
  double lanczos_lmin;     /* extreme eigenvalue estimates of P^{-1} A from   */
  double lanczos_lmax;     /*   the CG-Lanczos tridiagonal matrix              */
  double kappa_est;        /* lanczos_lmax / lanczos_lmin                      */
} iffd_pcg_stats;

/* ---- plan ---------------------------------------------------------------
 * iffd_plan_create: host-only.  Builds the univariate spline data for
 * S_{p,h,{0,1}} (Section 2): knots, banded K and M (Section 3), and, for
 * IFFD, the splitting S = S^reg (+) S^out (Section 4, eq:splitting) in the
 * special basis of Section 6 (boundary blocks V_reg,0 / V_reg,1), the
 * outlier basis V_out (L2-orthogonal to S^reg), the normalisation
 * Dt = diag(U^T V_reg^T M V_reg U)^{1/2} and the regular eigenvalues
 * (eq:Lambda reg2); for DENSE_FD, the full FP64 eigendecomposition of the
 * pencil (K, M) (eq:eigendecomposition).  The regular eigenvalues come from
 * the closed form of Lemma 4 (its stiffness symbol scaled by 1/h^2, as in its
 * proof), which equals the Rayleigh quotients of eq:Lambda reg2 without their
 * cancellation on smooth modes; Dt from the mass Rayleigh quotients (end of
 * Section 6).  Valid range: d in {2,3},
 * 1 <= p <= 8, n > p (the paper's standing assumption), m^d*max_rhs < 2^31
 * per pass and m^d < 2^28 (one right-hand side below 2 GiB in FP64, the
 * reach of the kernels' 32-bit buffer offsets); IFFD additionally needs n = 2^a or 3*2^a with 8 <= n <= 512
 * (IFFD_E_UNSUPPORTED otherwise).  For p = 1 IFFD has no outlier space
 * (S = S^reg, Section 4) and is the exact inverse by the DST-I alone.
 * *out receives the plan (NULL on error). */
int iffd_plan_create(iffd_plan** out, int d, int n, int p, const iffd_opts* opts);

/* Host-only, before iffd_plan_setup (IFFD_E_STATE after).  Makes the plan's
 * system matrix (iffd_kron_matvec, the PCG entry points) the Galerkin matrix of
 * the Poisson problem on Omega = F([0,1]^d) pulled back to the parameter cube
 * (Section 2):
 *   A_ij = int grad B_i^T G grad B_j dxi,  G = |det J| J^{-1} J^{-T},  J = dF/dxi,
 * with Gauss-Legendre rules of p_k + 1 points per element and direction,
 * applied matrix-free (per element sum factorization, then a fixed-order
 * gather).  The preconditioners stay those of A-hat, whose condition number
 * against A is bounded by the extremes of G (Section 3).  d = 2 or 3,
 * coef_a = 0.  In 2D the maps are the cross sections below (the annulus and
 * the plate without xi3, params {r_in, r_out} and {R, L}; the bump with
 * phi = sin(pi xi1) sin(pi xi2)).
 *   IFFD_GEOMETRY_BUMP     params {eps}, |eps| < 0.1: F(xi) = xi + eps phi(xi)
 *                          (1, 1, 1), phi = sin(pi xi1) sin(pi xi2) sin(pi xi3):
 *                          the unit cube with a non-separable parametrization
 *                          (A has no Kronecker structure).
 *   IFFD_GEOMETRY_ANNULUS  params {r_in, r_out, H}, 0 < r_in < r_out, H > 0:
 *                          F(xi) = (r c1(xi2), r c2(xi2), H xi3), r = r_in +
 *                          (r_out - r_in) xi1, c the quarter circle as the
 *                          rational quadratic with control points (1,0), (1,1),
 *                          (0,1) and weights 1, 1/sqrt(2), 1 (the thick quarter
 *                          of annulus of Section 7).
 *   IFFD_GEOMETRY_PLATE    params {R, L, H}, 0 < R < L, H > 0, n_1 even:
 *                          F(xi) = ((1 - xi2) R c(xi1) + xi2 o(xi1), H xi3),
 *                          the quarter of the plate [0, L]^2 outside the hole
 *                          of radius R at its corner, extruded to height H;
 *                          c the quarter circle above, o the two outer sides
 *                          (L, 0) -> (L, L) -> (0, L) at constant speed.  F
 *                          is only C^0 across the plane xi1 = 1/2 (from the
 *                          plate's corner to the hole, a breakpoint since n_1
 *                          is even), the setting of Section 7's plate with a
 *                          hole; with iffd_plan_set_knot(plan, 1, n_1 / 2, p_1)
 *                          the spline space is C^0 there too.
 *   IFFD_GEOMETRY_NONE     restores A-hat.
 * On a general plan with a repeated knot (iffd_plan_set_knot) the element
 * tables use the refined knot vector and the p+1 B-splines nonzero on element
 * e start at e, or at e + mult - 1 past the knot, so A is the mapped
 * operator of the reduced-regularity space (Remark rmk:reduced_regularity).
 * The operator needs a workspace of 8 * ls (p1+1)(p2+1)(p3+1) bytes per
 * right-hand side, ls = n1 n2 n3 rounded up to a multiple of 64, plus 32
 * (in 2D n3 = 1 and p3 + 1 = 1; iffd_plan_info.matvec_ws_bytes, included in
 * the PCG state sizes). */
int iffd_plan_set_geometry(iffd_plan* plan, int kind, const double* h_params, int nparams);

/* Sizes and dimensions of a plan.  Host-only, never fails on a valid plan.
 * For a general plan the scalar n, p, m, n_reg, n_out and fft_len are those
 * of direction 1 (iffd_plan_query_dirs gives every direction). */
int iffd_plan_query(const iffd_plan* plan, iffd_plan_info* info);

/* ---- general plans: per-direction n, p and boundary conditions ----------- */
typedef struct {
  int n, p;                       /* elements and degree of this direction    */
  int dirichlet_lo, dirichlet_hi; /* 1: Dirichlet at x_k = 0 / x_k = 1,
                                     0: natural (Neumann) condition            */
  int m;                          /* n + p - dirichlet_lo - dirichlet_hi       */
  int n_reg, n_out;               /* eq:reg_space_dim: n_reg = n - 1 (p odd,
                                     both ends Dirichlet), n + 1 (p odd, no
                                     Dirichlet end), n otherwise; n_out = m -
                                     n_reg                                     */
  int fft_len;                    /* complex FFT length of its transforms      */
} iffd_dir_info;

/* Host-only.  A plan whose direction k (1-based k = 1..d, direction 1 the
 * fastest index) has n[k-1] elements, degree p[k-1], and the boundary
 * conditions dirichlet[2(k-1)] (end x_k = 0) and dirichlet[2(k-1)+1] (end
 * x_k = 1), each 1 for a homogeneous Dirichlet and 0 for a natural (Neumann)
 * condition.  The spline space of direction k drops B_0 at a Dirichlet end 0
 * and the last B-spline at a Dirichlet end 1 (Section 2).  IFFD per
 * direction (Section 4 "other boundary conditions", Section 6): S^reg carries
 * the derivative conditions of eq:reg_space (even orders at Dirichlet ends,
 * odd orders at Neumann ends), its special basis reflects the cardinal
 * B-splines oddly at Dirichlet and evenly at Neumann ends (eq:special_basis),
 * U is the sine or cosine transform of Table 1 (DST-I..IV, DCT-I..IV),
 * computed through complex FFTs of length 2 n_k, and the regular eigenvalues
 * come from Lemma 4's closed form at the frequencies alpha_j / n_k of Table 1.
 * Every entry point takes general plans except iffd_plan_set_variant and
 * iffd_plan_tune (single FFT shape; tune is a no-op).  Valid range: d in
 * {2,3}; per direction 1 <= p <= 8, n > p, n = 2^a or 3*2^a with
 * 8 <= n <= 256 (IFFD_E_UNSUPPORTED otherwise); at least one Dirichlet end
 * (Neumann conditions on every face make the operator singular: the
 * constants; IFFD_E_UNSUPPORTED); opts: method IFFD_METHOD_FFT or
 * IFFD_METHOD_DENSE_FD (every direction's own dense eigendecomposition of
 * (K_k, M_k), the mode products on the matrix cores and the Kronecker-sum
 * scaling in a kernel of its own), apply_prec IFFD_PREC_F32 or IFFD_PREC_F64,
 * coef_a = 0 (IFFD_E_UNSUPPORTED or IFFD_E_INVAL otherwise).
 * iffd_kron_matvec and the PCG use the operator Ahat = sum_k M_d x .. x K_k
 * x .. x M_1 with each direction's own K, M. */
int iffd_plan_create_general(iffd_plan** out, int d, const int* n, const int* p,
                             const int* dirichlet, const iffd_opts* opts);

/* basis of S^reg of a general plan (iffd_plan_set_basis) */
#define IFFD_BASIS_SPECIAL  0  /* eq:special_basis: no interpolation solve      */
#define IFFD_BASIS_GENERIC  1  /* another basis: Q_reg = C^{-1} U D^{-1}        */

/* Host-only, general plans, before iffd_plan_setup (IFFD_E_STATE after;
 * IFFD_E_UNSUPPORTED for uniform plans; IFFD_E_INVAL for another value).
 * IFFD_BASIS_GENERIC writes Q_reg through a basis of S^reg that the sine
 * matrix does not diagonalize (eq:reg_eigenvectors): Q_reg = C^{-1} U D^{-1}
 * with C_ij = psi_j(x_i) the interpolation matrix at the nodes of Table 1
 * (banded; its LU factors, without pivoting, are part of the tables), U the
 * transform of Table 1 and D_jj = ||F_j||_L2 of the interpolants F_j
 * (eq:Dreg2).  The basis: the special basis of eq:special_basis with each of
 * its two end blocks replaced by the orthonormal factor Q of the block's QR
 * factorization (positive diagonal of R).  Every line transform then adds a
 * banded solve with C^T (forward) or C (backward) per line; P^{-1} r itself
 * does not depend on the basis (the same space S^reg, the same eigenvalues),
 * so this variant shows the cost that the special basis removes.  The plan's
 * tables are rebuilt; a mapped domain set before keeps its map.  Returns
 * IFFD_E_UNSUPPORTED if C would need pivoting. */
int iffd_plan_set_basis(iffd_plan* plan, int basis);

/* Host-only, general plans, before iffd_plan_setup (IFFD_E_STATE after).
 * Reduced regularity (Remark rmk:reduced_regularity, eq:reg_space2): the
 * breakpoint k / n_d of direction `direction` (1..d) is repeated `mult` times
 * (1 <= mult <= p_d; mult = 1 restores maximal smoothness; one knot per
 * direction: a later call on the same direction replaces it), so the spline
 * space of that direction is C^{p - mult} there and has mult - 1 more
 * B-splines (m grows by mult - 1; iffd_plan_query_dirs reports it).  S^reg
 * stays the space of C^{p-1} functions with the end conditions of
 * eq:reg_space, whose special-basis functions are written on the new
 * B-splines through the knot-insertion matrix E (Boehm's algorithm: the
 * identity away from the knot, a small block around it); S^out, its L2
 * complement, gains mult - 1 functions concentrated around the knot.  The
 * transforms read and write E^T / E on that window; the operator
 * (iffd_kron_matvec, PCG) uses K and M of the reduced space.  Valid: the
 * knot window at least p B-splines away from both end blocks (about 2p
 * elements from either end; IFFD_E_INVAL otherwise), at most 8 outlier
 * functions per direction, not with IFFD_BASIS_GENERIC (IFFD_E_UNSUPPORTED).
 * A mapped domain set before is rebuilt on the new space. */
int iffd_plan_set_knot(iffd_plan* plan, int direction, int k, int mult);

/* Per-direction sizes: h_out[k-1] describes direction k, for every plan
 * (uniform plans report Dirichlet ends).  count: capacity of h_out (>= d). */
int iffd_plan_query_dirs(const iffd_plan* plan, iffd_dir_info* h_out, int count);

/* Uploads the plan's tables into the caller's device buffer d_tables
 * (>= info.table_bytes bytes, 256-byte aligned), solves the small outlier
 * pencil (V_out^T K V_out, V_out^T M V_out) (eq:eigendecomposition_out) in
 * FP64 on the device, and synchronizes `stream` once.  Must be called before
 * any compute entry point; may be called again with another buffer.  Returns
 * IFFD_E_INVAL (plan not ready) if the outlier pencil's mass block is not
 * positive definite or its eigenpairs are not finite and positive. */
int iffd_plan_setup(iffd_plan* plan, void* d_tables, size_t table_bytes, void* stream);

/* Copies host-side plan data for inspection (tests, diagnostics).  `what`:
 *   0 lam_t  (m doubles: regular eigenvalues then outlier eigenvalues; for FD
 *            the m eigenvalues of (K,M)), 1 Dt (n_reg doubles),
 *   2 K band, 3 M band (m*(2p+1) doubles, row i holds columns i-p..i+p),
 *   4 V_reg,0 ((p-1)*floor(p/2) doubles, row-major), 5 V_reg,1 (same),
 *   6 Vt_out (n_out*m doubles: rows = Q_out-rotated outlier basis vectors,
 *            available after iffd_plan_setup; syncs `stream`),
 *   7 the system matrix's 1-D stiffness band (K_c of iffd_opts.coef_a, the
 *            same as 2 for coef_a = 0; m*(2p+1) doubles).
 * `count` is the capacity of h_out in doubles; returns IFFD_E_WORKSPACE if
 * too small. */
int iffd_plan_read(const iffd_plan* plan, int what, double* h_out, size_t count, void* stream);

/* iffd_plan_read for direction `direction` (1..d) of a general plan (for a
 * uniform plan every direction reads the same tables).  Sizes use that
 * direction's m, n_reg, n_out and p; tables 4 and 5 are its end blocks AL
 * (rl x cl) and AR (rr x cr) of V_reg = blkdiag(AL, I, AR), rl = p - (Dirichlet
 * at 0), cl = floor(p/2) (Dirichlet or p even) or (p+1)/2 (Neumann, p odd),
 * and the same for the end at 1; table 7 equals table 2.  For a general plan
 * iffd_plan_read reads direction 1. */
int iffd_plan_read_dir(const iffd_plan* plan, int direction, int what, double* h_out,
                       size_t count, void* stream);

void iffd_plan_destroy(iffd_plan* plan);

/* ---- compute ------------------------------------------------------------
 * z = P^{-1} r for nrhs right-hand sides (1 <= nrhs <= max_rhs), with
 *   IFFD:  P^{-1} = (Qt x .. x Qt)(sum_k Lt_k)^{-1}(Qt^T x .. x Qt^T)
 *          (eq:preconditioner), Qt = [V_reg U Dt^{-1}, V_out Q_out]
 *          (Sections 4 and 6), applied as d forward line transforms (boundary
 *          fold, sine transform by FFT, outlier dot products), a diagonal
 *          scaling, and d backward line transforms;
 *   FD:    the same with the dense eigenvectors of (K, M) (eq:exact_
 *          diagonalization), i.e. z = Ahat^{-1} r, by MFMA mode products.
 * d_r and d_z: [nrhs][m]^d FP64, must not overlap.  d_ws: >= apply_ws_bytes
 * for max_rhs (scaled by nrhs/max_rhs is enough), 256-byte aligned; may be
 * NULL when apply_ws_bytes is 0. */
int iffd_precond_apply(const iffd_plan* plan, const double* d_r, double* d_z, int nrhs,
                       void* d_ws, size_t ws_bytes, void* stream);

/* y = A x with the plan's system matrix A = sum_k M x .. x K_A (slot k) x .. x M
 * (eq:system_matrix and its 3-term analogue): K_A = K gives Ahat, K_A = K_c
 * for iffd_opts.coef_a != 0 (see iffd_opts).  FP64, matrix-free by sum
 * factorization with the banded 1-D matrices.  d_x, d_y: [nrhs][m]^d FP64, must not overlap.
 * d_ws: >= matvec_ws_bytes (for max_rhs), 256-byte aligned (NULL if 0). */
int iffd_kron_matvec(const iffd_plan* plan, const double* d_x, double* d_y, int nrhs,
                     void* d_ws, size_t ws_bytes, void* stream);

/* Solves A u = f (the plan's system matrix, see iffd_kron_matvec) for nrhs
 * right-hand sides by PCG with this plan's preconditioner (Section 3), which
 * is always built from Ahat; zero initial guess, stopping when
 * ||r_k||_2 <= rtol ||f||_2 for the recursively updated residual (protocol of
 * Section 7; the norm is the reading documented with the oracle) or after
 * maxit iterations.  All vectors, inner products and scalars are FP64 on the
 * device; the host polls convergence flags every `check_every` iterations
 * (<= 0: every iteration).  h_stats: nrhs entries (may be NULL).  Returns the
 * worst status over the batch.  d_ws >= pcg_ws_bytes (for max_rhs). */
int iffd_pcg_solve(const iffd_plan* plan, const double* d_f, double* d_u, int nrhs,
                   double rtol, int maxit, int check_every, iffd_pcg_stats* h_stats,
                   void* d_ws, size_t ws_bytes, void* stream);

/* Allocation-free form of iffd_precond_apply, for callers that cannot
 * allocate or pass device memory of their own (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same kernels
 * and the same result, bit for bit, with the apply's workspace taken from a
 * device array inside the library of IFFD_NOALLOC_SCRATCH_BYTES bytes (one
 * per device, held until the process ends).  The caller passes only r and z
 * (same layout and rules as iffd_precond_apply).  Returns IFFD_E_WORKSPACE
 * when the call needs more workspace than that (apply_ws_bytes scaled to
 * nrhs: 4 N nrhs bytes for the FP32 IFFD apply, none for the FP64 one,
 * 8 N nrhs for dense FD in FP32, 10 N nrhs + 4 N nrhs / m in FP16).  It calls
 * no allocating routine.  Calls on one device share its array: calls that
 * overlap on one device (other streams, other host threads) race and must be
 * serialized by the caller. */
#define IFFD_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int iffd_precond_apply_noalloc(const iffd_plan* plan, const double* d_r, double* d_z, int nrhs,
                               void* stream);

/* One pass of iffd_precond_apply (IFFD only), for per-kernel timing: the
 * apply is the sequence pass = 0 .. iffd_apply_pass_count()-1, where pass k
 * < d-1 is the forward line transform along direction k+1, pass d-1 the fused
 * forward transform / Kronecker-sum scaling / backward transform along
 * direction d, and the remaining passes the backward transforms along
 * directions d-1 .. 1.  Pass 0 reads d_r, the last pass writes d_z, the
 * others work in place on the workspace (FP32 apply) or on d_z (FP64 apply).
 * Same arguments and rules as iffd_precond_apply. */
int iffd_apply_pass_count(const iffd_plan* plan);
int iffd_apply_pass(const iffd_plan* plan, int pass, const double* d_r, double* d_z, int nrhs,
                    void* d_ws, size_t ws_bytes, void* stream);

/* FFT shape of one pass: variant 0 holds 16 (or 24) transform elements per
 * thread, variant 1 holds 8 (or 12) with twice the threads, variant 2 has
 * variant 1's shape with half the lines per workgroup (more workgroups for
 * small problems), variant 3 holds 4 elements per thread and variant 4 has
 * variant 3's shape with half the lines per workgroup (power-of-two transform
 * lengths up to 256; elsewhere both run variant 2).  All compute the same result; they
 * differ in speed.
 * iffd_plan_set_variant forces a choice (variant 0..4; diagnostics, tests);
 * iffd_plan_tune times every variant of every pass on
 * the device (reps launches each, events on `stream`, which it synchronizes)
 * and keeps the faster.  d_scratch: >= 16*N bytes + apply_ws_bytes for one
 * right-hand side, 256-byte aligned; its contents are overwritten.  Tuning
 * mutates the plan: do not run it while the plan is in use on other streams. */
int iffd_plan_set_variant(iffd_plan* plan, int pass, int variant);
int iffd_plan_get_variant(const iffd_plan* plan, int pass);
int iffd_plan_tune(iffd_plan* plan, void* d_scratch, size_t scratch_bytes, int reps, void* stream);

/* Small 2-D route of the IFFD apply (eq:preconditioner with Qt of Sections 4
 * and 6 held densely).  A 2-D plan of the FFT method with an FP32 apply whose
 * directions all have m <= 128 (and p <= 4, where the input may be rounded
 * to FP32 before the first product) also keeps, in its tables, each
 * direction's Qt = [V_reg U Dt^{-1}, V_out Q_out] as a dense FP32 m x m array
 * and its eigenvalues.  iffd_precond_apply, iffd_precond_apply_noalloc and
 * the preconditioner applies of iffd_pcg_solve and the stepped PCG (whose
 * residual update and r . z then run as kernels of their own) can compute
 *   Z = Qt_1 ((Qt_1^T R Qt_2) / (lam_1[a] + lam_2[b])) Qt_2^T
 * as two launches of LDS products: the same P^{-1} r to FP32 rounding, at
 * 4 m^3 multiply-adds per right-hand side instead of the transforms'
 * O(m^2 (log m + p)), but without the line passes' barrier chains, which is
 * what a small apply waits on.  iffd_apply_pass always runs the passes.
 *   IFFD_ROUTE_AUTO     the dense route where the plan has its tables and
 *                       max_rhs m_1 m_2 (m_1 + m_2) <= 2^24 (233
 *                       right-hand sides at m = 33, 30 at m = 65, 9 at
 *                       m = 97; larger batches fill the chip with the line
 *                       passes), else the passes (the default).  The route
 *                       depends on the plan only, never on nrhs, so a
 *                       right-hand side gets the same bits alone and in any
 *                       batch of the plan;
 *   IFFD_ROUTE_PASSES   always the line passes;
 *   IFFD_ROUTE_DENSE2D  always the dense route.
 * iffd_plan_set_route is host-only; it returns IFFD_E_UNSUPPORTED for
 * IFFD_ROUTE_DENSE2D on a plan without the dense tables and IFFD_E_INVAL for
 * another value.  iffd_plan_get_route returns the route an apply of nrhs
 * (>= 1) right-hand sides takes (IFFD_ROUTE_PASSES or IFFD_ROUTE_DENSE2D),
 * or a negative status.  Both are valid before and after iffd_plan_setup. */
#define IFFD_ROUTE_AUTO     0
#define IFFD_ROUTE_PASSES   1
#define IFFD_ROUTE_DENSE2D  2
int iffd_plan_set_route(iffd_plan* plan, int route);
int iffd_plan_get_route(const iffd_plan* plan, int nrhs);

/* ---- stepped PCG on resident state (continuous batching) -----------------
 * A state buffer holds `nslots` independent PCG solves of one plan: bytes =
 * state_bytes_fixed + nslots * state_bytes_per_slot.  Slots are independent:
 * a slot's arithmetic does not depend on the other slots (no cross-slot
 * reduction, fixed reduction order), so its result is the same alone or in a
 * batch.  All calls are asynchronous on `stream`.  1 <= nslots <= max_rhs.
 * The library records the plan and nslots each buffer was initialised with;
 * begin, iterate, poll, status and take return IFFD_E_STATE for a buffer
 * that was not initialised, or was initialised with another plan or another
 * nslots (the offsets inside the buffer follow from both). */

/* Zeroes the state (every slot free).  Must be called once per buffer. */
int iffd_pcg_state_init(const iffd_plan* plan, void* d_state, size_t state_bytes, int nslots,
                        void* stream);

/* Starts solves in the listed slots: copies f (count vectors, [count][m]^d
 * FP64) into the slots, sets x = 0, r = f, z = P^{-1} r, p = z, and marks them
 * active with tolerance rtol and iteration limit maxit.  h_slots: count slot
 * indices (host array), distinct, each < nslots. */
int iffd_pcg_begin(const iffd_plan* plan, void* d_state, int nslots, const int* h_slots,
                   int count, const double* d_f, double rtol, int maxit, void* stream);

/* Runs k PCG iterations on every active slot of the state (inactive and
 * free slots are skipped).  Capturable in a HIP graph. */
int iffd_pcg_iterate(const iffd_plan* plan, void* d_state, int nslots, int k, void* stream);

/* Enqueues a copy of the per-slot status into pinned or pageable host memory
 * h_out (nslots records of 4 doubles: active, converged-or-status code,
 * iterations, relres) and synchronizes `stream`. */
int iffd_pcg_poll(const iffd_plan* plan, const void* d_state, int nslots, double* h_out,
                  void* stream);

/* Asynchronous form of iffd_pcg_poll: enqueues on `stream` a kernel that
 * writes the same nslots records of 4 doubles into device memory d_out
 * (the caller copies them out and waits on an event of its own).  Lets a
 * scheduler watch many states without blocking on any one of them. */
int iffd_pcg_status(const iffd_plan* plan, const void* d_state, int nslots, double* d_out,
                    void* stream);

/* Copies the current iterate of slot `slot` into d_u ([m]^d FP64) and frees
 * the slot; slot = -1 copies every slot (d_u holds nslots vectors,
 * [nslots][m]^d) and frees them all.  Asynchronous. */
int iffd_pcg_take(const iffd_plan* plan, void* d_state, int nslots, int slot, double* d_u,
                  void* stream);

/* ---- diagnostics ---------------------------------------------------------- */
const char* iffd_status_string(int status);
const char* iffd_last_error(void);
/* 1 if the HIP device visible as current is gfx950, 0 otherwise. */
int iffd_device_ok(void);

#ifdef __cplusplus
}
#endif
#endif /* IFFD_H */
