// Internal plan structure shared by the host setup, the C ABI and the kernel
// launchers.  Not part of the public interface (include/iffd.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/iffd.h"

namespace iffd {

// Byte offsets of every table inside the caller's device table buffer.  Each
// array starts on a 256-byte boundary.  Arrays marked "64" are FP64, "32" FP32.
struct TableLayout {
  size_t lam64, s64, v0_64, v1_64, vt64, twl64, twp64, kb64, mb64, ao64, bo64, vout64;
  size_t qfd64, qtfd64, lamfd64;
  size_t kc64, mc64;  // compact band tables: 2p-1 end rows each side + 1 interior row
  size_t blob64, blob32;  // line-pass tables back to back (see Plan::bo_*)
  size_t lam32, s32, v0_32, v1_32, vt32, twl32, twp32;
  size_t qfd32, qtfd32, lamfd32;
  size_t qfd16, qtfd16, qs16;  // dense FD in FP16: Q / s_Q, Q^T / s_Q, s_Q (FP32)
  size_t dq32, dlam32;         // small 2-D route: dense Qt (m x m, row = dof) and lam, FP32
  size_t stat64;  // setup status word written by the outlier setup kernel (0 = ok)
  size_t unit64;  // general 2D plans: the third direction's band rows, K = 0 and M = 1
  size_t total;
};

// Workspace / state layout of the stepped PCG (all per-slot arrays are
// [nslots][...]).  Offsets in bytes from the start of the state buffer.
struct StateLayout {
  size_t scal;      // [nslots] SlotScalars
  size_t hist;      // [nslots][kHist] alpha/beta history (2 doubles each)
  size_t part;      // [3][nslots][npart] FP64 partial sums
  size_t x, r, p, qz;  // [nslots][N] FP64
  size_t ws;        // preconditioner workspace [nslots][N] (FP32 apply) or 0
  size_t mvws;      // operator workspace (3D: 2 [nslots][N] FP64) or 0
  size_t stat;      // [2][nslots][4] per-slot records for pipelined polling
  size_t fixed, per_slot, total;
  int npart;
};

constexpr int kHist = 256;  // alpha/beta history kept per slot for Lanczos
constexpr int kDenseMax = 128;  // largest m of the small 2-D route (its LDS tiles)

// One direction of a general plan (iffd_plan_create_general): its own n, p and
// boundary conditions.  The spline space drops B_0 when x = 0 is a Dirichlet
// end and the last B-spline when x = 1 is, so m = n + p - #Dirichlet ends.
// V_reg = blkdiag(AL, I, AR) in the special basis of Section 6 (end blocks of
// rl x cl and rr x cr entries, identity in between), U_{s,t} =
// sin(pi (s + sig)(t + tau) / n + beta), s, t = 0 .. n_reg - 1 (Table 1 with
// 0-based indices: sig = node offset, tau = frequency offset, beta = 0 or
// pi/2), S^out the L2-complement of S^reg.
struct GDir {
  int n = 0, p = 0, dlo = 1, dhi = 1;  // dlo / dhi: Dirichlet (1) or Neumann (0) at x = 0 / 1
  int m = 0, n_reg = 0, n_out = 0, L = 0;  // L = 2n: complex FFT length of the transforms
  int rl = 0, cl = 0, rr = 0, cr = 0;
  int sig2 = 0, tau2 = 0, beta = 0;  // 2 sig, 2 tau, beta / (pi / 2)
  std::vector<double> Kb, Mb;        // m x (2p+1) band rows
  std::vector<double> AL, AR;        // rl x cl, rr x cr (row-major)
  int pm = 0;                        // band width of the device copies: 2 pm + 1 (pm = max p)
  std::vector<double> Vout, Ao, Bo;  // n_out x m; outlier pencil n_out x n_out
  std::vector<double> Vt;            // n_out x m, Q_out-rotated (after setup)
  std::vector<double> lam, s, Dt;    // m, m, n_reg (lam's outlier part after setup)
  std::vector<double> tw;            // L complex twiddles e^{-2 pi i k / L}
  std::vector<double> tf;            // 4 n_reg complex twists: pre/post forward, pre/post backward
  int win32[2] = {0, 0}, win64[2] = {0, 0};  // outlier windows (as Plan::win32 / win64)
  // element offsets of this direction's tables inside its blob (FP64 blob and
  // FP32 blob share them): tw | tf | AL | AR | Vt | lam | s | Kb | Mb (the band
  // tables padded to 2 pm + 1 columns)
  int o_tw = 0, o_tf = 0, o_al = 0, o_ar = 0, o_vt = 0, o_lam = 0, o_s = 0, o_kb = 0, o_mb = 0;
  // generic basis of S^reg (eq:reg_eigenvectors): the LU factors of the
  // interpolation matrix C as bands, LB[i][k] = L[i][i - bl + k] (k < bl, unit
  // diagonal implied), UB[i][0] = 1 / U[i][i], UB[i][k] = U[i][i + k] (1 <= k <= bu)
  bool generic = false;
  int bl = 0, bu = 0;
  std::vector<double> LB, UB;
  int o_lb = 0, o_ub = 0;
  // reduced regularity (eq:reg_space2): the breakpoint kk / n repeated mult
  // times, rk = mult - 1 extra B-splines (m counts them, mo = m - rk does
  // not).  The knot insertion E (new kept B-splines x old ones) is the
  // identity on the old columns left of [wk0, wk1) and a shift by rk right of
  // them; EW holds its rows [wk0, wk1 + rk) x columns [wk0, wk1).  The rk
  // outlier vectors it adds are concentrated around the knot: outlier window
  // kwin32 / kwin64 = [kw0, kw1) besides the two end windows.
  int kk = 0, mult = 1, rk = 0, mo = 0, wk0 = 0, wk1 = 0;
  std::vector<double> EW;
  int o_ew = 0;
  int kwin32[2] = {0, 0}, kwin64[2] = {0, 0};
  // dense FD of a general plan (IFFD_METHOD_DENSE_FD): this direction's full
  // eigendecomposition Q^T K Q = diag(lamfd), Q^T M Q = I, and the byte
  // offsets of Q, Q^T and lamfd in the tables (FP64 and FP32 copies)
  std::vector<double> Qfd, lamfd;
  size_t fq64 = 0, fqt64 = 0, flam64 = 0, fq32 = 0, fqt32 = 0, flam32 = 0;
  // dense form of Qt = [V_reg U Dt^{-1}, V_out Q_out] for the small 2-D route:
  // row t < n_reg holds V_reg U e_t / Dt_t (m values, kept while building when
  // m <= kDenseMax), and the byte offsets of Qt (FP32, row i = dof i) and of
  // lam (FP32) in the tables
  std::vector<double> Qreg;
  size_t dq32 = 0, dlam32 = 0;
  int len = 0;
  size_t blob64 = 0, blob32 = 0;            // byte offsets of the blobs in the table buffer
  size_t ao64 = 0, bo64 = 0, vout64 = 0, stat64 = 0;  // outlier setup inputs / status (FP64)
};

// Geometry-mapped system matrix (iffd_plan_set_geometry): per direction the
// Gauss points, weights, and the values and derivatives of the p+1 B-splines of
// every element there (element offsets inside the tables at `off`)
// factors of a map per direction and Gauss point (the element tables' F)
#define GEO_FACTORS 6
struct GeoPlanDir {
  int n = 0, P = 0, lo = 0, m = 0;   // elements, p + 1, full index of kept entry 0, kept
  int kk = 0, rk = 0;                 // breakpoint kk / n repeated rk + 1 times
  int ulo = 0, uhi = -1;              // elements with one shared table (none: ulo > uhi)
  int o_x = 0, o_w = 0, o_v = 0, o_d = 0, o_f = 0;
};
struct GeoPlan {
  int kind = 0;   // IFFD_GEOMETRY_*
  double par[4] = {0, 0, 0, 0};
  GeoPlanDir dir[3];
  std::vector<double> tab;
  size_t off = 0;         // byte offset of the tables
  size_t base_total = 0;  // table bytes of the plan without them
};

struct Plan {
  int d = 0, n = 0, p = 0, m = 0, n_reg = 0, n_out = 0, half = 0, L = 0;
  int method = IFFD_METHOD_FFT, prec = IFFD_PREC_F32, max_rhs = 1;
  int64_t N = 0;

  // host-side FP64 data
  std::vector<double> Kb, Mb;       // m x (2p+1) band rows, column i-p..i+p
  double coef_a = 0.0;              // system matrix: K_c = int (1 + a x) B' B' (0: A-hat)
  std::vector<double> Kop;          // K_c band rows (= Kb for coef_a = 0)
  std::vector<double> V0, V1;       // (p-1) x half, row-major
  std::vector<double> Vout;         // n_out x m (rows = outlier basis vectors)
  std::vector<double> Ao, Bo;       // outlier pencil, n_out x n_out
  std::vector<double> lam;          // m: regular eigenvalues, then outliers
  std::vector<double> Dt;           // n_reg
  std::vector<double> s;            // m: Dt^{-2} on regular modes, 1 on outliers
  std::vector<double> Vt;           // n_out x m, Q_out-rotated (after setup)
  std::vector<double> twl, twp;     // FFT twiddles (interleaved complex)
  std::vector<double> Qfd, lamfd;   // dense FD: m x m (column j = eigvec j)
  std::vector<double> Kc, Mc;       // compact band tables (crows x (2p+1))
  int nbr = 0, crows = 0;
  std::vector<double> sn;           // sin(pi h / n), h = 0..n/2 (odd-p pre-twist)
  // element offsets of the line-pass tables inside one contiguous blob:
  // twl (2L) | Vt (n_out m) | V0 | V1 ((p-1) floor(p/2) each) | sn (n/2+1) |
  // twp (2(n+1)) | lam (m) | s (m)
  int bo_twl = 0, bo_twp = 0, bo_vt = 0, bo_v0 = 0, bo_v1 = 0, bo_lam = 0, bo_s = 0, blob_len = 0;
  int bo_sn = 0;
  // outlier windows per apply precision: Vt[q][j] is used for j < win[0] and
  // j >= win[1] (set at setup from Vt; the full row until then)
  int win32[2] = {0, 0}, win64[2] = {0, 0};

  int variant[5] = {1, 1, 1, 1, 1};  // FFT shape per apply pass (see fft_device.h)
  bool half_len = false;  // sine transforms through length-n FFTs (L = n), else L = 2n
  // FP32 apply: the forward pass along direction 1 (the one that reads the
  // FP64 input) computes in FP64 and writes FP32, so the input is never
  // rounded to FP32 before its first transform (set for p >= 5, where the
  // mass matrices' small eigenvalues amplify that rounding)
  bool first64 = false;

  // small 2-D route (IFFD_ROUTE_DENSE2D): both directions' Qt held densely
  // and applied as two launches of LDS products instead of the three line
  // passes.  dense2d: the plan qualifies (d = 2, FFT method, FP32 apply
  // without first64, every m <= kDenseMax); route: IFFD_ROUTE_*; Qreg: as
  // GDir::Qreg for uniform plans
  bool dense2d = false;
  int route = 0;
  std::vector<double> Qreg;

  // general plans: per-direction n, p and boundary conditions (dirs[0] is
  // direction 1, the fastest index); n, p, m, n_reg, n_out above then hold
  // direction 1's values
  bool gen = false;
  int basis = 0;   // IFFD_BASIS_*: the basis of S^reg of general plans
  GDir dirs[3];

  GeoPlan geo;

  TableLayout lay{};
  char* d_tables = nullptr;
  size_t table_bytes = 0;
  bool ready = false;
};

// host setup (plan.cpp)
int build_plan(Plan& P, int d, int n, int p, const iffd_opts* opts, std::string& err);
int build_plan_general(Plan& P, int d, const int* n, const int* p, const int* dirichlet,
                       const iffd_opts* opts, std::string& err);
int build_geometry(Plan& P, int kind, const double* par, int npar, std::string& err);
int set_plan_basis(Plan& P, int basis, std::string& err);
int set_plan_knot(Plan& P, int direction, int k, int mult, std::string& err);
void compute_layout(Plan& P);
StateLayout state_layout(const Plan& P, int nslots);
size_t apply_ws_bytes(const Plan& P, int nrhs);
int pcg_blocks(const Plan& P);  // number of partial sums per slot
int matvec_blocks(const Plan& P);  // workgroups of the operator per right-hand side
int apply_last_tiles_max(const Plan& P);  // partials of the apply's fused r.z
size_t matvec_ws_bytes(const Plan& P, int nrhs);

// whether an FFT length is supported by the built kernels
bool fft_len_supported(int L);

// records the thread-local message of iffd_last_error() and returns code
int set_last_error(int code, const std::string& msg);

}  // namespace iffd

// the opaque handle of the C ABI
struct iffd_plan {
  iffd::Plan P;
};
