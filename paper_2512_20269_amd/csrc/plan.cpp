// Host-side FP64 construction of the univariate IFFD / FD factors.
//
// Everything here runs once per plan (not on the timed path).  The
// construction follows the paper:
//   Section 2   p-open uniform knot vector, B-splines, Dirichlet reduction
//               (the first and last B-spline are dropped, m = n + p - 2);
//   Section 3   1-D stiffness K and mass M (banded, half-bandwidth p);
//   Section 4   splitting S = S^reg (+) S^out; V_reg has the block structure
//               blkdiag(V_reg,0, I, V_reg,1); S^out is the L2-orthogonal
//               complement, spanned by M^{-1} W with W spanning the Euclidean
//               complement of range(V_reg) (so V_reg^T M V_out = 0);
//   Section 6   the special basis (eq:special_basis_dirichlet): reflected
//               cardinal B-splines at the ends, plain ones inside, for which
//               Q_reg = U Dt^{-1} with U = [sin(x_i alpha_j)] (Table 1) and
//               Dt = diag(U^T V_reg^T M V_reg U)^{1/2};
//   Lemma 4     regular eigenvalues in closed form (the Rayleigh quotients
//               of eq:Lambda reg2 of the exact modes, without cancellation).
// The small outlier pencil is solved later on the device (setup kernel).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace iffd {
namespace {

constexpr long double kPi = 3.141592653589793238462643383279502884L;

// ---------------------------------------------------------------------------
// B-spline evaluation on a knot vector U (de Boor / Piegl-Tiller triangle).
// ---------------------------------------------------------------------------

int find_span(int nb, int p, double u, const std::vector<double>& U) {
  // span s in [p, nb-1] with U[s] <= u < U[s+1]; the right end belongs to
  // the last non-empty span
  if (u >= U[nb]) return nb - 1;
  int lo = p, hi = nb;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (u < U[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

// values (ders[0][j]) and first derivatives (ders[1][j]) of the p+1 B-splines
// N_{s-p+j}, j = 0..p, that are non-zero on span s.
void basis_and_derivative(int s, double u, int p, const std::vector<double>& U,
                          std::vector<double>& val, std::vector<double>& der) {
  std::vector<double> left(p + 1), right(p + 1);
  // ndu[j][r]: upper triangle = basis values of increasing degree,
  // lower triangle = knot differences
  std::vector<std::vector<double>> ndu(p + 1, std::vector<double>(p + 1, 0.0));
  ndu[0][0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = u - U[s + 1 - j];
    right[j] = U[s + j] - u;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      ndu[j][r] = right[r + 1] + left[j - r];
      double t = ndu[r][j - 1] / ndu[j][r];
      ndu[r][j] = saved + right[r + 1] * t;
      saved = left[j - r] * t;
    }
    ndu[j][j] = saved;
  }
  val.assign(p + 1, 0.0);
  der.assign(p + 1, 0.0);
  for (int j = 0; j <= p; ++j) val[j] = ndu[j][p];
  if (p == 0) return;
  // derivative from the degree p-1 values: N'_{i,p} = p N_{i,p-1}/(U_{i+p}-U_i)
  //                                               - p N_{i+1,p-1}/(U_{i+p+1}-U_{i+1})
  // ndu[j][p-1], j = 0..p-1, are N_{s-p+1+j, p-1}.
  for (int j = 0; j <= p; ++j) {
    int i = s - p + j;  // global index of the degree-p function
    double a = 0.0, b = 0.0;
    if (j >= 1) {        // N_{i,p-1} = ndu[j-1][p-1]
      double den = U[i + p] - U[i];
      if (den > 0) a = ndu[j - 1][p - 1] / den;
    }
    if (j <= p - 1) {    // N_{i+1,p-1} = ndu[j][p-1]
      double den = U[i + p + 1] - U[i + 1];
      if (den > 0) b = ndu[j][p - 1] / den;
    }
    der[j] = p * (a - b);
  }
}

// Gauss-Legendre rule on [-1,1] with q points (Newton on P_q).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    long double z = std::cos(kPi * (i + 0.75L) / (q + 0.5L));
    long double dp = 1;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = z; p0 = 1; }
      dp = q * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    // recompute the derivative at the converged node
    long double p0 = 1, p1 = z;
    for (int k = 2; k <= q; ++k) {
      long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (z * p1 - p0) / (z * z - 1);
    x[i] = (double)z;
    w[i] = (double)(2 / ((1 - z * z) * dp * dp));
  }
}

// Symmetric cardinal B-spline of degree p centred at 0 (support of width
// p+1), by the Cox-de Boor recursion on the uniform knots k - (p+1)/2.
template <typename R>
R cardinal_t(int p, R t) {
  std::vector<R> N(p + 1);
  R t0 = -(p + 1) / R(2);
  for (int i = 0; i <= p; ++i) {
    R a = t0 + i;
    N[i] = (t >= a && t < a + 1) ? R(1) : R(0);
  }
  for (int q = 1; q <= p; ++q)
    for (int i = 0; i + q <= p; ++i) {
      R a = t0 + i;
      N[i] = ((t - a) * N[i] + (a + q + 1 - t) * N[i + 1]) / q;
    }
  return N[0];
}
double cardinal(int p, double t) { return cardinal_t<double>(p, t); }

// Regular eigenvalue of mode j (Lemma 4, with the stiffness symbol's h
// scaling taken from its proof): with theta = j pi / n,
//   lambda_j = (2 - 2 cos theta) / h^2 * sK(theta) / sM(theta),
//   sM = sum_{|k| <= p} B_{2p+1}(k) cos(k theta),
//   sK = sum_{|k| <= p-1} B_{2p-1}(k) cos(k theta),
// B_q the symmetric cardinal B-spline of degree q.  It equals the Rayleigh
// quotient |F_j|^2_H1 / ||F_j||^2_L2 (eq:Lambda reg2) of the exact mode, but
// 2 - 2 cos theta is formed as 4 sin^2(theta / 2) in extended precision, so
// the smooth modes keep full relative accuracy (the quotient x^T K x /
// x^T M x of the FP64 band matrices cancels like eps * n^2 on them).
double lambda_reg_closed(int n, int p, int j) {
  typedef long double R;
  const R pi = kPi;
  R sM = cardinal_t<R>(2 * p + 1, R(0)), sK = cardinal_t<R>(2 * p - 1, R(0));
  for (int k = 1; k <= p; ++k) {
    // cos(k j pi / n) with the angle reduced exactly modulo 2 pi
    const long long a = ((long long)k * j) % (2LL * n);
    const R c = std::cos(pi * (R)a / (R)n);
    sM += 2 * cardinal_t<R>(2 * p + 1, (R)k) * c;
    if (k <= p - 1) sK += 2 * cardinal_t<R>(2 * p - 1, (R)k) * c;
  }
  const R s = std::sin(pi * (R)j / (R)(2 * n));
  return (double)(4 * (R)n * (R)n * s * s * sK / sM);
}

// The same closed form at theta = j2 pi / (2n) (j2 an integer), the
// frequencies alpha_j / n of every row of Table 1: j pi / n (Dirichlet at both
// ends), (j - 1/2) pi / n (one Dirichlet end), (j - 1) pi / n (none).
double lambda_reg_half(int n, int p, int j2) {
  typedef long double R;
  const R pi = kPi;
  R sM = cardinal_t<R>(2 * p + 1, R(0)), sK = cardinal_t<R>(2 * p - 1, R(0));
  for (int k = 1; k <= p; ++k) {
    const long long a = ((long long)k * j2) % (4LL * n);
    const R c = std::cos(pi * (R)a / (R)(2 * n));
    sM += 2 * cardinal_t<R>(2 * p + 1, (R)k) * c;
    if (k <= p - 1) sK += 2 * cardinal_t<R>(2 * p - 1, (R)k) * c;
  }
  const R s = std::sin(pi * (R)j2 / (R)(4 * n));
  return (double)(4 * (R)n * (R)n * s * s * sK / sM);
}

// Dense LU with partial pivoting; solves A X = B in place (A n x n, B n x k),
// both row-major.  Returns false if singular.
bool lu_solve(int n, std::vector<double> A, std::vector<double>& B, int k) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
      for (int j = 0; j < k; ++j) std::swap(B[c * k + j], B[piv * k + j]);
    }
    for (int r = c + 1; r < n; ++r) {
      double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      for (int j = 0; j < k; ++j) B[r * k + j] -= f * B[c * k + j];
    }
  }
  for (int c = n - 1; c >= 0; --c)
    for (int j = 0; j < k; ++j) {
      double s = B[c * k + j];
      for (int q = c + 1; q < n; ++q) s -= A[c * n + q] * B[q * k + j];
      B[c * k + j] = s / A[c * n + c];
    }
  return true;
}

// Cyclic Jacobi for a dense symmetric n x n matrix A (row-major, destroyed).
// On return w holds the eigenvalues and V (row-major, column j = eigenvector
// j), both unsorted.
void jacobi(int n, std::vector<double>& A, std::vector<double>& V, std::vector<double>& w) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        if (std::fabs(apq) <= std::max(eps * std::sqrt(std::fabs(app * aqq)), 1e-300)) continue;
        rotated = true;
        double th = (aqq - app) / (2 * apq);
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {  // rows p, q
          double a = A[(size_t)p * n + k], b = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * a - s * b;
          A[(size_t)q * n + k] = s * a + c * b;
        }
        for (int k = 0; k < n; ++k) {  // columns p, q
          double a = A[(size_t)k * n + p], b = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * a - s * b;
          A[(size_t)k * n + q] = s * a + c * b;
          double va = V[(size_t)k * n + p], vb = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * va - s * vb;
          V[(size_t)k * n + q] = s * va + c * vb;
        }
      }
    if (!rotated) break;
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

}  // namespace

bool fft_len_supported(int L) {
  static const int ok[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
  for (int v : ok)
    if (v == L) return true;
  return false;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// the small 2-D route needs both directions' dense Qt in FP32 with the input
// rounded to FP32 before its first product (so not where first64 is set)
static bool dense2d_ok(const Plan& P) {
  if (P.d != 2 || P.method != IFFD_METHOD_FFT || P.prec != IFFD_PREC_F32 || P.first64) return false;
  if (!P.gen) return P.m <= kDenseMax && P.Qreg.size() == (size_t)P.n_reg * P.m;
  for (int k = 0; k < 2; ++k) {
    const GDir& G = P.dirs[k];
    if (G.m > kDenseMax || G.Qreg.size() != (size_t)G.n_reg * G.m) return false;
  }
  return true;
}

void compute_layout(Plan& P) {
  TableLayout& t = P.lay;
  {
    const int nbh = (P.p - 1) * P.half;
    int o = 0;
    // ordered by use: every pass reads twl, Vt, V0, V1; odd p through
    // length-n FFTs also sn, even p twp; only the middle pass reads lam and s
    // (a pass stages just its prefix in LDS)
    P.bo_twl = o; o += 2 * std::max(P.L, 1);
    P.bo_vt = o;  o += P.n_out * P.m;
    P.bo_v0 = o;  o += nbh;
    P.bo_v1 = o;  o += nbh;
    P.bo_sn = o;  o += P.n / 2 + 1;
    o += o & 1;
    P.bo_twp = o; o += 2 * (P.n + 1);
    P.bo_lam = o; o += P.m;
    P.bo_s = o;   o += P.m;
    P.blob_len = o + (o & 1);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 8));
    return o;
  };
  const int m = P.m, bw = 2 * P.p + 1, nb = (P.p - 1) * P.half;
  const bool fd = P.method == IFFD_METHOD_DENSE_FD;
  const size_t mm = fd ? (size_t)m * m : 1;
  t.lam64 = take(8 * m);
  t.s64 = take(8 * m);
  t.v0_64 = take(8 * nb);
  t.v1_64 = take(8 * nb);
  t.vt64 = take(8 * (size_t)P.n_out * m);
  t.twl64 = take(16 * (size_t)std::max(P.L, 1));
  t.twp64 = take(16 * (size_t)(P.n + 1));
  t.kb64 = take(8 * (size_t)m * bw);
  t.mb64 = take(8 * (size_t)m * bw);
  t.ao64 = take(8 * (size_t)P.n_out * P.n_out);
  t.bo64 = take(8 * (size_t)P.n_out * P.n_out);
  t.vout64 = take(8 * (size_t)P.n_out * m);
  t.qfd64 = take(8 * mm);
  t.qtfd64 = take(8 * mm);
  t.lamfd64 = take(8 * m);
  t.kc64 = take(8 * (size_t)std::max(P.crows, 1) * bw);
  t.mc64 = take(8 * (size_t)std::max(P.crows, 1) * bw);
  t.lam32 = take(4 * m);
  t.s32 = take(4 * m);
  t.v0_32 = take(4 * nb);
  t.v1_32 = take(4 * nb);
  t.vt32 = take(4 * (size_t)P.n_out * m);
  t.twl32 = take(8 * (size_t)std::max(P.L, 1));
  t.twp32 = take(8 * (size_t)(P.n + 1));
  t.qfd32 = take(4 * mm);
  t.qtfd32 = take(4 * mm);
  t.lamfd32 = take(4 * m);
  const bool f16 = fd && (P.prec == IFFD_PREC_F16S || P.prec == IFFD_PREC_BF16S);
  t.qfd16 = take(f16 ? 2 * mm : 8);
  t.qtfd16 = take(f16 ? 2 * mm : 8);
  t.qs16 = take(8);
  P.dense2d = dense2d_ok(P);
  t.dq32 = take(P.dense2d ? 4 * (size_t)m * m : 8);
  t.dlam32 = take(P.dense2d ? 4 * (size_t)m : 8);
  t.stat64 = take(8);
  t.blob64 = take(8 * (size_t)P.blob_len);
  t.blob32 = take(4 * (size_t)P.blob_len);
  t.total = off;
}

int pcg_blocks(const Plan& P) {
  // partial sums per slot: one per 1024 elements, capped
  int64_t b = (P.N + 1023) / 1024;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 2048);
}

size_t apply_ws_bytes(const Plan& P, int nrhs) {
  // FD: two FP32 buffers, or one FP64 buffer used in turn with the output;
  // IFFD: one FP32 buffer (the FP64 apply works in place on the output)
  // FD in FP16: the two FP32 buffers, an FP16 copy of the operand and one FP32
  // scale per line
  if (P.method == IFFD_METHOD_DENSE_FD && (P.prec == IFFD_PREC_F16S || P.prec == IFFD_PREC_BF16S))
    return align256((size_t)8 * P.N * nrhs) + align256((size_t)2 * P.N * nrhs) +
           align256((size_t)4 * (P.N / P.m) * nrhs);
  if (P.method == IFFD_METHOD_DENSE_FD) return align256((size_t)8 * P.N * nrhs);
  if (P.prec == IFFD_PREC_F32) return align256((size_t)4 * P.N * nrhs);
  return 0;
}

StateLayout state_layout(const Plan& P, int nslots) {
  StateLayout s{};
  s.npart = std::max(std::max(pcg_blocks(P), matvec_blocks(P)), apply_last_tiles_max(P));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 8));
    return o;
  };
  s.scal = take((size_t)nslots * 16 * 8);
  s.hist = take((size_t)nslots * kHist * 2 * 8);
  s.part = take((size_t)3 * nslots * s.npart * 8);
  s.x = take((size_t)nslots * P.N * 8);
  s.r = take((size_t)nslots * P.N * 8);
  s.p = take((size_t)nslots * P.N * 8);
  s.qz = take((size_t)nslots * P.N * 8);
  size_t ws = apply_ws_bytes(P, nslots);
  s.ws = ws ? take(ws) : 0;
  size_t mw = matvec_ws_bytes(P, nslots);
  s.mvws = mw ? take(mw) : 0;
  s.stat = take((size_t)2 * nslots * 4 * 8);
  s.total = off;
  // linear in nslots up to alignment: report a safe per-slot bound
  s.per_slot = align256(16 * 8) + align256(kHist * 16) + align256((size_t)3 * s.npart * 8) +
               4 * align256((size_t)P.N * 8) + apply_ws_bytes(P, 1) + matvec_ws_bytes(P, 1) +
               align256(2 * 4 * 8) + 8 * 256;
  s.fixed = 4096;
  return s;
}

// Full generalized eigendecomposition of a banded pencil (K, M) (rows of
// 2p+1 band entries, m x m): M = L L^T (Cholesky), C = L^{-1} K L^{-T}
// (cyclic Jacobi), Q = L^{-T} Z, eigenpairs in ascending order; Q^T M Q = I,
// Q^T K Q = diag(w) (eq:eigendecomposition, the dense FD of Section 3).
static int dense_pencil(const std::vector<double>& Kb, const std::vector<double>& Mb, int m, int p,
                        std::vector<double>& Qfd, std::vector<double>& lamfd, std::string& err) {
  const int bw = 2 * p + 1;
  // full generalized eigendecomposition of (K, M): M = L L^T, C = L^-1 K L^-T
  std::vector<double> L((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    for (int i = j; i < std::min(m, j + p + 1); ++i) {
      double sum = Mb[(size_t)i * bw + (j - i + p)];
      for (int k = std::max(0, i - p); k < j; ++k) sum -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
      if (i == j) {
        if (!(sum > 0)) { err = "mass matrix not SPD"; return IFFD_E_INVAL; }
        L[(size_t)j * m + j] = std::sqrt(sum);
      } else {
        L[(size_t)i * m + j] = sum / L[(size_t)j * m + j];
      }
    }
  }
  // X = L^{-1} K (dense), then C = X L^{-T} = (L^{-1} X^T)^T
  std::vector<double> Kd((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int o = 0; o < bw; ++o) {
      int j = i + o - p;
      if (j >= 0 && j < m) Kd[(size_t)i * m + j] = Kb[(size_t)i * bw + o];
    }
  auto lower_solve_cols = [&](std::vector<double>& B) {  // B <- L^{-1} B (m x m)
    for (int c = 0; c < m; ++c)
      for (int i = 0; i < m; ++i) {
        double sum = B[(size_t)i * m + c];
        for (int k = std::max(0, i - p); k < i; ++k) sum -= L[(size_t)i * m + k] * B[(size_t)k * m + c];
        B[(size_t)i * m + c] = sum / L[(size_t)i * m + i];
      }
  };
  lower_solve_cols(Kd);
  std::vector<double> T((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) T[(size_t)i * m + j] = Kd[(size_t)j * m + i];
  lower_solve_cols(T);
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) {
      double a = 0.5 * (T[(size_t)i * m + j] + T[(size_t)j * m + i]);
      T[(size_t)i * m + j] = T[(size_t)j * m + i] = a;
    }
  std::vector<double> Z, w;
  jacobi(m, T, Z, w);
  // Q = L^{-T} Z (back substitution on each column)
  std::vector<double> Q = Z;
  for (int c = 0; c < m; ++c)
    for (int i = m - 1; i >= 0; --i) {
      double sum = Q[(size_t)i * m + c];
      for (int k = i + 1; k < std::min(m, i + p + 1); ++k) sum -= L[(size_t)k * m + i] * Q[(size_t)k * m + c];
      Q[(size_t)i * m + c] = sum / L[(size_t)i * m + i];
    }
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a] < w[b]; });
  Qfd.assign((size_t)m * m, 0.0);
  lamfd.assign(m, 0.0);
  for (int j = 0; j < m; ++j) {
    lamfd[j] = w[ord[j]];
    for (int i = 0; i < m; ++i) Qfd[(size_t)i * m + j] = Q[(size_t)i * m + ord[j]];
  }
  return IFFD_OK;
}

int build_plan(Plan& P, int d, int n, int p, const iffd_opts* opts, std::string& err) {
  if (d != 2 && d != 3) { err = "d must be 2 or 3"; return IFFD_E_INVAL; }
  if (p < 1 || p > 8) { err = "p must be in 1..8"; return IFFD_E_INVAL; }
  if (n <= p) { err = "n must exceed p"; return IFFD_E_INVAL; }
  if (n > 4096) { err = "n too large"; return IFFD_E_INVAL; }
  P.d = d; P.n = n; P.p = p;
  P.m = n + p - 2;
  P.n_reg = (p % 2) ? n - 1 : n;
  P.n_out = (p % 2) ? p - 1 : p - 2;
  P.half = p / 2;
  if (opts) {
    P.method = opts->method;
    P.prec = opts->apply_prec;
    P.max_rhs = opts->max_rhs;
    P.coef_a = opts->coef_a;
  }
  if (!(P.coef_a > -1.0 && P.coef_a <= 1000.0)) { err = "coef_a must lie in (-1, 1000]"; return IFFD_E_INVAL; }
  if (P.method != IFFD_METHOD_FFT && P.method != IFFD_METHOD_DENSE_FD) { err = "bad method"; return IFFD_E_INVAL; }
  if (P.prec != IFFD_PREC_F32 && P.prec != IFFD_PREC_F64 && P.prec != IFFD_PREC_F16S &&
      P.prec != IFFD_PREC_BF16S) { err = "bad apply_prec"; return IFFD_E_INVAL; }
  if ((P.prec == IFFD_PREC_F16S || P.prec == IFFD_PREC_BF16S) && P.method != IFFD_METHOD_DENSE_FD) {
    err = "IFFD_PREC_F16S and IFFD_PREC_BF16S are for dense FD only";
    return IFFD_E_INVAL;
  }
  if (P.max_rhs < 1) { err = "max_rhs must be >= 1"; return IFFD_E_INVAL; }
  P.N = 1;
  for (int k = 0; k < d; ++k) P.N *= P.m;
  if (P.N * (int64_t)P.max_rhs >= (int64_t(1) << 31)) { err = "problem too large for 32-bit indexing"; return IFFD_E_UNSUPPORTED; }
  // the kernels reach one right-hand side's FP64 tensor through buffer
  // resources, whose byte offsets stay below 2^31
  if (P.N * 8 >= (int64_t(1) << 31)) { err = "one right-hand side above 2 GiB in FP64 (m^d >= 2^28)"; return IFFD_E_UNSUPPORTED; }
  if (P.method == IFFD_METHOD_FFT) {
    // p = 1: S = S^reg (n_out = 0), the preconditioner is the exact inverse
    // by the DST-I alone (no boundary fold, no outliers)
    P.first64 = P.prec == IFFD_PREC_F32 && p >= 5;
    // odd p: DST-I through a length-2n FFT of the odd extension; even p:
    // DST-II / DST-III through a length-n FFT of a reordered sequence where
    // the kernels have that length, else through the length-2n extension
    P.half_len = fft_len_supported(n);
    // FP32 plans of odd degree >= 5 take the DST-I through the odd extension
    // of length 2n: the length-n route forms the odd coefficients as prefix
    // sums of FFT outputs, whose FP32 rounding the high-degree scaling damps
    // too little on the high modes (smooth data: 1.2e-5 at p = 5, 1.3e-4 at
    // p = 7 against the oracle); where 2n is not a built length the length-n
    // route stays
    if (P.prec == IFFD_PREC_F32 && (p & 1) && p >= 5 && fft_len_supported(2 * n)) P.half_len = false;
    P.L = P.half_len ? n : 2 * n;
    if (n > 512 || !fft_len_supported(P.L)) { err = "n must be 2^a or 3*2^a with 8 <= n <= 512 for the FFT kernels"; return IFFD_E_UNSUPPORTED; }
  }
  const int m = P.m, bw = 2 * p + 1, nb = n + p;  // nb: full basis size
  const double h = 1.0 / n;

  // --- knots and 1-D matrices (Sections 2, 3) -----------------------------
  std::vector<double> U(n + 2 * p + 1);
  for (int i = 0; i <= p; ++i) { U[i] = 0.0; U[n + p + i] = 1.0; }
  for (int k = 1; k < n; ++k) U[p + k] = (double)k / n;
  std::vector<double> gx, gw;
  gauss_legendre(p + 1, gx, gw);
  std::vector<double> Kf((size_t)nb * bw, 0.0), Mf((size_t)nb * bw, 0.0);  // full, banded
  // the system matrix's stiffness K_c (coefficient 1 + a x; exact quadrature:
  // the integrand has degree 2p - 1)
  const bool coef = P.coef_a != 0.0;
  std::vector<double> Kcf(coef ? (size_t)nb * bw : 0, 0.0);
  std::vector<double> val, der;
  for (int e = 0; e < n; ++e) {
    const int s = p + e;  // knot span of element e
    const double a = e * h;
    for (int g = 0; g < p + 1; ++g) {
      double x = a + 0.5 * h * (gx[g] + 1.0), wq = 0.5 * h * gw[g];
      basis_and_derivative(s, x, p, U, val, der);
      for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p; ++j) {
          int gi = s - p + i, gj = s - p + j;
          Mf[(size_t)gi * bw + (gj - gi + p)] += wq * val[i] * val[j];
          Kf[(size_t)gi * bw + (gj - gi + p)] += wq * der[i] * der[j];
          if (coef) Kcf[(size_t)gi * bw + (gj - gi + p)] += wq * (1.0 + P.coef_a * x) * der[i] * der[j];
        }
    }
  }
  // Dirichlet reduction: drop B_0 and B_{nb-1}; reduced row i = full row i+1
  P.Kb.assign((size_t)m * bw, 0.0);
  P.Mb.assign((size_t)m * bw, 0.0);
  for (int i = 0; i < m; ++i)
    for (int o = 0; o < bw; ++o) {
      int j = i + o - p;  // reduced column
      if (j < 0 || j >= m) continue;
      P.Kb[(size_t)i * bw + o] = Kf[(size_t)(i + 1) * bw + o];
      P.Mb[(size_t)i * bw + o] = Mf[(size_t)(i + 1) * bw + o];
    }
  P.Kop = P.Kb;
  if (coef)
    for (int i = 0; i < m; ++i)
      for (int o = 0; o < bw; ++o) {
        int j = i + o - p;
        if (j < 0 || j >= m) continue;
        P.Kop[(size_t)i * bw + o] = Kcf[(size_t)(i + 1) * bw + o];
      }

  // compact band tables: rows 0..nbr-1 and m-nbr..m-1 are special, the rows
  // in between equal the interior (Toeplitz) stencil
  // (the system matrix's band rows: with a coefficient every row differs)
  P.nbr = 2 * p - 1;
  P.crows = (!coef && m > 2 * P.nbr + 1) ? 2 * P.nbr + 1 : m;
  P.Kc.assign((size_t)P.crows * bw, 0.0);
  P.Mc.assign((size_t)P.crows * bw, 0.0);
  for (int cr = 0; cr < P.crows; ++cr) {
    int i;
    if (P.crows == m) i = cr;
    else if (cr < P.nbr) i = cr;
    else if (cr == P.nbr) i = m / 2;
    else i = m - P.nbr + (cr - P.nbr - 1);
    for (int o = 0; o < bw; ++o) {
      P.Kc[(size_t)cr * bw + o] = P.Kop[(size_t)i * bw + o];
      P.Mc[(size_t)cr * bw + o] = P.Mb[(size_t)i * bw + o];
    }
  }
  if (P.crows < m) {  // the interior rows must all match the stencil row
    const int mid = m / 2;
    for (int i = P.nbr; i < m - P.nbr; ++i)
      for (int o = 0; o < bw; ++o) {
        double a = P.Kb[(size_t)i * bw + o], b = P.Kb[(size_t)mid * bw + o];
        double c = P.Mb[(size_t)i * bw + o], d = P.Mb[(size_t)mid * bw + o];
        if (std::fabs(a - b) > 1e-12 * std::fabs(P.Kb[(size_t)mid * bw + p]) ||
            std::fabs(c - d) > 1e-12 * std::fabs(P.Mb[(size_t)mid * bw + p])) {
          err = "interior rows of K/M are not Toeplitz";
          return IFFD_E_INVAL;
        }
      }
  }

  P.lam.assign(m, 0.0);
  P.s.assign(m, 1.0);

  if (P.method == IFFD_METHOD_DENSE_FD) {
    const int rc = dense_pencil(P.Kb, P.Mb, m, p, P.Qfd, P.lamfd, err);
    if (rc != IFFD_OK) return rc;
    P.lam = P.lamfd;
    compute_layout(P);
    return IFFD_OK;
  }

  // --- special basis boundary blocks (Section 6) ---------------------------
  // Left end: Bhat_i = B~_i - B~_{dp - i}, i = 1..half, with B~_k(x) =
  // B~_p((x - x_k)/h), x_k = k h (p odd) or (k - 1/2) h (p even).  Each lives
  // on [0, p h], where only the reduced B-splines B_1..B_{p-1} are active; the
  // coefficients follow from interpolation at their Greville points.
  const int half = P.half, dp = (p % 2) ? 0 : 1, nbd = p - 1;
  auto node = [&](int k) { return (p % 2) ? k * h : (k - 0.5) * h; };
  std::vector<double> C((size_t)nbd * nbd), R((size_t)nbd * half);
  for (int r = 0; r < nbd; ++r) {
    int gi = r + 1;  // full index of reduced B_{r+1}
    double tau = 0;
    for (int k = 1; k <= p; ++k) tau += U[gi + k];
    tau /= p;
    int s = find_span(nb, p, tau, U);
    basis_and_derivative(s, tau, p, U, val, der);
    for (int c = 0; c < nbd; ++c) {
      int gc = c + 1, j = gc - (s - p);
      C[(size_t)r * nbd + c] = (j >= 0 && j <= p) ? val[j] : 0.0;
    }
    for (int c = 0; c < half; ++c) {
      int i = c + 1;
      R[(size_t)r * half + c] = cardinal(p, (tau - node(i)) / h) - cardinal(p, (tau - node(dp - i)) / h);
    }
  }
  if (!lu_solve(nbd, C, R, half)) { err = "collocation matrix singular"; return IFFD_E_INVAL; }
  P.V0 = R;  // (p-1) x half
  // Right end by reflection x -> 1 - x: the right function paired with left
  // function i is its mirror image, and B_j(1-x) = B_{m+1-j}(x).
  P.V1.assign((size_t)nbd * half, 0.0);
  for (int r = 0; r < nbd; ++r)
    for (int c = 0; c < half; ++c)
      P.V1[(size_t)r * half + c] = P.V0[(size_t)(nbd - 1 - r) * half + (half - 1 - c)];

  // --- outlier basis (Section 4): V_out = M^{-1} [W0; 0; W1] ----------------
  const int nh = nbd - half;  // outliers per end = floor((p-1)/2)
  std::vector<double> W0((size_t)nbd * nh, 0.0);  // complement of range(V0)
  if (nh > 0) {
    // Householder QR of V0 (nbd x half); the trailing columns of Q span
    // range(V0)'s orthogonal complement.
    std::vector<double> A = P.V0;
    std::vector<std::vector<double>> vs;
    for (int c = 0; c < half; ++c) {
      std::vector<double> v(nbd, 0.0);
      double nrm = 0;
      for (int r = c; r < nbd; ++r) nrm += A[(size_t)r * half + c] * A[(size_t)r * half + c];
      nrm = std::sqrt(nrm);
      double alpha = A[(size_t)c * half + c] >= 0 ? -nrm : nrm;
      for (int r = c; r < nbd; ++r) v[r] = A[(size_t)r * half + c];
      v[c] -= alpha;
      double vn = 0;
      for (int r = c; r < nbd; ++r) vn += v[r] * v[r];
      if (vn > 0)
        for (int cc = c; cc < half; ++cc) {
          double dot = 0;
          for (int r = c; r < nbd; ++r) dot += v[r] * A[(size_t)r * half + cc];
          for (int r = c; r < nbd; ++r) A[(size_t)r * half + cc] -= 2 * dot / vn * v[r];
        }
      vs.push_back(v);
    }
    // columns half..nbd-1 of Q = H_0 H_1 .. e_j
    for (int j = 0; j < nh; ++j) {
      std::vector<double> e(nbd, 0.0);
      e[half + j] = 1.0;
      for (int c = half - 1; c >= 0; --c) {
        const std::vector<double>& v = vs[c];
        double vn = 0, dot = 0;
        for (int r = 0; r < nbd; ++r) { vn += v[r] * v[r]; dot += v[r] * e[r]; }
        if (vn > 0)
          for (int r = 0; r < nbd; ++r) e[r] -= 2 * dot / vn * v[r];
      }
      for (int r = 0; r < nbd; ++r) W0[(size_t)r * nh + j] = e[r];
    }
  }
  // banded Cholesky of M (lower band, Lb[i][k] = L(i, i-p+k))
  std::vector<double> Lb((size_t)m * (p + 1), 0.0);
  auto Lat = [&](int i, int j) -> double& { return Lb[(size_t)i * (p + 1) + (j - i + p)]; };
  for (int i = 0; i < m; ++i)
    for (int j = std::max(0, i - p); j <= i; ++j) {
      double sum = P.Mb[(size_t)i * bw + (j - i + p)];
      for (int k = std::max(0, i - p); k < j; ++k) sum -= Lat(i, k) * Lat(j, k);
      if (i == j) {
        if (!(sum > 0)) { err = "mass matrix not SPD"; return IFFD_E_INVAL; }
        Lat(i, i) = std::sqrt(sum);
      } else {
        Lat(i, j) = sum / Lat(j, j);
      }
    }
  const int no = P.n_out;
  P.Vout.assign((size_t)no * m, 0.0);
  for (int c = 0; c < no; ++c) {
    std::vector<double> b(m, 0.0);
    if (c < nh) {
      for (int r = 0; r < nbd; ++r) b[r] = W0[(size_t)r * nh + c];
    } else {  // mirrored right-end column
      int cc = c - nh;
      for (int r = 0; r < nbd; ++r) b[m - 1 - r] = W0[(size_t)r * nh + cc];
    }
    for (int i = 0; i < m; ++i) {  // L y = b
      double sum = b[i];
      for (int k = std::max(0, i - p); k < i; ++k) sum -= Lat(i, k) * b[k];
      b[i] = sum / Lat(i, i);
    }
    for (int i = m - 1; i >= 0; --i) {  // L^T x = y
      double sum = b[i];
      for (int k = i + 1; k < std::min(m, i + p + 1); ++k) sum -= Lat(k, i) * b[k];
      b[i] = sum / Lat(i, i);
    }
    for (int i = 0; i < m; ++i) P.Vout[(size_t)c * m + i] = b[i];
  }
  auto band_mv = [&](const std::vector<double>& Bd, const double* x, double* y) {
    for (int i = 0; i < m; ++i) {
      double sum = 0;
      for (int o = 0; o < bw; ++o) {
        int j = i + o - p;
        if (j >= 0 && j < m) sum += Bd[(size_t)i * bw + o] * x[j];
      }
      y[i] = sum;
    }
  };
  P.Ao.assign((size_t)no * no, 0.0);
  P.Bo.assign((size_t)no * no, 0.0);
  {
    std::vector<double> kv(m), mv(m);
    for (int a = 0; a < no; ++a) {
      band_mv(P.Kb, &P.Vout[(size_t)a * m], kv.data());
      band_mv(P.Mb, &P.Vout[(size_t)a * m], mv.data());
      for (int b = 0; b < no; ++b) {
        double sk = 0, sm = 0;
        for (int i = 0; i < m; ++i) {
          sk += P.Vout[(size_t)b * m + i] * kv[i];
          sm += P.Vout[(size_t)b * m + i] * mv[i];
        }
        P.Ao[(size_t)a * no + b] = sk;
        P.Bo[(size_t)a * no + b] = sm;
      }
    }
    for (int a = 0; a < no; ++a)  // exact symmetry
      for (int b = a + 1; b < no; ++b) {
        double k2 = 0.5 * (P.Ao[(size_t)a * no + b] + P.Ao[(size_t)b * no + a]);
        double m2 = 0.5 * (P.Bo[(size_t)a * no + b] + P.Bo[(size_t)b * no + a]);
        P.Ao[(size_t)a * no + b] = P.Ao[(size_t)b * no + a] = k2;
        P.Bo[(size_t)a * no + b] = P.Bo[(size_t)b * no + a] = m2;
      }
  }

  // --- regular modes: Dt (end of Section 6) and Lambda_reg (Lemma 4) -------
  // U_ij = sin(x_i alpha_j), alpha_j = j pi: p odd sin(pi i j / n),
  // p even sin(pi (2i-1) j / (2n)); angles are reduced exactly modulo 2 pi.
  const int nr = P.n_reg;
  const int period = (p % 2) ? 2 * n : 4 * n;
  std::vector<double> sintab(period);
  for (int k = 0; k < period; ++k) sintab[k] = (double)std::sin(2 * kPi * k / period);
  P.Dt.assign(nr, 0.0);
  P.Qreg.assign(m <= kDenseMax ? (size_t)nr * m : 0, 0.0);
  std::vector<double> u(nr), v(m), mv(m);
  for (int j = 1; j <= nr; ++j) {
    for (int i = 1; i <= nr; ++i) {
      long long k = (p % 2) ? (long long)i * j : (long long)(2 * i - 1) * j;
      u[i - 1] = sintab[k % period];
    }
    // v = V_reg u
    std::fill(v.begin(), v.end(), 0.0);
    for (int r = 0; r < nbd; ++r) {
      double a = 0, b = 0;
      for (int c = 0; c < half; ++c) {
        a += P.V0[(size_t)r * half + c] * u[c];
        b += P.V1[(size_t)r * half + c] * u[nr - half + c];
      }
      v[r] = a;
      v[m - nbd + r] = b;
    }
    for (int i = half; i < nr - half; ++i) v[i + (p - 1 - half)] = u[i];
    band_mv(P.Mb, v.data(), mv.data());
    double sm = 0;
    for (int i = 0; i < m; ++i) sm += v[i] * mv[i];
    P.Dt[j - 1] = std::sqrt(sm);
    if (!P.Qreg.empty())
      for (int i = 0; i < m; ++i) P.Qreg[(size_t)(j - 1) * m + i] = v[i] / P.Dt[j - 1];
    P.lam[j - 1] = lambda_reg_closed(n, p, j);
    P.s[j - 1] = 1.0 / sm;
  }

  // --- FFT twiddles ------------------------------------------------------------
  P.twl.assign((size_t)2 * P.L, 0.0);
  for (int k = 0; k < P.L; ++k) {
    P.twl[2 * k] = (double)std::cos(2 * kPi * k / P.L);
    P.twl[2 * k + 1] = (double)-std::sin(2 * kPi * k / P.L);
  }
  P.sn.assign((size_t)n / 2 + 1, 0.0);
  for (int h = 0; h <= n / 2; ++h) P.sn[h] = (double)std::sin(kPi * h / n);
  P.twp.assign((size_t)2 * (n + 1), 0.0);
  for (int j = 0; j <= n; ++j) {
    P.twp[2 * j] = (double)std::cos(kPi * j / (2 * n));
    P.twp[2 * j + 1] = (double)-std::sin(kPi * j / (2 * n));
  }
  compute_layout(P);
  return IFFD_OK;
}

}  // namespace iffd

// ===========================================================================
// General plans: per direction its own n, p and Dirichlet / Neumann ends
// (Section 4, "other boundary conditions"; Table 1; Section 6).
// ===========================================================================
namespace iffd {
namespace {

// Left-end block of the special basis for one end type (eq:special_basis):
// the functions of B_L as combinations of the reduced B-splines 0 .. rows-1,
// rows = p - dir (dir = 1 for a Dirichlet end, whose B_0 is dropped).
//   Dirichlet:        Bt_i - Bt_{dp-i}, i = 1 .. floor(p/2)   (odd reflection)
//   Neumann, p even:  Bt_i + Bt_{1-i}, i = 1 .. p/2           (even reflection)
//   Neumann, p odd:   Bt_0, then Bt_i + Bt_{-i}, i = 1 .. (p-1)/2
// with Bt_k the cardinal B-spline centred at k h (p odd) or (k - 1/2) h (p
// even) and dp = 1 for even p, 0 for odd p.  The coefficients come from
// collocation at the Greville points of those B-splines and are checked at
// the element midpoints of the end region (each function must lie in their
// span).
int end_block(int n, int p, int dir, const std::vector<double>& U, std::vector<double>& A,
              int& rows, int& cols, std::string& err) {
  const double h = 1.0 / n;
  const int nb = n + p, dp = (p % 2) ? 0 : 1;
  std::vector<std::vector<std::pair<int, int>>> F;  // (sign, k) terms per function
  if (dir) {
    for (int i = 1; i <= p / 2; ++i) F.push_back({{1, i}, {-1, dp - i}});
  } else if (p % 2 == 0) {
    for (int i = 1; i <= p / 2; ++i) F.push_back({{1, i}, {1, 1 - i}});
  } else {
    F.push_back({{1, 0}});
    for (int i = 1; i <= (p - 1) / 2; ++i) F.push_back({{1, i}, {1, -i}});
  }
  rows = p - dir;
  cols = (int)F.size();
  A.assign((size_t)rows * cols, 0.0);
  if (rows == 0 || cols == 0) return IFFD_OK;
  auto fval = [&](int c, double x) {
    double v = 0.0;
    for (auto& t : F[c]) {
      const double ck = (p % 2) ? t.second * h : (t.second - 0.5) * h;
      v += t.first * cardinal(p, (x - ck) / h);
    }
    return v;
  };
  std::vector<double> val, der;
  auto bvals = [&](double x, std::vector<double>& row) {  // reduced B-splines 0..rows-1 at x
    const int s = find_span(nb, p, x, U);
    basis_and_derivative(s, x, p, U, val, der);
    row.assign(rows, 0.0);
    for (int c = 0; c < rows; ++c) {
      const int j = c + dir - (s - p);
      if (j >= 0 && j <= p) row[c] = val[j];
    }
  };
  std::vector<double> C((size_t)rows * rows), R((size_t)rows * cols), row;
  for (int r = 0; r < rows; ++r) {
    const int gi = r + dir;
    double tau = 0.0;
    for (int k = 1; k <= p; ++k) tau += U[gi + k];
    tau /= p;
    bvals(tau, row);
    for (int c = 0; c < rows; ++c) C[(size_t)r * rows + c] = row[c];
    for (int c = 0; c < cols; ++c) R[(size_t)r * cols + c] = fval(c, tau);
  }
  if (!lu_solve(rows, C, R, cols)) { err = "special basis collocation singular"; return IFFD_E_INVAL; }
  A = R;
  for (int e = 0; e < std::min(n, 2 * p + 2); ++e) {
    const double x = (e + 0.5) * h;
    bvals(x, row);
    for (int c = 0; c < cols; ++c) {
      double v = 0.0;
      for (int r = 0; r < rows; ++r) v += A[(size_t)r * cols + c] * row[r];
      if (std::fabs(v - fval(c, x)) > 1e-11) {
        err = "special basis function outside the end B-splines' span";
        return IFFD_E_INVAL;
      }
    }
  }
  return IFFD_OK;
}

// Orthonormal basis (rows x (rows - cols), row-major) of the orthogonal
// complement of range(A), A rows x cols of full column rank: the trailing
// columns of the Householder QR's Q.
std::vector<double> complement(const std::vector<double>& A0, int rows, int cols) {
  const int nc = rows - cols;
  std::vector<double> W((size_t)rows * std::max(nc, 0), 0.0);
  if (nc <= 0) return W;
  std::vector<double> A = A0;
  std::vector<std::vector<double>> vs;
  for (int c = 0; c < cols; ++c) {
    std::vector<double> v(rows, 0.0);
    double nrm = 0;
    for (int r = c; r < rows; ++r) nrm += A[(size_t)r * cols + c] * A[(size_t)r * cols + c];
    nrm = std::sqrt(nrm);
    const double alpha = A[(size_t)c * cols + c] >= 0 ? -nrm : nrm;
    for (int r = c; r < rows; ++r) v[r] = A[(size_t)r * cols + c];
    v[c] -= alpha;
    double vn = 0;
    for (int r = c; r < rows; ++r) vn += v[r] * v[r];
    if (vn > 0)
      for (int cc = c; cc < cols; ++cc) {
        double dot = 0;
        for (int r = c; r < rows; ++r) dot += v[r] * A[(size_t)r * cols + cc];
        for (int r = c; r < rows; ++r) A[(size_t)r * cols + cc] -= 2 * dot / vn * v[r];
      }
    vs.push_back(v);
  }
  for (int j = 0; j < nc; ++j) {
    std::vector<double> e(rows, 0.0);
    e[cols + j] = 1.0;
    for (int c = cols - 1; c >= 0; --c) {
      const std::vector<double>& v = vs[c];
      double vn = 0, dot = 0;
      for (int r = 0; r < rows; ++r) { vn += v[r] * v[r]; dot += v[r] * e[r]; }
      if (vn > 0)
        for (int r = 0; r < rows; ++r) e[r] -= 2 * dot / vn * v[r];
    }
    for (int r = 0; r < rows; ++r) W[(size_t)r * nc + j] = e[r];
  }
  return W;
}

// Knot insertion (Boehm): inserting x into the knot vector T of degree-p
// B-splines r times; returns E (row-major, new x old B-splines, full bases)
// with B^old_j = sum_i E[i][j] B^new_i, and T refined in place.
std::vector<double> insertion_matrix(std::vector<double>& T, int p, double x, int r, int& nbn) {
  int nb = (int)T.size() - p - 1;
  std::vector<double> E((size_t)nb * nb, 0.0);
  for (int j = 0; j < nb; ++j) E[(size_t)j * nb + j] = 1.0;
  int nb0 = nb;
  for (int it = 0; it < r; ++it) {
    const int s = find_span(nb, p, x, T);
    std::vector<double> E1((size_t)(nb + 1) * nb, 0.0);   // (nb+1) x nb
    for (int j = 0; j <= nb; ++j) {
      if (j <= s - p) {
        E1[(size_t)j * nb + j] = 1.0;
      } else if (j <= s) {
        const double a = (x - T[j]) / (T[j + p] - T[j]);
        E1[(size_t)j * nb + j] = a;
        E1[(size_t)j * nb + j - 1] = 1.0 - a;
      } else {
        E1[(size_t)j * nb + j - 1] = 1.0;
      }
    }
    std::vector<double> En((size_t)(nb + 1) * nb0, 0.0);
    for (int i = 0; i <= nb; ++i)
      for (int k = 0; k < nb; ++k) {
        const double e = E1[(size_t)i * nb + k];
        if (e != 0.0)
          for (int j = 0; j < nb0; ++j) En[(size_t)i * nb0 + j] += e * E[(size_t)k * nb0 + j];
      }
    E.swap(En);
    T.insert(T.begin() + s + 1, x);
    ++nb;
  }
  nbn = nb;
  return E;
}

int build_dir(GDir& G, int n, int p, int dlo, int dhi, std::string& err, int kk = 0, int mult = 1) {
  G.n = n; G.p = p; G.dlo = dlo; G.dhi = dhi;
  const int r = (kk > 0 && mult > 1) ? mult - 1 : 0;
  G.kk = r ? kk : 0;
  G.mult = r ? mult : 1;
  G.rk = r;
  const int nb = n + p + r, bw = 2 * p + 1;
  const int m = nb - dlo - dhi;
  G.m = m;
  G.mo = m - r;
  // eq:reg_space_dim
  if ((p % 2) && dlo && dhi) G.n_reg = n - 1;
  else if ((p % 2) && !dlo && !dhi) G.n_reg = n + 1;
  else G.n_reg = n;
  G.n_out = m - G.n_reg;
  G.L = 2 * n;
  const double h = 1.0 / n;

  // knots (the breakpoint kk / n repeated mult times: Remark
  // rmk:reduced_regularity), 1-D matrices of the full basis (Sections 2, 3),
  // reduction
  std::vector<double> U(n + 2 * p + 1);
  for (int i = 0; i <= p; ++i) { U[i] = 0.0; U[n + p + i] = 1.0; }
  for (int k = 1; k < n; ++k) U[p + k] = (double)k / n;
  const std::vector<double> U0 = U;   // the maximally smooth knots
  std::vector<double> Efull;          // knot insertion, full bases
  if (r) {
    int nbn = 0;
    Efull = insertion_matrix(U, p, (double)kk / n, r, nbn);
    if (nbn != nb) { err = "knot insertion size mismatch"; return IFFD_E_INVAL; }
  }
  std::vector<double> gx, gw, val, der;
  gauss_legendre(p + 1, gx, gw);
  std::vector<double> Kf((size_t)nb * bw, 0.0), Mf((size_t)nb * bw, 0.0);
  for (int e = 0; e < n; ++e) {
    const int s = p + e + (r && e >= kk ? r : 0);
    for (int g = 0; g < p + 1; ++g) {
      const double x = e * h + 0.5 * h * (gx[g] + 1.0), wq = 0.5 * h * gw[g];
      basis_and_derivative(s, x, p, U, val, der);
      for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p; ++j) {
          const int gi = s - p + i, gj = s - p + j;
          Mf[(size_t)gi * bw + (gj - gi + p)] += wq * val[i] * val[j];
          Kf[(size_t)gi * bw + (gj - gi + p)] += wq * der[i] * der[j];
        }
    }
  }
  G.Kb.assign((size_t)m * bw, 0.0);
  G.Mb.assign((size_t)m * bw, 0.0);
  for (int i = 0; i < m; ++i)
    for (int o = 0; o < bw; ++o) {
      const int j = i + o - p;
      if (j < 0 || j >= m) continue;
      G.Kb[(size_t)i * bw + o] = Kf[(size_t)(i + dlo) * bw + o];
      G.Mb[(size_t)i * bw + o] = Mf[(size_t)(i + dlo) * bw + o];
    }

  // end blocks of V_reg; the right end is the mirror image (x -> 1 - x) of a
  // left end of its type: B_j(1 - x) = B_{nb-1-j}(x), Bt_k(1 - x) = Bt_{n+dp-k}(x)
  std::vector<double> Bl, Br;
  int rows, cols;
  int rc = end_block(n, p, dlo, U0, Bl, rows, cols, err);
  if (rc != IFFD_OK) return rc;
  G.rl = rows; G.cl = cols; G.AL = Bl;
  rc = end_block(n, p, dhi, U0, Br, rows, cols, err);
  if (rc != IFFD_OK) return rc;
  G.rr = rows; G.cr = cols;
  G.AR.assign((size_t)rows * cols, 0.0);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c)
      G.AR[(size_t)(rows - 1 - r) * cols + (cols - 1 - c)] = Br[(size_t)r * cols + c];
  const int nint = G.n_reg - G.cl - G.cr;
  const int mo = G.mo;
  if (nint < 0 || nint != mo - G.rl - G.rr) { err = "special basis does not fit the space"; return IFFD_E_INVAL; }
  // the knot window of E on the kept bases: old kept column j is new kept
  // column j left of the window, j + r right of it
  if (r) {
    const int nb0 = nb - r;
    auto Ek = [&](int i, int j) { return Efull[(size_t)(i + dlo) * nb0 + (j + dlo)]; };
    int lo = mo, hi = -1;
    for (int j = 0; j < mo; ++j)
      for (int i = 0; i < m; ++i) {
        const double want = (i == j && j < mo) ? 1.0 : 0.0;
        const double shifted = (i == j + r) ? 1.0 : 0.0;
        const double e = Ek(i, j);
        if (e != want && e != shifted) { lo = std::min(lo, j); hi = std::max(hi, j); }
      }
    if (hi < lo) { err = "knot insertion without a window"; return IFFD_E_INVAL; }
    G.wk0 = lo;
    G.wk1 = hi + 1;
    for (int j = 0; j < mo; ++j)
      for (int i = 0; i < m; ++i) {
        const double e = Ek(i, j);
        double want;
        if (j < G.wk0) want = i == j ? 1.0 : 0.0;
        else if (j >= G.wk1) want = i == j + r ? 1.0 : 0.0;
        else want = (i >= G.wk0 && i < G.wk1 + r) ? e : 0.0;
        if (std::fabs(e - want) > 1e-14) { err = "knot insertion outside its window"; return IFFD_E_INVAL; }
      }
    if (G.wk0 < G.rl + p || G.wk1 > mo - G.rr - p) {
      err = "the repeated knot must lie at least 2p elements from both ends";
      return IFFD_E_INVAL;
    }
    const int wr_ = G.wk1 - G.wk0 + r, wc_ = G.wk1 - G.wk0;
    G.EW.assign((size_t)wr_ * wc_, 0.0);
    for (int i = 0; i < wr_; ++i)
      for (int c = 0; c < wc_; ++c) G.EW[(size_t)i * wc_ + c] = Ek(G.wk0 + i, G.wk0 + c);
  } else {
    G.wk0 = G.wk1 = 0;
    G.EW.clear();
  }

  // Table 1 with 0-based indices: x_s = (s + sig) h, alpha_t = (t + tau) pi
  G.sig2 = (p % 2) ? (dlo ? 2 : 0) : 1;
  G.tau2 = (dlo && dhi) ? 2 : ((dlo || dhi) ? 1 : 0);
  G.beta = dlo ? 0 : 1;

  // outlier basis V_out = M^{-1} [W_L; W_K; W_R] (Section 4): W_K spans the
  // complement of the knot window's columns of E V_reg (reduced regularity)
  const std::vector<double> WL = complement(G.AL, G.rl, G.cl), WR = complement(G.AR, G.rr, G.cr);
  const int nl = G.rl - G.cl, nr_ = G.rr - G.cr;
  const int wrows = r ? G.wk1 - G.wk0 + r : 0, wcols = r ? G.wk1 - G.wk0 : 0;
  const std::vector<double> WK = r ? complement(G.EW, wrows, wcols) : std::vector<double>();
  if (nl + r + nr_ != G.n_out) { err = "outlier dimension mismatch"; return IFFD_E_INVAL; }
  std::vector<double> Lb((size_t)m * (p + 1), 0.0);
  auto Lat = [&](int i, int j) -> double& { return Lb[(size_t)i * (p + 1) + (j - i + p)]; };
  for (int i = 0; i < m; ++i)
    for (int j = std::max(0, i - p); j <= i; ++j) {
      double sum = G.Mb[(size_t)i * bw + (j - i + p)];
      for (int k = std::max(0, i - p); k < j; ++k) sum -= Lat(i, k) * Lat(j, k);
      if (i == j) {
        if (!(sum > 0)) { err = "mass matrix not SPD"; return IFFD_E_INVAL; }
        Lat(i, i) = std::sqrt(sum);
      } else {
        Lat(i, j) = sum / Lat(j, j);
      }
    }
  const int no = G.n_out;
  G.Vout.assign((size_t)no * m, 0.0);
  for (int c = 0; c < no; ++c) {
    std::vector<double> b(m, 0.0);
    if (c < nl) for (int i = 0; i < G.rl; ++i) b[i] = WL[(size_t)i * nl + c];
    else if (c < nl + r) for (int i = 0; i < wrows; ++i) b[G.wk0 + i] = WK[(size_t)i * r + (c - nl)];
    else for (int i = 0; i < G.rr; ++i) b[m - G.rr + i] = WR[(size_t)i * nr_ + (c - nl - r)];
    for (int i = 0; i < m; ++i) {
      double sum = b[i];
      for (int k = std::max(0, i - p); k < i; ++k) sum -= Lat(i, k) * b[k];
      b[i] = sum / Lat(i, i);
    }
    for (int i = m - 1; i >= 0; --i) {
      double sum = b[i];
      for (int k = i + 1; k < std::min(m, i + p + 1); ++k) sum -= Lat(k, i) * b[k];
      b[i] = sum / Lat(i, i);
    }
    for (int i = 0; i < m; ++i) G.Vout[(size_t)c * m + i] = b[i];
  }
  auto band_mv = [&](const std::vector<double>& Bd, const double* x, double* y) {
    for (int i = 0; i < m; ++i) {
      double sum = 0;
      for (int o = 0; o < bw; ++o) {
        const int j = i + o - p;
        if (j >= 0 && j < m) sum += Bd[(size_t)i * bw + o] * x[j];
      }
      y[i] = sum;
    }
  };
  G.Ao.assign((size_t)no * no, 0.0);
  G.Bo.assign((size_t)no * no, 0.0);
  {
    std::vector<double> kv(m), mv(m);
    for (int a = 0; a < no; ++a) {
      band_mv(G.Kb, &G.Vout[(size_t)a * m], kv.data());
      band_mv(G.Mb, &G.Vout[(size_t)a * m], mv.data());
      for (int b = 0; b < no; ++b) {
        double sk = 0, sm = 0;
        for (int i = 0; i < m; ++i) {
          sk += G.Vout[(size_t)b * m + i] * kv[i];
          sm += G.Vout[(size_t)b * m + i] * mv[i];
        }
        G.Ao[(size_t)a * no + b] = sk;
        G.Bo[(size_t)a * no + b] = sm;
      }
    }
    for (int a = 0; a < no; ++a)
      for (int b = a + 1; b < no; ++b) {
        const double k2 = 0.5 * (G.Ao[(size_t)a * no + b] + G.Ao[(size_t)b * no + a]);
        const double m2 = 0.5 * (G.Bo[(size_t)a * no + b] + G.Bo[(size_t)b * no + a]);
        G.Ao[(size_t)a * no + b] = G.Ao[(size_t)b * no + a] = k2;
        G.Bo[(size_t)a * no + b] = G.Bo[(size_t)b * no + a] = m2;
      }
  }

  // regular modes: Dt = ||V_reg U e_t||_M, Lambda_reg by the closed form at
  // theta_t = alpha_t / n (Lemma 4).  Angles in units of 2 pi / (8n), reduced
  // exactly; beta = pi/2 is 2n units.
  const int nrg = G.n_reg, per = 8 * n;
  std::vector<double> sintab(per), costab(per);
  for (int k = 0; k < per; ++k) {
    sintab[k] = (double)std::sin(2 * kPi * k / per);
    costab[k] = (double)std::cos(2 * kPi * k / per);
  }
  G.lam.assign(m, 0.0);
  G.s.assign(m, 1.0);
  G.Dt.assign(nrg, 0.0);
  G.Qreg.assign(m <= kDenseMax ? (size_t)nrg * m : 0, 0.0);
  std::vector<double> u(nrg), vo(mo), v(m), mv(m);
  for (int t = 0; t < nrg; ++t) {
    for (int s = 0; s < nrg; ++s) {
      const long long a = ((long long)(2 * s + G.sig2) * (2 * t + G.tau2) + 2LL * n * G.beta) % per;
      u[s] = sintab[a];
    }
    std::fill(vo.begin(), vo.end(), 0.0);
    for (int i = 0; i < G.rl; ++i) {
      double acc = 0;
      for (int c = 0; c < G.cl; ++c) acc += G.AL[(size_t)i * G.cl + c] * u[c];
      vo[i] = acc;
    }
    for (int i = 0; i < nint; ++i) vo[G.rl + i] = u[G.cl + i];
    for (int i = 0; i < G.rr; ++i) {
      double acc = 0;
      for (int c = 0; c < G.cr; ++c) acc += G.AR[(size_t)i * G.cr + c] * u[nrg - G.cr + c];
      vo[mo - G.rr + i] = acc;
    }
    // v = E vo on the reduced space's B-splines (the same function)
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int j = 0; j < mo; ++j) {
      if (!r || j < G.wk0) v[j] += vo[j];
      else if (j >= G.wk1) v[j + r] += vo[j];
    }
    for (int i = 0; i < wrows; ++i)
      for (int c = 0; c < wcols; ++c) v[G.wk0 + i] += G.EW[(size_t)i * wcols + c] * vo[G.wk0 + c];
    band_mv(G.Mb, v.data(), mv.data());
    double sm = 0;
    for (int i = 0; i < m; ++i) sm += v[i] * mv[i];
    G.Dt[t] = std::sqrt(sm);
    if (!G.Qreg.empty())
      for (int i = 0; i < m; ++i) G.Qreg[(size_t)t * m + i] = v[i] / G.Dt[t];
    G.s[t] = 1.0 / sm;
    G.lam[t] = lambda_reg_half(n, p, 2 * t + G.tau2);
  }

  // FFT twiddles and the four twists of the transforms through length-2n FFTs:
  //   forward  y_t = sum_s g_s U_{s,t}:  pre  e^{-i pi s tau / n},
  //                                       post e^{-i (beta + pi sig (t + tau) / n)};
  //   backward c_s = sum_t y_t U_{s,t}:  pre  e^{-i pi t sig / n},
  //                                       post e^{-i (beta + pi tau (s + sig) / n)}
  G.tw.assign((size_t)2 * G.L, 0.0);
  for (int k = 0; k < G.L; ++k) {
    G.tw[2 * k] = (double)std::cos(2 * kPi * k / G.L);
    G.tw[2 * k + 1] = (double)-std::sin(2 * kPi * k / G.L);
  }
  G.tf.assign((size_t)8 * nrg, 0.0);
  auto put = [&](int slot, int i, long long a) {
    a %= per;
    G.tf[(size_t)2 * (slot * nrg + i)] = costab[a];
    G.tf[(size_t)2 * (slot * nrg + i) + 1] = -sintab[a];
  };
  for (int i = 0; i < nrg; ++i) {
    put(0, i, 2LL * i * G.tau2);
    put(1, i, (long long)G.sig2 * (2 * i + G.tau2) + 2LL * n * G.beta);
    put(2, i, 2LL * i * G.sig2);
    put(3, i, (long long)G.tau2 * (2 * i + G.sig2) + 2LL * n * G.beta);
  }
  return IFFD_OK;
}

// Q of the QR factorization (positive diagonal of R) of a rows x cols block
// (row-major) of full column rank, in place: Gram-Schmidt with a second
// orthogonalization pass
void orthonormal_columns(std::vector<double>& A, int rows, int cols) {
  for (int c = 0; c < cols; ++c) {
    for (int pass = 0; pass < 2; ++pass)
      for (int c2 = 0; c2 < c; ++c2) {
        double dot = 0.0;
        for (int r = 0; r < rows; ++r) dot += A[(size_t)r * cols + c2] * A[(size_t)r * cols + c];
        for (int r = 0; r < rows; ++r) A[(size_t)r * cols + c] -= dot * A[(size_t)r * cols + c2];
      }
    double nrm = 0.0;
    for (int r = 0; r < rows; ++r) nrm += A[(size_t)r * cols + c] * A[(size_t)r * cols + c];
    nrm = std::sqrt(nrm);
    for (int r = 0; r < rows; ++r) A[(size_t)r * cols + c] /= nrm;
  }
}

// A generic basis of S^reg for eq:reg_eigenvectors, Q_reg = C^{-1} U D^{-1}:
// the special basis with each end block (AL, AR) replaced by its orthonormal
// QR factor, the interior B-splines kept.  C_ij = psi_j(x_i) at the nodes
// x_i = (i + sig) h of Table 1 is banded; its LU factors (no pivoting) are
// kept as bands.  D_t = ||F_t||_L2 for the interpolant F_t = V_reg C^{-1} U e_t
// (eq:Dreg2; s_t = 1 / D_t^2), and Lambda_reg, which does not depend on the
// basis, is checked against F_t's Rayleigh quotient (eq:Lambda reg2).  The
// outlier space (and V_out) is the same as for the special basis.
int make_generic(GDir& G, std::string& err) {
  const int n = G.n, p = G.p, m = G.m, nr = G.n_reg, nb = n + p, bw = 2 * p + 1;
  const int cl = G.cl, cr = G.cr, rl = G.rl, rr = G.rr, nint = nr - cl - cr;
  std::vector<double> AL = G.AL, AR = G.AR;
  orthonormal_columns(AL, rl, cl);
  orthonormal_columns(AR, rr, cr);
  std::vector<double> U(n + 2 * p + 1);
  for (int i = 0; i <= p; ++i) { U[i] = 0.0; U[n + p + i] = 1.0; }
  for (int k = 1; k < n; ++k) U[p + k] = (double)k / n;
  // the interpolation matrix
  std::vector<double> C((size_t)nr * nr, 0.0), val, der, brow(m);
  for (int i = 0; i < nr; ++i) {
    const double x = (2.0 * i + G.sig2) / (2.0 * n);
    const int sp = find_span(nb, p, x, U);
    basis_and_derivative(sp, x, p, U, val, der);
    std::fill(brow.begin(), brow.end(), 0.0);
    for (int j = 0; j <= p; ++j) {
      const int r = sp - p + j - G.dlo;
      if (r >= 0 && r < m) brow[r] = val[j];
    }
    for (int j = 0; j < cl; ++j) {
      double v = 0.0;
      for (int r = 0; r < rl; ++r) v += AL[(size_t)r * cl + j] * brow[r];
      C[(size_t)i * nr + j] = v;
    }
    for (int j = 0; j < nint; ++j) C[(size_t)i * nr + cl + j] = brow[rl + j];
    for (int j = 0; j < cr; ++j) {
      double v = 0.0;
      for (int r = 0; r < rr; ++r) v += AR[(size_t)r * cr + j] * brow[m - rr + r];
      C[(size_t)i * nr + nr - cr + j] = v;
    }
  }
  int bl = 0, bu = 0;
  double cmax = 0.0;
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nr; ++j)
      if (C[(size_t)i * nr + j] != 0.0) {
        bl = std::max(bl, i - j);
        bu = std::max(bu, j - i);
        cmax = std::max(cmax, std::fabs(C[(size_t)i * nr + j]));
      }
  // LU without pivoting inside the band (the fill stays in it)
  for (int k = 0; k < nr; ++k) {
    const double piv = C[(size_t)k * nr + k];
    if (!(std::fabs(piv) > 1e-10 * cmax)) {
      err = "generic basis: the interpolation matrix needs pivoting";
      return IFFD_E_UNSUPPORTED;
    }
    for (int i = k + 1; i <= std::min(nr - 1, k + bl); ++i) {
      const double l = C[(size_t)i * nr + k] / piv;
      C[(size_t)i * nr + k] = l;
      if (l != 0.0)
        for (int j = k + 1; j <= std::min(nr - 1, k + bu); ++j) C[(size_t)i * nr + j] -= l * C[(size_t)k * nr + j];
    }
  }
  G.bl = bl;
  G.bu = bu;
  G.LB.assign((size_t)nr * std::max(bl, 1), 0.0);
  G.UB.assign((size_t)nr * (bu + 1), 0.0);
  for (int i = 0; i < nr; ++i) {
    for (int k = 0; k < bl; ++k) {
      const int j = i - bl + k;
      if (j >= 0) G.LB[(size_t)i * bl + k] = C[(size_t)i * nr + j];
    }
    G.UB[(size_t)i * (bu + 1)] = 1.0 / C[(size_t)i * nr + i];
    for (int k = 1; k <= bu; ++k)
      if (i + k < nr) G.UB[(size_t)i * (bu + 1) + k] = C[(size_t)i * nr + i + k];
  }
  // D_t and the eigenvalue check
  auto band_dot = [&](const std::vector<double>& Bd, const std::vector<double>& v) {
    double acc = 0.0;
    for (int i = 0; i < m; ++i)
      for (int o = 0; o < bw; ++o) {
        const int j = i + o - p;
        if (j >= 0 && j < m) acc += v[i] * Bd[(size_t)i * bw + o] * v[j];
      }
    return acc;
  };
  const int per = 8 * n;
  double lmax = 0.0;
  for (int t = 0; t < nr; ++t) lmax = std::max(lmax, G.lam[t]);
  std::vector<double> w(nr), v(m);
  G.Qreg.assign(m <= kDenseMax ? (size_t)nr * m : 0, 0.0);
  for (int t = 0; t < nr; ++t) {
    for (int i = 0; i < nr; ++i) {
      const long long a = ((long long)(2 * i + G.sig2) * (2 * t + G.tau2) + 2LL * n * G.beta) % per;
      w[i] = std::sin(2 * kPi * (double)a / per);
    }
    for (int i = 0; i < nr; ++i)   // L y = u
      for (int j = std::max(0, i - bl); j < i; ++j) w[i] -= C[(size_t)i * nr + j] * w[j];
    for (int i = nr - 1; i >= 0; --i) {   // U w = y
      for (int j = i + 1; j <= std::min(nr - 1, i + bu); ++j) w[i] -= C[(size_t)i * nr + j] * w[j];
      w[i] /= C[(size_t)i * nr + i];
    }
    for (int r = 0; r < rl; ++r) {
      double acc = 0.0;
      for (int c = 0; c < cl; ++c) acc += AL[(size_t)r * cl + c] * w[c];
      v[r] = acc;
    }
    for (int i = 0; i < nint; ++i) v[rl + i] = w[cl + i];
    for (int r = 0; r < rr; ++r) {
      double acc = 0.0;
      for (int c = 0; c < cr; ++c) acc += AR[(size_t)r * cr + c] * w[nr - cr + c];
      v[m - rr + r] = acc;
    }
    const double sm = band_dot(G.Mb, v), sk = band_dot(G.Kb, v);
    if (!(sm > 0.0)) { err = "generic basis: an interpolant has no mass"; return IFFD_E_INVAL; }
    if (std::fabs(sk / sm - G.lam[t]) > 1e-8 * G.lam[t] + 1e-12 * lmax) {
      err = "generic basis: eigenvalue check failed";
      return IFFD_E_INVAL;
    }
    G.s[t] = 1.0 / sm;
    G.Dt[t] = std::sqrt(sm);
    if (!G.Qreg.empty())
      for (int i = 0; i < m; ++i) G.Qreg[(size_t)t * m + i] = v[i] / G.Dt[t];
  }
  G.AL = AL;
  G.AR = AR;
  G.generic = true;
  return IFFD_OK;
}

// the dense FD tables of a direction of a dense-FD general plan
int finish_dir(const Plan& P, GDir& G, std::string& err) {
  if (P.method != IFFD_METHOD_DENSE_FD) return IFFD_OK;
  return dense_pencil(G.Kb, G.Mb, G.m, G.p, G.Qfd, G.lamfd, err);
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

void compute_layout_general(Plan& P) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = al256(off + std::max<size_t>(bytes, 8));
    return o;
  };
  int pm = 1;
  for (int k = 0; k < P.d; ++k) pm = std::max(pm, P.dirs[k].p);
  P.dense2d = dense2d_ok(P);
  const bool dense = P.dense2d;
  for (int k = 0; k < P.d; ++k) {
    GDir& G = P.dirs[k];
    G.pm = pm;
    const int bw = 2 * pm + 1;
    int o = 0;
    G.o_tw = o;  o += 2 * G.L;
    G.o_tf = o;  o += 8 * G.n_reg;
    G.o_al = o;  o += G.rl * G.cl;
    G.o_ar = o;  o += G.rr * G.cr;
    G.o_vt = o;  o += G.n_out * G.m;
    G.o_lam = o; o += G.m;
    G.o_s = o;   o += G.m;
    G.o_kb = o;  o += G.m * bw;
    G.o_mb = o;  o += G.m * bw;
    G.o_lb = o;  o += G.generic ? G.n_reg * G.bl : 0;
    G.o_ub = o;  o += G.generic ? G.n_reg * (G.bu + 1) : 0;
    G.o_ew = o;  o += (int)G.EW.size();
    G.len = o + (o & 1);
    G.blob64 = take((size_t)8 * G.len);
    G.blob32 = take((size_t)4 * G.len);
    if (P.method == IFFD_METHOD_DENSE_FD) {
      const size_t mm = (size_t)G.m * G.m;
      G.fq64 = take(8 * mm);
      G.fqt64 = take(8 * mm);
      G.flam64 = take((size_t)8 * G.m);
      G.fq32 = take(4 * mm);
      G.fqt32 = take(4 * mm);
      G.flam32 = take((size_t)4 * G.m);
    }
    G.dq32 = G.dlam32 = 0;
    if (dense) {
      G.dq32 = take((size_t)4 * G.m * G.m);
      G.dlam32 = take((size_t)4 * G.m);
    }
    G.ao64 = take((size_t)8 * G.n_out * G.n_out);
    G.bo64 = take((size_t)8 * G.n_out * G.n_out);
    G.vout64 = take((size_t)8 * G.n_out * G.m);
    G.stat64 = take(8);
  }
  const size_t unit = take((size_t)8 * 2 * (2 * pm + 1));
  P.lay.unit64 = unit;
  P.lay.total = off;
}

}  // namespace

int build_plan_general(Plan& P, int d, const int* nv, const int* pv, const int* dirichlet,
                       const iffd_opts* opts, std::string& err) {
  if (d != 2 && d != 3) { err = "d must be 2 or 3"; return IFFD_E_INVAL; }
  if (!nv || !pv || !dirichlet) { err = "null n, p or dirichlet array"; return IFFD_E_INVAL; }
  if (opts) {
    P.method = opts->method;
    P.prec = opts->apply_prec;
    P.max_rhs = opts->max_rhs;
    P.coef_a = opts->coef_a;
  }
  if (P.method != IFFD_METHOD_FFT && P.method != IFFD_METHOD_DENSE_FD) { err = "bad method"; return IFFD_E_INVAL; }
  if (P.prec != IFFD_PREC_F32 && P.prec != IFFD_PREC_F64) { err = "general plans take IFFD_PREC_F32 or IFFD_PREC_F64"; return IFFD_E_INVAL; }
  if (P.coef_a != 0.0) { err = "general plans take coef_a = 0 (the Kronecker-sum operator)"; return IFFD_E_UNSUPPORTED; }
  if (P.max_rhs < 1) { err = "max_rhs must be >= 1"; return IFFD_E_INVAL; }
  bool any_dirichlet = false;
  int pmax = 0;
  for (int k = 0; k < d; ++k) {
    const int n = nv[k], p = pv[k], a = dirichlet[2 * k], b = dirichlet[2 * k + 1];
    if (p < 1 || p > 8) { err = "p must be in 1..8"; return IFFD_E_INVAL; }
    if (n <= p) { err = "n must exceed p"; return IFFD_E_INVAL; }
    if ((a != 0 && a != 1) || (b != 0 && b != 1)) { err = "dirichlet flags must be 0 or 1"; return IFFD_E_INVAL; }
    if (n > 256 || !fft_len_supported(2 * n)) {
      err = "general plans need n = 2^a or 3*2^a with 8 <= n <= 256 in every direction";
      return IFFD_E_UNSUPPORTED;
    }
    any_dirichlet = any_dirichlet || a || b;
    pmax = std::max(pmax, p);
  }
  if (!any_dirichlet) {
    err = "Neumann conditions on every face: the operator is singular (the constants)";
    return IFFD_E_UNSUPPORTED;
  }
  P.gen = true;
  P.d = d;
  P.N = 1;
  for (int k = 0; k < d; ++k) {
    int rc = build_dir(P.dirs[k], nv[k], pv[k], dirichlet[2 * k], dirichlet[2 * k + 1], err);
    if (rc == IFFD_OK) rc = finish_dir(P, P.dirs[k], err);
    if (rc != IFFD_OK) return rc;
    P.N *= P.dirs[k].m;
  }
  if (P.N * (int64_t)P.max_rhs >= (int64_t(1) << 31)) { err = "problem too large for 32-bit indexing"; return IFFD_E_UNSUPPORTED; }
  if (P.N * 8 >= (int64_t(1) << 31)) { err = "one right-hand side above 2 GiB in FP64"; return IFFD_E_UNSUPPORTED; }
  const GDir& G = P.dirs[0];
  P.n = G.n; P.p = G.p; P.m = G.m; P.n_reg = G.n_reg; P.n_out = G.n_out; P.L = G.L;
  P.half = G.p / 2;
  P.first64 = P.prec == IFFD_PREC_F32 && pmax >= 5;
  P.lay = TableLayout{};
  compute_layout_general(P);
  return IFFD_OK;
}

int set_plan_basis(Plan& P, int basis, std::string& err) {
  if (basis != IFFD_BASIS_SPECIAL && basis != IFFD_BASIS_GENERIC) { err = "unknown basis"; return IFFD_E_INVAL; }
  if (!P.gen) { err = "the basis choice needs a general plan (iffd_plan_create_general)"; return IFFD_E_UNSUPPORTED; }
  if (basis == P.basis) return IFFD_OK;
  GDir dirs[3];
  for (int k = 0; k < P.d; ++k) {
    const GDir& G = P.dirs[k];
    if (basis == IFFD_BASIS_GENERIC && G.rk) {
      err = "the generic basis is not built for a repeated knot";
      return IFFD_E_UNSUPPORTED;
    }
    int rc = build_dir(dirs[k], G.n, G.p, G.dlo, G.dhi, err, G.kk, G.mult);
    if (rc == IFFD_OK && basis == IFFD_BASIS_GENERIC) rc = make_generic(dirs[k], err);
    if (rc == IFFD_OK) rc = finish_dir(P, dirs[k], err);
    if (rc != IFFD_OK) return rc;
  }
  for (int k = 0; k < P.d; ++k) P.dirs[k] = dirs[k];
  P.basis = basis;
  // the tables of a mapped domain follow the plan's own
  const int gk = P.geo.kind;
  double gp[4];
  for (int i = 0; i < 4; ++i) gp[i] = P.geo.par[i];
  P.geo = GeoPlan{};
  P.lay = TableLayout{};
  compute_layout_general(P);
  if (gk) return build_geometry(P, gk, gp, 4, err);
  return IFFD_OK;
}

int set_plan_knot(Plan& P, int direction, int k, int mult, std::string& err) {
  if (!P.gen) { err = "a repeated knot needs a general plan (iffd_plan_create_general)"; return IFFD_E_UNSUPPORTED; }
  if (direction < 1 || direction > P.d) { err = "direction out of range"; return IFFD_E_INVAL; }
  GDir& G = P.dirs[direction - 1];
  if (mult < 1 || mult > G.p) { err = "multiplicity must be in 1..p"; return IFFD_E_INVAL; }
  if (mult > 1 && (k < 1 || k >= G.n)) { err = "the knot k / n must be an interior breakpoint"; return IFFD_E_INVAL; }
  if (P.basis == IFFD_BASIS_GENERIC && mult > 1) {
    err = "the generic basis is not built for a repeated knot";
    return IFFD_E_UNSUPPORTED;
  }
  GDir nd;
  int rc = build_dir(nd, G.n, G.p, G.dlo, G.dhi, err, mult > 1 ? k : 0, mult);
  if (rc == IFFD_OK) rc = finish_dir(P, nd, err);
  if (rc != IFFD_OK) return rc;
  if (nd.n_out > 8) { err = "at most 8 outlier functions per direction"; return IFFD_E_UNSUPPORTED; }
  int64_t N = 1;
  for (int j = 0; j < P.d; ++j) N *= (j == direction - 1 ? nd.m : P.dirs[j].m);
  if (N * (int64_t)P.max_rhs >= (int64_t(1) << 31) || N * 8 >= (int64_t(1) << 31)) {
    err = "problem too large for 32-bit indexing";
    return IFFD_E_UNSUPPORTED;
  }
  G = nd;
  P.N = N;
  const GDir& G1 = P.dirs[0];
  P.m = G1.m; P.n_reg = G1.n_reg; P.n_out = G1.n_out;
  // the tables of a mapped domain follow the new space
  const int gk = P.geo.kind;
  double gp[4];
  for (int i = 0; i < 4; ++i) gp[i] = P.geo.par[i];
  P.geo = GeoPlan{};
  P.lay = TableLayout{};
  compute_layout_general(P);
  if (gk) return build_geometry(P, gk, gp, 4, err);
  return IFFD_OK;
}

// ---------------------------------------------------------------------------
// Geometry-mapped system matrix: per-direction element tables
// ---------------------------------------------------------------------------
// the quarter of the unit circle from (1, 0) to (0, 1) as the rational
// quadratic with control points (1,0), (1,1), (0,1) and weights 1, 1/sqrt 2,
// 1: c = (c1, c2) and c' at t
static void quarter_circle(double t, double c[4]) {
  const double w = 0.70710678118654752440;
  const double b0 = (1 - t) * (1 - t), b1 = 2 * t * (1 - t), b2 = t * t;
  const double db0 = -2 * (1 - t), db1 = 2 - 4 * t, db2 = 2 * t;
  const double den = b0 + w * b1 + b2, dden = db0 + w * db1 + db2;
  const double n1 = b0 + w * b1, n2 = w * b1 + b2;
  const double dn1 = db0 + w * db1, dn2 = w * db1 + db2;
  c[0] = n1 / den;
  c[1] = n2 / den;
  c[2] = (dn1 * den - n1 * dden) / (den * den);
  c[3] = (dn2 * den - n2 * dden) / (den * den);
}

// one-dimensional factors of the map along direction k at xi (the element
// kernels form G from them, closed forms in geo.hip):
//   bump     f = (sin(pi xi), cos(pi xi))
//   annulus  direction 1: (r(xi)); direction 2: (c1, c2, c1', c2') at t = xi
//   plate    direction 1: (o - R c, R c', o' - R c') with the hole's arc R c
//            and the outer sides o ((L, 2 L xi) below xi = 1/2, (2 L (1 - xi),
//            L) above); direction 2: (xi)
static void geo_map_factors(int kind, const double* par, int k, double xi,
                            double f[GEO_FACTORS]) {
  for (int i = 0; i < GEO_FACTORS; ++i) f[i] = 0.0;
  if (kind == IFFD_GEOMETRY_BUMP) {
    const double pi = 3.14159265358979323846;
    f[0] = std::sin(pi * xi);
    f[1] = std::cos(pi * xi);
  } else if (kind == IFFD_GEOMETRY_ANNULUS) {
    if (k == 0) f[0] = par[0] + (par[1] - par[0]) * xi;
    if (k == 1) quarter_circle(xi, f);
  } else if (kind == IFFD_GEOMETRY_PLATE) {
    if (k == 0) {
      const double R = par[0], L = par[1];
      double c[4];
      quarter_circle(xi, c);
      const bool first = xi < 0.5;   // on the side x = L, else on y = L
      const double o1 = first ? L : 2 * L * (1 - xi), o2 = first ? 2 * L * xi : L;
      const double do1 = first ? 0.0 : -2 * L, do2 = first ? 2 * L : 0.0;
      f[0] = o1 - R * c[0];
      f[1] = o2 - R * c[1];
      f[2] = R * c[2];
      f[3] = R * c[3];
      f[4] = do1 - R * c[2];
      f[5] = do2 - R * c[3];
    }
    if (k == 1) f[0] = xi;
  }
}

int build_geometry(Plan& P, int kind, const double* par, int npar, std::string& err) {
  if (P.geo.kind == 0) P.geo.base_total = P.lay.total;
  if (kind == IFFD_GEOMETRY_NONE) {
    P.lay.total = P.geo.base_total;
    P.geo = GeoPlan{};
    return IFFD_OK;
  }
  if (P.d != 2 && P.d != 3) { err = "a mapped domain needs d = 2 or 3"; return IFFD_E_UNSUPPORTED; }
  if (P.coef_a != 0.0) { err = "a mapped domain replaces coef_a; create the plan with coef_a = 0"; return IFFD_E_INVAL; }
  if (P.method != IFFD_METHOD_FFT && P.method != IFFD_METHOD_DENSE_FD) { err = "bad method"; return IFFD_E_INVAL; }
  GeoPlan G;
  G.kind = kind;
  G.base_total = P.geo.kind == 0 ? P.lay.total : P.geo.base_total;
  if (kind == IFFD_GEOMETRY_BUMP) {
    if (!par || npar < 1 || !(std::fabs(par[0]) < 0.1)) { err = "bump map: params {eps}, |eps| < 0.1"; return IFFD_E_INVAL; }
    G.par[0] = par[0];
  } else if (kind == IFFD_GEOMETRY_ANNULUS) {
    // 2D: the cross section {r_in, r_out} (the prism's H is 1 and unused)
    if (!par || npar < P.d || !(par[0] > 0.0 && par[1] > par[0] && (P.d == 2 || par[2] > 0.0))) {
      err = P.d == 3 ? "annulus map: params {r_in, r_out, H}, 0 < r_in < r_out, H > 0"
                     : "annulus map (2D): params {r_in, r_out}, 0 < r_in < r_out";
      return IFFD_E_INVAL;
    }
    for (int i = 0; i < 3; ++i) G.par[i] = i < 2 || P.d == 3 ? par[i] : 1.0;
  } else if (kind == IFFD_GEOMETRY_PLATE) {
    if (!par || npar < P.d || !(par[0] > 0.0 && par[1] > par[0] && (P.d == 2 || par[2] > 0.0))) {
      err = P.d == 3 ? "plate map: params {R, L, H}, 0 < R < L, H > 0"
                     : "plate map (2D): params {R, L}, 0 < R < L";
      return IFFD_E_INVAL;
    }
    const int n1 = P.gen ? P.dirs[0].n : P.n;
    if (n1 % 2) {
      err = "plate map: n_1 must be even (the corner plane xi_1 = 1/2 on a breakpoint)";
      return IFFD_E_INVAL;
    }
    for (int i = 0; i < 3; ++i) G.par[i] = i < 2 || P.d == 3 ? par[i] : 1.0;
  } else {
    err = "unknown geometry kind";
    return IFFD_E_INVAL;
  }
  // In 2D the third direction is a single element with one point, V = 1,
  // D = 0 and w = 1 (factors (1, 0, ..)): the 3D operator then is the 2D one
  // (no xi_3 derivative, the bump's third gradient entry 0, the prisms' H 1).
  int o = 0;
  for (int k = 0; k < 3; ++k) {
    GeoPlanDir& g = G.dir[k];
    int n, p, lo, m, kk = 0, rk = 0;
    if (k >= P.d) {
      n = 1; p = 0; lo = 0; m = 1;
    } else if (P.gen) {
      n = P.dirs[k].n; p = P.dirs[k].p; lo = P.dirs[k].dlo; m = P.dirs[k].m;
      if (P.dirs[k].rk) { kk = P.dirs[k].kk; rk = P.dirs[k].rk; }
    } else {
      n = P.n; p = P.p; lo = 1; m = P.m;
    }
    if (p + 1 > 9) { err = "p <= 8"; return IFFD_E_INVAL; }
    g.n = n; g.P = p + 1; g.lo = lo; g.m = m; g.kk = kk; g.rk = rk;
    g.o_x = o; o += n * g.P;
    g.o_w = o; o += n * g.P;
    g.o_v = o; o += n * g.P * g.P;
    g.o_d = o; o += n * g.P * g.P;
    g.o_f = o; o += n * g.P * GEO_FACTORS;
  }
  G.tab.assign((size_t)o, 0.0);
  std::vector<double> gx, gw, val, der;
  for (int k = 0; k < 3; ++k) {
    GeoPlanDir& g = G.dir[k];
    const int n = g.n, p = g.P - 1;
    if (k >= P.d) {   // the 2D plan's dummy direction
      G.tab[(size_t)g.o_x] = 0.5;
      G.tab[(size_t)g.o_w] = 1.0;
      G.tab[(size_t)g.o_v] = 1.0;
      G.tab[(size_t)g.o_d] = 0.0;
      G.tab[(size_t)g.o_f] = 1.0;
      g.ulo = 0;
      g.uhi = -1;
      continue;
    }
    // open knots with the breakpoint kk / n repeated rk more times
    std::vector<double> U;
    for (int i = 0; i <= p; ++i) U.push_back(0.0);
    for (int j = 1; j < n; ++j)
      for (int r = 0; r <= (j == g.kk ? g.rk : 0); ++r) U.push_back((double)j / n);
    for (int i = 0; i <= p; ++i) U.push_back(1.0);
    gauss_legendre(p + 1, gx, gw);
    const double h = 1.0 / n;
    for (int e = 0; e < n; ++e) {
      // span of element e: B-splines f .. f+p, f = e (+ rk past the breakpoint)
      const int s = p + e + (e >= g.kk ? g.rk : 0);
      for (int q = 0; q <= p; ++q) {
        const double x = e * h + 0.5 * h * (gx[q] + 1.0);
        G.tab[(size_t)g.o_x + e * g.P + q] = x;
        G.tab[(size_t)g.o_w + e * g.P + q] = 0.5 * h * gw[q];
        geo_map_factors(kind, G.par, k, x, &G.tab[(size_t)g.o_f + ((size_t)e * g.P + q) * GEO_FACTORS]);
        basis_and_derivative(s, x, p, U, val, der);
        for (int a = 0; a <= p; ++a) {
          G.tab[(size_t)g.o_v + ((size_t)e * g.P + q) * g.P + a] = val[a];
          G.tab[(size_t)g.o_d + ((size_t)e * g.P + q) * g.P + a] = der[a];
        }
      }
    }
    // On the uniform knots the p+1 B-splines of elements p .. n-1-p are
    // translates of one another (their knot windows are uniform), so their
    // tables agree up to rounding: they get the table of element p exactly,
    // and the element kernel reads it once for a whole run of such elements.
    if (g.rk == 0 && n - 1 - p >= p) {
      g.ulo = p;
      g.uhi = n - 1 - p;
      const size_t PP = (size_t)g.P * g.P;
      for (int e = g.ulo + 1; e <= g.uhi; ++e)
        for (size_t j = 0; j < PP; ++j) {
          G.tab[(size_t)g.o_v + e * PP + j] = G.tab[(size_t)g.o_v + g.ulo * PP + j];
          G.tab[(size_t)g.o_d + e * PP + j] = G.tab[(size_t)g.o_d + g.ulo * PP + j];
        }
    }
  }
  G.off = (G.base_total + 255) & ~(size_t)255;
  P.lay.total = G.off + (((size_t)8 * o + 255) & ~(size_t)255);
  P.geo = G;
  return IFFD_OK;
}

}  // namespace iffd
