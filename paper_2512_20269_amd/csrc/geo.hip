// The system matrix of the Poisson problem on a mapped domain (3D):
//   A_ij = int_[0,1]^3 grad B_i^T G grad B_j dxi,  G = |det J| J^{-1} J^{-T},
// J = dF/dxi for a built-in analytic map F (Section 2's problem on
// Omega = F([0,1]^3); the preconditioners stay those of A-hat, Section 3).
// Gauss-Legendre rules with p_k + 1 points per element and direction.
//
// Matrix-free, in two kernels:
//   geo_element  per element (several per workgroup; one lane per line of the
//                element tensor when p_1 = p_2 = p_3, geo_element_lines,
//                else one lane per local index): gather the (p_1+1)(p_2+1)
//                (p_3+1) local coefficients, sum factorization to the
//                gradients at the Gauss points (three contractions), G from
//                the map at each point, the transposed contractions back to
//                the local functions; the local result goes to a workspace
//                slot of its own (no atomics), stored local index major
//                (all elements of one local index contiguous) so that the
//                gather reads whole cache lines;
//   geo_gather   one thread per kept coefficient: the sum of the (at most
//                (p+1)^3) element contributions in a fixed order, plus
//                per-block partial sums of x . y or (f - y)^2 for PCG.
// Deterministic: no result depends on scheduling.
//
// Every map is built from one-dimensional factors (the bump's sin(pi xi_k),
// the annulus' radius and circle, the plate's circle and outer sides): the
// host tabulates them at the p_k + 1 Gauss points of every element and
// direction, and G at a point is a few products of them (closed forms in
// geo_metric).
#include <hip/hip_runtime.h>

#include "launch.h"

namespace iffd {

// factors of the map per direction and Gauss point, tabulated on the host
// with the element tables (geo_map_factors in plan.cpp):
//   bump:     f = (sin(pi xi), cos(pi xi))
//   annulus:  direction 1: f = (r(xi)), direction 2: f = (c1, c2, c1', c2')
//             of the quarter circle at t = xi, direction 3: unused
//   plate:    direction 1: with the hole's arc R c(xi) and the outer sides
//             o(xi), f = (o - R c, R c', o' - R c') (two entries each),
//             direction 2: f = (xi), direction 3: unused
constexpr int GEO_NF = GEO_FACTORS;

// G = |det J| J^{-1} J^{-T} at one point from the factors of the three
// directions, stored G00 G11 G22 G01 G02 G12 (symmetric), in closed form for
// each map:
//   bump     J = I + 1 g^T with g = eps grad phi (every row of dF/dxi - I is
//            grad of eps phi): det J = 1 + g . 1 (matrix determinant lemma),
//            J^{-1} = I - 1 g^T / det (Sherman-Morrison), so
//            G_kl = det delta_kl - (g_k + g_l) + |g|^2 / det; det >= 1 - 3 pi
//            |eps| > 0 for the admitted |eps| < 0.1;
//   annulus  J = [[dr c1, r c1', 0], [dr c2, r c2', 0], [0, 0, H]]: with the
//            2 x 2 block K and k = det K, G = (H / |k|) adj(K) adj(K)^T on
//            that block and G22 = |k| / H;
//   plate    the same form with the columns dF/dxi_1 = R c' + xi_2 (o' - R c')
//            and dF/dxi_2 = o - R c of K.
__device__ __forceinline__ void geo_metric(int kind, const double* par, const double* f1,
                                           const double* f2, const double* f3, double G[6]) {
  if (kind == IFFD_GEOMETRY_BUMP) {
    // F = xi + eps phi (1, 1, 1), phi = sin(pi xi1) sin(pi xi2) sin(pi xi3)
    const double pe = 3.14159265358979323846 * par[0];
    const double g0 = pe * f1[1] * f2[0] * f3[0], g1 = pe * f1[0] * f2[1] * f3[0],
                 g2 = pe * f1[0] * f2[0] * f3[1];
    const double det = 1.0 + g0 + g1 + g2;
    const double q = (g0 * g0 + g1 * g1 + g2 * g2) / det;
    G[0] = det - 2.0 * g0 + q;
    G[1] = det - 2.0 * g1 + q;
    G[2] = det - 2.0 * g2 + q;
    G[3] = q - g0 - g1;
    G[4] = q - g0 - g2;
    G[5] = q - g1 - g2;
  } else {
    // the 2 x 2 block K = [[k00, k01], [k10, k11]] of J (columns dF/dxi_1,
    // dF/dxi_2) over a prism of height H
    double k00, k10, k01, k11;
    const double H = par[2];
    if (kind == IFFD_GEOMETRY_ANNULUS) {
      // F = (r c1(xi2), r c2(xi2), H xi3), r = r_in + (r_out - r_in) xi1
      const double dr = par[1] - par[0], r = f1[0];
      k00 = dr * f2[0]; k10 = dr * f2[1]; k01 = r * f2[2]; k11 = r * f2[3];
    } else {
      // F = ((1 - xi2) R c(xi1) + xi2 o(xi1), H xi3)
      const double s = f2[0];
      k00 = f1[2] + s * f1[4]; k10 = f1[3] + s * f1[5]; k01 = f1[0]; k11 = f1[1];
    }
    const double k = fabs(k00 * k11 - k01 * k10);
    const double h = H / k;
    G[0] = h * (k11 * k11 + k01 * k01);
    G[1] = h * (k10 * k10 + k00 * k00);
    G[3] = -h * (k11 * k10 + k01 * k00);
    G[2] = k / H;
    G[4] = 0.0;
    G[5] = 0.0;
  }
  (void)f3;
}

// per-direction element tables (FP64): Gauss points x[e][q], weights w[e][q]
// (h/2 times the reference weights), values V[e][q][a] and derivatives
// D[e][q][a] of the B-splines e .. e+p (full basis) at them
struct GeoDir {
  const double* x;
  const double* F;   // F[e][q][GEO_NF]: the map's factors at the points
  const double* w;
  const double* V;
  const double* D;
  int n, P, lo, m;   // elements, p + 1, full index of kept entry 0 (Dirichlet at 0), kept
  int kk, rk;        // breakpoint kk / n repeated rk + 1 times (rk = 0: none)
  int ulo, uhi;      // elements ulo..uhi hold one table (the basis is translation
                     // invariant there); ulo > uhi: none
};

// full index of the first B-spline nonzero on element e: past a breakpoint of
// multiplicity rk + 1 the rk extra functions come first
__device__ __forceinline__ int geo_first(const GeoDir& g, int e) {
  return e + (e >= g.kk ? g.rk : 0);
}
// the element on which full function gi is local function a, or a value
// outside 0 .. n - 1 when there is none
__device__ __forceinline__ int geo_elem(const GeoDir& g, int gi, int a) {
  const int e = gi - a;
  if (e < g.kk) return e;
  const int e2 = e - g.rk;
  return e2 >= g.kk ? e2 : -1;
}

struct GeoArgs {
  GeoDir d[3];
  int kind;
  double par[4];
  int N;      // kept coefficients per right-hand side
  int nloc;   // P1 P2 P3
  int nel;    // n1 n2 n3
  int ls;     // workspace stride of one local index: nel padded to an odd
              // multiple of 32 doubles (256 bytes), so that the (p+1)^3 streams
              // of a workgroup do not start on the same HBM channel
};

constexpr int GEO_T = 1024;    // gather threads per block (its block count is the PCG partial count)
constexpr int GEO_MAXP = 9;    // p <= 8

// PM3: the capacity along xi_3 (PM, or 1 for a 2D plan's one-point third
// direction, which then packs more elements into a workgroup)
template <int PM, int PM3 = PM>
struct GeoCfg {
  static constexpr int CUBE = PM * PM * PM3;
  // lanes: one per local index up to 256 (one to four wavefronts)
  static constexpr int NT = CUBE <= 64 ? 64 : (CUBE <= 128 ? 128 : 256);
  static constexpr int E = 2 * CUBE > NT ? 1 : NT / CUBE;   // elements per workgroup
  static constexpr int PP = PM * PM;
};

// PM >= max_k P_k.  Lane t of the workgroup takes the items t, t + NT, ... of
// the E * nloc (element, local index) pairs; every stage ends in a barrier.
// UNI: P_1 = P_2 = P_3 = PM, known at compile time (every index split by a
// constant); otherwise the P_k <= PM come from the plan.
template <int PM, bool UNI, int PM3 = PM>
__global__ void __launch_bounds__((GeoCfg<PM, PM3>::NT))
geo_element(const double* __restrict__ x, double* __restrict__ loc, GeoArgs a,
            const double* __restrict__ active, int astride) {
  using C = GeoCfg<PM, PM3>;
  constexpr int E = C::E, CU = C::CUBE, PP = C::PP, NT = C::NT;
  __shared__ double U[E * CU], A1[E * CU], A2[E * CU];
  __shared__ double B1[E * CU], B2[E * CU], B3[E * CU];
  __shared__ double tv[E][3][PP], td[E][3][PP];
  __shared__ double tw[E][3][PM], tf[E][3][PM][GEO_NF];
  const int rhs = blockIdx.y;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const GeoDir &d1 = a.d[0], &d2 = a.d[1], &d3 = a.d[2];
  const int P1 = UNI ? PM : d1.P, P2 = UNI ? PM : d2.P, P3 = UNI ? PM : d3.P;
  const int nloc = UNI ? CU : a.nloc;
  const int tid = threadIdx.x;
  const int el0 = xcd_linear(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, a.nel - el0);   // elements of this workgroup
  const int items = ne * nloc;
  // element tables and the map's factors at the Gauss points
  for (int t = tid; t < ne * 3 * PP; t += NT) {
    const int ee = t / (3 * PP), r = t - ee * 3 * PP, k = r / PP, j = r - k * PP;
    const GeoDir& g = a.d[k];
    const int el = el0 + ee;
    const int ek = k == 0 ? el % d1.n : (k == 1 ? (el / d1.n) % d2.n : el / (d1.n * d2.n));
    if (UNI || j < g.P * g.P) {
      tv[ee][k][j] = g.V[(size_t)ek * g.P * g.P + j];
      td[ee][k][j] = g.D[(size_t)ek * g.P * g.P + j];
    }
  }
  for (int t = tid; t < ne * 3 * PM; t += NT) {
    const int ee = t / (3 * PM), r = t - ee * 3 * PM, k = r / PM, q = r - k * PM;
    const GeoDir& g = a.d[k];
    const int el = el0 + ee;
    const int ek = k == 0 ? el % d1.n : (k == 1 ? (el / d1.n) % d2.n : el / (d1.n * d2.n));
    if (UNI || q < g.P) {
      tw[ee][k][q] = g.w[(size_t)ek * g.P + q];
#pragma unroll
      for (int i = 0; i < GEO_NF; ++i) tf[ee][k][q][i] = g.F[((size_t)ek * g.P + q) * GEO_NF + i];
    }
  }
  // local coefficients U[a3][a2][a1] (0 for dropped B-splines)
  const double* xr = x + (size_t)rhs * a.N;
  for (int t = tid; t < items; t += NT) {
    const int ee = t / nloc, i = t - ee * nloc;
    const int el = el0 + ee;
    const int e1 = el % d1.n, e2 = (el / d1.n) % d2.n, e3 = el / (d1.n * d2.n);
    const int a1 = i % P1, a2 = (i / P1) % P2, a3 = i / (P1 * P2);
    const int r1 = geo_first(d1, e1) + a1 - d1.lo, r2 = geo_first(d2, e2) + a2 - d2.lo,
              r3 = geo_first(d3, e3) + a3 - d3.lo;
    const bool ok = r1 >= 0 && r1 < d1.m && r2 >= 0 && r2 < d2.m && r3 >= 0 && r3 < d3.m;
    U[ee * CU + i] = ok ? xr[(size_t)r1 + (size_t)d1.m * (r2 + (size_t)d2.m * r3)] : 0.0;
  }
  __syncthreads();
  // direction 1: A1 = V1 U, A2 = D1 U   ([a3][a2][q1])
  for (int t = tid; t < items; t += NT) {
    const int ee = t / nloc, i = t - ee * nloc;
    const int q1 = i % P1, rest = i / P1;
    const double* u = U + ee * CU + rest * P1;
    const double *v = tv[ee][0] + q1 * P1, *dd = td[ee][0] + q1 * P1;
    double s = 0.0, w = 0.0;
    for (int a1 = 0; a1 < P1; ++a1) {
      s += v[a1] * u[a1];
      w += dd[a1] * u[a1];
    }
    A1[ee * CU + i] = s;
    A2[ee * CU + i] = w;
  }
  __syncthreads();
  // direction 2: B1 = V2 A1, B2 = D2 A1, B3 = V2 A2   ([a3][q2][q1])
  for (int t = tid; t < items; t += NT) {
    const int ee = t / nloc, i = t - ee * nloc;
    const int q1 = i % P1, q2 = (i / P1) % P2, a3 = i / (P1 * P2);
    const double *v = tv[ee][1] + q2 * P2, *dd = td[ee][1] + q2 * P2;
    const double* x1 = A1 + ee * CU + a3 * P2 * P1 + q1;
    const double* x2 = A2 + ee * CU + a3 * P2 * P1 + q1;
    double s = 0.0, w = 0.0, u = 0.0;
    for (int a2 = 0; a2 < P2; ++a2) {
      s += v[a2] * x1[a2 * P1];
      w += dd[a2] * x1[a2 * P1];
      u += v[a2] * x2[a2 * P1];
    }
    B1[ee * CU + i] = s;
    B2[ee * CU + i] = w;
    B3[ee * CU + i] = u;
  }
  __syncthreads();
  // direction 3 and the coefficient: gradients at the Gauss points, then
  // w G grad u ([q3][q2][q1]), kept in U, A1, A2
  for (int t = tid; t < items; t += NT) {
    const int ee = t / nloc, i = t - ee * nloc;
    const int q1 = i % P1, q2 = (i / P1) % P2, q3 = i / (P1 * P2);
    const double *v = tv[ee][2] + q3 * P3, *dd = td[ee][2] + q3 * P3;
    const int base = ee * CU + q2 * P1 + q1;
    double g1 = 0.0, g2 = 0.0, g3 = 0.0;
    for (int a3 = 0; a3 < P3; ++a3) {
      const int j = base + a3 * P2 * P1;
      g1 += v[a3] * B3[j];    // D1 V2 V3
      g2 += v[a3] * B2[j];    // V1 D2 V3
      g3 += dd[a3] * B1[j];   // V1 V2 D3
    }
    double G[6];
    geo_metric(a.kind, a.par, tf[ee][0][q1], tf[ee][1][q2], tf[ee][2][q3], G);
    const double wq = tw[ee][0][q1] * tw[ee][1][q2] * tw[ee][2][q3];
    U[ee * CU + i] = wq * (G[0] * g1 + G[3] * g2 + G[4] * g3);
    A1[ee * CU + i] = wq * (G[3] * g1 + G[1] * g2 + G[5] * g3);
    A2[ee * CU + i] = wq * (G[4] * g1 + G[5] * g2 + G[2] * g3);
  }
  __syncthreads();
  // back along direction 3: B1 = V3^T F1, B2 = V3^T F2, B3 = D3^T F3   ([a3][q2][q1])
  for (int t = tid; t < items; t += NT) {
    const int ee = t / nloc, i = t - ee * nloc;
    const int q1 = i % P1, q2 = (i / P1) % P2, a3 = i / (P1 * P2);
    const int base = ee * CU + q2 * P1 + q1;
    double s = 0.0, w = 0.0, u = 0.0;
    for (int q3 = 0; q3 < P3; ++q3) {
      const int j = base + q3 * P2 * P1;
      const double v = tv[ee][2][q3 * P3 + a3], dd = td[ee][2][q3 * P3 + a3];
      s += v * U[j];
      w += v * A1[j];
      u += dd * A2[j];
    }
    B1[ee * CU + i] = s;
    B2[ee * CU + i] = w;
    B3[ee * CU + i] = u;
  }
  __syncthreads();
  // back along direction 2: A1 = V2^T B1 (takes D1), A2 = D2^T B2 + V2^T B3 (takes V1)
  for (int t = tid; t < items; t += NT) {
    const int ee = t / nloc, i = t - ee * nloc;
    const int q1 = i % P1, a2 = (i / P1) % P2, a3 = i / (P1 * P2);
    const int base = ee * CU + a3 * P2 * P1 + q1;
    double s = 0.0, w = 0.0;
    for (int q2 = 0; q2 < P2; ++q2) {
      const int j = base + q2 * P1;
      const double v = tv[ee][1][q2 * P2 + a2], dd = td[ee][1][q2 * P2 + a2];
      s += v * B1[j];
      w += dd * B2[j] + v * B3[j];
    }
    A1[ee * CU + i] = s;
    A2[ee * CU + i] = w;
  }
  __syncthreads();
  // back along direction 1: the element's contribution to its local functions,
  // stored at loc[(rhs nloc + i) ls + el]
  double* out = loc + (size_t)rhs * nloc * a.ls;
  for (int t = tid; t < items; t += NT) {
    const int ee = t / nloc, i = t - ee * nloc;
    const int a1 = i % P1, rest = i / P1;
    const double* y1 = A1 + ee * CU + rest * P1;
    const double* y2 = A2 + ee * CU + rest * P1;
    double s = 0.0;
    for (int q1 = 0; q1 < P1; ++q1) s += td[ee][0][q1 * P1 + a1] * y1[q1] + tv[ee][0][q1 * P1 + a1] * y2[q1];
    out[(size_t)i * a.ls + el0 + ee] = s;
  }
}

// Line-wise sum factorization for P_1 = P_2 = P_3 = P: lane (element, line)
// holds one line of the element's P^3 tensor in registers and applies the
// one-dimensional factor along it; the result goes back to the same line
// positions, so three LDS arrays serve all stages and only the change of
// direction between stages needs a barrier.  Direction 3's forward
// contraction, the coefficient G at the P points of the line and the
// backward contraction along direction 3 are one stage.
//   stage 1  lines along xi_1 (a2, a3):  A1 = V1 U, A2 = D1 U
//   stage 2  lines along xi_2 (q1, a3):  B1 = V2 A1, B2 = D2 A1, B3 = V2 A2
//   stage 3  lines along xi_3 (q1, q2):  grad u at the points, F = w G grad u,
//                                        C1 = V3^T F1, C2 = V3^T F2, C3 = D3^T F3
//   stage 4  lines along xi_2 (q1, a3):  A1 = V2^T C1, A2 = D2^T C2 + V2^T C3
//   stage 5  lines along xi_1 (a2, a3):  y_loc = D1^T A1 + V1^T A2 -> workspace
template <int P>
struct GeoLineCfg {
  static constexpr int L = P * P;                         // lines per element
  static constexpr int NT = P <= 4 ? 64 : (P <= 8 ? 128 : 256);   // lanes
  static constexpr int E = NT / L;                        // elements per workgroup
  // LDS strides (doubles) of a2, a3 and of the elements: padded so that the
  // lanes of one access (P^2 lines of each of E elements, along any of the three
  // directions) spread over the banks; the padded values come from a search
  // over S1 in [P, P+8], S2 and ES up to 16 and 32 past their minimum, scored by
  // the most lanes on one bank in groups of 16 and 32 lanes (16 and 32 banks
  // of 8 bytes); where the best needs more LDS (P = 6, 7, 9: fewer waves per
  // compute unit, measured slower at P = 6) the odd strides stay
  static constexpr int S1 = P == 2 ? 3 : P == 4 ? 5 : P == 8 ? 9 : (P | 1);
  static constexpr int S2 = P == 2 ? 6 : P == 4 ? 20 : P == 8 ? 72 : (S1 * P) | 1;
  static constexpr int ES = P == 2 ? 12 : P == 4 ? 80 : P == 8 ? 576 : (S2 * P) | 1;
  static_assert(S1 >= P && S2 >= S1 * P && ES >= S2 * P, "strides must not overlap");
};

template <int P>
__global__ void __launch_bounds__(GeoLineCfg<P>::NT)
geo_element_lines(const double* __restrict__ x, double* __restrict__ loc, GeoArgs a,
                  const double* __restrict__ active, int astride) {
  using C = GeoLineCfg<P>;
  constexpr int E = C::E, L = C::L, NT = C::NT, S1 = C::S1, S2 = C::S2, ES = C::ES;
  constexpr int PP = P * P, CU = P * P * P;
  __shared__ double X0[E * ES], X1[E * ES], X2[E * ES];
  __shared__ double tv[E][PP], td[E][PP];        // direction 1, per element
  __shared__ double tw1[E][P], tf1[E][P][GEO_NF];
  __shared__ double tw23[2][P], tf23[2][P][GEO_NF];   // directions 2 and 3, one element each
  const int rhs = blockIdx.y;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const GeoDir &d1 = a.d[0], &d2 = a.d[1], &d3 = a.d[2];
  const int tid = threadIdx.x;
  // a workgroup takes up to E consecutive elements of one row along xi_1: they
  // share e2 and e3, so the tables of directions 2 and 3 are the same for the
  // whole wave and are read with scalar loads, not from LDS
  const int bpr = (d1.n + E - 1) / E;
  const int b = xcd_linear(blockIdx.x, gridDim.x);
  const int row = b / bpr;
  const int e10 = (b - row * bpr) * E;
  const int ne = min(E, d1.n - e10);
  const int e2 = row % d2.n, e3 = row / d2.n;
  const int el0 = row * d1.n + e10;
  // direction 1's tables: where every element of the workgroup lies in the
  // translation-invariant range they are one table, read with scalar loads;
  // otherwise per element from LDS
  const bool u1 = e10 >= d1.ulo && e10 + ne - 1 <= d1.uhi;
  const double* V1 = d1.V + (size_t)(u1 ? d1.ulo : 0) * PP;
  const double* D1 = d1.D + (size_t)(u1 ? d1.ulo : 0) * PP;
  const double* V2 = d2.V + (size_t)e2 * PP;
  const double* D2 = d2.D + (size_t)e2 * PP;
  const double* V3 = d3.V + (size_t)e3 * PP;
  const double* D3 = d3.D + (size_t)e3 * PP;
  if (!u1)
    for (int t = tid; t < ne * PP; t += NT) {
      tv[0][t] = d1.V[(size_t)e10 * PP + t];
      td[0][t] = d1.D[(size_t)e10 * PP + t];
    }
  for (int t = tid; t < ne * P; t += NT) {
    tw1[0][t] = d1.w[(size_t)e10 * P + t];
#pragma unroll
    for (int i = 0; i < GEO_NF; ++i) tf1[0][t][i] = d1.F[((size_t)e10 * P + t) * GEO_NF + i];
  }
  if (tid < 2 * P) {
    const int k = tid / P, q = tid - k * P;
    const GeoDir& g = k ? d3 : d2;
    const int e = k ? e3 : e2;
    tw23[k][q] = g.w[(size_t)e * P + q];
#pragma unroll
    for (int i = 0; i < GEO_NF; ++i) tf23[k][q][i] = g.F[((size_t)e * P + q) * GEO_NF + i];
  }
  const double* xr = x + (size_t)rhs * a.N;
  const int f2 = geo_first(d2, e2) - d2.lo, f3 = geo_first(d3, e3) - d3.lo;
  for (int t = tid; t < ne * CU; t += NT) {
    const int ee = t / CU, i = t - ee * CU;
    const int a1 = i % P, a2 = (i / P) % P, a3 = i / PP;
    const int r1 = geo_first(d1, e10 + ee) + a1 - d1.lo, r2 = f2 + a2, r3 = f3 + a3;
    const bool ok = r1 >= 0 && r1 < d1.m && r2 >= 0 && r2 < d2.m && r3 >= 0 && r3 < d3.m;
    X0[ee * ES + a1 + S1 * a2 + S2 * a3] =
        ok ? xr[(size_t)r1 + (size_t)d1.m * (r2 + (size_t)d2.m * r3)] : 0.0;
  }
  __syncthreads();
  const int ee = tid / L, ln = tid - ee * L;
  const bool live = ee < ne;
  const int la = ln % P, lb = ln / P;     // the line's two fixed indices
  double* Y0 = X0 + ee * ES;
  double* Y1 = X1 + ee * ES;
  double* Y2 = X2 + ee * ES;
  // In every stage the outer loop runs over the output (or input) index along
  // the line without unrolling; what it indexes is read from LDS as it goes
  // (this lane owns the line, so reading and rewriting it in place is safe),
  // and only the unrolled inner index lives in registers.
  // stage 1: line (a2, a3) = (la, lb) along a1
  auto stage1 = [&](const double* V, const double* D) {
    if (!live) return;
    const int o = S1 * la + S2 * lb;
    double u[P];
#pragma unroll
    for (int j = 0; j < P; ++j) u[j] = Y0[o + j];
#pragma unroll 1
    for (int q = 0; q < P; ++q) {
      double s = 0.0, w = 0.0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        s += V[q * P + j] * u[j];
        w += D[q * P + j] * u[j];
      }
      Y0[o + q] = s;
      Y1[o + q] = w;
    }
  };
  if (u1)
    stage1(V1, D1);
  else
    stage1(tv[ee], td[ee]);
  __syncthreads();
  // stage 2: line (q1, a3) = (la, lb) along a2
  if (live) {
    const int o = la + S2 * lb;
    double u1[P], u2[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      u1[j] = Y0[o + S1 * j];
      u2[j] = Y1[o + S1 * j];
    }
#pragma unroll 1
    for (int q = 0; q < P; ++q) {
      double s = 0.0, w = 0.0, v = 0.0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double vv = V2[q * P + j], dd = D2[q * P + j];
        s += vv * u1[j];
        w += dd * u1[j];
        v += vv * u2[j];
      }
      Y0[o + S1 * q] = s;
      Y1[o + S1 * q] = w;
      Y2[o + S1 * q] = v;
    }
  }
  __syncthreads();
  // stage 3: line (q1, q2) = (la, lb) along a3 / q3
  if (live) {
    const int o = la + S1 * lb;
    double b1[P], b2[P], b3[P], c1[P], c2[P], c3[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      b1[j] = Y0[o + S2 * j];
      b2[j] = Y1[o + S2 * j];
      b3[j] = Y2[o + S2 * j];
      c1[j] = c2[j] = c3[j] = 0.0;
    }
    const double w12 = tw1[ee][la] * tw23[0][lb];
    // the annulus and the plate are prisms over xi_3 (G does not depend on
    // xi_3): G of the line's points is computed once
    const bool prism = a.kind == IFFD_GEOMETRY_ANNULUS || a.kind == IFFD_GEOMETRY_PLATE;
    double G[6];
    if (prism) geo_metric(a.kind, a.par, tf1[ee][la], tf23[0][lb], tf23[1][0], G);
#pragma unroll 1
    for (int q = 0; q < P; ++q) {
      double g1 = 0.0, g2 = 0.0, g3 = 0.0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double vv = V3[q * P + j], dd = D3[q * P + j];
        g1 += vv * b3[j];   // D1 V2 V3
        g2 += vv * b2[j];   // V1 D2 V3
        g3 += dd * b1[j];   // V1 V2 D3
      }
      if (!prism) geo_metric(a.kind, a.par, tf1[ee][la], tf23[0][lb], tf23[1][q], G);
      const double wq = w12 * tw23[1][q];
      const double f1 = wq * (G[0] * g1 + G[3] * g2 + G[4] * g3);
      const double f2 = wq * (G[3] * g1 + G[1] * g2 + G[5] * g3);
      const double f3 = wq * (G[4] * g1 + G[5] * g2 + G[2] * g3);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double vv = V3[q * P + j], dd = D3[q * P + j];
        c1[j] += vv * f1;
        c2[j] += vv * f2;
        c3[j] += dd * f3;
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      Y0[o + S2 * j] = c1[j];
      Y1[o + S2 * j] = c2[j];
      Y2[o + S2 * j] = c3[j];
    }
  }
  __syncthreads();
  // stage 4: line (q1, a3) = (la, lb) along q2 -> a2
  if (live) {
    const int o = la + S2 * lb;
    double s1[P], s2[P];
#pragma unroll
    for (int j = 0; j < P; ++j) s1[j] = s2[j] = 0.0;
#pragma unroll 1
    for (int q = 0; q < P; ++q) {
      const double c1 = Y0[o + S1 * q], c2 = Y1[o + S1 * q], c3 = Y2[o + S1 * q];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double vv = V2[q * P + j], dd = D2[q * P + j];
        s1[j] += vv * c1;
        s2[j] += dd * c2 + vv * c3;
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
      Y0[o + S1 * j] = s1[j];
      Y1[o + S1 * j] = s2[j];
    }
  }
  __syncthreads();
  // stage 5: line (a2, a3) = (la, lb) along q1 -> a1, to loc[(rhs nloc + i) ls + el]
  auto stage5 = [&](const double* V, const double* D) {
    if (!live) return;
    const int o = S1 * la + S2 * lb;
    double s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) s[j] = 0.0;
#pragma unroll 1
    for (int q = 0; q < P; ++q) {
      const double y1 = Y0[o + q], y2 = Y1[o + q];
#pragma unroll
      for (int j = 0; j < P; ++j)
        s[j] += D[q * P + j] * y1 + V[q * P + j] * y2;
    }
    double* out = loc + ((size_t)rhs * CU + (size_t)P * ln) * a.ls + el0 + ee;
#pragma unroll
    for (int j = 0; j < P; ++j) out[(size_t)j * a.ls] = s[j];
  };
  if (u1)
    stage5(V1, D1);
  else
    stage5(tv[ee], td[ee]);
}

// the gather for P_1 = P_2 = P_3 = P: the same fixed order, every load of a
// row issued unconditionally from a clamped address
template <int P>
__global__ void __launch_bounds__(GEO_T)
geo_gather_uni(const double* __restrict__ loc, double* __restrict__ y, GeoArgs a, int nblk,
               const double* __restrict__ xd, const double* __restrict__ fres,
               double* __restrict__ part, int npart, const double* __restrict__ active,
               int astride) {
  __shared__ double red[GEO_T / 64];
  const int rhs = blockIdx.x / nblk, blk = blockIdx.x - rhs * nblk;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const GeoDir &d1 = a.d[0], &d2 = a.d[1], &d3 = a.d[2];
  const int c = (a.N + nblk - 1) / nblk;
  const int lo = min(a.N, blk * c), hi = min(a.N, lo + c);
  const size_t ro = (size_t)rhs * a.N;
  const size_t nel = (size_t)a.ls;   // the stride of one local index
  const double* lr = loc + (size_t)rhs * (P * P * P) * nel;
  double dot = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += GEO_T) {
    const int r1 = i % d1.m, r2 = (i / d1.m) % d2.m, r3 = i / (d1.m * d2.m);
    const int g1 = r1 + d1.lo, g2 = r2 + d2.lo, g3 = r3 + d3.lo;   // full indices
    double s = 0.0;
    for (int a3 = 0; a3 < P; ++a3) {
      const int e3 = geo_elem(d3, g3, a3);
      if (e3 < 0 || e3 >= d3.n) continue;
      for (int a2 = 0; a2 < P; ++a2) {
        const int e2 = geo_elem(d2, g2, a2);
        if (e2 < 0 || e2 >= d2.n) continue;
        const double* row = lr + (size_t)((a3 * P + a2) * P) * nel + (size_t)d1.n * (e2 + (size_t)d2.n * e3);
        double v[P];
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) {
          const int e1 = geo_elem(d1, g1, a1);
          const bool ok = e1 >= 0 && e1 < d1.n;
          v[a1] = row[(size_t)a1 * nel + (ok ? e1 : 0)];
          v[a1] = ok ? v[a1] : 0.0;
        }
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) s += v[a1];
      }
    }
    y[ro + i] = s;
    if (part) {
      if (fres) {
        const double dv = fres[ro + i] - s;
        dot += dv * dv;
      } else {
        dot += xd[ro + i] * s;
      }
    }
  }
  if (!part) return;
  for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s2 = 0.0;
    for (int w = 0; w < GEO_T / 64; ++w) s2 += red[w];
    part[(size_t)rhs * npart + blk] = s2;
  }
}

// y at every kept coefficient: the element contributions in a fixed order
// (local index a3, a2, a1 descending through the elements e = g - a);
// per-block partial sums (x . y, or (f - y)^2 when fres is given)
__global__ void __launch_bounds__(GEO_T)
geo_gather(const double* __restrict__ loc, double* __restrict__ y, GeoArgs a, int nblk,
           const double* __restrict__ xd, const double* __restrict__ fres,
           double* __restrict__ part, int npart, const double* __restrict__ active, int astride) {
  __shared__ double red[GEO_T / 64];
  const int rhs = blockIdx.x / nblk, blk = blockIdx.x - rhs * nblk;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const GeoDir &d1 = a.d[0], &d2 = a.d[1], &d3 = a.d[2];
  const int c = (a.N + nblk - 1) / nblk;
  const int lo = min(a.N, blk * c), hi = min(a.N, lo + c);
  const size_t ro = (size_t)rhs * a.N;
  const double* lr = loc + (size_t)rhs * a.nloc * a.ls;
  double dot = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += GEO_T) {
    const int r1 = i % d1.m, r2 = (i / d1.m) % d2.m, r3 = i / (d1.m * d2.m);
    const int g1 = r1 + d1.lo, g2 = r2 + d2.lo, g3 = r3 + d3.lo;   // full indices
    double s = 0.0;
    for (int a3 = 0; a3 < d3.P; ++a3) {
      const int e3 = geo_elem(d3, g3, a3);
      if (e3 < 0 || e3 >= d3.n) continue;
      for (int a2 = 0; a2 < d2.P; ++a2) {
        const int e2 = geo_elem(d2, g2, a2);
        if (e2 < 0 || e2 >= d2.n) continue;
        const double* row = lr + (size_t)((a3 * d2.P + a2) * d1.P) * a.ls +
                            (size_t)d1.n * (e2 + (size_t)d2.n * e3);
        for (int a1 = 0; a1 < d1.P; ++a1) {
          const int e1 = geo_elem(d1, g1, a1);
          if (e1 >= 0 && e1 < d1.n) s += row[(size_t)a1 * a.ls + e1];
        }
      }
    }
    y[ro + i] = s;
    if (part) {
      if (fres) {
        const double dv = fres[ro + i] - s;
        dot += dv * dv;
      } else {
        dot += xd[ro + i] * s;
      }
    }
  }
  if (!part) return;
  for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s2 = 0.0;
    for (int w = 0; w < GEO_T / 64; ++w) s2 += red[w];
    part[(size_t)rhs * npart + blk] = s2;
  }
}

static int geo_local_stride(int nel) { return (nel + 63) / 64 * 64 + 32; }

static GeoArgs geo_args(const Plan& P) {
  GeoArgs a;
  const double* t = (const double*)(P.d_tables + P.geo.off);
  for (int k = 0; k < 3; ++k) {
    const GeoPlanDir& g = P.geo.dir[k];
    a.d[k].x = t + g.o_x;
    a.d[k].F = t + g.o_f;
    a.d[k].w = t + g.o_w;
    a.d[k].V = t + g.o_v;
    a.d[k].D = t + g.o_d;
    a.d[k].n = g.n;
    a.d[k].P = g.P;
    a.d[k].lo = g.lo;
    a.d[k].m = g.m;
    a.d[k].kk = g.kk;
    a.d[k].rk = g.rk;
    a.d[k].ulo = g.ulo;
    a.d[k].uhi = g.uhi;
  }
  a.kind = P.geo.kind;
  for (int i = 0; i < 4; ++i) a.par[i] = P.geo.par[i];
  a.N = (int)P.N;
  a.nloc = a.d[0].P * a.d[1].P * a.d[2].P;
  a.nel = a.d[0].n * a.d[1].n * a.d[2].n;
  a.ls = geo_local_stride(a.nel);
  return a;
}

size_t geo_matvec_ws_bytes(const Plan& P, int nrhs) {
  size_t nel = 1, nloc = 1;
  for (int k = 0; k < 3; ++k) {
    nel *= (size_t)P.geo.dir[k].n;
    nloc *= (size_t)P.geo.dir[k].P;
  }
  return 8 * (size_t)geo_local_stride((int)nel) * nloc * (size_t)nrhs;
}

int geo_matvec_blocks(const Plan& P) { return pcg_blocks(P); }

template <int PM>
static void launch_geo_element(const GeoArgs& a, const double* x, double* loc, double* y,
                               int nrhs, int nb, double* part, int npart, const double* act,
                               int as, hipStream_t s, const double* fres) {
  const bool uni = a.d[0].P == PM && a.d[1].P == PM && a.d[2].P == PM;
  if (uni) {
    constexpr int E = GeoLineCfg<PM>::E, NT = GeoLineCfg<PM>::NT;
    // whole rows along xi_1, E elements per workgroup
    const unsigned nwg = (unsigned)((a.d[0].n + E - 1) / E * a.d[1].n * a.d[2].n);
    hipLaunchKernelGGL(geo_element_lines<PM>, dim3(nwg, (unsigned)nrhs), dim3(NT), 0, s, x, loc,
                       a, act, as);
    hipLaunchKernelGGL(geo_gather_uni<PM>, dim3((unsigned)(nb * nrhs)), dim3(GEO_T), 0, s,
                       (const double*)loc, y, a, nb, x, fres, part, npart, act, as);
  } else if (a.d[2].P == 1) {   // 2D: the one-point third direction
    constexpr int E = GeoCfg<PM, 1>::E, NT = GeoCfg<PM, 1>::NT;
    const unsigned nwg = (unsigned)((a.nel + E - 1) / E);
    hipLaunchKernelGGL((geo_element<PM, false, 1>), dim3(nwg, (unsigned)nrhs), dim3(NT), 0, s, x,
                       loc, a, act, as);
    hipLaunchKernelGGL(geo_gather, dim3((unsigned)(nb * nrhs)), dim3(GEO_T), 0, s,
                       (const double*)loc, y, a, nb, x, fres, part, npart, act, as);
  } else {
    constexpr int E = GeoCfg<PM>::E, NT = GeoCfg<PM>::NT;
    const unsigned nwg = (unsigned)((a.nel + E - 1) / E);
    hipLaunchKernelGGL((geo_element<PM, false>), dim3(nwg, (unsigned)nrhs), dim3(NT), 0, s, x,
                       loc, a, act, as);
    hipLaunchKernelGGL(geo_gather, dim3((unsigned)(nb * nrhs)), dim3(GEO_T), 0, s,
                       (const double*)loc, y, a, nb, x, fres, part, npart, act, as);
  }
}

hipError_t launch_geo_matvec(const Plan& P, const double* x, double* y, int nrhs, void* ws,
                             double* part, int npart, const double* act, int as, hipStream_t s,
                             const double* fres) {
  if (!ws) return hipErrorInvalidValue;
  const GeoArgs a = geo_args(P);
  const int pm = std::max(a.d[0].P, std::max(a.d[1].P, a.d[2].P));
  if (pm < 2 || pm > GEO_MAXP) return hipErrorInvalidValue;
  const int nb = geo_matvec_blocks(P);
  if (part && npart < nb) return hipErrorInvalidValue;
  double* loc = (double*)ws;
#define IFFD_GEO_CASE(PM_)                                                                   \
  case PM_:                                                                                  \
    launch_geo_element<PM_>(a, x, loc, y, nrhs, nb, part, npart, act, as, s, fres);            \
    break;
  switch (pm) {
    IFFD_GEO_CASE(2)
    IFFD_GEO_CASE(3)
    IFFD_GEO_CASE(4)
    IFFD_GEO_CASE(5)
    IFFD_GEO_CASE(6)
    IFFD_GEO_CASE(7)
    IFFD_GEO_CASE(8)
    default: launch_geo_element<9>(a, x, loc, y, nrhs, nb, part, npart, act, as, s, fres); break;
  }
#undef IFFD_GEO_CASE
  return hipGetLastError();
}

}  // namespace iffd
