// The system matrix of the Poisson problem on a mapped domain (3D):
//   A_ij = int_[0,1]^3 grad B_i^T G grad B_j dxi,  G = |det J| J^{-1} J^{-T},
// J = dF/dxi for a built-in analytic map F (Section 2's problem on
// Omega = F([0,1]^3); the preconditioners stay those of A-hat, Section 3).
// Gauss-Legendre rules with p_k + 1 points per element and direction.
//
// Matrix-free, in two kernels:
//   geo_element  one workgroup per element: gather the (p_1+1)(p_2+1)(p_3+1)
//                local coefficients, sum factorization to the gradients at
//                the Gauss points (three contractions), G(xi) from the map at
//                each point, the transposed contractions back to the local
//                functions; the local result is written to a workspace slot
//                of its own (no atomics);
//   geo_gather   one thread per kept coefficient: the sum of the (at most
//                (p+1)^3) element contributions in a fixed order, plus
//                per-block partial sums of x . y or (f - y)^2 for PCG.
// Deterministic: no result depends on scheduling.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace iffd {

// the map's Jacobian J[i][k] = dF_i / dxi_k at xi
__device__ __forceinline__ void geo_jacobian(int kind, const double* par, const double* xi,
                                             double J[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) J[i][k] = 0.0;
  if (kind == IFFD_GEOMETRY_BUMP) {
    // F = xi + eps phi (1, 1, 1), phi = sin(pi xi1) sin(pi xi2) sin(pi xi3)
    const double pi = 3.14159265358979323846;
    const double eps = par[0];
    double s[3], c[3];
    for (int k = 0; k < 3; ++k) sincos(pi * xi[k], &s[k], &c[k]);
    const double g[3] = {pi * c[0] * s[1] * s[2], pi * s[0] * c[1] * s[2], pi * s[0] * s[1] * c[2]};
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < 3; ++k) J[i][k] = eps * g[k];
      J[i][i] += 1.0;
    }
  } else {
    // thick quarter of annulus: F = (r c1(t), r c2(t), H xi3), r = r_in + (r_out - r_in) xi1,
    // t = xi2, c the quarter circle as a rational quadratic (weights 1, 1/sqrt 2, 1)
    const double r_in = par[0], r_out = par[1], H = par[2];
    const double t = xi[1], w = 0.70710678118654752440;
    const double b0 = (1 - t) * (1 - t), b1 = 2 * t * (1 - t), b2 = t * t;
    const double db0 = -2 * (1 - t), db1 = 2 - 4 * t, db2 = 2 * t;
    const double den = b0 + w * b1 + b2, dden = db0 + w * db1 + db2;
    const double n1 = b0 + w * b1, n2 = w * b1 + b2;
    const double dn1 = db0 + w * db1, dn2 = w * db1 + db2;
    const double c1 = n1 / den, c2 = n2 / den;
    const double dc1 = (dn1 * den - n1 * dden) / (den * den);
    const double dc2 = (dn2 * den - n2 * dden) / (den * den);
    const double r = r_in + (r_out - r_in) * xi[0];
    J[0][0] = (r_out - r_in) * c1;
    J[1][0] = (r_out - r_in) * c2;
    J[0][1] = r * dc1;
    J[1][1] = r * dc2;
    J[2][2] = H;
  }
}

// G = |det J| (J^T J)^{-1} = |det J| J^{-1} J^{-T}, symmetric: G00 G11 G22 G01 G02 G12
__device__ __forceinline__ void geo_coefficient(int kind, const double* par, const double* xi,
                                                double G[6]) {
  double J[3][3];
  geo_jacobian(kind, par, xi, J);
  // cofactors: J^{-1} = adj(J) / det, so J^{-1} J^{-T} = adj adj^T / det^2
  double C[3][3];
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  C[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  C[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * C[0][0] + J[0][1] * C[1][0] + J[0][2] * C[2][0];
  const double f = 1.0 / fabs(det);   // |det| / det^2
  auto row = [&](int a, int b) { return C[a][0] * C[b][0] + C[a][1] * C[b][1] + C[a][2] * C[b][2]; };
  G[0] = f * row(0, 0);
  G[1] = f * row(1, 1);
  G[2] = f * row(2, 2);
  G[3] = f * row(0, 1);
  G[4] = f * row(0, 2);
  G[5] = f * row(1, 2);
}

// per-direction element tables (FP64): Gauss points x[e][q], weights w[e][q]
// (h/2 times the reference weights), values V[e][q][a] and derivatives
// D[e][q][a] of the B-splines e .. e+p (full basis) at them
struct GeoDir {
  const double* x;
  const double* w;
  const double* V;
  const double* D;
  int n, P, lo, m;   // elements, p + 1, full index of kept entry 0 (Dirichlet at 0), kept
};

struct GeoArgs {
  GeoDir d[3];
  int kind;
  double par[4];
  int N;      // kept coefficients per right-hand side
  int nloc;   // P1 P2 P3
  int nel;    // n1 n2 n3
};

constexpr int GEO_T = 256;
constexpr int GEO_MAXP = 9;   // p <= 8
constexpr int GEO_CUBE = GEO_MAXP * GEO_MAXP * GEO_MAXP;

__global__ void __launch_bounds__(GEO_T)
geo_element(const double* __restrict__ x, double* __restrict__ loc, GeoArgs a,
            const double* __restrict__ active, int astride) {
  __shared__ double U[GEO_CUBE], A1[GEO_CUBE], A2[GEO_CUBE];
  __shared__ double B1[GEO_CUBE], B2[GEO_CUBE], B3[GEO_CUBE];
  __shared__ double tv[3][GEO_MAXP * GEO_MAXP], td[3][GEO_MAXP * GEO_MAXP];
  __shared__ double tx[3][GEO_MAXP], tw[3][GEO_MAXP];
  const int el = blockIdx.x, rhs = blockIdx.y;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const GeoDir &d1 = a.d[0], &d2 = a.d[1], &d3 = a.d[2];
  const int e1 = el % d1.n, e2 = (el / d1.n) % d2.n, e3 = el / (d1.n * d2.n);
  const int P1 = d1.P, P2 = d2.P, P3 = d3.P;
  const int tid = threadIdx.x;
  const int e[3] = {e1, e2, e3};
  for (int k = 0; k < 3; ++k) {
    const GeoDir& g = a.d[k];
    const int PP = g.P * g.P;
    for (int i = tid; i < PP; i += GEO_T) {
      tv[k][i] = g.V[(size_t)e[k] * PP + i];
      td[k][i] = g.D[(size_t)e[k] * PP + i];
    }
    if (tid < g.P) {
      tx[k][tid] = g.x[(size_t)e[k] * g.P + tid];
      tw[k][tid] = g.w[(size_t)e[k] * g.P + tid];
    }
  }
  // local coefficients U[a3][a2][a1] (0 for dropped B-splines)
  const double* xr = x + (size_t)rhs * a.N;
  for (int i = tid; i < a.nloc; i += GEO_T) {
    const int a1 = i % P1, a2 = (i / P1) % P2, a3 = i / (P1 * P2);
    const int r1 = e1 + a1 - d1.lo, r2 = e2 + a2 - d2.lo, r3 = e3 + a3 - d3.lo;
    const bool ok = r1 >= 0 && r1 < d1.m && r2 >= 0 && r2 < d2.m && r3 >= 0 && r3 < d3.m;
    U[i] = ok ? xr[(size_t)r1 + (size_t)d1.m * (r2 + (size_t)d2.m * r3)] : 0.0;
  }
  __syncthreads();
  // direction 1: A1 = V1 U, A2 = D1 U   ([a3][a2][q1])
  for (int i = tid; i < a.nloc; i += GEO_T) {
    const int q1 = i % P1, rest = i / P1;
    double s = 0.0, t = 0.0;
    for (int a1 = 0; a1 < P1; ++a1) {
      const double u = U[rest * P1 + a1];
      s += tv[0][q1 * P1 + a1] * u;
      t += td[0][q1 * P1 + a1] * u;
    }
    A1[i] = s;
    A2[i] = t;
  }
  __syncthreads();
  // direction 2: B1 = V2 A1, B2 = D2 A1, B3 = V2 A2   ([a3][q2][q1])
  for (int i = tid; i < a.nloc; i += GEO_T) {
    const int q1 = i % P1, q2 = (i / P1) % P2, a3 = i / (P1 * P2);
    double s = 0.0, t = 0.0, u = 0.0;
    for (int a2 = 0; a2 < P2; ++a2) {
      const int j = (a3 * P2 + a2) * P1 + q1;
      s += tv[1][q2 * P2 + a2] * A1[j];
      t += td[1][q2 * P2 + a2] * A1[j];
      u += tv[1][q2 * P2 + a2] * A2[j];
    }
    B1[i] = s;
    B2[i] = t;
    B3[i] = u;
  }
  __syncthreads();
  // direction 3 and the coefficient: gradients at the Gauss points, then
  // F = w G grad u ([q3][q2][q1]), kept in U, A1, A2
  for (int i = tid; i < a.nloc; i += GEO_T) {
    const int q1 = i % P1, q2 = (i / P1) % P2, q3 = i / (P1 * P2);
    double g1 = 0.0, g2 = 0.0, g3 = 0.0;
    for (int a3 = 0; a3 < P3; ++a3) {
      const int j = (a3 * P2 + q2) * P1 + q1;
      const double v3 = tv[2][q3 * P3 + a3], d3v = td[2][q3 * P3 + a3];
      g1 += v3 * B3[j];   // D1 V2 V3
      g2 += v3 * B2[j];   // V1 D2 V3
      g3 += d3v * B1[j];  // V1 V2 D3
    }
    const double xi[3] = {tx[0][q1], tx[1][q2], tx[2][q3]};
    double G[6];
    geo_coefficient(a.kind, a.par, xi, G);
    const double wq = tw[0][q1] * tw[1][q2] * tw[2][q3];
    U[i] = wq * (G[0] * g1 + G[3] * g2 + G[4] * g3);
    A1[i] = wq * (G[3] * g1 + G[1] * g2 + G[5] * g3);
    A2[i] = wq * (G[4] * g1 + G[5] * g2 + G[2] * g3);
  }
  __syncthreads();
  // back along direction 3: B1 = V3^T F1, B2 = V3^T F2, B3 = D3^T F3   ([a3][q2][q1])
  for (int i = tid; i < a.nloc; i += GEO_T) {
    const int q1 = i % P1, q2 = (i / P1) % P2, a3 = i / (P1 * P2);
    double s = 0.0, t = 0.0, u = 0.0;
    for (int q3 = 0; q3 < P3; ++q3) {
      const int j = (q3 * P2 + q2) * P1 + q1;
      s += tv[2][q3 * P3 + a3] * U[j];
      t += tv[2][q3 * P3 + a3] * A1[j];
      u += td[2][q3 * P3 + a3] * A2[j];
    }
    B1[i] = s;
    B2[i] = t;
    B3[i] = u;
  }
  __syncthreads();
  // back along direction 2: A1 = V2^T B1 (takes D1), A2 = D2^T B2 + V2^T B3 (takes V1)
  for (int i = tid; i < a.nloc; i += GEO_T) {
    const int q1 = i % P1, a2 = (i / P1) % P2, a3 = i / (P1 * P2);
    double s = 0.0, t = 0.0;
    for (int q2 = 0; q2 < P2; ++q2) {
      const int j = (a3 * P2 + q2) * P1 + q1;
      s += tv[1][q2 * P2 + a2] * B1[j];
      t += td[1][q2 * P2 + a2] * B2[j] + tv[1][q2 * P2 + a2] * B3[j];
    }
    A1[i] = s;
    A2[i] = t;
  }
  __syncthreads();
  // back along direction 1: the element's contribution to its local functions
  double* out = loc + ((size_t)rhs * a.nel + el) * a.nloc;
  for (int i = tid; i < a.nloc; i += GEO_T) {
    const int a1 = i % P1, rest = i / P1;
    double s = 0.0;
    for (int q1 = 0; q1 < P1; ++q1) {
      const int j = rest * P1 + q1;
      s += td[0][q1 * P1 + a1] * A1[j] + tv[0][q1 * P1 + a1] * A2[j];
    }
    out[i] = s;
  }
}

// y at every kept coefficient: the element contributions in a fixed order;
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
  const double* lr = loc + (size_t)rhs * a.nel * a.nloc;
  double dot = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += GEO_T) {
    const int r1 = i % d1.m, r2 = (i / d1.m) % d2.m, r3 = i / (d1.m * d2.m);
    const int g1 = r1 + d1.lo, g2 = r2 + d2.lo, g3 = r3 + d3.lo;   // full indices
    double s = 0.0;
    for (int e3 = max(0, g3 - d3.P + 1); e3 <= min(d3.n - 1, g3); ++e3)
      for (int e2 = max(0, g2 - d2.P + 1); e2 <= min(d2.n - 1, g2); ++e2)
        for (int e1 = max(0, g1 - d1.P + 1); e1 <= min(d1.n - 1, g1); ++e1) {
          const size_t el = (size_t)e1 + (size_t)d1.n * (e2 + (size_t)d2.n * e3);
          const int a1 = g1 - e1, a2 = g2 - e2, a3 = g3 - e3;
          s += lr[el * a.nloc + (a3 * d2.P + a2) * d1.P + a1];
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

static GeoArgs geo_args(const Plan& P) {
  GeoArgs a;
  const double* t = (const double*)(P.d_tables + P.geo.off);
  for (int k = 0; k < 3; ++k) {
    const GeoPlanDir& g = P.geo.dir[k];
    a.d[k].x = t + g.o_x;
    a.d[k].w = t + g.o_w;
    a.d[k].V = t + g.o_v;
    a.d[k].D = t + g.o_d;
    a.d[k].n = g.n;
    a.d[k].P = g.P;
    a.d[k].lo = g.lo;
    a.d[k].m = g.m;
  }
  a.kind = P.geo.kind;
  for (int i = 0; i < 4; ++i) a.par[i] = P.geo.par[i];
  a.N = (int)P.N;
  a.nloc = a.d[0].P * a.d[1].P * a.d[2].P;
  a.nel = a.d[0].n * a.d[1].n * a.d[2].n;
  return a;
}

size_t geo_matvec_ws_bytes(const Plan& P, int nrhs) {
  size_t nel = 1, nloc = 1;
  for (int k = 0; k < 3; ++k) {
    nel *= (size_t)P.geo.dir[k].n;
    nloc *= (size_t)P.geo.dir[k].P;
  }
  return 8 * nel * nloc * (size_t)nrhs;
}

int geo_matvec_blocks(const Plan& P) { return pcg_blocks(P); }

hipError_t launch_geo_matvec(const Plan& P, const double* x, double* y, int nrhs, void* ws,
                             double* part, int npart, const double* act, int as, hipStream_t s,
                             const double* fres) {
  if (!ws) return hipErrorInvalidValue;
  const GeoArgs a = geo_args(P);
  if (a.nloc > GEO_CUBE) return hipErrorInvalidValue;
  const int nb = geo_matvec_blocks(P);
  if (part && npart < nb) return hipErrorInvalidValue;
  double* loc = (double*)ws;
  hipLaunchKernelGGL(geo_element, dim3((unsigned)a.nel, (unsigned)nrhs), dim3(GEO_T), 0, s, x,
                     loc, a, act, as);
  hipLaunchKernelGGL(geo_gather, dim3((unsigned)(nb * nrhs)), dim3(GEO_T), 0, s,
                     (const double*)loc, y, a, nb, x, fres, part, npart, act, as);
  return hipGetLastError();
}

}  // namespace iffd
