// General plans (per direction n, p and Dirichlet / Neumann ends): the
// sequence of line passes that forms z = P^{-1} r, the matrix-free operator
// and the device part of the setup.
#include "gen_impl.h"

namespace iffd {

// each length's passes are compiled in their own translation unit (gen_l*.hip)
extern template IFFD_GEN_PASS_LEN(16);
extern template IFFD_GEN_PASS_LEN(24);
extern template IFFD_GEN_PASS_LEN(32);
extern template IFFD_GEN_PASS_LEN(48);
extern template IFFD_GEN_PASS_LEN(64);
extern template IFFD_GEN_PASS_LEN(96);
extern template IFFD_GEN_PASS_LEN(128);
extern template IFFD_GEN_PASS_LEN(192);
extern template IFFD_GEN_PASS_LEN(256);
extern template IFFD_GEN_PASS_LEN(384);
extern template IFFD_GEN_PASS_LEN(512);

static hipError_t gen_line(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                           void* out, int nrhs, const double* a, int as, hipStream_t s) {
  switch (P.dirs[axis - 1].L) {
    case 16: return gen_pass_len<16>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 24: return gen_pass_len<24>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 32: return gen_pass_len<32>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 48: return gen_pass_len<48>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 64: return gen_pass_len<64>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 96: return gen_pass_len<96>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 128: return gen_pass_len<128>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 192: return gen_pass_len<192>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 256: return gen_pass_len<256>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 384: return gen_pass_len<384>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 512: return gen_pass_len<512>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    default: return hipErrorInvalidValue;
  }
}

// pass k of the apply: forward along directions 1 .. d-1, the middle pass
// along d, backward along d-1 .. 1.  The FP64 apply works in place on z, the
// FP32 apply on the FP32 workspace; pass 0 reads r, the last pass writes z.
hipError_t launch_gen_pass(const Plan& P, int pass, const double* r, double* z, int nrhs, void* ws,
                           const double* a, int as, hipStream_t s) {
  const int d = P.d;
  const bool f64 = P.prec == IFFD_PREC_F64;
  const int et = f64 ? ELEM_F64 : ELEM_F32;
  void* w = f64 ? (void*)z : ws;
  if (pass < d - 1) {
    const bool p0 = pass == 0;
    return gen_line(P, PASS_FWD, pass + 1, p0 ? ELEM_F64 : et, p0 ? (const void*)r : w, et, w,
                    nrhs, a, as, s);
  }
  if (pass == d - 1) return gen_line(P, PASS_MID, d, et, w, et, w, nrhs, a, as, s);
  if (pass < 2 * d - 1) {
    const int axis = 2 * d - 1 - pass;
    return gen_line(P, PASS_BWD, axis, et, w, axis == 1 ? ELEM_F64 : et,
                    axis == 1 ? (void*)z : w, nrhs, a, as, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gen_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                            const double* a, int as, hipStream_t s) {
  for (int k = 0; k < 2 * P.d - 1; ++k) {
    hipError_t e = launch_gen_pass(P, k, r, z, nrhs, ws, a, as, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---- the operator y = Ahat x with per-direction banded K_k, M_k -------------
// Sum factorization, one banded product per direction and pass:
//   2D:  a = M1 x, b = K1 x;           y = K2 a + M2 b
//   3D:  a = M1 x, b = K1 x;  c = M2 a, e = K2 a + M2 b;  y = K3 c + M3 e
// i.e. sum_k (x) of K in slot k and M elsewhere (eq:system_matrix and its
// 3-term analogue).  One thread per output entry; the last pass also forms
// per-workgroup partial sums of x . y (or (f - y)^2 for a true residual) in
// a fixed order.

constexpr int GMV_T = 256;

__device__ __forceinline__ double gmv_sum(const double* __restrict__ B, const double* __restrict__ u,
                                          int i, int p, int m, size_t base, int S) {
  const int bw = 2 * p + 1;
  const int j0 = i - p < 0 ? 0 : i - p, j1 = i + p > m - 1 ? m - 1 : i + p;
  const double* row = B + (size_t)i * bw + (p - i);
  double acc = 0.0;
  for (int j = j0; j <= j1; ++j) acc += row[j] * u[base + (size_t)j * S];
  return acc;
}

__global__ void __launch_bounds__(GMV_T)
gmv_pass(const double* __restrict__ u, const double* __restrict__ v, double* __restrict__ o1,
         double* __restrict__ o2, const double* __restrict__ A, const double* __restrict__ B,
         const double* __restrict__ Cm, const double* __restrict__ Dm, int p, int m, int S, int N,
         int nblk, const double* __restrict__ xd, const double* __restrict__ fres,
         double* __restrict__ part, int npart, const double* __restrict__ active, int astride) {
  __shared__ double red[GMV_T / 64];
  const int rhs = blockIdx.x / nblk, blk = blockIdx.x - rhs * nblk;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const int c = (N + nblk - 1) / nblk;
  const int lo = min(N, blk * c), hi = min(N, lo + c);
  const size_t ro = (size_t)rhs * N;
  double dot = 0.0;
  for (int e = lo + (int)threadIdx.x; e < hi; e += GMV_T) {
    const int i = (e / S) % m;
    const size_t base = ro + (size_t)(e - i * S);
    double y1 = gmv_sum(A, u, i, p, m, base, S);
    if (v && B) y1 += gmv_sum(B, v, i, p, m, base, S);
    o1[ro + e] = y1;
    if (o2) {
      double y2 = gmv_sum(Cm, u, i, p, m, base, S);
      if (v && Dm) y2 += gmv_sum(Dm, v, i, p, m, base, S);
      o2[ro + e] = y2;
    }
    if (part) {
      if (fres) {
        const double rr = fres[ro + e] - y1;
        dot += rr * rr;
      } else {
        dot += xd[ro + e] * y1;
      }
    }
  }
  if (!part) return;
  for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dot;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < GMV_T / 64; ++w) s += red[w];
    part[(size_t)rhs * npart + blk] = s;
  }
}

int gen_matvec_blocks(const Plan& P) {
  const int64_t b = (P.N + 4 * GMV_T - 1) / (4 * GMV_T);
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 2048);
}

size_t gen_matvec_ws_bytes(const Plan& P, int nrhs) {
  return (size_t)(P.d == 3 ? 4 : 2) * 8 * P.N * nrhs;
}

hipError_t launch_gen_matvec(const Plan& P, const double* x, double* y, int nrhs, void* ws,
                             double* part, int npart, const double* act, int as, hipStream_t s,
                             const double* fres) {
  const int N = (int)P.N, nb = gen_matvec_blocks(P);
  if (part && npart < nb) return hipErrorInvalidValue;
  if (!ws) return hipErrorInvalidValue;
  double* wa = (double*)ws;
  double* wb = wa + (size_t)N * nrhs;
  auto band = [&](int k, bool stiff) {
    const GDir& G = P.dirs[k];
    return (const double*)(P.d_tables + G.blob64) + (stiff ? G.o_kb : G.o_mb);
  };
  const dim3 grid((unsigned)(nb * nrhs)), block(GMV_T);
  const GDir& g1 = P.dirs[0];
  const GDir& g2 = P.dirs[1];
  // direction 1: a = M1 x, b = K1 x
  hipLaunchKernelGGL(gmv_pass, grid, block, 0, s, x, (const double*)nullptr, wa, wb, band(0, false),
                     (const double*)nullptr, band(0, true), (const double*)nullptr, g1.p, g1.m, 1,
                     N, nb, (const double*)nullptr, (const double*)nullptr, (double*)nullptr, 0,
                     act, as);
  if (P.d == 2) {
    hipLaunchKernelGGL(gmv_pass, grid, block, 0, s, (const double*)wa, (const double*)wb, y,
                       (double*)nullptr, band(1, true), band(1, false), (const double*)nullptr,
                       (const double*)nullptr, g2.p, g2.m, g1.m, N, nb, x, fres, part, npart, act,
                       as);
    return hipGetLastError();
  }
  double* wc = wb + (size_t)N * nrhs;
  double* we = wc + (size_t)N * nrhs;
  const GDir& g3 = P.dirs[2];
  // direction 2: c = M2 a, e = K2 a + M2 b
  hipLaunchKernelGGL(gmv_pass, grid, block, 0, s, (const double*)wa, (const double*)wb, wc, we,
                     band(1, false), (const double*)nullptr, band(1, true), band(1, false), g2.p,
                     g2.m, g1.m, N, nb, (const double*)nullptr, (const double*)nullptr,
                     (double*)nullptr, 0, act, as);
  // direction 3: y = K3 c + M3 e
  hipLaunchKernelGGL(gmv_pass, grid, block, 0, s, (const double*)wc, (const double*)we, y,
                     (double*)nullptr, band(2, true), band(2, false), (const double*)nullptr,
                     (const double*)nullptr, g3.p, g3.m, g1.m * g2.m, N, nb, x, fres, part, npart,
                     act, as);
  return hipGetLastError();
}

}  // namespace iffd
