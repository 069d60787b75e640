// Matrix-free Galerkin operator y = Ahat x on gfx950 (FP64).
//
// Ahat = sum_k M (x) .. (x) K (slot k) (x) .. (x) M (eq:system_matrix and its
// 3-term analogue) with the banded 1-D matrices K, M (half-bandwidth p,
// Section 3).  Sum factorization in two passes (3D):
//   pass 1, along direction 3:   t = M3 x,  s = K3 x
//   pass 2, per plane i3:        u = M2 t,  v = K2 t + M2 s   (direction 2)
//                                y = K1 u + M1 v              (direction 1)
// which is M3 M2 K1 x + M3 K2 M1 x + K3 M2 M1 x, i.e. 7 banded 1-D products
// per point, the minimum for the Kronecker sum.  In 2D pass 2 runs on x with
// s = 0 (y = K1 M2 x + M1 K2 x).
//
// Pass 1: one thread per (i1, i2) column and chunk of C3 planes; the thread
// loads its window of C3 + 2p values at once, so every load is in flight
// together, and writes C3 values of t and s.  Pass 2: one workgroup per
// TY x TX tile of a plane; the tile of t and s with a p-wide halo goes
// through LDS, the direction-2 products are formed for the tile rows over the
// halo columns, then the direction-1 products for the tile.  Pass 2 also
// forms the per-workgroup partial of x . y that PCG needs for p . Ap.
// The 1-D matrices are Toeplitz away from the ends, so they are held
// compactly: the 2p-1 special rows at each end plus one interior row.
#include "launch.h"

namespace iffd {

__device__ __forceinline__ int crow(int i, int m, int nbr, int crows) {
  if (crows == m) return i;
  if (i < nbr) return i;
  if (i >= m - nbr) return i - (m - nbr) + nbr + 1;
  return nbr;
}

constexpr int MV1_THREADS = 256;
constexpr int MV1_C3 = 16;  // planes per thread in pass 1

template <int P>
__global__ void __launch_bounds__(MV1_THREADS)
mv_axis3(const double* __restrict__ x, double* __restrict__ t3, double* __restrict__ s3, int m,
         int N, int nch, const double* __restrict__ kc, const double* __restrict__ mc, int nbr,
         int crows, const double* __restrict__ active, int astride) {
  constexpr int BW = 2 * P + 1;
  constexpr int WIN = MV1_C3 + 2 * P;
  const int plane = m * m;
  const int cols_blocks = (plane + MV1_THREADS - 1) / MV1_THREADS;
  int bid = blockIdx.x;
  const int per_rhs = cols_blocks * nch;
  const int rhs = bid / per_rhs;
  bid -= rhs * per_rhs;
  const int ch = bid / cols_blocks;
  const int col = (bid - ch * cols_blocks) * MV1_THREADS + threadIdx.x;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  if (col >= plane) return;
  const int c0 = ch * MV1_C3;
  const double* xr = x + (size_t)rhs * N + col;
  double w[WIN];
#pragma unroll
  for (int k = 0; k < WIN; ++k) {
    const int c = c0 - P + k;
    w[k] = (c >= 0 && c < m) ? xr[(size_t)c * plane] : 0.0;
  }
  double* tr = t3 + (size_t)rhs * N + col;
  double* sr = s3 + (size_t)rhs * N + col;
#pragma unroll
  for (int k = 0; k < MV1_C3; ++k) {
    const int i3 = c0 + k;
    if (i3 < m) {
      const int cr = crow(i3, m, nbr, crows);
      const double* krow = kc + cr * BW;
      const double* mrow = mc + cr * BW;
      double tv = 0.0, sv = 0.0;
#pragma unroll
      for (int o = 0; o < BW; ++o) {
        tv += mrow[o] * w[k + o];
        sv += krow[o] * w[k + o];
      }
      tr[(size_t)i3 * plane] = tv;
      sr[(size_t)i3 * plane] = sv;
    }
  }
}

constexpr int MV2_THREADS = 256;
constexpr int MV2_TX = 64;  // tile columns (direction 1)
template <int P>
constexpr int mv2_ty() { return P <= 4 ? 16 : 8; }  // tile rows (direction 2)

template <int P, bool HAS_S>
__global__ void __launch_bounds__(MV2_THREADS)
mv_plane(const double* __restrict__ xin, const double* __restrict__ t3,
         const double* __restrict__ s3, double* __restrict__ y, int m, int N, int ntx, int nty,
         const double* __restrict__ kc, const double* __restrict__ mc, int nbr, int crows,
         double* __restrict__ part, int npart, const double* __restrict__ active, int astride) {
  constexpr int BW = 2 * P + 1;
  constexpr int MV2_TY = mv2_ty<P>();
  constexpr int XW = MV2_TX + 2 * P;   // tile width with the column halo
  constexpr int RH = MV2_TY + 2 * P;   // tile height with the row halo
  __shared__ double ts[RH * XW];
  __shared__ double ss[HAS_S ? RH * XW : 1];
  __shared__ double us[MV2_TY * XW];
  __shared__ double vs[MV2_TY * XW];
  __shared__ double kcs[(4 * P - 1) * BW];
  __shared__ double mcs[(4 * P - 1) * BW];
  __shared__ double red[MV2_THREADS / 64];

  const int t = threadIdx.x;
  const int tiles = ntx * nty;
  const int planes = N / (m * m);
  int bid = blockIdx.x;
  const int per_rhs = tiles * planes;
  const int rhs = bid / per_rhs;
  bid -= rhs * per_rhs;
  const int pl = bid / tiles;
  const int tl = bid - pl * tiles;
  const int by = tl / ntx, bx = tl - by * ntx;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const size_t base = (size_t)rhs * N + (size_t)pl * m * m;
  const int r0 = by * MV2_TY, q0 = bx * MV2_TX;

  for (int e = t; e < crows * BW; e += MV2_THREADS) {
    kcs[e] = kc[e];
    mcs[e] = mc[e];
  }
  // tile of t (and s) with halo, zero outside the domain
  for (int e0 = t; e0 < RH * XW; e0 += MV2_THREADS * 4) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * MV2_THREADS;
      const int r = e / XW, c = e - (e / XW) * XW;
      const int i2 = r0 + r - P, i1 = q0 + c - P;
      const bool in = e < RH * XW && i2 >= 0 && i2 < m && i1 >= 0 && i1 < m;
      const size_t gi = base + (size_t)i2 * m + i1;
      a[u] = in ? t3[gi] : 0.0;
      b[u] = (HAS_S && in) ? s3[gi] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * MV2_THREADS;
      if (e < RH * XW) {
        ts[e] = a[u];
        if (HAS_S) ss[e] = b[u];
      }
    }
  }
  __syncthreads();
  // direction 2 on the tile rows, over the halo columns: u = M2 t, v = K2 t + M2 s
  for (int e = t; e < MV2_TY * XW; e += MV2_THREADS) {
    const int r = e / XW, c = e - (e / XW) * XW;
    const int i2 = r0 + r;
    double uv = 0.0, vv = 0.0;
    if (i2 < m) {
      const int cr = crow(i2, m, nbr, crows);
      const double* krow = kcs + cr * BW;
      const double* mrow = mcs + cr * BW;
#pragma unroll
      for (int o = 0; o < BW; ++o) {
        const double tv = ts[(r + o) * XW + c];
        uv += mrow[o] * tv;
        vv += krow[o] * tv;
        if (HAS_S) vv += mrow[o] * ss[(r + o) * XW + c];
      }
    }
    us[e] = uv;
    vs[e] = vv;
  }
  __syncthreads();
  // direction 1: y = K1 u + M1 v
  double dot = 0.0;
  for (int e = t; e < MV2_TY * MV2_TX; e += MV2_THREADS) {
    const int r = e / MV2_TX, c = e - (e / MV2_TX) * MV2_TX;
    const int i2 = r0 + r, i1 = q0 + c;
    if (i2 >= m || i1 >= m) continue;
    const int cr = crow(i1, m, nbr, crows);
    const double* krow = kcs + cr * BW;
    const double* mrow = mcs + cr * BW;
    double yv = 0.0;
#pragma unroll
    for (int o = 0; o < BW; ++o) yv += krow[o] * us[r * XW + c + o] + mrow[o] * vs[r * XW + c + o];
    const size_t gi = base + (size_t)i2 * m + i1;
    y[gi] = yv;
    if (part) dot += xin[gi] * yv;
  }
  if (part) {
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
    if ((t & 63) == 0) red[t >> 6] = dot;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int w = 0; w < MV2_THREADS / 64; ++w) s += red[w];
      part[(size_t)rhs * npart + (blockIdx.x - rhs * per_rhs)] = s;
    }
  }
}

// workgroups of the operator per right-hand side (pass 2 produces the partials)
int matvec_blocks(const Plan& P_) {
  const int m = P_.m;
  const int ty = P_.p <= 4 ? 16 : 8;
  const int ntx = (m + MV2_TX - 1) / MV2_TX, nty = (m + ty - 1) / ty;
  return ntx * nty * (P_.d == 3 ? m : 1);
}

size_t matvec_ws_bytes(const Plan& P_, int nrhs) {
  return P_.d == 3 ? (size_t)2 * 8 * P_.N * nrhs : 0;
}

template <int P>
static hipError_t mv_launch(const Plan& P_, const double* x, double* y, int nrhs, void* ws,
                            double* part, int npart, const double* a, int as, hipStream_t s) {
  const int m = P_.m, N = (int)P_.N;
  const char* b = P_.d_tables;
  const double* kc = (const double*)(b + P_.lay.kc64);
  const double* mc = (const double*)(b + P_.lay.mc64);
  const int nbr = 2 * P - 1, crows = P_.crows;
  const int ntx = (m + MV2_TX - 1) / MV2_TX, nty = (m + mv2_ty<P>() - 1) / mv2_ty<P>();
  const int per_rhs = matvec_blocks(P_);
  if (part && per_rhs > npart) return hipErrorInvalidValue;
  if (P_.d == 3) {
    if (!ws) return hipErrorInvalidValue;
    double* t3 = (double*)ws;
    double* s3 = t3 + (size_t)N * nrhs;
    const int nch = (m + MV1_C3 - 1) / MV1_C3;
    const int cb = (m * m + MV1_THREADS - 1) / MV1_THREADS;
    hipLaunchKernelGGL(mv_axis3<P>, dim3(cb * nch * nrhs), dim3(MV1_THREADS), 0, s, x, t3, s3, m,
                       N, nch, kc, mc, nbr, crows, a, as);
    hipLaunchKernelGGL((mv_plane<P, true>), dim3(per_rhs * nrhs), dim3(MV2_THREADS), 0, s, x, t3,
                       s3, y, m, N, ntx, nty, kc, mc, nbr, crows, part, npart, a, as);
  } else {
    hipLaunchKernelGGL((mv_plane<P, false>), dim3(per_rhs * nrhs), dim3(MV2_THREADS), 0, s, x, x,
                       (const double*)nullptr, y, m, N, ntx, nty, kc, mc, nbr, crows, part, npart,
                       a, as);
  }
  return hipGetLastError();
}

hipError_t launch_matvec(const Plan& P_, const double* x, double* y, int nrhs, void* ws,
                         double* part, int npart, const double* a, int as, hipStream_t s) {
  switch (P_.p) {
    case 1: return mv_launch<1>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    case 2: return mv_launch<2>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    case 3: return mv_launch<3>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    case 4: return mv_launch<4>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    case 5: return mv_launch<5>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    case 6: return mv_launch<6>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    case 7: return mv_launch<7>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    case 8: return mv_launch<8>(P_, x, y, nrhs, ws, part, npart, a, as, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace iffd
