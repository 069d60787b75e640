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
// together, and writes C3 values of t and s.  Pass 2 (below) forms both
// in-plane directions and the per-workgroup partial of x . y that PCG needs
// for p . Ap.
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
  int bid = xcd_linear(blockIdx.x, gridDim.x);   // chunks of a column meet in one L2
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

// Pass 2: one wave per (plane, strip of 64 - 2p columns, chunk of 8 rows).
// Lane c owns column i1 = strip start - p + c and walks down its rows with a
// register window of C2 + 2p values of t (and s): direction 2 is formed in
// registers (the band row is the same for every lane), direction 1 moves the
// neighbouring columns' terms across the lanes by DPP shifts, so the pass
// needs no LDS tile and no barrier.  The outer p lanes on each side only feed
// their neighbours.  Each workgroup of four waves writes one partial of x . y.
constexpr int MV2_THREADS = 256;

// whole-wave lane shifts of a double by one lane (DPP wave_shr:1 / wave_shl:1;
// the lane that has no source receives 0)
__device__ __forceinline__ double wave_from_lower(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, 0x138, 0xF, 0xF, true),
                          __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double wave_from_upper(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, 0x130, 0xF, 0xF, true),
                          __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xF, 0xF, true));
}

template <int P>
constexpr int mv2_rows() { return 8; }

__host__ __device__ inline void mv2_geom(int m, int planes, int P, int& ncs, int& nch, int& bpr) {
  const int out = 64 - 2 * P;
  const int c2 = 8;
  ncs = (m + out - 1) / out;
  nch = (m + c2 - 1) / c2;
  const long long items = (long long)planes * ncs * nch;
  bpr = (int)((items + MV2_THREADS / 64 - 1) / (MV2_THREADS / 64));
}

template <int P, bool HAS_S>
__global__ void __launch_bounds__(MV2_THREADS)
mv_rows(const double* __restrict__ xin, const double* __restrict__ t3,
        const double* __restrict__ s3, double* __restrict__ y, int m, int N, int ncs, int nch,
        int bpr, const double* __restrict__ kc, const double* __restrict__ mc, int nbr, int crows,
        double* __restrict__ part, int npart, const double* __restrict__ active, int astride,
        const double* __restrict__ fres) {
  constexpr int BW = 2 * P + 1;
  constexpr int C2 = mv2_rows<P>();
  constexpr int WIN = C2 + 2 * P;
  constexpr int OUT = 64 - 2 * P;
  __shared__ double red[MV2_THREADS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lin = xcd_linear(blockIdx.x, gridDim.x);   // halo rows meet in one L2
  const int rhs = lin / bpr;
  const int blk = lin - rhs * bpr;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const int plane = m * m;
  const int planes = N / plane;
  const int ipp = ncs * nch;
  const int item = blk * (MV2_THREADS / 64) + w;
  double dot = 0.0;
  if (item < planes * ipp) {
    // row chunks vary fastest, so the waves of a workgroup take consecutive
    // chunks of one strip and share their p-row halos through the cache
    const int pl = item / ipp;
    const int rem = item - pl * ipp;
    const int cs = rem / nch;
    const int ch = rem - cs * nch;
    const int i1 = cs * OUT - P + lane;
    const bool col = i1 >= 0 && i1 < m;
    const int r0 = ch * C2;
    const size_t base = (size_t)rhs * N + (size_t)pl * plane;
    double wt[WIN], wsv[WIN];
#pragma unroll
    for (int k = 0; k < WIN; ++k) {
      const int i2 = r0 - P + k;
      const bool in = col && i2 >= 0 && i2 < m;
      const size_t gi = base + (size_t)(in ? i2 : 0) * m + (in ? i1 : 0);
      wt[k] = in ? t3[gi] : 0.0;
      wsv[k] = (HAS_S && in) ? s3[gi] : 0.0;
    }
    // x (or f for the residual) at the output points, for the partial sums
    // (loaded with the window so that no load waits inside the row loop)
    const bool out = lane >= P && lane < 64 - P && col;
    const double* xsrc = fres ? fres : xin;
    double xv[C2];
#pragma unroll
    for (int r = 0; r < C2; ++r) {
      const bool in = part && out && r0 + r < m;
      xv[r] = in ? xsrc[base + (size_t)(r0 + r) * m + i1] : 0.0;
    }
    // row by row: direction 2 from the register window, direction 1 from the
    // neighbouring lanes through DPP whole-wave shifts (VALU moves, no LDS)
    // direction-1 coefficients: the centre of this column's band row, and
    // what columns i1 + d (kl, ml) and i1 - d (kh, mh) apply to column i1
    const int cr1 = crow(col ? i1 : 0, m, nbr, crows);
    const double k1c = kc[cr1 * BW + P], m1c = mc[cr1 * BW + P];
    double kl[P + 1], ml[P + 1], kh[P + 1], mh[P + 1];
#pragma unroll
    for (int d = 1; d <= P; ++d) {
      const int jl = i1 + d, jh = i1 - d;
      const int crl = crow(jl >= 0 && jl < m ? jl : 0, m, nbr, crows);
      const int crh = crow(jh >= 0 && jh < m ? jh : 0, m, nbr, crows);
      kl[d] = kc[crl * BW + P - d];
      ml[d] = mc[crl * BW + P - d];
      kh[d] = kc[crh * BW + P + d];
      mh[d] = mc[crh * BW + P + d];
    }
#pragma unroll
    for (int r = 0; r < C2; ++r) {
      // the band row is the same for the whole wave: scalar loads
      const int cr2 = __builtin_amdgcn_readfirstlane(crow(min(r0 + r, m - 1), m, nbr, crows));
      const double* k2 = kc + cr2 * BW;
      const double* m2 = mc + cr2 * BW;
      double u = 0.0, v = 0.0;
#pragma unroll
      for (int o = 0; o < BW; ++o) {
        u += m2[o] * wt[r + o];
        v += k2[o] * wt[r + o];
        if (HAS_S) v += m2[o] * wsv[r + o];
      }
      // column i1 takes the terms of columns i1 -+ d, formed on their lanes
      // with column i1's coefficients and accumulated along single-lane
      // shifts (Horner's scheme): P shifts per direction
      double lo = kl[P] * u + ml[P] * v;
      double hi = kh[P] * u + mh[P] * v;
#pragma unroll
      for (int d = P - 1; d >= 1; --d) {
        lo = wave_from_lower(lo);
        hi = wave_from_upper(hi);
        lo = fma(kl[d], u, fma(ml[d], v, lo));
        hi = fma(kh[d], u, fma(mh[d], v, hi));
      }
      lo = wave_from_lower(lo);
      hi = wave_from_upper(hi);
      const double yv = fma(k1c, u, fma(m1c, v, lo + hi));
      if (out && r0 + r < m) {
        y[base + (size_t)(r0 + r) * m + i1] = yv;
        const double dv = xv[r] - yv;
        dot += fres ? dv * dv : xv[r] * yv;
      }
    }
  }
  if (part) {
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
    if (lane == 0) red[w] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < MV2_THREADS / 64; ++k) s += red[k];
      part[(size_t)rhs * npart + blk] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// 3D, p <= 4: one fused pass.  A workgroup of 8 waves owns a tile of 32
// columns (direction 1) x 16 rows (direction 2) x MVF_C3 planes (direction 3);
// each wave holds two rows, one per half-wave, a lane per column.  The outer
// p columns and rows of the tile only feed their neighbours.  Every thread
// loads its column of x over the tile's planes plus a p-plane halo at once
// (all loads in flight), forms t = M3 x and s = K3 x for one plane at a time
// in registers and passes them through LDS (double-buffered by plane parity,
// one barrier per plane); the waves holding output rows form u = M2 t and
// v = K2 t + M2 s down the rows and y = K1 u + M1 v across the lanes with DPP
// whole-wave shifts (a shift never crosses from one half into the other's
// output lanes).  x is read once per tile plus halos (largely from L2) and y
// written once, against 48 bytes per point for the two passes above.  Small
// workgroups let several share a compute unit, so one's barrier waits are
// covered by another's work.  The partial x . y of a workgroup uses the x
// value at the window centre.
constexpr int MVF_C3 = 8;
constexpr int MVF_RT = 16;   // tile rows
constexpr int MVF_CW = 32;   // tile columns (half a wave)
constexpr int MVF_THREADS = MVF_RT * MVF_CW;

__host__ __device__ inline void mvf_geom(int m, int P, int& ncs, int& nrb, int& n3c) {
  ncs = (m + (MVF_CW - 2 * P) - 1) / (MVF_CW - 2 * P);
  nrb = (m + (MVF_RT - 2 * P) - 1) / (MVF_RT - 2 * P);
  n3c = (m + MVF_C3 - 1) / MVF_C3;
}

static bool mv_fused(const Plan& P_) { return P_.d == 3 && P_.p <= 4; }

template <int P>
__global__ void __launch_bounds__(MVF_THREADS)
mv_fused3(const double* __restrict__ x, double* __restrict__ y, int m, int N, int ncs, int nrb,
          int n3c, const double* __restrict__ kc, const double* __restrict__ mc, int nbr,
          int crows, double* __restrict__ part, int npart, const double* __restrict__ active,
          int astride, const double* __restrict__ fres) {
  constexpr int BW = 2 * P + 1;
  constexpr int WIN = MVF_C3 + 2 * P;
  constexpr int OUT = MVF_CW - 2 * P, R2 = MVF_RT - 2 * P;
  __shared__ double ts[2][2][MVF_RT][MVF_CW];   // [plane parity][t, s][row][column]
  __shared__ double b1[2][BW][MVF_CW];           // direction-1 band rows of the columns
  __shared__ double b2[2][MVF_RT][BW];           // direction-2 band rows of the rows
  __shared__ double red[MVF_THREADS / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int cl = lane & (MVF_CW - 1);
  const int ty = 2 * wv + (lane >> 5);
  const int bpr = ncs * nrb * n3c;
  const int lin = xcd_linear(blockIdx.x, gridDim.x);   // neighbouring tiles share halos in one L2
  const int rhs = lin / bpr;
  const int blk = lin - rhs * bpr;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  // plane chunks vary fastest, then row blocks, then column strips
  const int ch = blk % n3c;
  const int rb = (blk / n3c) % nrb;
  const int cs = blk / (n3c * nrb);
  const int i1 = cs * OUT - P + cl;
  const int i2 = rb * R2 - P + ty;
  const int c0 = ch * MVF_C3;
  const bool colrow = i1 >= 0 && i1 < m && i2 >= 0 && i2 < m;
  const int plane = m * m;
  // x column window, planes c0 - P .. c0 + C3 + P - 1 (0 outside the tensor)
  const auto rs = buf_rsrc(x + (size_t)rhs * N, (unsigned)N * 8u);
  const unsigned vo = colrow ? (unsigned)(i2 * m + i1) * 8u : BUF_OOB;
  double w[WIN];
#pragma unroll
  for (int k = 0; k < WIN; ++k) {
    const int c = c0 - P + k;
    w[k] = (c >= 0 && c < m) ? buf_ld<double>(rs, vo + (unsigned)(c * plane) * 8u) : 0.0;
  }
  // band rows of the tile's columns and rows (read after the first barrier)
  for (int e = threadIdx.x; e < BW * MVF_CW; e += MVF_THREADS) {
    const int o = e / MVF_CW, c = e - o * MVF_CW;
    const int j1 = cs * OUT - P + c;
    const int cr = crow(j1 >= 0 && j1 < m ? j1 : 0, m, nbr, crows);
    b1[0][o][c] = kc[cr * BW + o];
    b1[1][o][c] = mc[cr * BW + o];
  }
  for (int e = threadIdx.x; e < BW * MVF_RT; e += MVF_THREADS) {
    const int r = e / BW, o = e - r * BW;
    const int j2 = rb * R2 - P + r;
    const int cr = crow(j2 >= 0 && j2 < m ? j2 : 0, m, nbr, crows);
    b2[0][r][o] = kc[cr * BW + o];
    b2[1][r][o] = mc[cr * BW + o];
  }
  // waves with an output row in either half do the in-plane work
  const bool owave = 2 * wv + 1 >= P && 2 * wv < P + R2;
  const bool out = ty >= P && ty < P + R2 && i2 < m && cl >= P && cl < MVF_CW - P && i1 < m;
  const int ta = ty >= P && ty < P + R2 ? ty : P;   // rows the halo half-wave reads (discarded)
  const auto ws = buf_rsrc(y + (size_t)rhs * N, (unsigned)N * 8u);
  const auto fr = buf_rsrc(fres ? fres + (size_t)rhs * N : y, fres ? (unsigned)N * 8u : 0u);
  // a tile whose columns and rows all take the interior (Toeplitz) band row
  // reads its coefficients from scalar registers instead of LDS
  const bool inter = crows < m && cs * OUT - P >= nbr && cs * OUT - P + MVF_CW <= m - nbr &&
                     rb * R2 - P >= nbr && rb * R2 - P + MVF_RT <= m - nbr;
  double dot = 0.0;
  auto run = [&](auto tag) {
    constexpr bool INTER = decltype(tag)::value;
    const double* ki = kc + nbr * BW;   // the interior row
    const double* mi = mc + nbr * BW;
    auto K1 = [&](int o) { return INTER ? ki[o] : b1[0][o][cl]; };
    auto M1 = [&](int o) { return INTER ? mi[o] : b1[1][o][cl]; };
    // coefficient that column cl + d (L) or cl - d (H) applies to this
    // column's u and v; a column outside the half-wave is no output column
    auto K1L = [&](int d) { return INTER ? ki[P - d] : b1[0][P - d][(cl + d) & (MVF_CW - 1)]; };
    auto M1L = [&](int d) { return INTER ? mi[P - d] : b1[1][P - d][(cl + d) & (MVF_CW - 1)]; };
    auto K1H = [&](int d) { return INTER ? ki[P + d] : b1[0][P + d][(cl - d) & (MVF_CW - 1)]; };
    auto M1H = [&](int d) { return INTER ? mi[P + d] : b1[1][P + d][(cl - d) & (MVF_CW - 1)]; };
    auto K2 = [&](int o) { return INTER ? ki[o] : b2[0][ta][o]; };
    auto M2 = [&](int o) { return INTER ? mi[o] : b2[1][ta][o]; };
#pragma unroll
    for (int k = 0; k < MVF_C3; ++k) {
      const int i3 = c0 + k;
      if (i3 >= m) break;   // uniform
      const int cr3 = __builtin_amdgcn_readfirstlane(crow(i3, m, nbr, crows));
      const double* k3 = kc + cr3 * BW;
      const double* m3 = mc + cr3 * BW;
      double t = 0.0, sv = 0.0;
#pragma unroll
      for (int o = 0; o < BW; ++o) {
        t += m3[o] * w[k + o];
        sv += k3[o] * w[k + o];
      }
      ts[k & 1][0][ty][cl] = t;
      ts[k & 1][1][ty][cl] = sv;
      __syncthreads();
      if (owave) {
        double u = 0.0, v = 0.0;
#pragma unroll
        for (int o = 0; o < BW; ++o) {
          const double tt = ts[k & 1][0][ta - P + o][cl];
          const double ss = ts[k & 1][1][ta - P + o][cl];
          u += M2(o) * tt;
          v += K2(o) * tt + M2(o) * ss;
        }
        // direction 1: column j takes K1[j][j-d] u + M1[j][j-d] v of column
        // j - d and the same of column j + d (d = 1..P).  The lane of column
        // j - d forms that term with column j's coefficients and the terms
        // ride one lane per step towards their column, each step adding the
        // next nearer one (Horner's scheme): P shifts per direction in all.
        double lo = K1L(P) * u + M1L(P) * v;
        double hi = K1H(P) * u + M1H(P) * v;
#pragma unroll
        for (int d = P - 1; d >= 1; --d) {
          lo = wave_from_lower(lo);
          hi = wave_from_upper(hi);
          lo = fma(K1L(d), u, fma(M1L(d), v, lo));
          hi = fma(K1H(d), u, fma(M1H(d), v, hi));
        }
        lo = wave_from_lower(lo);   // sum over d of the terms of columns j - d
        hi = wave_from_upper(hi);   // and of columns j + d
        const double yv = fma(K1(P), u, fma(M1(P), v, lo + hi));
        if (out) {
          const unsigned oo = (unsigned)(i3 * plane + i2 * m + i1) * 8u;
          buf_st<double>(yv, ws, oo);
          if (fres) {   // uniform
            const double dv = buf_ld<double>(fr, oo) - yv;
            dot += dv * dv;
          } else {
            dot += w[k + P] * yv;
          }
        }
      }
    }
  };
  if (inter) run(std::integral_constant<bool, true>{});
  else run(std::integral_constant<bool, false>{});
  if (part) {
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
    if (lane == 0) red[wv] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s2 = 0.0;
      for (int k = 0; k < MVF_THREADS / 64; ++k) s2 += red[k];
      part[(size_t)rhs * npart + blk] = s2;
    }
  }
}

// workgroups of the operator per right-hand side (the pass that produces the
// partials)
// Uniform plans keep the kernels above: measured at n = 256 against the
// one-pass rolling kernel of mvroll.hip (which serves general plans), the
// fused tile ties it for p <= 4 (182 vs 185 us at p = 3) and the two passes
// beat it for p >= 6 (283 vs 488 us at p = 6, 379 vs 1602 us at p = 8, where
// its register windows spill).
int matvec_blocks(const Plan& P_) {
  if (P_.geo.kind) return geo_matvec_blocks(P_);
  if (P_.gen) return gen_matvec_blocks(P_);
  if (mv_fused(P_)) {
    int ncs, nrb, n3c;
    mvf_geom(P_.m, P_.p, ncs, nrb, n3c);
    return ncs * nrb * n3c;
  }
  int ncs, nch, bpr;
  mv2_geom(P_.m, P_.d == 3 ? P_.m : 1, P_.p, ncs, nch, bpr);
  return bpr;
}

size_t matvec_ws_bytes(const Plan& P_, int nrhs) {
  if (P_.geo.kind) return geo_matvec_ws_bytes(P_, nrhs);
  if (P_.gen) return gen_matvec_ws_bytes(P_, nrhs);
  return (P_.d == 3 && !mv_fused(P_)) ? (size_t)2 * 8 * P_.N * nrhs : 0;
}

template <int P>
static hipError_t mv_launch(const Plan& P_, const double* x, double* y, int nrhs, void* ws,
                            double* part, int npart, const double* a, int as, hipStream_t s,
                            const double* fres) {
  const int m = P_.m, N = (int)P_.N;
  const char* b = P_.d_tables;
  const double* kc = (const double*)(b + P_.lay.kc64);
  const double* mc = (const double*)(b + P_.lay.mc64);
  const int nbr = 2 * P - 1, crows = P_.crows;
  if constexpr (P <= 4) {
    if (mv_fused(P_)) {
      int ncs, nrb, n3c;
      mvf_geom(m, P, ncs, nrb, n3c);
      const int bpr = ncs * nrb * n3c;
      if (part && bpr > npart) return hipErrorInvalidValue;
      hipLaunchKernelGGL(mv_fused3<P>, dim3(bpr * nrhs), dim3(MVF_THREADS), 0, s, x, y, m, N, ncs,
                         nrb, n3c, kc, mc, nbr, crows, part, npart, a, as, fres);
      return hipGetLastError();
    }
  }
  int ncs, nch, bpr;
  mv2_geom(m, P_.d == 3 ? m : 1, P, ncs, nch, bpr);
  if (part && bpr > npart) return hipErrorInvalidValue;
  if (P_.d == 3) {
    if (!ws) return hipErrorInvalidValue;
    double* t3 = (double*)ws;
    double* s3 = t3 + (size_t)N * nrhs;
    const int n3 = (m + MV1_C3 - 1) / MV1_C3;
    const int cb = (m * m + MV1_THREADS - 1) / MV1_THREADS;
    hipLaunchKernelGGL(mv_axis3<P>, dim3(cb * n3 * nrhs), dim3(MV1_THREADS), 0, s, x, t3, s3, m,
                       N, n3, kc, mc, nbr, crows, a, as);
    hipLaunchKernelGGL((mv_rows<P, true>), dim3(bpr * nrhs), dim3(MV2_THREADS), 0, s, x, t3, s3,
                       y, m, N, ncs, nch, bpr, kc, mc, nbr, crows, part, npart, a, as, fres);
  } else {
    hipLaunchKernelGGL((mv_rows<P, false>), dim3(bpr * nrhs), dim3(MV2_THREADS), 0, s, x, x,
                       (const double*)nullptr, y, m, N, ncs, nch, bpr, kc, mc, nbr, crows, part,
                       npart, a, as, fres);
  }
  return hipGetLastError();
}

hipError_t launch_matvec(const Plan& P_, const double* x, double* y, int nrhs, void* ws,
                         double* part, int npart, const double* a, int as, hipStream_t s,
                         const double* fres) {
  if (P_.geo.kind) return launch_geo_matvec(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
  if (P_.gen) return launch_gen_matvec(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
  switch (P_.p) {
    case 1: return mv_launch<1>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    case 2: return mv_launch<2>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    case 3: return mv_launch<3>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    case 4: return mv_launch<4>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    case 5: return mv_launch<5>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    case 6: return mv_launch<6>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    case 7: return mv_launch<7>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    case 8: return mv_launch<8>(P_, x, y, nrhs, ws, part, npart, a, as, s, fres);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace iffd
