// Matrix-free operator y = A x in one pass for general plans (2D and 3D):
// A = sum_k M_3 (x) .. K_k .. (x) M_1 with per-direction
// banded K_k, M_k (eq:system_matrix and its 3-term analogue; in 2D the third
// direction has one entry, M_3 = 1 and K_3 = 0).
//
// A workgroup of 8 waves owns a tile of 64 columns (direction 1, one lane
// each) x 32 rows (direction 2, four per wave) and walks a chunk of planes
// (direction 3) in order.  Each thread keeps, for its four rows, a rolling
// register window of the 2 PM + 1 planes of x around the current plane:
// every plane of x is loaded once per tile (each load is issued 2 to 4
// planes ahead of its use), t = M3 x and s = K3 x come from the window, then t and s go
// through LDS (double-buffered by plane parity, one LDS-only barrier per plane, so
// the loads in flight are not drained) so that each wave forms, for a run of
// consecutive output rows (reading every t and s row it needs once),
// u = M2 t and v = K2 t + M2 s down the rows and
// y = K1 u + M1 v across the lanes with DPP whole-wave shifts (Horner's
// scheme, PM shifts each way).  The outer PM columns and rows of a tile only
// feed their neighbours; a chunk reads PM halo planes on each side.  The band
// tables are m_k x (2 PM + 1), PM >= every direction's p (rows padded with
// zeros), so one kernel serves per-direction degrees.  The last step also
// forms per-workgroup partial sums of x . y, or of (f - y)^2 for a true
// residual, in a fixed order.
#include "launch.h"

namespace iffd {

constexpr int MR_W = 8;     // waves per workgroup
constexpr int MR_RPT = 4;   // rows per thread
constexpr int MR_TR = MR_W * MR_RPT;  // tile rows
constexpr int MR_C3 = 16;   // planes per workgroup
// planes of x in flight ahead of the window (fewer for the wide windows of
// high degrees, whose registers are scarce)
template <int PM>
constexpr int mr_pf() { return PM <= 5 ? 4 : 2; }
constexpr int MR_THREADS = 64 * MR_W;

// whole-wave lane shifts of a double by one lane (DPP wave_shr:1 / wave_shl:1;
// the lane without a source receives 0)
__device__ __forceinline__ double roll_from_lower(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, 0x138, 0xF, 0xF, true),
                          __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double roll_from_upper(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, 0x130, 0xF, 0xF, true),
                          __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xF, 0xF, true));
}

void mv_roll_geom(const RollBands& B, int& ncs, int& nrb, int& n3c) {
  const int oc = 64 - 2 * B.pm, orr = MR_TR - 2 * B.pm;
  ncs = (B.n[0] + oc - 1) / oc;
  nrb = (B.n[1] + orr - 1) / orr;
  n3c = (B.n[2] + MR_C3 - 1) / MR_C3;
}

int mv_roll_blocks(const RollBands& B) {
  int a, b, c;
  mv_roll_geom(B, a, b, c);
  return a * b * c;
}

template <int PM>
__global__ void __launch_bounds__(MR_THREADS)
mv_roll(const double* __restrict__ x, double* __restrict__ y, RollBands B, int N, int ncs,
        int nrb, int n3c, double* __restrict__ part, int npart, const double* __restrict__ active,
        int astride, const double* __restrict__ fres) {
  constexpr int BW = 2 * PM + 1;
  constexpr int OC = 64 - 2 * PM, OR = MR_TR - 2 * PM;
  // degrees above 4 keep the direction-1 coefficients in LDS, not registers
  // (the windows of four rows already take 8 PM + 4 registers)
  constexpr bool RC = PM <= 4;
  constexpr int MR_PF = mr_pf<PM>();
  // output rows per wave in the in-plane step
  constexpr int RB = (OR + MR_W - 1) / MR_W;
  __shared__ double ts[2][2][MR_TR][64];   // [plane parity][t, s][row][column]
  __shared__ double xs[2][MR_TR][64];      // [plane parity][row][column]: x at the plane
  __shared__ double b2[2][MR_TR][BW];      // direction-2 band rows of the tile's rows: K, M
  __shared__ double b3[2][MR_C3][BW];      // direction-3 band rows of the chunk's planes
  __shared__ double c1[RC ? 1 : 4][RC ? 1 : PM + 1][64];   // kl, ml, kh, mh per lane
  __shared__ double red[MR_W];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m1 = B.n[0], m2 = B.n[1], m3 = B.n[2];
  const int bpr = ncs * nrb * n3c;
  const int lin = xcd_linear(blockIdx.x, gridDim.x);   // neighbouring tiles share halos in one L2
  const int rhs = lin / bpr;
  const int blk = lin - rhs * bpr;
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  // plane chunks vary fastest, then row blocks, then column strips
  const int ch = blk % n3c;
  const int rb = (blk / n3c) % nrb;
  const int cs = blk / (n3c * nrb);
  const int i1 = cs * OC - PM + lane;
  const bool colok = i1 >= 0 && i1 < m1;
  const int c0 = ch * MR_C3;
  const int plane = m1 * m2;
  const double* K1 = B.k[0];
  const double* M1 = B.m[0];
  const double* K3 = B.k[2];
  const double* M3 = B.m[2];

  // direction-2 band rows of the tile's rows
  for (int e = threadIdx.x; e < MR_TR * BW; e += MR_THREADS) {
    const int r = e / BW, o = e - r * BW;
    const int j2 = rb * OR - PM + r;
    const bool ok = j2 >= 0 && j2 < m2;
    b2[0][r][o] = ok ? B.k[1][(size_t)j2 * BW + o] : 0.0;
    b2[1][r][o] = ok ? B.m[1][(size_t)j2 * BW + o] : 0.0;
  }
  for (int e = threadIdx.x; e < MR_C3 * BW; e += MR_THREADS) {
    const int c = e / BW, o = e - c * BW;
    const int j3 = c0 + c;
    const bool ok = j3 < m3;
    b3[0][c][o] = ok ? K3[(size_t)j3 * BW + o] : 0.0;
    b3[1][c][o] = ok ? M3[(size_t)j3 * BW + o] : 0.0;
  }
  // direction-1 coefficients of this lane: its own band row's centre, and what
  // the columns i1 + d (L) and i1 - d (H) apply to it (zero outside)
  double k1c = 0.0, m1c = 0.0, kl[RC ? PM + 1 : 1], ml[RC ? PM + 1 : 1], kh[RC ? PM + 1 : 1],
         mh[RC ? PM + 1 : 1];
  if (colok) {
    k1c = K1[(size_t)i1 * BW + PM];
    m1c = M1[(size_t)i1 * BW + PM];
  }
#pragma unroll
  for (int d = 1; d <= PM; ++d) {
    const int jl = i1 + d, jh = i1 - d;
    const bool okl = colok && jl < m1, okh = colok && jh >= 0;
    const double a = okl ? K1[(size_t)jl * BW + PM - d] : 0.0;
    const double b = okl ? M1[(size_t)jl * BW + PM - d] : 0.0;
    const double c = okh ? K1[(size_t)jh * BW + PM + d] : 0.0;
    const double e = okh ? M1[(size_t)jh * BW + PM + d] : 0.0;
    if constexpr (RC) {
      kl[d] = a; ml[d] = b; kh[d] = c; mh[d] = e;
    } else if (wv == 0) {
      c1[0][d][lane] = a; c1[1][d][lane] = b; c1[2][d][lane] = c; c1[3][d][lane] = e;
    }
  }
  auto KL = [&](int d) { if constexpr (RC) return kl[d]; else return c1[0][d][lane]; };
  auto ML = [&](int d) { if constexpr (RC) return ml[d]; else return c1[1][d][lane]; };
  auto KH = [&](int d) { if constexpr (RC) return kh[d]; else return c1[2][d][lane]; };
  auto MH = [&](int d) { if constexpr (RC) return mh[d]; else return c1[3][d][lane]; };

  // rolling windows: w[j][o] = x at plane i3 - PM + o of row j
  const auto rs = buf_rsrc(x + (size_t)rhs * N, (unsigned)N * 8u);
  unsigned vo[MR_RPT];
  int i2r[MR_RPT];
#pragma unroll
  for (int j = 0; j < MR_RPT; ++j) {
    const int r = wv + MR_W * j;
    i2r[j] = rb * OR - PM + r;
    const bool ok = colok && i2r[j] >= 0 && i2r[j] < m2;
    vo[j] = ok ? (unsigned)(i2r[j] * m1 + i1) * 8u : BUF_OOB;
  }
  auto ldp = [&](int j, int c) -> double {
    return (c >= 0 && c < m3) ? buf_ld<double>(rs, vo[j] + (unsigned)(c * plane) * 8u) : 0.0;
  };
  // w: the window; nx[j][.]: the MR_PF planes after the window, loading (slot
  // q holds the plane that enters the window at the steps k = q mod MR_PF)
  double w[MR_RPT][BW], nx[MR_RPT][MR_PF];
#pragma unroll
  for (int j = 0; j < MR_RPT; ++j) {
#pragma unroll
    for (int o = 1; o < BW; ++o) w[j][o] = ldp(j, c0 - PM - 1 + o);
#pragma unroll
    for (int q = 0; q < MR_PF; ++q) nx[j][q] = ldp(j, c0 + PM + q);
  }
  const auto ws = buf_rsrc(y + (size_t)rhs * N, (unsigned)N * 8u);
  const auto fr = buf_rsrc(fres ? fres + (size_t)rhs * N : y, fres ? (unsigned)N * 8u : 0u);
  const bool outc = lane >= PM && lane < 64 - PM && colok;
  double dot = 0.0;
  const int kend = min(MR_C3, m3 - c0);
  lds_barrier();   // the band rows staged above
  for (int k0 = 0; k0 < kend; k0 += MR_PF) {
#pragma unroll
    for (int q = 0; q < MR_PF; ++q) {
      const int k = k0 + q;
      if (k >= kend) break;   // uniform
      const int i3 = c0 + k;
      // advance the windows; plane i3 + PM + MR_PF goes out in the freed slot
#pragma unroll
      for (int j = 0; j < MR_RPT; ++j) {
#pragma unroll
        for (int o = 0; o < BW - 1; ++o) w[j][o] = w[j][o + 1];
        w[j][BW - 1] = nx[j][q];
        nx[j][q] = ldp(j, i3 + PM + MR_PF);
      }
      const double* k3 = b3[0][k];   // LDS broadcasts: no global round trip per plane
      const double* m3r = b3[1][k];
      const int pb = k & 1;
#pragma unroll
      for (int j = 0; j < MR_RPT; ++j) {
        double t = 0.0, sv = 0.0;
#pragma unroll
        for (int o = 0; o < BW; ++o) {
          t += m3r[o] * w[j][o];
          sv += k3[o] * w[j][o];
        }
        ts[pb][0][wv + MR_W * j][lane] = t;
        ts[pb][1][wv + MR_W * j][lane] = sv;
        xs[pb][wv + MR_W * j][lane] = w[j][PM];   // x at the point, for the partial sums
      }
      lds_barrier();   // the planes in flight stay in flight
      // wave wv forms the RB consecutive output rows r0 .. r0 + RB - 1: the
      // RB + 2 PM rows of t and s they need are read from LDS once
      const int r0 = PM + wv * RB;
      if (r0 < PM + OR) {   // uniform per wave
        double tv[RB + 2 * PM], sv2[RB + 2 * PM];
#pragma unroll
        for (int q = 0; q < RB + 2 * PM; ++q) {
          const int rr = min(r0 - PM + q, MR_TR - 1);   // rows past the tile feed no output
          tv[q] = ts[pb][0][rr][lane];
          sv2[q] = ts[pb][1][rr][lane];
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const int r = r0 + b;
          const int i2 = rb * OR - PM + r;
          if (r >= PM + OR || i2 >= m2) break;   // uniform per wave
          double u = 0.0, v = 0.0;
#pragma unroll
          for (int o = 0; o < BW; ++o) {
            u += b2[1][r][o] * tv[b + o];
            v += b2[0][r][o] * tv[b + o] + b2[1][r][o] * sv2[b + o];
          }
          double lo = KL(PM) * u + ML(PM) * v;
          double hi = KH(PM) * u + MH(PM) * v;
#pragma unroll
          for (int d = PM - 1; d >= 1; --d) {
            lo = roll_from_lower(lo);
            hi = roll_from_upper(hi);
            lo = fma(KL(d), u, fma(ML(d), v, lo));
            hi = fma(KH(d), u, fma(MH(d), v, hi));
          }
          lo = roll_from_lower(lo);
          hi = roll_from_upper(hi);
          const double yv = fma(k1c, u, fma(m1c, v, lo + hi));
          if (outc) {
            const unsigned oo = (unsigned)(i3 * plane + i2 * m1 + i1) * 8u;
            buf_st<double>(yv, ws, oo);
            if (part) {
              if (fres) {
                const double dv = buf_ld<double>(fr, oo) - yv;
                dot += dv * dv;
              } else {
                dot += xs[pb][r][lane] * yv;
              }
            }
          }
        }
      }
    }
  }
  if (part) {
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
    if (lane == 0) red[wv] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s2 = 0.0;
      for (int k = 0; k < MR_W; ++k) s2 += red[k];
      part[(size_t)rhs * npart + blk] = s2;
    }
  }
}

template <int PM>
static hipError_t roll_t(const RollBands& B, const double* x, double* y, int nrhs, int N,
                         double* part, int npart, const double* a, int as, hipStream_t s,
                         const double* fres) {
  int ncs, nrb, n3c;
  mv_roll_geom(B, ncs, nrb, n3c);
  const int bpr = ncs * nrb * n3c;
  if (part && bpr > npart) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mv_roll<PM>, dim3(bpr * nrhs), dim3(MR_THREADS), 0, s, x, y, B, N, ncs, nrb,
                     n3c, part, npart, a, as, fres);
  return hipGetLastError();
}

hipError_t launch_mv_roll(const RollBands& B, const double* x, double* y, int nrhs, int N,
                          double* part, int npart, const double* a, int as, hipStream_t s,
                          const double* fres) {
  switch (B.pm) {
    case 1: return roll_t<1>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    case 2: return roll_t<2>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    case 3: return roll_t<3>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    case 4: return roll_t<4>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    case 5: return roll_t<5>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    case 6: return roll_t<6>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    case 7: return roll_t<7>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    case 8: return roll_t<8>(B, x, y, nrhs, N, part, npart, a, as, s, fres);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace iffd
