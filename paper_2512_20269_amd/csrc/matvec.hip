// Matrix-free Galerkin operator y = Ahat x on gfx950 (FP64).
//
// Ahat = sum_k M (x) .. (x) K (slot k) (x) .. (x) M (eq:system_matrix and its
// 3-term analogue) with the banded 1-D matrices K, M (half-bandwidth p,
// Section 3).  Sum factorization per plane c (fixed i3):
//     t = M2 x_c,  s = K2 x_c          (along direction 2)
//     w = K1 t + M1 s,  v = M1 t       (along direction 1)
// so that w = (M2 (x) K1 + K2 (x) M1) x_c and v = (M2 (x) M1) x_c, and
//     y_{i3} = sum_c M3[i3,c] w_c + K3[i3,c] v_c     (along direction 3).
// In 2D the result is w.  That is 7 (3D) or 4 (2D) banded 1-D products per
// point, i.e. the minimum for the Kronecker sum.
//
// A workgroup owns a TY x TX tile of (i2, i1) and marches over a chunk of
// planes i3; each plane's contribution is pushed into a register ring of
// 2p+1 partial output planes, and the oldest plane is complete (and stored)
// once the march has passed p planes beyond it.  Halo values outside the
// domain are zero.  The 1-D matrices are Toeplitz away from the ends, so they
// are held compactly: the 2p-1 special rows at each end plus one interior
// stencil row.
#include "launch.h"

namespace iffd {

struct MvGeom {
  int m, N, TX, TY, ntx, nty, C3, nch, nbr, crows, d;
  const double* active;
  int astride;
  int npart;
};

__device__ __forceinline__ int crow(int i, int m, int nbr, int crows) {
  if (crows == m) return i;
  if (i < nbr) return i;
  if (i >= m - nbr) return i - (m - nbr) + nbr + 1;
  return nbr;
}

constexpr int MV_THREADS = 256;
constexpr int MV_PPT = 4;   // output points per thread per plane
constexpr int MV_XE = 10;   // x-tile elements per thread per plane (max)
constexpr int MV_TE = 8;    // t/s elements per thread per plane (max)

template <int P>
__global__ void __launch_bounds__(MV_THREADS)
matvec_kernel(const double* __restrict__ x, double* __restrict__ y, MvGeom g,
              const double* __restrict__ kc, const double* __restrict__ mc,
              double* __restrict__ part) {
  constexpr int BW = 2 * P + 1;
  extern __shared__ __align__(16) char smem[];
  const int m = g.m, TX = g.TX, TY = g.TY;
  const int XW = TX + 2 * P;
  double* xs = reinterpret_cast<double*>(smem);                  // (TY+2P) x XW
  double* ts = xs + (TY + 2 * P) * XW;                           // TY x XW
  double* ss = ts + TY * XW;                                     // TY x XW
  double* kcs = ss + TY * XW;                                    // crows x BW
  double* mcs = kcs + g.crows * BW;
  __shared__ double red[MV_THREADS / 64];

  const int t = threadIdx.x;
  int bid = blockIdx.x;
  const int tiles = g.ntx * g.nty;
  const int per_rhs = tiles * g.nch;
  const int rhs = bid / per_rhs;
  bid -= rhs * per_rhs;
  const int ch = bid / tiles;
  const int tl = bid - ch * tiles;
  const int by = tl / g.ntx, bx = tl - by * g.ntx;
  if (g.active && g.active[(size_t)rhs * g.astride] == 0.0) return;
  const int c0 = ch * g.C3, c1 = min(m, c0 + g.C3);
  const int d3 = g.d == 3;
  const double* xr = x + (size_t)rhs * g.N;
  double* yr = y + (size_t)rhs * g.N;
  const int nbr = g.nbr, crows = g.crows;

  for (int e = t; e < crows * BW; e += MV_THREADS) {
    kcs[e] = kc[e];
    mcs[e] = mc[e];
  }

  // x-tile elements of this thread (fixed for every plane)
  int xoff[MV_XE];
  const int xn = (TY + 2 * P) * XW;
#pragma unroll
  for (int k = 0; k < MV_XE; ++k) {
    const int e = t + MV_THREADS * k;
    xoff[k] = -2;  // -2: not mine, -1: outside the domain
    if (e < xn) {
      const int r = e / XW, cc = e - (e / XW) * XW;
      const int i2 = by * TY + r - P, i1 = bx * TX + cc - P;
      xoff[k] = (i2 >= 0 && i2 < m && i1 >= 0 && i1 < m) ? i2 * m + i1 : -1;
    }
  }
  // t/s elements: LDS row base and compact coefficient row of direction 2
  int tbase[MV_TE], tcr[MV_TE];
  const int tn = TY * XW;
#pragma unroll
  for (int k = 0; k < MV_TE; ++k) {
    const int e = t + MV_THREADS * k;
    tbase[k] = -1;
    tcr[k] = 0;
    if (e < tn) {
      const int r = e / XW, cc = e - (e / XW) * XW;
      const int i2 = by * TY + r;
      if (i2 < m) {
        tbase[k] = r * XW + cc;
        tcr[k] = crow(i2, m, nbr, crows);
      }
    }
  }
  // output points
  int pbase[MV_PPT], pcr[MV_PPT], poff[MV_PPT];
#pragma unroll
  for (int k = 0; k < MV_PPT; ++k) {
    const int pt = t + MV_THREADS * k;
    poff[k] = -1;
    pbase[k] = 0;
    pcr[k] = 0;
    if (pt < TY * TX) {
      const int r = pt / TX, cc = pt - (pt / TX) * TX;
      const int i2 = by * TY + r, i1 = bx * TX + cc;
      if (i2 < m && i1 < m) {
        poff[k] = i2 * m + i1;
        pbase[k] = r * XW + cc;
        pcr[k] = crow(i1, m, nbr, crows);
      }
    }
  }

  double acc[MV_PPT][BW];
#pragma unroll
  for (int k = 0; k < MV_PPT; ++k)
#pragma unroll
    for (int j = 0; j < BW; ++j) acc[k][j] = 0.0;
  double dot = 0.0;
  const int plane = m * m;
  const int cstart = d3 ? c0 - P : 0, cend = d3 ? c1 + P : 1;

  for (int c = cstart; c < cend; ++c) {
    const bool live = (c >= 0 && c < (d3 ? m : 1));
    if (live) {
      __syncthreads();
      const double* xp = xr + (size_t)c * plane;
#pragma unroll
      for (int k = 0; k < MV_XE; ++k) {
        const int e = t + MV_THREADS * k;
        if (xoff[k] >= -1) xs[e] = xoff[k] >= 0 ? xp[xoff[k]] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < MV_TE; ++k) {
        if (tbase[k] < 0) {
          const int e = t + MV_THREADS * k;
          if (e < tn) { ts[e] = 0.0; ss[e] = 0.0; }
          continue;
        }
        double tv = 0.0, sv = 0.0;
        const double* mrow = mcs + tcr[k] * BW;
        const double* krow = kcs + tcr[k] * BW;
#pragma unroll
        for (int j = 0; j < BW; ++j) {
          const double xv = xs[tbase[k] + j * XW];
          tv += mrow[j] * xv;
          sv += krow[j] * xv;
        }
        ts[t + MV_THREADS * k] = tv;
        ss[t + MV_THREADS * k] = sv;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < MV_PPT; ++k) {
        if (poff[k] < 0) continue;
        double w = 0.0, v = 0.0;
        const double* mrow = mcs + pcr[k] * BW;
        const double* krow = kcs + pcr[k] * BW;
#pragma unroll
        for (int j = 0; j < BW; ++j) {
          const double tv = ts[pbase[k] + j], sv = ss[pbase[k] + j];
          w += krow[j] * tv + mrow[j] * sv;
          v += mrow[j] * tv;
        }
        if (!d3) {
          acc[k][0] = w;
        } else {
#pragma unroll
          for (int kk = 0; kk < BW; ++kk) {
            const int i3 = c - P + kk;
            if (i3 >= 0 && i3 < m) {
              const int cr3 = crow(i3, m, nbr, crows);
              const int o = 2 * P - kk;  // band column of c in row i3
              acc[k][kk] += mcs[cr3 * BW + o] * w + kcs[cr3 * BW + o] * v;
            }
          }
        }
      }
    }
    // output plane oc is complete
    const int oc = d3 ? c - P : 0;
    if (oc >= c0 && oc < (d3 ? c1 : 1)) {
#pragma unroll
      for (int k = 0; k < MV_PPT; ++k) {
        if (poff[k] < 0) continue;
        const size_t gi = (size_t)oc * plane + poff[k];
        yr[gi] = acc[k][0];
        if (part) dot += xr[gi] * acc[k][0];
      }
    }
    if (d3) {
#pragma unroll
      for (int k = 0; k < MV_PPT; ++k) {
#pragma unroll
        for (int j = 0; j < BW - 1; ++j) acc[k][j] = acc[k][j + 1];
        acc[k][BW - 1] = 0.0;
      }
    }
  }
  if (part) {
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
    if ((t & 63) == 0) red[t >> 6] = dot;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int w = 0; w < MV_THREADS / 64; ++w) s += red[w];
      part[(size_t)rhs * g.npart + blockIdx.x - rhs * per_rhs] = s;
    }
  }
}

static bool mv_geometry(const Plan& P_, MvGeom& g) {
  const int P = P_.p;
  const int m = P_.m;
  g.m = m;
  g.N = (int)P_.N;
  g.d = P_.d;
  g.ntx = (m + 63) / 64;
  g.TX = (m + g.ntx - 1) / g.ntx;
  // rows: bounded by the per-thread register budgets
  int TY = (MV_THREADS * MV_PPT) / g.TX;
  while (TY > 0 && (TY + 2 * P) * (g.TX + 2 * P) > MV_THREADS * MV_XE) --TY;
  while (TY > 0 && TY * (g.TX + 2 * P) > MV_THREADS * MV_TE) --TY;
  if (TY > m) TY = m;
  if (TY < 1) return false;
  g.TY = TY;
  g.nty = (m + TY - 1) / TY;
  if (P_.d == 3) {
    // enough workgroups per right-hand side to fill the chip, with chunks long
    // enough to amortise the 2p-plane halo of the march.  The split depends
    // on the plan only, so the partial sums of a right-hand side are grouped
    // the same way in every batch.
    const int tiles = g.ntx * g.nty;
    int C3 = m;
    while (C3 > 4 * P && tiles * ((m + C3 - 1) / C3) < 1024) C3 = (C3 + 1) / 2;
    g.C3 = C3;
    g.nch = (m + C3 - 1) / C3;
  } else {
    g.C3 = 1;
    g.nch = 1;
  }
  g.nbr = 2 * P - 1;
  g.crows = P_.crows;
  return true;
}

int matvec_blocks(const Plan& P_) {
  MvGeom g;
  if (!mv_geometry(P_, g)) return 1;
  return g.ntx * g.nty * g.nch;
}

template <int P>
static hipError_t mv_launch(const Plan& P_, const double* x, double* y, int nrhs, double* part,
                            int npart, const double* a, int as, hipStream_t s) {
  MvGeom g;
  if (!mv_geometry(P_, g)) return hipErrorInvalidValue;
  const int TY = g.TY;
  g.active = a;
  g.astride = as;
  g.npart = npart;
  const int per_rhs = g.ntx * g.nty * g.nch;
  if (part && per_rhs > npart) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * ((size_t)(TY + 2 * P) * (g.TX + 2 * P) +
                                       2 * (size_t)TY * (g.TX + 2 * P) + 2 * (size_t)g.crows * (2 * P + 1));
  if (lds > 65536) {
    static bool done = false;
    if (!done) {
      hipError_t e = hipFuncSetAttribute((const void*)matvec_kernel<P>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      if (e != hipSuccess) return e;
      done = true;
    }
  }
  const char* b = P_.d_tables;
  hipLaunchKernelGGL(matvec_kernel<P>, dim3(per_rhs * nrhs), dim3(MV_THREADS), lds, s, x, y, g,
                     (const double*)(b + P_.lay.kc64), (const double*)(b + P_.lay.mc64), part);
  return hipGetLastError();
}

hipError_t launch_matvec(const Plan& P_, const double* x, double* y, int nrhs, double* part,
                         int npart, const double* a, int as, hipStream_t s) {
  switch (P_.p) {
    case 1: return mv_launch<1>(P_, x, y, nrhs, part, npart, a, as, s);
    case 2: return mv_launch<2>(P_, x, y, nrhs, part, npart, a, as, s);
    case 3: return mv_launch<3>(P_, x, y, nrhs, part, npart, a, as, s);
    case 4: return mv_launch<4>(P_, x, y, nrhs, part, npart, a, as, s);
    case 5: return mv_launch<5>(P_, x, y, nrhs, part, npart, a, as, s);
    case 6: return mv_launch<6>(P_, x, y, nrhs, part, npart, a, as, s);
    case 7: return mv_launch<7>(P_, x, y, nrhs, part, npart, a, as, s);
    case 8: return mv_launch<8>(P_, x, y, nrhs, part, npart, a, as, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace iffd
