#pragma once
// IFFD line passes of general plans on gfx950: every direction has its own n,
// p and Dirichlet / Neumann ends (Section 4, "other boundary conditions";
// Table 1; Section 6).  Kernel templates; instantiated per FFT length in
// gen_l*.hip, dispatched in gen.hip.
//
// Per line along direction k (length m), with V_reg = blkdiag(AL, I, AR) in
// the special basis and U_{s,t} = sin(pi (s + sig)(t + tau) / n + beta) the
// transform of Table 1 (sig, tau in {0, 1/2, 1}, beta in {0, pi/2}):
//   forward   y_reg = U^T fold(x),  y_out = Vt x
//   backward  x = unfold(U y_reg) + Vt^T y_out
// fold = V_reg^T (AL^T on the first rl entries, AR^T on the last rr, the
// interior passes through), unfold = V_reg.  Both products with U run through
// one complex FFT of length L = 2n per pair of real lines a, b:
//   y_t = -Im[ post_t * A_t ],  A_t = sum_s g_s pre_s e^{-2 pi i s t / L},
// with pre_s = e^{-i pi s tau / n}, post_t = e^{-i (beta + pi sig (t + tau) / n)}
// (forward; sig and tau swap roles backward).  A_t has the symmetry
// conj(A_t) = A_{-t - 2 tau}, so the transform Z of (g_a + i g_b) pre splits
// into A = (Z_t + conj Z_t') / 2 and B = (Z_t - conj Z_t') / (2i), t' = -t -
// 2 tau mod L, which gives y_a = -Im[post (Z_t + conj Z_t')] / 2 and
// y_b = Re[post (Z_t - conj Z_t')] / 2.
//
// One workgroup owns TW lines of one right-hand side, staged through LDS with
// coalesced loads (lines along direction 1 are contiguous rows; lines along a
// strided direction are taken TW at a time from consecutive positions of the
// faster directions, each padded run of direction-1 positions having an even
// length so that the two lines of an FFT pair always belong to one run).  The
// middle pass (along direction d) runs forward, scales by the Kronecker sum
// of the eigenvalues and runs backward without leaving LDS.
#include "fft_device.h"
#include "launch.h"

namespace iffd {

// FFT shape: 8 (or 12) elements per thread (variant 1 of fft_device.h; the
// 16-element shape measured 1.6x slower on these passes), up to 32 line pairs
// and 256 threads per workgroup
template <typename T, int L>
struct GCfg {
  static constexpr int V = 1;
  static constexpr int E = FftPlan<L, V>::E;
  static constexpr int NT = L / E;   // threads per transform
  static constexpr int CAP = 256 / NT;
  static constexpr int FPW = CAP >= 32 ? 32 : (CAP < 1 ? 1 : CAP);  // line pairs per workgroup
  static constexpr int TW = 2 * FPW;  // lines per workgroup (a power of two)
  static constexpr int NTH = FPW * NT;
};

// one direction's tables in its blob (element offsets) and sizes
template <typename T>
struct GDirDev {
  const T* blob;  // tw | tf | AL | AR | Vt | lam | s | ...
  int o_tw, o_tf, o_al, o_ar, o_vt, o_lam, o_s;
  int m, n_reg, n_out, rl, cl, rr, cr;
  int mir_f, mir_b;  // 2 tau, 2 sig: the index shift of the spectral symmetry
  int wl, wr;        // outlier windows: Vt[q][j] used for j < wl and j >= wr
  // generic basis of S^reg (eq:reg_eigenvectors): nonzero gb adds the banded
  // solves with the interpolation matrix C = L U (bands at o_lb, o_ub; see GDir)
  int gb, bl, bu, o_lb, o_ub;
  // reduced regularity (a repeated knot, eq:reg_space2): the line has m
  // entries on the reduced space's B-splines, mo = m - rk of them on the
  // maximally smooth space's; E (knot insertion) is the identity below the
  // old position wk0, a shift by rk from wk1 on, and the block EW (rows
  // wk0 .. wk1 + rk, columns wk0 .. wk1) in between (wk0 = wk1 = 2^30 without
  // a knot).  Outlier window [kw0, kw1) around the knot.
  int rk, wk0, wk1, o_ew, kw0, kw1, mo;
};

template <typename T>
struct GPassArgs {
  GDirDev<T> dir;
  int S;    // element stride along the pass's direction
  int m1;   // extent of direction 1
  int mr;   // S > 1: padded run of direction-1 positions (m1 rounded up to even)
  int sm;   // S > 1: S / m1
  int lpr;  // lines per right-hand side (padded for S > 1)
  int tpr;  // tiles per right-hand side
  int N;    // elements per right-hand side
  // middle pass: eigenvalues and scalings of direction 1 and (3D) direction 2
  const T* lam1;
  const T* s1;
  const T* lam2;
  const T* s2;
  const double* active;  // per-RHS flags (0 = skip) or null
  int astride;
};

struct GLds {
  size_t tw, x, f, gb, yo, kb, lb, lo, so, total;
};

__host__ __device__ inline size_t gup16(size_t x) { return (x + 15) & ~(size_t)15; }

template <typename T, int L, class C = GCfg<T, L>>
__host__ __device__ inline GLds gen_lds(int m) {
  const int MP = m | 1;
  GLds r;
  size_t o = 0;
  r.tw = o; o = gup16(o + 2 * sizeof(T) * L);
  r.x = o;  o = gup16(o + sizeof(T) * C::TW * MP);
  r.f = o;  o = gup16(o + 2 * sizeof(T) * C::FPW * fft_region<L>());
  r.gb = o; o = gup16(o + sizeof(T) * C::TW * 8);
  r.yo = o; o = gup16(o + sizeof(T) * C::TW * 8);
  r.kb = o; o = gup16(o + sizeof(T) * C::TW * 16);
  r.lb = o; o = gup16(o + sizeof(int) * C::TW);
  r.lo = o; o = gup16(o + sizeof(T) * C::TW);
  r.so = o; o = gup16(o + sizeof(T) * C::TW);
  r.total = o;
  return r;
}

// First element of line q of the pass (-1 if q is a padding line); for the
// middle pass also the line's spectral positions along directions 1 and 2.
template <typename T>
__device__ __forceinline__ int gen_line(const GPassArgs<T>& a, int q, int& i1, int& i2) {
  i1 = 0;
  i2 = 0;
  if (q >= a.lpr) return -1;
  if (a.S == 1) return q * a.dir.m;
  const int r = q % a.mr, rest = q / a.mr;
  if (r >= a.m1) return -1;
  const int j2 = rest % a.sm, outer = rest / a.sm;
  i1 = r;
  i2 = j2;
  return outer * a.dir.m * a.S + j2 * a.m1 + r;
}

// The transforms of one tile of TW lines held in LDS (X[l][i], row pitch MP).
// All threads of the workgroup call each step; every step ends with a barrier.
template <typename T, int L, class C>
struct GTile {
  cpx<T>* tw;  // L twiddles
  T* X;        // TW x MP
  cpx<T>* F;   // FPW FFT regions
  T* GB;       // TW x 8: folded end values
  T* YO;       // TW x 8: outlier coefficients
  T* KB;       // TW x 16: E^T x on the knot window (reduced regularity)
  const T* LO; // TW: sum of the other directions' eigenvalues (middle pass)
  const T* SO; // TW: product of their scalings (middle pass)
  int MP;

  // generic basis: w <- C^{-T} w on the folded lines w = X[l][off .. off + n_reg),
  // one thread per line (C^T = U^T L^T: forward substitution with U^T, then
  // backward substitution with L^T)
  __device__ __forceinline__ void solve_ct(const GDirDev<T>& D) const {
    const int nr = D.n_reg, bl = D.bl, bu = D.bu, off = D.rl - D.cl;
    const T* LB = D.blob + D.o_lb;
    const T* UB = D.blob + D.o_ub;
    for (int l = threadIdx.x; l < C::TW; l += C::NTH) {
      T* w = X + l * MP + off;
      for (int i = 0; i < nr; ++i) {
        T acc = w[i];
        for (int j = max(0, i - bu); j < i; ++j) acc -= UB[j * (bu + 1) + (i - j)] * w[j];
        w[i] = acc * UB[i * (bu + 1)];
      }
      for (int i = nr - 1; i >= 0; --i) {
        T acc = w[i];
        const int je = min(nr - 1, i + bl);
        for (int j = i + 1; j <= je; ++j) acc -= LB[j * bl + (i - j + bl)] * w[j];
        w[i] = acc;
      }
    }
  }

  // generic basis: c <- C^{-1} c on the lines c = X[l][off .. off + n_reg)
  // (L y = c forward, U c = y backward)
  __device__ __forceinline__ void solve_c(const GDirDev<T>& D) const {
    const int nr = D.n_reg, bl = D.bl, bu = D.bu, off = D.rl - D.cl;
    const T* LB = D.blob + D.o_lb;
    const T* UB = D.blob + D.o_ub;
    for (int l = threadIdx.x; l < C::TW; l += C::NTH) {
      T* w = X + l * MP + off;
      for (int i = 0; i < nr; ++i) {
        T acc = w[i];
        for (int j = max(0, i - bl); j < i; ++j) acc -= LB[i * bl + (j - i + bl)] * w[j];
        w[i] = acc;
      }
      for (int i = nr - 1; i >= 0; --i) {
        T acc = w[i];
        const int je = min(nr - 1, i + bu);
        for (int j = i + 1; j <= je; ++j) acc -= UB[i * (bu + 1) + (j - i)] * w[j];
        w[i] = acc * UB[i * (bu + 1)];
      }
    }
  }

  // X[l][0..m) = x  ->  X[l][0..n_reg) = U^T V_reg^T x, YO[l] = Vt x; with MID
  // both scaled by s_t * SO[l] / (lambda_t + LO[l]).  A generic basis
  // (D.gb) writes the folded line in place, X[l][off + s] = (V_reg^T x)_s, and
  // solves with C^T before the transform.
  template <bool MID>
  __device__ __forceinline__ void forward(const GDirDev<T>& D) const {
    constexpr int TW = C::TW, NTH = C::NTH, NT = C::NT;
    const int m = D.m, nr = D.n_reg, no = D.n_out, cl = D.cl, cr = D.cr, rl = D.rl, rr = D.rr;
    const int off = rl - cl, ncr = nr - cr;
    const T* AL = D.blob + D.o_al;
    const T* AR = D.blob + D.o_ar;
    const T* Vt = D.blob + D.o_vt;
    const cpx<T>* TF = reinterpret_cast<const cpx<T>*>(D.blob + D.o_tf);
    const int tid = threadIdx.x;
    const int f = tid / NT, lane = tid - f * NT;
    cpx<T>* buf = F + f * fft_region<L>();
    const int la = 2 * f, lb = 2 * f + 1;
    // boundary fold values, outlier coefficients and, with a repeated knot,
    // E^T x on the knot window
    const int nbv = cl + cr;
    const int nkw = D.rk ? D.wk1 - D.wk0 : 0;
    const T* EW = D.blob + D.o_ew;
    // the short ones (end blocks, knot window) one thread each
    for (int w = tid; w < TW * (nbv + nkw); w += NTH) {
      const int l = w & (TW - 1), k = w / TW;
      const T* x = X + l * MP;
      T acc = T(0);
      if (k < cl) {
        for (int r = 0; r < rl; ++r) acc += AL[r * cl + k] * x[r];
        GB[l * 8 + k] = acc;
      } else if (k < nbv) {
        const int kk = k - cl;
        for (int r = 0; r < rr; ++r) acc += AR[r * cr + kk] * x[m - rr + r];
        GB[l * 8 + k] = acc;
      } else {
        const int c = k - nbv;
        for (int i = 0; i < nkw + D.rk; ++i) acc += EW[i * nkw + c] * x[D.wk0 + i];
        KB[l * 16 + c] = acc;
      }
    }
    // the outlier dots over their windows (tens of entries): tpd adjacent
    // lanes of one wave per dot, summed by shuffles in a fixed order; every
    // thread runs every round so that the shuffles see all lanes
    if (no > 0) {
      const int ndots = TW * no;
      int tpd = 1;
      while (tpd < 64 && ndots * tpd * 2 <= NTH) tpd *= 2;
      const int per = NTH / tpd;
      const int rounds = (ndots + per - 1) / per;
      const int sub = tid & (tpd - 1);
      const int nl = D.wl, nk = D.kw1 - D.kw0, nw = D.wl + nk + (m - D.wr);
      for (int rd = 0; rd < rounds; ++rd) {
        const int di = tid / tpd + rd * per;
        T acc = T(0);
        if (di < ndots) {
          const int l = di & (TW - 1), q = di / TW;
          const T* x = X + l * MP;
          const T* v = Vt + q * m;
          for (int u = sub; u < nw; u += tpd) {
            const int j = u < nl ? u : (u < nl + nk ? D.kw0 + (u - nl) : D.wr + (u - nl - nk));
            acc += v[j] * x[j];
          }
        }
        for (int o = 1; o < tpd; o <<= 1) acc += __shfl_xor(acc, o);
        if (sub == 0 && di < ndots) YO[(di & (TW - 1)) * 8 + di / TW] = acc;
      }
    }
    __syncthreads();
    const bool gbas = D.gb != 0;
    if (gbas) {
      for (int w = tid; w < TW * nbv; w += NTH) {
        const int l = w & (TW - 1), k = w / TW;
        X[l * MP + off + (k < cl ? k : ncr + k - cl)] = GB[l * 8 + k];
      }
      __syncthreads();
      solve_ct(D);
      __syncthreads();
    }
    {
      const T* xa = X + la * MP;
      const T* xb = X + lb * MP;
      const T* ga = GB + la * 8;
      const T* gbb = GB + lb * 8;
      const T* ka = KB + la * 16;
      const T* kbb = KB + lb * 16;
      const int wk0 = D.wk0, wk1 = D.wk1, rk = D.rk;
      // the folded line: end blocks, then x on the old interior positions
      // through the knot window
      auto fold = [&](const T* x, const T* g, const T* kw, int s) -> T {
        if (s < cl) return g[s];
        if (s >= ncr) return g[cl + s - ncr];
        const int j = s + off;
        if (j < wk0) return x[j];
        if (j >= wk1) return x[j + rk];
        return kw[j - wk0];
      };
      auto ld = [&](int k, bool, bool, bool) -> cpx<T> {
        if (k >= nr) return cpx<T>{T(0), T(0)};
        const cpx<T> v = gbas ? cpx<T>{xa[off + k], xb[off + k]}
                              : cpx<T>{fold(xa, ga, ka, k), fold(xb, gbb, kbb, k)};
        return c_mul(v, TF[k]);
      };
      auto st = [&](int k, cpx<T> v) { buf[fpad<L>(k)] = v; };
      fft_forward<T, L, C::V>(buf, lane, tw, ld, st);
    }
    __syncthreads();
    {
      const cpx<T>* post = TF + nr;
      const int mir = D.mir_f;
      const T* lamd = D.blob + D.o_lam;
      const T* sd = D.blob + D.o_s;
      for (int t = lane; t < nr; t += NT) {
        const cpx<T> z1 = buf[fpad<L>(t)];
        int t2 = L - t - mir;
        if (t2 >= L) t2 -= L;
        cpx<T> z2 = buf[fpad<L>(t2)];
        z2.y = -z2.y;
        const cpx<T> P = post[t];
        const cpx<T> sp = c_mul(P, c_add(z1, z2)), sm = c_mul(P, c_sub(z1, z2));
        T ya = -sp.y * T(0.5), yb = sm.x * T(0.5);
        if constexpr (MID) {
          const T l = lamd[t], s = sd[t];
          ya *= s * SO[la] / (l + LO[la]);
          yb *= s * SO[lb] / (l + LO[lb]);
        }
        X[la * MP + t] = ya;
        X[lb * MP + t] = yb;
      }
      if constexpr (MID) {
        for (int w = tid; w < TW * no; w += NTH) {
          const int l = w & (TW - 1), q = w / TW;
          YO[l * 8 + q] *= SO[l] / (lamd[nr + q] + LO[l]);
        }
      }
    }
    __syncthreads();
  }

  // entry i of the spectral line l after forward(): y_reg, then y_out
  __device__ __forceinline__ T spectral(const GDirDev<T>& D, int l, int i) const {
    return i < D.n_reg ? X[l * MP + i] : YO[l * 8 + i - D.n_reg];
  }

  // X[l][0..n_reg) = y_reg and YO[l] = y_out  ->  c = U y_reg at X[l][off + s]
  // (off = rl - cl), where the interior rows of x = V_reg c read it in place;
  // a generic basis (D.gb) then solves with C: c = C^{-1} U y_reg
  __device__ __forceinline__ void backward(const GDirDev<T>& D) const {
    constexpr int NT = C::NT;
    const int nr = D.n_reg, off = D.rl - D.cl;
    const cpx<T>* TF = reinterpret_cast<const cpx<T>*>(D.blob + D.o_tf);
    const int tid = threadIdx.x;
    const int f = tid / NT, lane = tid - f * NT;
    cpx<T>* buf = F + f * fft_region<L>();
    const int la = 2 * f, lb = 2 * f + 1;
    {
      const T* xa = X + la * MP;
      const T* xb = X + lb * MP;
      const cpx<T>* pre = TF + 2 * nr;
      auto ld = [&](int k, bool, bool, bool) -> cpx<T> {
        if (k >= nr) return cpx<T>{T(0), T(0)};
        return c_mul(cpx<T>{xa[k], xb[k]}, pre[k]);
      };
      auto st = [&](int k, cpx<T> v) { buf[fpad<L>(k)] = v; };
      fft_forward<T, L, C::V>(buf, lane, tw, ld, st);
    }
    __syncthreads();
    {
      const cpx<T>* post = TF + 3 * nr;
      const int mir = D.mir_b;
      for (int t = lane; t < nr; t += NT) {
        const cpx<T> z1 = buf[fpad<L>(t)];
        int t2 = L - t - mir;
        if (t2 >= L) t2 -= L;
        cpx<T> z2 = buf[fpad<L>(t2)];
        z2.y = -z2.y;
        const cpx<T> P = post[t];
        const cpx<T> sp = c_mul(P, c_add(z1, z2)), sm = c_mul(P, c_sub(z1, z2));
        X[la * MP + off + t] = -sp.y * T(0.5);
        X[lb * MP + off + t] = sm.x * T(0.5);
      }
    }
    __syncthreads();
    if (D.gb) {
      solve_c(D);
      __syncthreads();
    }
  }

  // entry r of line l after backward(): x = V_reg c + Vt^T y_out
  __device__ __forceinline__ T value(const GDirDev<T>& D, int l, int r) const {
    const int m = D.m, cl = D.cl, cr = D.cr, rl = D.rl, rr = D.rr, off = rl - cl;
    const T* AL = D.blob + D.o_al;
    const T* AR = D.blob + D.o_ar;
    const T* Vt = D.blob + D.o_vt;
    const T* x = X + l * MP;
    T v;
    if (r < rl) {
      v = T(0);
      for (int c = 0; c < cl; ++c) v += AL[r * cl + c] * x[off + c];
    } else if (r >= m - rr) {
      const int rr0 = r - (m - rr);
      v = T(0);
      for (int c = 0; c < cr; ++c) v += AR[rr0 * cr + c] * x[D.mo - rr + c];
    } else if (r < D.wk0) {
      v = x[r];
    } else if (r >= D.wk1 + D.rk) {
      v = x[r - D.rk];
    } else {   // E on the knot window
      const int nkw = D.wk1 - D.wk0;
      const T* EW = D.blob + D.o_ew + (r - D.wk0) * nkw;
      v = T(0);
      for (int c = 0; c < nkw; ++c) v += EW[c] * x[D.wk0 + c];
    }
    if (r < D.wl || r >= D.wr || (r >= D.kw0 && r < D.kw1)) {
      const T* yo = YO + l * 8;
      for (int q = 0; q < D.n_out; ++q) v += Vt[q * m + r] * yo[q];
    }
    return v;
  }
};

template <typename T, int L, class C>
__device__ __forceinline__ GTile<T, L, C> gen_tile(char* smem, const GLds& ly, int m) {
  GTile<T, L, C> g;
  g.tw = reinterpret_cast<cpx<T>*>(smem + ly.tw);
  g.X = reinterpret_cast<T*>(smem + ly.x);
  g.F = reinterpret_cast<cpx<T>*>(smem + ly.f);
  g.GB = reinterpret_cast<T*>(smem + ly.gb);
  g.YO = reinterpret_cast<T*>(smem + ly.yo);
  g.KB = reinterpret_cast<T*>(smem + ly.kb);
  g.LO = reinterpret_cast<const T*>(smem + ly.lo);
  g.SO = reinterpret_cast<const T*>(smem + ly.so);
  g.MP = m | 1;
  return g;
}

template <typename Tin, typename Tout, typename T, int MODE, int L>
__global__ void __launch_bounds__((GCfg<T, L>::NTH))
gen_line_pass(const Tin* __restrict__ in, Tout* __restrict__ out, GPassArgs<T> a) {
  using C = GCfg<T, L>;
  constexpr int TW = C::TW, NTH = C::NTH;
  extern __shared__ __align__(16) char smem[];
  const GDirDev<T>& D = a.dir;
  const int m = D.m, nr = D.n_reg, no = D.n_out;
  const int MP = m | 1;
  const GLds ly = gen_lds<T, L>(m);
  const GTile<T, L, C> G = gen_tile<T, L, C>(smem, ly, m);
  T* X = G.X;
  int* LB = reinterpret_cast<int*>(smem + ly.lb);
  T* LO = reinterpret_cast<T*>(smem + ly.lo);
  T* SO = reinterpret_cast<T*>(smem + ly.so);
  const int tid = threadIdx.x;

  const int b = xcd_linear(blockIdx.x, gridDim.x);
  const int rhs = b / a.tpr, tile = b - rhs * a.tpr;
  if (a.active && a.active[(size_t)rhs * a.astride] == 0.0) return;
  const int q0 = tile * TW;
  const Tin* src = in + (size_t)rhs * a.N;
  Tout* dst = out + (size_t)rhs * a.N;

  {
    const cpx<T>* g = reinterpret_cast<const cpx<T>*>(D.blob + D.o_tw);
    for (int k = tid; k < L; k += NTH) G.tw[k] = g[k];
  }
  if (tid < TW) {
    int i1, i2;
    LB[tid] = gen_line(a, q0 + tid, i1, i2);
    if constexpr (MODE == PASS_MID) {
      T lo = a.lam1[i1], so = a.s1[i1];
      if (a.lam2) {
        lo += a.lam2[i2];
        so *= a.s2[i2];
      }
      LO[tid] = lo;
      SO[tid] = so;
    }
  }
  __syncthreads();

  // ---- load the tile: X[l][i] = line l, entry i ----
  if (a.S == 1) {
    const int nl = min(TW, a.lpr - q0);
    const size_t base = (size_t)q0 * m;
    for (int e = tid; e < TW * m; e += NTH) {
      const int l = e / m;
      X[l * MP + (e - l * m)] = l < nl ? (T)src[base + e] : T(0);
    }
  } else {
    for (int e = tid; e < TW * m; e += NTH) {
      const int l = e & (TW - 1), i = e / TW;
      const int bl = LB[l];
      X[l * MP + i] = bl >= 0 ? (T)src[(size_t)bl + (size_t)i * a.S] : T(0);
    }
  }
  __syncthreads();

  if constexpr (MODE == PASS_FWD) {
    G.template forward<false>(D);
    // ---- store y = [y_reg; y_out] ----
    if (a.S == 1) {
      const int nl = min(TW, a.lpr - q0);
      const size_t base = (size_t)q0 * m;
      for (int e = tid; e < nl * m; e += NTH) {
        const int l = e / m, i = e - l * m;
        dst[base + e] = (Tout)G.spectral(D, l, i);
      }
    } else {
      for (int e = tid; e < TW * m; e += NTH) {
        const int l = e & (TW - 1), i = e / TW;
        const int bl = LB[l];
        if (bl >= 0) dst[(size_t)bl + (size_t)i * a.S] = (Tout)G.spectral(D, l, i);
      }
    }
    return;
  } else {
    if constexpr (MODE == PASS_MID) {
      G.template forward<true>(D);
    } else {
      // outlier coefficients of the spectral input
      for (int w = tid; w < TW * no; w += NTH) {
        const int l = w & (TW - 1), q = w / TW;
        G.YO[l * 8 + q] = X[l * MP + nr + q];
      }
      __syncthreads();
    }
    G.backward(D);
    // ---- x = V_reg c + Vt^T y_out, stored ----
    if (a.S == 1) {
      const int nl = min(TW, a.lpr - q0);
      const size_t base = (size_t)q0 * m;
      for (int e = tid; e < nl * m; e += NTH) {
        const int l = e / m, r = e - l * m;
        dst[base + e] = (Tout)G.value(D, l, r);
      }
    } else {
      for (int e = tid; e < TW * m; e += NTH) {
        const int l = e & (TW - 1), r = e / TW;
        const int bl = LB[l];
        if (bl >= 0) dst[(size_t)bl + (size_t)r * a.S] = (Tout)G.value(D, l, r);
      }
    }
  }
}

// device view of one direction's tables
template <typename T>
GDirDev<T> gen_dir_dev(const Plan& P, const GDir& G) {
  const bool f64 = sizeof(T) == 8;
  GDirDev<T> d;
  d.blob = (const T*)(P.d_tables + (f64 ? G.blob64 : G.blob32));
  d.o_tw = G.o_tw; d.o_tf = G.o_tf; d.o_al = G.o_al; d.o_ar = G.o_ar;
  d.o_vt = G.o_vt; d.o_lam = G.o_lam; d.o_s = G.o_s;
  d.m = G.m; d.n_reg = G.n_reg; d.n_out = G.n_out;
  d.rl = G.rl; d.cl = G.cl; d.rr = G.rr; d.cr = G.cr;
  d.mir_f = G.tau2;
  d.mir_b = G.sig2;
  d.wl = f64 ? G.win64[0] : G.win32[0];
  d.wr = f64 ? G.win64[1] : G.win32[1];
  d.rk = G.rk;
  d.wk0 = G.rk ? G.wk0 : (1 << 30);
  d.wk1 = G.rk ? G.wk1 : (1 << 30);
  d.o_ew = G.o_ew;
  d.kw0 = f64 ? G.kwin64[0] : G.kwin32[0];
  d.kw1 = f64 ? G.kwin64[1] : G.kwin32[1];
  d.mo = G.mo;
  d.gb = G.generic ? 1 : 0;
  d.bl = G.bl;
  d.bu = G.bu;
  d.o_lb = G.o_lb;
  d.o_ub = G.o_ub;
  return d;
}

// launch of one pass (host side); the plan's direction `axis` (1-based)
template <typename Tin, typename Tout, typename T, int MODE, int L>
hipError_t gen_launch(const Plan& P, int axis, const void* in, void* out, int nrhs,
                      const double* active, int astride, hipStream_t s) {
  using C = GCfg<T, L>;
  const GDir& G = P.dirs[axis - 1];
  if (G.L != L || G.n_out > 8 || G.cl + G.cr > 8 || (G.rk && G.wk1 - G.wk0 > 16))
    return hipErrorInvalidValue;
  const bool f64 = sizeof(T) == 8;
  GPassArgs<T> a;
  const char* tb = P.d_tables;
  auto blob_of = [&](const GDir& g) { return (const T*)(tb + (f64 ? g.blob64 : g.blob32)); };
  a.dir = gen_dir_dev<T>(P, G);
  int S = 1;
  for (int k = 0; k < axis - 1; ++k) S *= P.dirs[k].m;
  a.S = S;
  a.m1 = P.dirs[0].m;
  a.N = (int)P.N;
  if (S == 1) {
    a.mr = a.m1;
    a.sm = 1;
    a.lpr = (int)(P.N / G.m);
  } else {
    a.mr = a.m1 + (a.m1 & 1);
    a.sm = S / a.m1;
    a.lpr = (int)(P.N / G.m / a.m1) * a.mr;
  }
  a.tpr = (a.lpr + C::TW - 1) / C::TW;
  a.lam1 = a.s1 = a.lam2 = a.s2 = nullptr;
  if (MODE == PASS_MID) {
    const GDir& g1 = P.dirs[0];
    a.lam1 = blob_of(g1) + g1.o_lam;
    a.s1 = blob_of(g1) + g1.o_s;
    if (P.d == 3) {
      const GDir& g2 = P.dirs[1];
      a.lam2 = blob_of(g2) + g2.o_lam;
      a.s2 = blob_of(g2) + g2.o_s;
    }
  }
  a.active = active;
  a.astride = astride;
  const GLds ly = gen_lds<T, L>(G.m);
  if (ly.total > 160 * 1024) return hipErrorInvalidValue;   // beyond a workgroup's LDS
  static bool attr = false;
  if (ly.total > 65536 && !attr) {
    hipError_t e = hipFuncSetAttribute((const void*)gen_line_pass<Tin, Tout, T, MODE, L>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((gen_line_pass<Tin, Tout, T, MODE, L>), dim3((unsigned)(a.tpr * nrhs)),
                     dim3(C::NTH), ly.total, s, (const Tin*)in, (Tout*)out, a);
  return hipGetLastError();
}

// element types of one pass for one FFT length (instantiated per length)
template <int L>
hipError_t gen_pass_len(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                        void* out, int nrhs, const double* a, int as, hipStream_t s) {
  if (P.prec == IFFD_PREC_F64) {
    if (tin != ELEM_F64 || tout != ELEM_F64) return hipErrorInvalidValue;
    if (mode == PASS_FWD) return gen_launch<double, double, double, PASS_FWD, L>(P, axis, in, out, nrhs, a, as, s);
    if (mode == PASS_MID) return gen_launch<double, double, double, PASS_MID, L>(P, axis, in, out, nrhs, a, as, s);
    return gen_launch<double, double, double, PASS_BWD, L>(P, axis, in, out, nrhs, a, as, s);
  }
  if (mode == PASS_FWD) {
    if (tin == ELEM_F64 && tout == ELEM_F32 && P.first64)
      return gen_launch<double, float, double, PASS_FWD, L>(P, axis, in, out, nrhs, a, as, s);
    if (tin == ELEM_F64 && tout == ELEM_F32)
      return gen_launch<double, float, float, PASS_FWD, L>(P, axis, in, out, nrhs, a, as, s);
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return gen_launch<float, float, float, PASS_FWD, L>(P, axis, in, out, nrhs, a, as, s);
  } else if (mode == PASS_BWD) {
    if (tin == ELEM_F32 && tout == ELEM_F64)
      return gen_launch<float, double, float, PASS_BWD, L>(P, axis, in, out, nrhs, a, as, s);
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return gen_launch<float, float, float, PASS_BWD, L>(P, axis, in, out, nrhs, a, as, s);
  } else {
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return gen_launch<float, float, float, PASS_MID, L>(P, axis, in, out, nrhs, a, as, s);
  }
  return hipErrorInvalidValue;
}

#define IFFD_GEN_PASS_LEN(L)                                                                  \
  hipError_t gen_pass_len<L>(const Plan&, int, int, int, const void*, int, void*, int,        \
                             const double*, int, hipStream_t)


}  // namespace iffd
