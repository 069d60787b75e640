#pragma once
// IFFD line passes on gfx950 (kernel templates; instantiated per FFT length
// in apply_l*.hip, dispatched in apply.hip).
//
// The preconditioner of eq:preconditioner is applied mode-wise: for every
// direction k, each line of the coefficient tensor along k is transformed by
// Qt_k^T (forward), the tensor is divided by the Kronecker sum of the
// eigenvalues, and every line is transformed back by Qt_k (backward).  With
// Qt = [V_reg U Dt^{-1}, V_out Q_out] (Sections 4 and 6) one line transform is
//   forward   y_reg = U^T fold(x),          y_out = Vt x
//   backward  x = unfold(U y_reg) + Vt^T y_out
// where fold = V_reg^T (the p-1 boundary entries at each end collapse to
// floor(p/2) values through the special-basis blocks, interior entries pass
// through), unfold = V_reg, U is the sine matrix of Table 1 (DST-I for odd p,
// DST-II / DST-III for even p) and Vt = (V_out Q_out)^T is the dense
// n_out x m outlier block.  The Dt^{-1} factors of both sides are folded into
// the diagonal scaling: z_hat = y * prod_k s_k / sum_k lam_k with
// s = Dt^{-2} on regular modes and 1 on outliers.
//
// Sine transforms by FFT: two real lines a, b are packed as a + i b into one
// complex FFT.  Where n is a supported FFT length (n >= 16) the FFT has length
// L = n (PK_ODD_N: DST-I by a pre-twist, the sine part of the spectrum and
// prefix sums of its cosine part, see dst1n; PK_EVEN_N: DST-II / DST-III by a
// reordering and a quarter-wave twiddle).  For n = 8, 12 it has length L = 2n
// and runs on an odd extension:
//   DST-I  (n-1 values g):  z = [0, g, 0, -reverse(g)],  X_a = -Im C / 2,
//          X_b = Re C / 2 at indices 1..n-1;
//   DST-II (n values):      z = [g, -reverse(g)], W = e^{-i pi k/(2n)} C,
//          X_a = -Im W / 2, X_b = Re W / 2 at 1..n;
//   DST-III (n values c, full weight on c_n): with wbar_j = c_a,j - i c_b,j,
//          z_j = conj(t_j) wbar_j (0<j<n), z_n = 2i wbar_n,
//          z_{2n-j} = -t_j wbar_j, t_j = e^{-i pi j/(2n)};
//          x_a = -Im C / 2, x_b = -Re C / 2 at 1..n.
//
// One workgroup owns a tile of TW lines of one right-hand side (pairs never
// straddle two right-hand sides, so a result does not depend on the batch it
// is computed in).  The tile is staged through LDS with coalesced loads (lines
// along direction 1 are contiguous; lines along a strided direction are taken
// TW at a time from consecutive positions of the faster directions, so each
// row of the tile is one contiguous run), transformed in registers and LDS,
// and written back the same way.  Passes along strided directions work in
// place.
#include "fft_device.h"
#include "launch.h"

namespace iffd {

enum { PK_ODD = 0, PK_EVEN_2N = 1, PK_EVEN_N = 2, PK_ODD_N = 3 };

template <typename T>
struct Tabs {
  const T* blob;  // twl | Vt | V0 | V1 | sn | twp | lam | s, element offsets below
  int o_twl, o_twp, o_vt, o_v0, o_v1, o_lam, o_s, len;
  int o_sn;
  int nch;  // 16-byte chunks covering the staged prefix (the blob is padded)
};

struct Geom {
  int m, n, p, n_reg, n_out, half, nbd, c0;
  int S;       // element stride along the axis
  int lpr;     // lines per right-hand side (padded line space for S > 1, see line_at)
  int mr;      // S > 1: lines per row of the padded line space (m, or m + 1 for odd m)
  int sm;      // S > 1: S / m
  int tpr;     // tiles per right-hand side
  int N;       // elements per right-hand side
  int d;
  int tpd_log;  // log2 of the threads per outlier dot
  int wl, wr;   // outlier rows Vt[q][j] are used for j < wl and j >= wr only: beyond
                // these windows at the two ends every entry is below the working
                // precision relative to the largest (the outlier basis decays
                // geometrically away from the ends)
  const double* dr;  // fused dr . out partials (backward pass along direction 1), or null
  const double* fq;  // fused in <- in - alpha q (forward pass along direction 1), or null
  const double* falpha;
  double* fr;        // = in, written back
  double* dpart;     // per-tile partials of either fused step
  int dnpart;
  const double* active;  // per-RHS flags or null
  int active_stride;
};

// Tile shape of variant V: E transform elements per thread (variant 2 takes
// variant 1's FFT shape, variant 3 has 4, variant 4 takes variant 3's), FPW
// line pairs per workgroup (variants 2 and 4 half as many, for problems too
// small to fill the chip with full tiles).
template <typename T, int L, int V>
struct Cfg {
  static constexpr int E = FftPlan<L, V>::E;
  static constexpr int NT = L / E;
  static constexpr int CAP = (sizeof(T) == 8 ? 128 : 256) / ((V == 2 || V == 4) ? 2 * NT : NT);
  static constexpr int FPW = CAP >= 32 ? 32 : (CAP < 1 ? 1 : CAP);
  static constexpr int TW = 2 * FPW;
  static constexpr int NTH = FPW * NT;
};

__host__ __device__ inline size_t up16(size_t x) { return (x + 15) & ~(size_t)15; }

struct LdsMap {
  size_t x, blob, g, co, lo, so, lb, dm, total;
};

template <typename T, int L, int V>
__host__ __device__ inline LdsMap lds_map(int m, int n, int n_out, int half, int p, int blen) {
  using C = Cfg<T, L, V>;
  const int MP = m | 1;
  size_t xs = (size_t)C::TW * MP;
  size_t fs = (size_t)C::FPW * fft_region<L>() * 2;
  LdsMap r;
  size_t off = 0;
  r.x = off;   off = up16(off + sizeof(T) * (xs > fs ? xs : fs));
  r.blob = off; off = up16(off + sizeof(T) * blen);
  r.g = off;   off = up16(off + sizeof(T) * C::TW * 2 * (p > 1 ? p - 1 : 1));
  r.co = off;  off = up16(off + sizeof(T) * C::TW * (n_out > 0 ? n_out : 1));
  r.lo = off;  off = up16(off + sizeof(T) * C::TW);
  r.so = off;  off = up16(off + sizeof(T) * C::TW);
  r.lb = off;  off = up16(off + sizeof(int) * C::TW);
  r.dm = off;  off = up16(off + sizeof(T) * 2 * C::NTH);
  r.total = off;
  return r;
}

// copy a small table from global memory to LDS with several loads in flight
template <typename T>
__device__ __forceinline__ void to_lds(T* dst, const T* src, int count, int t, int nth) {
  for (int e0 = t; e0 < count; e0 += 4 * nth) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * nth;
      v[u] = e < count ? src[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * nth;
      if (e < count) dst[e] = v[u];
    }
  }
}

template <int V>
constexpr int ilog2() { return V <= 1 ? 0 : 1 + ilog2<V / 2>(); }

// Line q of a pass along a strided direction (S > 1).  Its lines are indexed
// by (outer, i2, a): a the index along direction 1 (fastest), i2 along the
// directions between 1 and the pass's own, outer along the slower ones.  The
// line space is padded so that every run of lines with the same (outer, i2)
// has an even length mr (a dummy line a = m when m is odd): the two lines of
// an FFT pair (2f, 2f+1) then never straddle two runs.  A straddling pair
// would share one complex FFT between the last line of a run (for a spectral
// direction 1 an outlier coefficient, often near zero) and the first line of
// the next (the smoothest mode, the largest), and FP32 rounding of the large
// line would leak into the small one.  Returns whether q is a real line; base
// is its first entry, inner its index in [0, S).
__device__ __forceinline__ bool line_at(const Geom& g, int q, int& base, int& inner) {
  const int a = q % g.mr, rest = q / g.mr;
  const int i2 = rest % g.sm, outer = rest / g.sm;
  inner = i2 * g.m + a;
  base = outer * g.m * g.S + inner;
  return a < g.m;
}

// Tile layout in LDS: row l of X holds line l (m entries, row stride MP).
// The folded sequence g = V_reg^T x (n_reg entries) is kept in place at
// X[l][c0 + idx], c0 = p-1-floor(p/2): interior entries of x already sit
// there, and the floor(p/2) folded values of each end land inside that end's
// p-1 boundary slots.  So every FFT input is one branch-free LDS read.  The
// same holds backwards: U c is written to X[l][c0 + idx] and the p-1 boundary
// values of each end are then unfolded in place.
// PK: the sine transform route, fixed per kernel: PK_ODD (DST-I, L = 2n),
// PK_EVEN_2N (DST-II / DST-III, L = 2n), PK_EVEN_N (DST-II / DST-III, L = n),
// PK_ODD_N (DST-I, L = n).
// UPD: the forward pass of FP64 input along direction 1 also applies the PCG
// residual update r <- r - alpha q to its input (g.fq, g.falpha, g.fr, partial
// sums of the updated r^2 in g.dpart); a kernel of its own (line_pass_upd), so
// that the plain pass keeps its registers.
template <typename Tin, typename Tout, typename T, int MODE, int L, int V, int PK, bool UPD>
__device__ __forceinline__ void line_pass_body(const Tin* __restrict__ in, Tout* __restrict__ out,
                                               const Geom& g, const Tabs<T>& tb) {
  using C = Cfg<T, L, V>;
  constexpr int TW = C::TW, NTH = C::NTH, NT = C::NT;
  constexpr int LTW = ilog2<TW>();
  // contiguous lines (direction 1): RW lanes walk one line, NG lines at once
  constexpr int RW = NTH < 64 ? NTH : 64;
  constexpr int NG = NTH / RW;
  // m = n + p - 2 <= n + 6, with n = L (length-n routes) or L / 2
  constexpr int MMAX = (PK == PK_ODD || PK == PK_EVEN_2N) ? L / 2 + 6 : L + 6;
  constexpr int UMAX = (MMAX + RW - 1) / RW;   // row chunks of a stored contiguous line
  constexpr int CH = 8;                       // loads in flight per thread (generic path)
  // m = n + p - 2 <= n + 6; the loads of a tile row go in batches of MB entries,
  // one batch when L = 2n, two when L = n (even p, length-n transforms)
  constexpr int MB = L / 2 + 6;
  constexpr int UMX = (MB + RW - 1) / RW;     // row chunks of a contiguous line per batch
  constexpr int LPT = (TW + NG - 1) / NG;     // contiguous lines per thread
  extern __shared__ __align__(16) char smem[];
  const int m = g.m, n = g.n, n_reg = g.n_reg, n_out = g.n_out, half = g.half;
  const int MP = m | 1;
  const LdsMap mp = lds_map<T, L, V>(m, n, n_out, half, g.p, tb.len);
  T* X = reinterpret_cast<T*>(smem + mp.x);
  cpx<T>* F = reinterpret_cast<cpx<T>*>(smem + mp.x);  // aliases X
  T* BL = reinterpret_cast<T*>(smem + mp.blob);
  cpx<T>* twl = reinterpret_cast<cpx<T>*>(BL + tb.o_twl);
  cpx<T>* twp = reinterpret_cast<cpx<T>*>(BL + tb.o_twp);
  const T* SN = BL + tb.o_sn;   // sin(pi h / n): contiguous, so the pre-twist reads hit distinct banks
  T* GB = reinterpret_cast<T*>(smem + mp.g);  // per-line boundary values
  T* CO = reinterpret_cast<T*>(smem + mp.co);
  T* LO = reinterpret_cast<T*>(smem + mp.lo);
  T* SO = reinterpret_cast<T*>(smem + mp.so);
  int* LB = reinterpret_cast<int*>(smem + mp.lb);
  T* VT = BL + tb.o_vt;
  T* V0 = BL + tb.o_v0;
  T* V1 = BL + tb.o_v1;
  T* LAM = BL + tb.o_lam;
  T* SS = BL + tb.o_s;
  const int nbd = g.nbd;
  T* DM = reinterpret_cast<T*>(smem + mp.dm);  // sink for discarded FFT outputs
  const int GW = 2 * nbd;

  const int t = threadIdx.x;
  // XCD-aware order: tiles that share cache lines (neighbouring lines of a
  // strided pass) meet in one L2
  T* sink = DM + 2 * t;  // per-thread slot for discarded values
  const int lin = xcd_linear(blockIdx.x, gridDim.x);
  const int rhs = lin / g.tpr;
  const int tile = lin - rhs * g.tpr;
  if (g.active && g.active[(size_t)rhs * g.active_stride] == 0.0) return;
  const int q0 = tile * TW;
  const int nv = min(TW, g.lpr - q0);
  const int S = g.S;
  const int c0 = g.c0;
  constexpr bool odd = PK == PK_ODD || PK == PK_ODD_N;
  constexpr int MAXO = 6;   // n_out <= 6 (p <= 8)

  // ---- tables, twiddles and per-line data into LDS ---------------------------
  if constexpr (NTH % TW != 0) {   // line bases for the generic strided path
    if (S > 1)
      for (int l = t; l < TW; l += NTH) {
        int base, inner;
        const bool real = line_at(g, q0 + l, base, inner);
        LB[l] = (l < nv && real) ? rhs * g.N + base : -1;
      }
  }
  // issue the table loads (16-byte chunks) now; they land in LDS after the
  // tile loads are issued
  constexpr int BCH = 4;
  const auto trs = buf_rsrc(tb.blob, (unsigned)tb.nch * 16u);
  u32x4 bv[BCH];
#pragma unroll
  for (int u = 0; u < BCH; ++u) bv[u] = buf_ld16(trs, (unsigned)(t + u * NTH) * 16u);

  // ---- load the tile: X[l][j] = in(line l, position j); missing lines = 0 --
  // (buffer loads: entries past the tile or the tensor read as 0)
  // the fused residual update (forward pass of FP64 input along direction 1)
  constexpr bool FU = UPD && MODE == PASS_FWD && sizeof(Tin) == 8;
  double racc = 0.0;   // this thread's share of the updated r^2
  if (S == 1) {
    // every load of a batch is issued before its first LDS write
    const auto rs = buf_rsrc(in + (size_t)rhs * g.N + (size_t)q0 * m,
                             (unsigned)(nv * m * (int)sizeof(Tin)));
    const int lane = t % RW, grp = t / RW;
    const unsigned vo = (unsigned)(grp * m + lane) * sizeof(Tin);
    const unsigned frec = FU ? (unsigned)(nv * m * 8) : 0u;
    const size_t fo = (size_t)rhs * g.N + (size_t)q0 * m;
    const auto qs = buf_rsrc(FU ? g.fq + fo : (const double*)in, frec);
    const auto rw = buf_rsrc(FU ? g.fr + fo : (const double*)in, frec);
    const double alpha = FU ? g.falpha[(size_t)rhs * g.active_stride] : 0.0;
    for (int jb = 0; jb < m; jb += UMX * RW) {
      Tin v[LPT][UMX];
#pragma unroll
      for (int a = 0; a < LPT; ++a)
#pragma unroll
        for (int u = 0; u < UMX; ++u)
          v[a][u] = buf_ld<Tin>(rs, vo + (unsigned)((a * NG * m + jb + RW * u) * (int)sizeof(Tin)));
      if constexpr (FU) {
        // r <- r - alpha q, written back once per entry (line l < nv, j < m)
        double qv[LPT][UMX];
#pragma unroll
        for (int a = 0; a < LPT; ++a)
#pragma unroll
          for (int u = 0; u < UMX; ++u)
            qv[a][u] = buf_ld<double>(qs, vo + (unsigned)((a * NG * m + jb + RW * u) * 8));
#pragma unroll
        for (int a = 0; a < LPT; ++a)
#pragma unroll
          for (int u = 0; u < UMX; ++u) {
            const int j = jb + lane + RW * u, l = grp + a * NG;
            const bool own = j < m && l < nv;
            const double rv = (double)v[a][u] - alpha * qv[a][u];
            v[a][u] = (Tin)rv;
            buf_st<double>(rv, rw, own ? vo + (unsigned)((a * NG * m + jb + RW * u) * 8) : BUF_OOB);
            racc += own ? rv * rv : 0.0;
          }
      }
      // entries past the row go to a sink (a select, not a branch, so the
      // compiler keeps every load of the batch ahead of the first write)
#pragma unroll
      for (int u = 0; u < UMX; ++u) {
        const int j = jb + lane + RW * u;
#pragma unroll
        for (int a = 0; a < LPT; ++a) {
          const int l = grp + a * NG;
          *((j < m && l < TW) ? X + l * MP + j : sink) = (T)v[a][u];
        }
      }
    }
  } else if constexpr (NTH % TW == 0) {
    // every thread keeps one line l = t mod TW and takes its rows j0, j0 + JS, ..
    // (rows of the tile are runs of TW consecutive entries of the tensor)
    constexpr int JS = NTH / TW;
    const int l = t & (TW - 1), j0 = t >> LTW;
    int base, inner;
    const bool real = line_at(g, q0 + l, base, inner) && l < nv;
    const auto rs = buf_rsrc(in + (size_t)rhs * g.N, (unsigned)(g.N * (int)sizeof(Tin)));
    const unsigned vo = real ? (unsigned)(base + j0 * S) * sizeof(Tin) : BUF_OOB;
    T* dst = X + l * MP + j0;
    const int cnt = j0 < m ? (m - j0 + JS - 1) / JS : 0;
    const int step = JS * S * (int)sizeof(Tin);
    constexpr int KMAX = (MB + JS - 1) / JS;   // rows per thread and batch, all in flight
    const int kend = (m + JS - 1) / JS;        // the most rows any thread has
    for (int kb = 0; kb < kend; kb += KMAX) {
      Tin v[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) v[k] = buf_ld<Tin>(rs, vo + (unsigned)((kb + k) * step));
#pragma unroll
      for (int k = 0; k < KMAX; ++k) *(kb + k < cnt ? dst + (kb + k) * JS : sink) = (T)v[k];
    }
  } else {
    __syncthreads();  // LB
    const int cnt = TW * m;
    for (int e0 = t; e0 < cnt; e0 += NTH * CH) {
      Tin v[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = e0 + u * NTH;
        const int l = e & (TW - 1), j = e >> LTW;
        v[u] = (e < cnt && l < nv && LB[l] >= 0) ? in[LB[l] + j * S] : Tin(0);
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = e0 + u * NTH;
        const int l = e & (TW - 1), j = e >> LTW;
        if (e < cnt) X[l * MP + j] = (T)v[u];
      }
    }
  }
  {
    u32x4* B4 = reinterpret_cast<u32x4*>(BL);
#pragma unroll
    for (int u = 0; u < BCH; ++u)
      if (t + u * NTH < tb.nch) B4[t + u * NTH] = bv[u];
    for (int c = t + BCH * NTH; c < tb.nch; c += NTH) B4[c] = buf_ld16(trs, (unsigned)c * 16u);
  }
  __syncthreads();
  if constexpr (FU) {   // fixed-order sum of the updated r^2 over the workgroup
    double* red = reinterpret_cast<double*>(DM);   // NTH doubles fit in DM
    if constexpr (NTH % 64 == 0) {
      for (int o = 32; o > 0; o >>= 1) racc += __shfl_xor(racc, o);
      if ((t & 63) == 0) red[t >> 6] = racc;
    } else {
      red[t] = racc;   // a partial wave: no shuffles
    }
    __syncthreads();
    if (t == 0) {
      constexpr int NR = NTH % 64 == 0 ? NTH / 64 : NTH;
      double sum = 0.0;
      for (int k = 0; k < NR; ++k) sum += red[k];
      g.dpart[(size_t)rhs * g.dnpart + tile] = sum;
    }
    __syncthreads();   // DM takes discarded values again below
  }
  if (MODE == PASS_MID) {
    // spectral indices of each line in the other directions (the middle pass
    // runs along the last direction, so the inner index holds them all);
    // read after the next barrier, by the forward transform's output stage
    for (int l = t; l < TW; l += NTH) {
      T lo = T(0), so = T(1);
      int base, i;
      if (l < nv && line_at(g, q0 + l, base, i)) {
        const int j1 = i % m, j2 = i / m;
        lo = LAM[j1];
        so = SS[j1];
        if (g.d == 3) { lo += LAM[j2]; so *= SS[j2]; }
      }
      LO[l] = lo;
      SO[l] = so;
    }
  }

  // Kronecker-sum scaling of spectral entry j of line l (middle pass)
  auto fac = [&](int l, int j) -> T {
    if constexpr (sizeof(T) == 4)   // hardware reciprocal (1 ulp) for the FP32 apply
      return SS[j] * SO[l] * __builtin_amdgcn_rcpf(LAM[j] + LO[l]);
    else
      return SS[j] * SO[l] / (LAM[j] + LO[l]);
  };

  const int f = t / NT, tid = t - (t / NT) * NT;
  const int la = 2 * f, lb = 2 * f + 1;
  cpx<T>* buf = F + f * fft_region<L>();
  T* Xa = X + la * MP;
  T* Xb = X + lb * MP;
  T* Ga = Xa + c0;  // g (or U c) of line a
  T* Gb = Xb + c0;
  T* dmy = DM + 2 * t;

  // DST-I of the two lines of this pair by one length-n FFT (odd p, L = n).
  // With v_0 = v_n = 0, S_j = sin(pi j / n) and
  //   y_j = S_j (v_j + v_{n-j}) + (v_j - v_{n-j}) / 2,
  // the transform Y_k = sum_j y_j e^{-2 pi i jk/n} = A_k - i B_k gives the sine
  // coefficients F_k = sum_j v_j sin(pi jk/n) as F_2k = B_k and
  // F_2k+1 = F_2k-1 + A_k with F_-1 = -F_1, i.e. F_2k+1 = A_0 + .. + A_k - A_0/2
  // (the sine part of y is odd about n/2 and the difference part even, and
  // 2 sin(pi j/n) cos(2 pi jk/n) = sin(pi j(2k+1)/n) - sin(pi j(2k-1)/n)).
  // The two lines go in as y_a + i y_b; thread tid of the pair then takes
  // k = tid + NT c, and the prefix sums of A run as cross-lane scans over the
  // pair's NT lanes, block by block.
  // Input v_j at sa/sb[j-1], output F_k at da/db[k-1] (times the Kronecker-sum
  // factor when SCALE).
  auto dst1n = [&](const T* sa, const T* sb, T* da, T* db, auto scale_tag) {
    constexpr bool SCALE = decltype(scale_tag)::value;
    constexpr int N = L;
    auto ldo = [&](int j, bool, bool j0, bool) -> cpx<T> {
      const int jj = j0 ? 1 : j;   // y_0 = 0; keeps the reads in range
      const T va = sa[jj - 1], vb = sb[jj - 1];
      const T wa = sa[N - jj - 1], wb = sb[N - jj - 1];
      const int h = jj <= N / 2 ? jj : N - jj;
      const T sj = SN[h];
      const T ya = sj * (va + wa) + T(0.5) * (va - wa);
      const T yb = sj * (vb + wb) + T(0.5) * (vb - wb);
      return j0 ? cpx<T>{T(0), T(0)} : cpx<T>{ya, yb};
    };
    auto sto = [&](int k, cpx<T> v) { buf[fpad<L>(k)] = v; };
    fft_forward<T, L, V>(buf, tid, twl, ldo, sto);
    __syncthreads();
    // thread tid takes k = tid + NT c (c < CK): the reads of W_k and W_{n-k}
    // and the writes below run over consecutive k across lanes; the prefix
    // sums of A run as a cross-lane scan per block of NT values plus the
    // running total of the blocks before
    constexpr int CK = N / (2 * NT);
    T fo_a[CK], fo_b[CK], fe_a[CK], fe_b[CK];   // F_2k+1 and F_2k of both lines
    T carry_a = T(0), carry_b = T(0), a0a = T(0), a0b = T(0);
#pragma unroll
    for (int c = 0; c < CK; ++c) {
      const int k = tid + NT * c;
      const cpx<T> wk = buf[fpad<L>(k)], wm = buf[fpad<L>(k == 0 ? 0 : N - k)];
      // line a: (W_k + conj W_{n-k}) / 2, line b: -i (W_k - conj W_{n-k}) / 2
      const T aa = T(0.5) * (wk.x + wm.x), ab = T(0.5) * (wk.y + wm.y);
      fe_a[c] = T(0.5) * (wm.y - wk.y);
      fe_b[c] = T(0.5) * (wk.x - wm.x);
      if (c == 0) {   // A_0 from the group's first lane
        a0a = __shfl(aa, 0, NT);
        a0b = __shfl(ab, 0, NT);
      }
      const T sa = group_inclusive_scan<NT>(aa, tid), sb = group_inclusive_scan<NT>(ab, tid);
      fo_a[c] = carry_a + sa;
      fo_b[c] = carry_b + sb;
      if (c + 1 < CK) {
        carry_a += __shfl(sa, NT - 1, NT);
        carry_b += __shfl(sb, NT - 1, NT);
      }
    }
    __syncthreads();   // every W is read before the rows (aliasing the regions) are written
    // one write instruction covers the odd coefficient of half the lanes and
    // the even one of the other half (positions 2k and 2k - 1), so a group's
    // lanes hit distinct banks
    const bool hi16 = (tid & 16) != 0;
#pragma unroll
    for (int c = 0; c < CK; ++c) {
      const int k = tid + NT * c;
      T fa = fo_a[c] - T(0.5) * a0a, fb = fo_b[c] - T(0.5) * a0b;   // F_2k+1, position 2k
      T ga = fe_a[c], gb = fe_b[c];                                   // F_2k, position 2k-1
      if constexpr (SCALE) {
        fa *= fac(la, 2 * k); fb *= fac(lb, 2 * k);
        if (k >= 1) { ga *= fac(la, 2 * k - 1); gb *= fac(lb, 2 * k - 1); }
      }
      const bool ev = k >= 1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool odd_now = (h == 0) != hi16;
        const int pos = odd_now ? 2 * k : 2 * k - 1;
        const bool ok = odd_now || ev;
        *(ok ? da + pos : dmy) = odd_now ? fa : ga;
        *(ok ? db + pos : dmy + 1) = odd_now ? fb : gb;
      }
    }
  };

  if (MODE == PASS_FWD || MODE == PASS_MID) {
    // ---- outlier dots; boundary fold into the g slots ----------------------
    // 1 << tl threads per dot (chosen on the host) within one wave read the
    // window entries of their line from the tile in LDS and sum by shuffles,
    // so no partial crosses a wave (per-wave partials of a strided tile summed
    // across waves measured slower: that sum ran on a few lanes between two
    // barriers).  Every thread runs the same number of rounds so the shuffles
    // see all lanes; the dot runs over the window entries u < nw, entry
    // j = u (left) or u - wl + wr (right).
    if (n_out > 0) {
      const int tl = g.tpd_log, tpd = 1 << tl;
      const int ndots = TW * n_out;
      const int per = NTH >> tl;
      const int rounds = (ndots + per - 1) / per;
      const int sub = t & (tpd - 1);
      const int wl = g.wl, nw = g.wl + (m - g.wr), sh = g.wr - g.wl;
      for (int rd = 0; rd < rounds; ++rd) {
        const int di = (t >> tl) + rd * per;
        T acc = T(0);
        const int l = di & (TW - 1), q = di >> LTW;
        if (di < ndots) {
          const T* vr = VT + q * m;
          const T* xr = X + l * MP;
          // four independent partial sums keep several LDS reads in flight
          T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
          int u = sub;
          auto jx = [&](int uu) { return uu < wl ? uu : uu + sh; };
          for (; u + 3 * tpd < nw; u += 4 * tpd) {
            const int j_0 = jx(u), j_1 = jx(u + tpd), j_2 = jx(u + 2 * tpd), j_3 = jx(u + 3 * tpd);
            a0 += vr[j_0] * xr[j_0];
            a1 += vr[j_1] * xr[j_1];
            a2 += vr[j_2] * xr[j_2];
            a3 += vr[j_3] * xr[j_3];
          }
          for (; u < nw; u += tpd) {
            const int j_0 = jx(u);
            a0 += vr[j_0] * xr[j_0];
          }
          acc = (a0 + a1) + (a2 + a3);
        }
        for (int o = 1; o < tpd; o <<= 1) acc += __shfl_xor(acc, o);
        if (sub == 0 && di < ndots) CO[l * n_out + q] = acc;
      }
    }
    for (int e = t; e < TW * 2 * half; e += NTH) {
      const int l = e % TW, c = e / TW;
      T acc = T(0);
      if (c < half) {
        for (int r = 0; r < nbd; ++r) acc += V0[r * half + c] * X[l * MP + r];
      } else {
        for (int r = 0; r < nbd; ++r) acc += V1[r * half + (c - half)] * X[l * MP + m - nbd + r];
      }
      GB[l * GW + c] = acc;
    }
    __syncthreads();
    for (int e = t; e < TW * 2 * half; e += NTH) {
      const int l = e % TW, c = e / TW;
      const int pos = c < half ? c0 + c : m - nbd + (c - half);
      X[l * MP + pos] = GB[l * GW + c];
    }
    if (MODE == PASS_MID) {   // the outlier coefficients take the same scaling
      for (int e = t; e < TW * n_out; e += NTH) {
        const int l = e & (TW - 1), q = e >> LTW;
        CO[l * n_out + q] *= fac(l, n_reg + q);
      }
    }
    __syncthreads();

    // ---- forward transform: X[l][0..n_reg) = U^T g_l (scaled in the middle) --
    auto ld = [&](int k, bool lo, bool k0, bool kh) -> cpx<T> {
      int idx;
      if (odd) idx = lo ? k - 1 : 2 * n - k - 1;   // k = 0, n give 0 (below)
      else idx = lo ? k : 2 * n - 1 - k;
      idx = idx < 0 ? 0 : idx;
      T a = Ga[idx], b = Gb[idx];
      const bool zero = odd && (k0 || kh);
      a = zero ? T(0) : (lo ? a : -a);
      b = zero ? T(0) : (lo ? b : -b);
      return {a, b};
    };
    auto st = [&](int k, cpx<T> v) {
      const bool ok = k >= 1 && k <= n_reg;
      const int j = ok ? k - 1 : 0;
      if (!odd) v = c_mul(v, twp[k <= n ? k : n]);
      T a = T(-0.5) * v.y, b = T(0.5) * v.x;
      if (MODE == PASS_MID) {  // scaling fused into the transform output
        a *= fac(la, j);
        b *= fac(lb, j);
      }
      *(ok ? Xa + j : dmy) = a;
      *(ok ? Xb + j : dmy + 1) = b;
    };
    if constexpr (PK == PK_ODD_N) {
      dst1n(Ga, Gb, Xa, Xb, std::integral_constant<bool, MODE == PASS_MID>{});
      __syncthreads();
    } else if constexpr (PK != PK_EVEN_N) {
      fft_forward<T, L, V>(buf, tid, twl, ld, st);
      __syncthreads();
    } else {
      // even p with L = n: the length-n transform of the reordered sequence
      // v_i = g_2i, v_{n-1-i} = -g_{2i+1} (two lines packed as real and
      // imaginary parts) stays in this transform's LDS region in natural order;
      // the pair (W_k, W_{n-k}) then gives the coefficients n-k and k of both
      // lines: V = (W_k + conj W_{n-k})/2 for line a, -i (W_k - conj W_{n-k})/2
      // for line b, C(k) = Re(t_k V), C(n-k) = Re(t_{n-k} conj V), t = twp.
      constexpr int N = L;
      auto ldh = [&](int k, bool lo, bool, bool) -> cpx<T> {
        const int idx = lo ? 2 * k : 2 * N - 1 - 2 * k;
        const T a = Ga[idx], b = Gb[idx];
        return {lo ? a : -a, lo ? b : -b};
      };
      auto sth = [&](int k, cpx<T> v) { buf[fpad<L>(k)] = v; };
      fft_forward<T, L, V>(buf, tid, twl, ldh, sth);
      __syncthreads();
      constexpr int NP = (N / 2 + 1 + NT - 1) / NT;   // pairs per thread
      T ra[NP][2], rb[NP][2];
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int k = tid + NT * u;
        const int kk = k <= N / 2 ? k : 0;
        const cpx<T> wk = buf[fpad<L>(kk)], wm = buf[fpad<L>(kk == 0 ? 0 : N - kk)];
        const cpx<T> va = {T(0.5) * (wk.x + wm.x), T(0.5) * (wk.y - wm.y)};
        const cpx<T> vb = {T(0.5) * (wk.y + wm.y), T(-0.5) * (wk.x - wm.x)};
        const cpx<T> tk = twp[kk], tm = twp[N - kk];
        ra[u][0] = tk.x * va.x - tk.y * va.y;   // C_a(k)
        rb[u][0] = tk.x * vb.x - tk.y * vb.y;
        ra[u][1] = tm.x * va.x + tm.y * va.y;   // C_a(n-k)
        rb[u][1] = tm.x * vb.x + tm.y * vb.y;
      }
      __syncthreads();   // every W is read before the rows (aliasing the regions) are written
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        const int k = tid + NT * u;
        if (k <= N / 2) {
          // coefficient j = n - k at position n-k-1, coefficient k at position k-1
          const int p0 = N - k - 1;
          T a0 = ra[u][0], b0 = rb[u][0];
          if (MODE == PASS_MID) { a0 *= fac(la, p0); b0 *= fac(lb, p0); }
          Xa[p0] = a0;
          Xb[p0] = b0;
          if (k >= 1 && 2 * k < N) {
            const int p1 = k - 1;
            T a1 = ra[u][1], b1 = rb[u][1];
            if (MODE == PASS_MID) { a1 *= fac(la, p1); b1 *= fac(lb, p1); }
            Xa[p1] = a1;
            Xb[p1] = b1;
          }
        }
      }
      __syncthreads();
    }
    if (MODE == PASS_FWD) {
      for (int e = t; e < TW * n_out; e += NTH) {
        const int l = e & (TW - 1), q = e >> LTW;
        X[l * MP + n_reg + q] = CO[l * n_out + q];
      }
      __syncthreads();
    }
  } else {
    for (int e = t; e < TW * n_out; e += NTH) {
      const int l = e & (TW - 1), q = e >> LTW;
      CO[l * n_out + q] = X[l * MP + n_reg + q];
    }
  }

  if (MODE == PASS_BWD || MODE == PASS_MID) {
    // ---- backward transform: X[l][c0 + idx] = (U c_l)[idx] -------------------
    auto ld = [&](int k, bool lo, bool k0, bool kh) -> cpx<T> {
      if (odd) {
        int idx = lo ? k - 1 : 2 * n - k - 1;
        idx = idx < 0 ? 0 : idx;
        const bool zero = k0 || kh;
        const T a = Xa[idx], b = Xb[idx];
        return {zero ? T(0) : (lo ? a : -a), zero ? T(0) : (lo ? b : -b)};
      }
      // DST-III by the anti-Hermitian extension of wbar = c_a - i c_b
      const bool le = lo || kh;   // k <= n
      int j = le ? k : 2 * n - k;
      j = k0 ? 1 : j;
      const cpx<T> wb = {Xa[j - 1], -Xb[j - 1]};
      const cpx<T> tw = twp[j];
      cpx<T> z;
      if (le) {
        z = c_mul(wb, cpx<T>{tw.x, -tw.y});
        const T s2 = kh ? T(2) : T(1);
        z = {s2 * z.x, s2 * z.y};
      } else {
        const cpx<T> u = c_mul(wb, tw);
        z = {-u.x, -u.y};
      }
      return k0 ? cpx<T>{T(0), T(0)} : z;
    };
    auto st = [&](int k, cpx<T> v) {
      const bool ok = k >= 1 && k <= n_reg;
      const int j = ok ? k - 1 : 0;
      *(ok ? Ga + j : dmy) = T(-0.5) * v.y;
      *(ok ? Gb + j : dmy + 1) = odd ? T(0.5) * v.x : T(-0.5) * v.x;
    };
    if constexpr (PK == PK_ODD_N) {
      dst1n(Xa, Xb, Ga, Gb, std::integral_constant<bool, false>{});
    } else if constexpr (PK != PK_EVEN_N) {
      fft_forward<T, L, V>(buf, tid, twl, ld, st);
    } else {
      // even p with L = n: with d_k = c_{n-k} (d_n = 0), the Hermitian sequence
      // Z_0 = d_0, Z_k = t_k (d_k + i d_{n-k}) / 2 has a real transform v; two
      // lines packed as Z_a + i Z_b, and x_2i = v_i, x_{2i+1} = -v_{n-1-i}
      constexpr int N = L;
      auto ldh = [&](int k, bool, bool k0, bool) -> cpx<T> {
        const T ak = Xa[N - k - 1], bk = Xb[N - k - 1];
        const int km = k0 ? 0 : k - 1;
        const T am = k0 ? T(0) : Xa[km], bm = k0 ? T(0) : Xb[km];
        const cpx<T> tk = twp[k];
        const cpx<T> za = c_mul(tk, cpx<T>{ak, am}), zb = c_mul(tk, cpx<T>{bk, bm});
        const cpx<T> ya = k0 ? cpx<T>{ak, T(0)} : cpx<T>{T(0.5) * za.x, T(0.5) * za.y};
        const cpx<T> yb = k0 ? cpx<T>{bk, T(0)} : cpx<T>{T(0.5) * zb.x, T(0.5) * zb.y};
        return {ya.x - yb.y, ya.y + yb.x};
      };
      auto sth = [&](int k, cpx<T> v) {
        const bool lo = k < N / 2;
        const int idx = lo ? 2 * k : 2 * (N - 1 - k) + 1;
        Ga[idx] = lo ? v.x : -v.x;
        Gb[idx] = lo ? v.y : -v.y;
      };
      fft_forward<T, L, V>(buf, tid, twl, ldh, sth);
    }
    __syncthreads();
    // ---- unfold the ends in place: x = V_reg,0 g_left, V_reg,1 g_right --------
    for (int e = t; e < TW * 2 * nbd; e += NTH) {
      const int l = e % TW, r = e / TW;
      const T* gl = X + l * MP;
      T acc = T(0);
      if (r < nbd) {
        for (int c = 0; c < half; ++c) acc += V0[r * half + c] * gl[c0 + c];
      } else {
        const int rr = r - nbd;
        for (int c = 0; c < half; ++c) acc += V1[rr * half + c] * gl[m - nbd + c];
      }
      GB[l * GW + r] = acc;
    }
    __syncthreads();
    for (int e = t; e < TW * 2 * nbd; e += NTH) {
      const int l = e % TW, r = e / TW;
      const int pos = r < nbd ? r : m - nbd + (r - nbd);
      X[l * MP + pos] = GB[l * GW + r];
    }
    __syncthreads();
  }

  // ---- store: the tile row, plus the outlier block after the backward pass --
  // a line's outlier coefficients are held in registers (n_out <= MAXO)
  auto load_co = [&](int l, T* co) {
#pragma unroll
    for (int q = 0; q < MAXO; ++q) co[q] = (MODE != PASS_FWD && q < n_out) ? CO[l * n_out + q] : T(0);
  };
  auto value = [&](int l, int j, const T* co) -> T {
    T v = X[l * MP + j];
    if (MODE != PASS_FWD && (j < g.wl || j >= g.wr)) {
#pragma unroll
      for (int q = 0; q < MAXO; ++q)
        if (q < n_out) v += VT[q * m + j] * co[q];
    }
    return v;
  };
  if (S == 1) {
    const auto rs = buf_rsrc(out + (size_t)rhs * g.N + (size_t)q0 * m,
                             (unsigned)(nv * m * (int)sizeof(Tout)));
    const int lane = t % RW, grp = t / RW;
    // fused partial dr . out of the tile (the values as stored, FP64)
    const bool fdot = MODE == PASS_BWD && sizeof(Tout) == 8 && g.dr != nullptr;
    const auto rd = buf_rsrc(fdot ? g.dr + (size_t)rhs * g.N + (size_t)q0 * m : (const double*)out,
                             fdot ? (unsigned)(nv * m * 8) : 0u);
    double dacc = 0.0;
    for (int l = grp; l < nv; l += NG) {
      T co[MAXO];
      load_co(l, co);
#pragma unroll
      for (int u = 0; u < UMAX; ++u) {
        const int j = lane + RW * u;
        if (RW * u < m) {   // uniform: skip chunks past every row
          const int jj = j < m ? j : 0;
          const unsigned off = j < m ? (unsigned)(l * m + j) : BUF_OOB / 8u;
          const Tout v = (Tout)value(l, jj, co);
          buf_st<Tout>(v, rs, off * (unsigned)sizeof(Tout));
          if (fdot) dacc += (double)v * buf_ld<double>(rd, off * 8u);
        }
      }
    }
    if (fdot) {   // uniform; fixed-order sum over the workgroup
      double* red = reinterpret_cast<double*>(DM);   // NTH doubles fit in DM
      if constexpr (NTH % 64 == 0) {
        for (int o = 32; o > 0; o >>= 1) dacc += __shfl_xor(dacc, o);
        if ((t & 63) == 0) red[t >> 6] = dacc;
      } else {
        red[t] = dacc;   // a partial wave: no shuffles
      }
      __syncthreads();
      if (t == 0) {
        constexpr int NR = NTH % 64 == 0 ? NTH / 64 : NTH;
        double sum = 0.0;
        for (int k = 0; k < NR; ++k) sum += red[k];
        g.dpart[(size_t)rhs * g.dnpart + tile] = sum;
      }
    }
  } else if constexpr (NTH % TW == 0) {
    constexpr int JS = NTH / TW;
    const int l = t & (TW - 1), j0 = t >> LTW;
    int base, inner;
    const bool real = line_at(g, q0 + l, base, inner);
    if (l < nv && real && j0 < m) {
      T co[MAXO];
      load_co(l, co);
      const auto rs = buf_rsrc(out + (size_t)rhs * g.N, (unsigned)(g.N * (int)sizeof(Tout)));
      const unsigned vo = (unsigned)(base + j0 * S) * sizeof(Tout);
      const int cnt = (m - j0 + JS - 1) / JS;
      const int step = JS * S * (int)sizeof(Tout);
      // rows k < kl and k >= kr lie in the outlier windows; the rows between
      // are stored as they are
      const int kl = MODE == PASS_FWD ? 0 : min(cnt, j0 < g.wl ? (g.wl - 1 - j0) / JS + 1 : 0);
      const int kr = MODE == PASS_FWD ? 0 : max(kl, g.wr <= j0 ? 0 : (g.wr - j0 + JS - 1) / JS);
      for (int k = 0; k < kl; ++k)
        buf_st<Tout>((Tout)value(l, j0 + k * JS, co), rs, vo + (unsigned)(k * step));
      for (int k = kl; k < kr; ++k)
        buf_st<Tout>((Tout)X[l * MP + j0 + k * JS], rs, vo + (unsigned)(k * step));
      for (int k = max(kr, kl); k < cnt; ++k)
        buf_st<Tout>((Tout)value(l, j0 + k * JS, co), rs, vo + (unsigned)(k * step));
    }
  } else {
    const int cnt = TW * m;
    for (int e0 = t; e0 < cnt; e0 += NTH * CH) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = e0 + u * NTH;
        const int l = e & (TW - 1), j = e >> LTW;
        if (e < cnt && l < nv && LB[l] >= 0) {
          T co[MAXO];
          load_co(l, co);
          out[LB[l] + j * S] = (Tout)value(l, j, co);
        }
      }
    }
  }
}

template <typename Tin, typename Tout, typename T, int MODE, int L, int V, int PK>
__global__ void __launch_bounds__((Cfg<T, L, V>::NTH))
line_pass(const Tin* __restrict__ in, Tout* __restrict__ out, Geom g, Tabs<T> tb) {
  line_pass_body<Tin, Tout, T, MODE, L, V, PK, false>(in, out, g, tb);
}

template <typename Tin, typename Tout, typename T, int MODE, int L, int V, int PK>
__global__ void __launch_bounds__((Cfg<T, L, V>::NTH))
line_pass_upd(const Tin* __restrict__ in, Tout* __restrict__ out, Geom g, Tabs<T> tb) {
  line_pass_body<Tin, Tout, T, MODE, L, V, PK, true>(in, out, g, tb);
}

// the tables a pass stages in LDS: a prefix of the blob (odd p needs no twp,
// only the middle pass needs lam and s)
template <typename T>
static Tabs<T> tables_of(const Plan& P, int mode) {
  const char* b = P.d_tables + (sizeof(T) == 8 ? P.lay.blob64 : P.lay.blob32);
  const int len = mode == PASS_MID ? P.blob_len
                                    : ((P.p & 1) ? (P.half_len ? P.bo_twp : P.bo_sn) : P.bo_lam);
  const int nch = (int)((len * sizeof(T) + 15) / 16);
  return {(const T*)b, P.bo_twl, P.bo_twp, P.bo_vt, P.bo_v0, P.bo_v1, P.bo_lam, P.bo_s, len, P.bo_sn,
          nch};
}

template <typename Tin, typename Tout, typename T, int MODE, int L, int V, int PK>
static hipError_t launch_t(const Plan& P, int axis, const void* in, void* out, int nrhs,
                           const double* active, int astride, hipStream_t s, const PassHook* hk) {
  using C = Cfg<T, L, V>;
  Geom g;
  g.m = P.m; g.n = P.n; g.p = P.p; g.n_reg = P.n_reg; g.n_out = P.n_out; g.half = P.half;
  g.nbd = P.p - 1; g.c0 = P.p - 1 - P.half;
  int S = 1;
  for (int k = 1; k < axis; ++k) S *= P.m;
  g.S = S;
  g.N = (int)P.N;
  g.lpr = (int)(P.N / P.m);
  g.mr = P.m;
  g.sm = S > 1 ? S / P.m : 1;
  if (S > 1 && (P.m & 1)) {   // pad every run of lines to an even length (see line_at)
    g.mr = P.m + 1;
    g.lpr = (int)(P.N / P.m / P.m) * g.mr;
  }
  g.tpr = (g.lpr + C::TW - 1) / C::TW;
  g.d = P.d;
  g.active = active;
  g.active_stride = astride;
  g.wl = sizeof(T) == 8 ? P.win64[0] : P.win32[0];
  g.wr = sizeof(T) == 8 ? P.win64[1] : P.win32[1];
  g.dr = nullptr;
  g.fq = nullptr;
  g.falpha = nullptr;
  g.fr = nullptr;
  g.dpart = nullptr;
  g.dnpart = 0;
  if (hk) {
    const bool dot = MODE == PASS_BWD && sizeof(Tout) == 8 && hk->dr && !hk->q;
    const bool upd = MODE == PASS_FWD && sizeof(Tin) == 8 && hk->q && hk->alpha &&
                     hk->r_out == in && !hk->dr;
    if (axis != 1 || !(dot || upd) || !hk->part || g.tpr > hk->npart) return hipErrorInvalidValue;
    g.dr = hk->dr;
    g.fq = hk->q;
    g.falpha = hk->alpha;
    g.fr = hk->r_out;
    g.dpart = hk->part;
    g.dnpart = hk->npart;
    hk->tiles = g.tpr;
  }
  {
    // threads per outlier dot: as many as the workgroup allows, up to a wave
    const int ndots = C::TW * P.n_out;
    int tpd = 1;
    while (tpd < 64 && ndots * tpd * 2 <= C::NTH) tpd *= 2;
    if (ndots * tpd < C::NTH && tpd < 64) tpd *= 2;
    int tl = 0;
    while ((1 << tl) < tpd) ++tl;
    g.tpd_log = tl;
  }
  const Tabs<T> tb = tables_of<T>(P, MODE);
  const LdsMap mp = lds_map<T, L, V>(P.m, P.n, P.n_out, P.half, P.p, tb.len);
  dim3 grid((unsigned)(g.tpr * nrhs)), block(C::NTH);
  if constexpr (MODE == PASS_FWD && sizeof(Tin) == 8) {
    if (g.fq) {
      static bool attr_upd = false;
      if (mp.total > 65536 && !attr_upd) {
        hipError_t e = hipFuncSetAttribute((const void*)line_pass_upd<Tin, Tout, T, MODE, L, V, PK>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_upd = true;
      }
      hipLaunchKernelGGL((line_pass_upd<Tin, Tout, T, MODE, L, V, PK>), grid, block, mp.total, s,
                         (const Tin*)in, (Tout*)out, g, tb);
      return hipGetLastError();
    }
  }
  static bool attr_set = false;
  if (mp.total > 65536 && !attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)line_pass<Tin, Tout, T, MODE, L, V, PK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((line_pass<Tin, Tout, T, MODE, L, V, PK>), grid, block, mp.total, s,
                     (const Tin*)in, (Tout*)out, g, tb);
  return hipGetLastError();
}

template <typename Tin, typename Tout, typename T, int MODE, int L, int PK>
static hipError_t by_shape(const Plan& P, int var, int axis, const void* in, void* out, int nrhs,
                           const double* a, int as, hipStream_t s, const PassHook* hk) {
  if (var == 0) return launch_t<Tin, Tout, T, MODE, L, 0, PK>(P, axis, in, out, nrhs, a, as, s, hk);
  if (var == 1) return launch_t<Tin, Tout, T, MODE, L, 1, PK>(P, axis, in, out, nrhs, a, as, s, hk);
  if constexpr (fft_has_v3<L>()) {
    if (var == 3) return launch_t<Tin, Tout, T, MODE, L, 3, PK>(P, axis, in, out, nrhs, a, as, s, hk);
    if (var == 4) return launch_t<Tin, Tout, T, MODE, L, 4, PK>(P, axis, in, out, nrhs, a, as, s, hk);
  }
  return launch_t<Tin, Tout, T, MODE, L, 2, PK>(P, axis, in, out, nrhs, a, as, s, hk);
}

template <typename Tin, typename Tout, typename T, int MODE, int L>
static hipError_t by_variant(const Plan& P, int var, int axis, const void* in, void* out, int nrhs,
                             const double* a, int as, hipStream_t s, const PassHook* hk) {
  // one kernel per transform route: L = n where n is a supported length
  // (n >= 16), L = 2n for n = 8 and 12
  const bool odd = (P.p & 1) != 0;
  if constexpr (L <= 24) {
    if (!P.half_len) {
      if (odd) {
        return by_shape<Tin, Tout, T, MODE, L, PK_ODD>(P, var, axis, in, out, nrhs, a, as, s, hk);
      }
      return by_shape<Tin, Tout, T, MODE, L, PK_EVEN_2N>(P, var, axis, in, out, nrhs, a, as, s, hk);
    }
  } else if constexpr (sizeof(Tin) == 4 || sizeof(Tout) == 4) {
    // FP32 plans of odd degree >= 5: the odd extension of length 2n (no
    // prefix sums over FFT outputs, see build_plan)
    if (!P.half_len && odd)
      return by_shape<Tin, Tout, T, MODE, L, PK_ODD>(P, var, axis, in, out, nrhs, a, as, s, hk);
  }
  if constexpr (L <= 512) {
    if (P.half_len) {
      if (odd) {
        return by_shape<Tin, Tout, T, MODE, L, PK_ODD_N>(P, var, axis, in, out, nrhs, a, as, s, hk);
      }
      return by_shape<Tin, Tout, T, MODE, L, PK_EVEN_N>(P, var, axis, in, out, nrhs, a, as, s, hk);
    }
  }
  return hipErrorInvalidValue;
}

// the element types and variants of the line pass for one FFT length and mode
// (each (L, MODE) pair is instantiated in its own translation unit)
template <int L, int MODE>
hipError_t line_pass_mode(const Plan& P, int var, int axis, int tin, const void* in, int tout,
                          void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  if (P.prec == IFFD_PREC_F64) {
    if (tin != ELEM_F64 || tout != ELEM_F64) return hipErrorInvalidValue;
    return by_variant<double, double, double, MODE, L>(P, var, axis, in, out, nrhs, a, as, s, hk);
  }
  if constexpr (MODE == PASS_FWD) {
    // the pass that reads the FP64 input computes in FP64 when first64 is set
    if (tin == ELEM_F64 && tout == ELEM_F32 && P.first64)
      return by_variant<double, float, double, PASS_FWD, L>(P, var, axis, in, out, nrhs, a, as, s, hk);
    if (tin == ELEM_F64 && tout == ELEM_F32)
      return by_variant<double, float, float, PASS_FWD, L>(P, var, axis, in, out, nrhs, a, as, s, hk);
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return by_variant<float, float, float, PASS_FWD, L>(P, var, axis, in, out, nrhs, a, as, s, hk);
  } else if constexpr (MODE == PASS_BWD) {
    if (tin == ELEM_F32 && tout == ELEM_F64)
      return by_variant<float, double, float, PASS_BWD, L>(P, var, axis, in, out, nrhs, a, as, s, hk);
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return by_variant<float, float, float, PASS_BWD, L>(P, var, axis, in, out, nrhs, a, as, s, hk);
  } else {
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return by_variant<float, float, float, PASS_MID, L>(P, var, axis, in, out, nrhs, a, as, s, hk);
  }
  return hipErrorInvalidValue;
}

#define IFFD_LINE_PASS_MODE(L, MODE)                                                         \
  hipError_t line_pass_mode<L, MODE>(const Plan&, int, int, int, const void*, int, void*, int, \
                                     const double*, int, hipStream_t, const PassHook*)

}  // namespace iffd
