// IFFD line passes on gfx950.
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
// complex FFT of length L = 2n of an odd extension:
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

template <typename T>
struct Tabs {
  const T* lam;
  const T* s;
  const T* V0;
  const T* V1;
  const T* Vt;
  const cpx<T>* twl;
  const cpx<T>* twp;
};

struct Geom {
  int m, n, p, n_reg, n_out, half, nbd, c0;
  int S;       // element stride along the axis
  int lpr;     // lines per right-hand side
  int tpr;     // tiles per right-hand side
  int N;       // elements per right-hand side
  int d;
  const double* active;  // per-RHS flags or null
  int active_stride;
};

template <typename T, int L>
struct Cfg {
  static constexpr int E = FftPlan<L>::E;
  static constexpr int NT = L / E;
  static constexpr int CAP = (sizeof(T) == 8 ? 128 : 256) / NT;
  static constexpr int FPW = CAP >= 32 ? 32 : (CAP < 1 ? 1 : CAP);
  static constexpr int TW = 2 * FPW;
  static constexpr int NTH = FPW * NT;
};

__host__ __device__ inline size_t up16(size_t x) { return (x + 15) & ~(size_t)15; }

struct LdsMap {
  size_t x, twl, twp, g, co, lo, so, lb, total;
};

template <typename T, int L>
__host__ __device__ inline LdsMap lds_map(int m, int n, int n_out, int half) {
  using C = Cfg<T, L>;
  const int MP = m | 1;
  size_t xs = (size_t)C::TW * MP;
  size_t fs = (size_t)C::FPW * fft_region<L>() * 2;
  LdsMap r;
  size_t off = 0;
  r.x = off;   off = up16(off + sizeof(T) * (xs > fs ? xs : fs));
  r.twl = off; off = up16(off + sizeof(T) * 2 * L);
  r.twp = off; off = up16(off + sizeof(T) * 2 * (n + 1));
  r.g = off;   off = up16(off + sizeof(T) * C::TW * 2 * (half > 0 ? half : 1));
  r.co = off;  off = up16(off + sizeof(T) * C::TW * (n_out > 0 ? n_out : 1));
  r.lo = off;  off = up16(off + sizeof(T) * C::TW);
  r.so = off;  off = up16(off + sizeof(T) * C::TW);
  r.lb = off;  off = up16(off + sizeof(int) * C::TW);
  r.total = off;
  return r;
}

template <typename Tin, typename Tout, typename T, int MODE, int L>
__global__ void __launch_bounds__((Cfg<T, L>::NTH))
line_pass(const Tin* in, Tout* out, Geom g, Tabs<T> tb) {
  using C = Cfg<T, L>;
  constexpr int TW = C::TW, NTH = C::NTH, NT = C::NT;
  extern __shared__ __align__(16) char smem[];
  const int m = g.m, n = g.n, n_reg = g.n_reg, n_out = g.n_out, half = g.half;
  const int MP = m | 1;
  const LdsMap mp = lds_map<T, L>(m, n, n_out, half);
  T* X = reinterpret_cast<T*>(smem + mp.x);
  cpx<T>* F = reinterpret_cast<cpx<T>*>(smem + mp.x);  // aliases X
  cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem + mp.twl);
  cpx<T>* twp = reinterpret_cast<cpx<T>*>(smem + mp.twp);
  T* G = reinterpret_cast<T*>(smem + mp.g);
  T* CO = reinterpret_cast<T*>(smem + mp.co);
  T* LO = reinterpret_cast<T*>(smem + mp.lo);
  T* SO = reinterpret_cast<T*>(smem + mp.so);
  int* LB = reinterpret_cast<int*>(smem + mp.lb);
  const int GW = 2 * (half > 0 ? half : 1);

  const int t = threadIdx.x;
  const int rhs = blockIdx.x / g.tpr;
  const int tile = blockIdx.x - rhs * g.tpr;
  if (g.active && g.active[(size_t)rhs * g.active_stride] == 0.0) return;
  const int q0 = tile * TW;
  const int nv = min(TW, g.lpr - q0);
  const int S = g.S;

  // per-line data (a block may have fewer threads than the tile has lines)
  for (int l = t; l < TW; l += NTH) {
    const int ql = q0 + l;
    LB[l] = (l < nv) ? rhs * g.N + (ql / S) * m * S + (ql % S) : 0;
    if (MODE == PASS_MID) {
      // spectral indices of the line in the other directions (the middle pass
      // runs along the last direction, so the inner index holds them all)
      T lo = T(0), so = T(1);
      if (l < nv) {
        const int i = ql % S;
        const int j1 = i % m, j2 = i / m;
        lo = tb.lam[j1];
        so = tb.s[j1];
        if (g.d == 3) { lo += tb.lam[j2]; so *= tb.s[j2]; }
      }
      LO[l] = lo;
      SO[l] = so;
    }
  }
  for (int k = t; k < L; k += NTH) twl[k] = tb.twl[k];
  if (MODE != PASS_FWD || (g.p % 2) == 0)
    for (int k = t; k <= n; k += NTH) twp[k] = tb.twp[k];
  __syncthreads();

  // ---- load the tile: X[l][j] = in(line l, position j) ---------------------
  if (S == 1) {
    const Tin* src = in + LB[0];
    const int tot = nv * m;
    int l = t / m, j = t - (t / m) * m;
    const int sl = NTH / m, sj = NTH - sl * m;
    for (int e = t; e < tot; e += NTH) {
      X[l * MP + j] = (T)src[e];
      j += sj;
      l += sl;
      if (j >= m) { j -= m; ++l; }
    }
  } else {
    for (int e = t; e < TW * m; e += NTH) {
      const int l = e % TW, j = e / TW;
      if (l < nv) X[l * MP + j] = (T)in[LB[l] + j * S];
    }
  }
  // zero rows of missing lines (they share FFTs with real lines)
  for (int e = nv * MP + t; e < TW * MP; e += NTH) X[e] = T(0);
  __syncthreads();

  // ---- outlier dots and boundary fold (forward) / save outlier coefs -------
  if (MODE == PASS_FWD || MODE == PASS_MID) {
    if (n_out > 0) {
      const int ndots = TW * n_out;
      int tpd = 1;
      while (tpd < 64 && ndots * tpd * 2 <= NTH) tpd *= 2;
      const int sub = t % tpd;
      for (int di = t / tpd; di < (ndots + (NTH / tpd) - 1) / (NTH / tpd) * (NTH / tpd);
           di += NTH / tpd) {
        T acc = T(0);
        const int l = di % TW, q = di / TW;
        if (di < ndots) {
          const T* vr = tb.Vt + (size_t)q * m;
          const T* xr = X + l * MP;
          for (int j = sub; j < m; j += tpd) acc += vr[j] * xr[j];
        }
        for (int o = 1; o < tpd; o <<= 1) acc += __shfl_xor(acc, o);
        if (sub == 0 && di < ndots) CO[l * n_out + q] = acc;
      }
    }
    const int nbd = g.nbd;
    for (int e = t; e < TW * 2 * half; e += NTH) {
      const int l = e % TW, c = e / TW;
      T acc = T(0);
      if (c < half) {
        for (int r = 0; r < nbd; ++r) acc += tb.V0[r * half + c] * X[l * MP + r];
      } else {
        for (int r = 0; r < nbd; ++r)
          acc += tb.V1[r * half + (c - half)] * X[l * MP + m - nbd + r];
      }
      G[l * GW + c] = acc;
    }
  } else {
    for (int e = t; e < TW * n_out; e += NTH) {
      const int l = e / n_out, q = e - (e / n_out) * n_out;
      CO[e] = X[l * MP + n_reg + q];
    }
  }
  __syncthreads();

  const int f = t / NT, tid = t - (t / NT) * NT;
  const int la = 2 * f, lb = 2 * f + 1;
  cpx<T>* buf = F + f * fft_region<L>();
  const int c0 = g.c0;
  const bool odd = (g.p & 1) != 0;

  auto gval = [&](int l, int idx) -> T {
    if (idx < half) return G[l * GW + idx];
    if (idx >= n_reg - half) return G[l * GW + half + idx - (n_reg - half)];
    return X[l * MP + idx + c0];
  };

  // ---- forward transform: X[l][0..n_reg) = U^T fold(x_l) -------------------
  auto forward = [&]() {
    auto ld = [&](int k) -> cpx<T> {
      int idx;
      T sg = T(1);
      if (odd) {
        if (k == 0 || k == n) return {T(0), T(0)};
        if (k < n) idx = k - 1;
        else { idx = 2 * n - k - 1; sg = T(-1); }
      } else {
        if (k < n) idx = k;
        else { idx = 2 * n - 1 - k; sg = T(-1); }
      }
      return {sg * gval(la, idx), sg * gval(lb, idx)};
    };
    auto st = [&](int k, cpx<T> v) {
      if (odd) {
        if (k >= 1 && k <= n - 1) {
          X[la * MP + k - 1] = T(-0.5) * v.y;
          X[lb * MP + k - 1] = T(0.5) * v.x;
        }
      } else {
        if (k >= 1 && k <= n) {
          cpx<T> w = c_mul(v, twp[k]);
          X[la * MP + k - 1] = T(-0.5) * w.y;
          X[lb * MP + k - 1] = T(0.5) * w.x;
        }
      }
    };
    fft_forward<T, L>(buf, tid, twl, ld, st);
  };

  // ---- backward transform: g = U c, stored as X interior + G ends ----------
  auto backward = [&]() {
    auto ld = [&](int k) -> cpx<T> {
      if (odd) {
        int idx;
        T sg = T(1);
        if (k == 0 || k == n) return {T(0), T(0)};
        if (k < n) idx = k - 1;
        else { idx = 2 * n - k - 1; sg = T(-1); }
        return {sg * X[la * MP + idx], sg * X[lb * MP + idx]};
      }
      if (k == 0) return {T(0), T(0)};
      const int j = k <= n ? k : 2 * n - k;
      const cpx<T> wb = {X[la * MP + j - 1], -X[lb * MP + j - 1]};
      if (k == n) return {T(-2) * wb.y, T(2) * wb.x};
      const cpx<T> tw = twp[j];
      if (k < n) return c_mul(wb, cpx<T>{tw.x, -tw.y});
      const cpx<T> u = c_mul(wb, tw);
      return {-u.x, -u.y};
    };
    auto put = [&](int l, int idx, T v) {
      if (idx < half) G[l * GW + idx] = v;
      else if (idx >= n_reg - half) G[l * GW + half + idx - (n_reg - half)] = v;
      else X[l * MP + idx + c0] = v;
    };
    auto st = [&](int k, cpx<T> v) {
      if (k >= 1 && k <= n_reg) {
        put(la, k - 1, T(-0.5) * v.y);
        put(lb, k - 1, odd ? T(0.5) * v.x : T(-0.5) * v.x);
      }
    };
    fft_forward<T, L>(buf, tid, twl, ld, st);
  };

  if (MODE == PASS_FWD || MODE == PASS_MID) forward();
  __syncthreads();

  if (MODE == PASS_MID) {
    // diagonal scaling by prod s / sum lam (regular modes in X, outliers in CO)
    for (int e = t; e < TW * m; e += NTH) {
      const int l = e % TW, j = e / TW;
      const T fac = tb.s[j] * SO[l] / (tb.lam[j] + LO[l]);
      if (j < n_reg) X[l * MP + j] *= fac;
      else CO[l * n_out + (j - n_reg)] *= fac;
    }
    __syncthreads();
  }

  if (MODE == PASS_BWD || MODE == PASS_MID) {
    backward();
    __syncthreads();
  }

  // ---- store ---------------------------------------------------------------
  const int nbd = g.nbd;
  auto value = [&](int l, int j) -> T {
    if (MODE == PASS_FWD) return j < n_reg ? X[l * MP + j] : CO[l * n_out + (j - n_reg)];
    T v;
    if (j < nbd) {
      v = T(0);
      for (int c = 0; c < half; ++c) v += tb.V0[j * half + c] * G[l * GW + c];
    } else if (j >= m - nbd) {
      v = T(0);
      const int r = j - (m - nbd);
      for (int c = 0; c < half; ++c) v += tb.V1[r * half + c] * G[l * GW + half + c];
    } else {
      v = X[l * MP + j];
    }
    for (int q = 0; q < n_out; ++q) v += tb.Vt[(size_t)q * m + j] * CO[l * n_out + q];
    return v;
  };
  if (S == 1) {
    Tout* dst = out + LB[0];
    const int tot = nv * m;
    int l = t / m, j = t - (t / m) * m;
    const int sl = NTH / m, sj = NTH - sl * m;
    for (int e = t; e < tot; e += NTH) {
      dst[e] = (Tout)value(l, j);
      j += sj;
      l += sl;
      if (j >= m) { j -= m; ++l; }
    }
  } else {
    for (int e = t; e < TW * m; e += NTH) {
      const int l = e % TW, j = e / TW;
      if (l < nv) out[LB[l] + j * S] = (Tout)value(l, j);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
static Tabs<T> tables_of(const Plan& P);

template <>
Tabs<float> tables_of<float>(const Plan& P) {
  const char* b = P.d_tables;
  const TableLayout& t = P.lay;
  return {(const float*)(b + t.lam32), (const float*)(b + t.s32), (const float*)(b + t.v0_32),
          (const float*)(b + t.v1_32), (const float*)(b + t.vt32),
          (const cpx<float>*)(b + t.twl32), (const cpx<float>*)(b + t.twp32)};
}
template <>
Tabs<double> tables_of<double>(const Plan& P) {
  const char* b = P.d_tables;
  const TableLayout& t = P.lay;
  return {(const double*)(b + t.lam64), (const double*)(b + t.s64), (const double*)(b + t.v0_64),
          (const double*)(b + t.v1_64), (const double*)(b + t.vt64),
          (const cpx<double>*)(b + t.twl64), (const cpx<double>*)(b + t.twp64)};
}

template <typename Tin, typename Tout, typename T, int MODE, int L>
static hipError_t launch_t(const Plan& P, int axis, const void* in, void* out, int nrhs,
                           const double* active, int astride, hipStream_t s) {
  using C = Cfg<T, L>;
  Geom g;
  g.m = P.m; g.n = P.n; g.p = P.p; g.n_reg = P.n_reg; g.n_out = P.n_out; g.half = P.half;
  g.nbd = P.p - 1; g.c0 = P.p - 1 - P.half;
  int S = 1;
  for (int k = 1; k < axis; ++k) S *= P.m;
  g.S = S;
  g.N = (int)P.N;
  g.lpr = (int)(P.N / P.m);
  g.tpr = (g.lpr + C::TW - 1) / C::TW;
  g.d = P.d;
  g.active = active;
  g.active_stride = astride;
  const LdsMap mp = lds_map<T, L>(P.m, P.n, P.n_out, P.half);
  static bool attr_set = false;
  if (mp.total > 65536 && !attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)line_pass<Tin, Tout, T, MODE, L>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid((unsigned)(g.tpr * nrhs)), block(C::NTH);
  hipLaunchKernelGGL((line_pass<Tin, Tout, T, MODE, L>), grid, block, mp.total, s,
                     (const Tin*)in, (Tout*)out, g, tables_of<T>(P));
  return hipGetLastError();
}

template <typename Tin, typename Tout, typename T, int MODE>
static hipError_t dispatch_L(const Plan& P, int axis, const void* in, void* out, int nrhs,
                             const double* a, int as, hipStream_t s) {
  switch (P.L) {
    case 16: return launch_t<Tin, Tout, T, MODE, 16>(P, axis, in, out, nrhs, a, as, s);
    case 24: return launch_t<Tin, Tout, T, MODE, 24>(P, axis, in, out, nrhs, a, as, s);
    case 32: return launch_t<Tin, Tout, T, MODE, 32>(P, axis, in, out, nrhs, a, as, s);
    case 48: return launch_t<Tin, Tout, T, MODE, 48>(P, axis, in, out, nrhs, a, as, s);
    case 64: return launch_t<Tin, Tout, T, MODE, 64>(P, axis, in, out, nrhs, a, as, s);
    case 96: return launch_t<Tin, Tout, T, MODE, 96>(P, axis, in, out, nrhs, a, as, s);
    case 128: return launch_t<Tin, Tout, T, MODE, 128>(P, axis, in, out, nrhs, a, as, s);
    case 192: return launch_t<Tin, Tout, T, MODE, 192>(P, axis, in, out, nrhs, a, as, s);
    case 256: return launch_t<Tin, Tout, T, MODE, 256>(P, axis, in, out, nrhs, a, as, s);
    case 384: return launch_t<Tin, Tout, T, MODE, 384>(P, axis, in, out, nrhs, a, as, s);
    case 512: return launch_t<Tin, Tout, T, MODE, 512>(P, axis, in, out, nrhs, a, as, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_line_pass(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                            void* out, int nrhs, const double* a, int as, hipStream_t s) {
  if (P.prec == IFFD_PREC_F64) {
    if (tin != ELEM_F64 || tout != ELEM_F64) return hipErrorInvalidValue;
    if (mode == PASS_FWD) return dispatch_L<double, double, double, PASS_FWD>(P, axis, in, out, nrhs, a, as, s);
    if (mode == PASS_BWD) return dispatch_L<double, double, double, PASS_BWD>(P, axis, in, out, nrhs, a, as, s);
    return dispatch_L<double, double, double, PASS_MID>(P, axis, in, out, nrhs, a, as, s);
  }
  if (mode == PASS_FWD) {
    if (tin == ELEM_F64 && tout == ELEM_F32)
      return dispatch_L<double, float, float, PASS_FWD>(P, axis, in, out, nrhs, a, as, s);
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return dispatch_L<float, float, float, PASS_FWD>(P, axis, in, out, nrhs, a, as, s);
  } else if (mode == PASS_BWD) {
    if (tin == ELEM_F32 && tout == ELEM_F64)
      return dispatch_L<float, double, float, PASS_BWD>(P, axis, in, out, nrhs, a, as, s);
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return dispatch_L<float, float, float, PASS_BWD>(P, axis, in, out, nrhs, a, as, s);
  } else {
    if (tin == ELEM_F32 && tout == ELEM_F32)
      return dispatch_L<float, float, float, PASS_MID>(P, axis, in, out, nrhs, a, as, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_iffd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                             const double* a, int as, hipStream_t s) {
  hipError_t e;
  if (P.prec == IFFD_PREC_F64) {
    // in place on z after the first pass
    e = launch_line_pass(P, PASS_FWD, 1, ELEM_F64, r, ELEM_F64, z, nrhs, a, as, s);
    if (e != hipSuccess) return e;
    if (P.d == 3) {
      e = launch_line_pass(P, PASS_FWD, 2, ELEM_F64, z, ELEM_F64, z, nrhs, a, as, s);
      if (e != hipSuccess) return e;
    }
    e = launch_line_pass(P, PASS_MID, P.d, ELEM_F64, z, ELEM_F64, z, nrhs, a, as, s);
    if (e != hipSuccess) return e;
    if (P.d == 3) {
      e = launch_line_pass(P, PASS_BWD, 2, ELEM_F64, z, ELEM_F64, z, nrhs, a, as, s);
      if (e != hipSuccess) return e;
    }
    return launch_line_pass(P, PASS_BWD, 1, ELEM_F64, z, ELEM_F64, z, nrhs, a, as, s);
  }
  float* w = (float*)ws;
  e = launch_line_pass(P, PASS_FWD, 1, ELEM_F64, r, ELEM_F32, w, nrhs, a, as, s);
  if (e != hipSuccess) return e;
  if (P.d == 3) {
    e = launch_line_pass(P, PASS_FWD, 2, ELEM_F32, w, ELEM_F32, w, nrhs, a, as, s);
    if (e != hipSuccess) return e;
  }
  e = launch_line_pass(P, PASS_MID, P.d, ELEM_F32, w, ELEM_F32, w, nrhs, a, as, s);
  if (e != hipSuccess) return e;
  if (P.d == 3) {
    e = launch_line_pass(P, PASS_BWD, 2, ELEM_F32, w, ELEM_F32, w, nrhs, a, as, s);
    if (e != hipSuccess) return e;
  }
  return launch_line_pass(P, PASS_BWD, 1, ELEM_F32, w, ELEM_F64, z, nrhs, a, as, s);
}

}  // namespace iffd
