// Device-side building blocks for batched short complex FFTs on gfx950:
// complex helpers, small DFT codelets (radix 2, 3, 4, 8, 16) held in
// registers, and a Stockham autosort stage that exchanges through LDS.
//
// An FFT of length L is split into stages of radices R_1 .. R_s (product L).
// NT = L / E threads cooperate on one transform, each holding E elements
// (E divisible by every radix, so a thread runs E / R butterflies per
// stage).  Stage with radix R after a span NS = R_1 .. R_{s-1}:
//   butterfly j (0 <= j < L/R) reads x[j + r L/R], r < R, multiplies by the
//   twiddles w_L^{(j mod NS) r L/(NS R)}, runs a radix-R DFT and writes to
//   (j div NS) NS R + (j mod NS) + r NS.  The final order is natural.
// All transforms are forward (kernel e^{-2 pi i jk/L}).
#pragma once

#include <hip/hip_runtime.h>

namespace iffd {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> c_add(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_sub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_mul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i
template <typename T>
__device__ __forceinline__ cpx<T> c_mi(cpx<T> a) { return {a.y, -a.x}; }

// ---- codelets: in-place forward DFT of v[0..R-1] --------------------------

template <typename T>
__device__ __forceinline__ void dft2(cpx<T>& a, cpx<T>& b) {
  cpx<T> t = a;
  a = c_add(t, b);
  b = c_sub(t, b);
}

template <typename T>
__device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  cpx<T> s0 = c_add(a0, a2), d0 = c_sub(a0, a2);
  cpx<T> s1 = c_add(a1, a3), d1 = c_mi(c_sub(a1, a3));
  a0 = c_add(s0, s1);
  a2 = c_sub(s0, s1);
  a1 = c_add(d0, d1);
  a3 = c_sub(d0, d1);
}

template <typename T>
__device__ __forceinline__ void dft3(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2) {
  const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
  cpx<T> s = c_add(a1, a2), d = c_sub(a1, a2);
  cpx<T> m = {a0.x - T(0.5) * s.x, a0.y - T(0.5) * s.y};
  // -i h d
  cpx<T> r = {h * d.y, -h * d.x};
  a0 = c_add(a0, s);
  a1 = c_add(m, r);
  a2 = c_sub(m, r);
}

template <typename T>
__device__ __forceinline__ void dft8(cpx<T>* v) {
  const T q = T(0.70710678118654752440084436210485);
  // even / odd split, each a radix-4 DFT
  cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // w8^1 = q(1 - i), w8^2 = -i, w8^3 = q(-1 - i)
  o1 = {q * (o1.x + o1.y), q * (o1.y - o1.x)};
  o2 = c_mi(o2);
  o3 = {q * (o3.y - o3.x), -q * (o3.x + o3.y)};
  v[0] = c_add(e0, o0); v[4] = c_sub(e0, o0);
  v[1] = c_add(e1, o1); v[5] = c_sub(e1, o1);
  v[2] = c_add(e2, o2); v[6] = c_sub(e2, o2);
  v[3] = c_add(e3, o3); v[7] = c_sub(e3, o3);
}

template <typename T>
__device__ __forceinline__ void dft16(cpx<T>* v) {
  // 4 x 4: B[n2][k1] = DFT4 over n1 of v[4 n1 + n2], twiddle w16^{n2 k1},
  // X[k1 + 4 k2] = DFT4 over n2.
  const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
  const T q = T(0.70710678118654752440084436210485);
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // now v[4 k1 + n2] = B[n2][k1]
  // twiddles w16^{n2 k1}: (n2,k1) -> exponent n2*k1
  v[5] = {c1 * v[5].x + s1 * v[5].y, c1 * v[5].y - s1 * v[5].x};      // w^1
  v[9] = {q * (v[9].x + v[9].y), q * (v[9].y - v[9].x)};              // w^2
  v[13] = {s1 * v[13].x + c1 * v[13].y, s1 * v[13].y - c1 * v[13].x};  // w^3
  v[6] = {q * (v[6].x + v[6].y), q * (v[6].y - v[6].x)};              // w^2
  v[10] = c_mi(v[10]);                                                // w^4
  v[14] = {q * (v[14].y - v[14].x), -q * (v[14].x + v[14].y)};         // w^6
  v[7] = {s1 * v[7].x + c1 * v[7].y, s1 * v[7].y - c1 * v[7].x};      // w^3
  v[11] = {q * (v[11].y - v[11].x), -q * (v[11].x + v[11].y)};         // w^6
  v[15] = {-c1 * v[15].x - s1 * v[15].y, s1 * v[15].x - c1 * v[15].y}; // w^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // v[4 k1 + k2] = X[k1 + 4 k2]: transpose the 4x4 index into natural order
  cpx<T> t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}

template <typename T, int R>
__device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 2) dft2(v[0], v[1]);
  else if constexpr (R == 3) dft3(v[0], v[1], v[2]);
  else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8(v);
  else if constexpr (R == 16) dft16(v);
  else static_assert(R == 2, "unsupported radix");
}

// ---- radix plans per FFT length ------------------------------------------
// Variant V = 0 holds E = 16 (or 24) elements per thread, V = 1 holds 8 (or
// 12): twice the threads per transform and one more stage, which raises the
// number of waves in flight for small problems.

template <int L, int V> struct FftPlan;
template <> struct FftPlan<16, 0>  { static constexpr int E = 16; };
template <> struct FftPlan<24, 0>  { static constexpr int E = 24; };
template <> struct FftPlan<32, 0>  { static constexpr int E = 16; };
template <> struct FftPlan<48, 0>  { static constexpr int E = 12; };
template <> struct FftPlan<64, 0>  { static constexpr int E = 16; };
template <> struct FftPlan<96, 0>  { static constexpr int E = 24; };
template <> struct FftPlan<128, 0> { static constexpr int E = 16; };
template <> struct FftPlan<192, 0> { static constexpr int E = 24; };
template <> struct FftPlan<256, 0> { static constexpr int E = 16; };
template <> struct FftPlan<384, 0> { static constexpr int E = 24; };
template <> struct FftPlan<512, 0> { static constexpr int E = 16; };
template <> struct FftPlan<16, 1>  { static constexpr int E = 8; };
template <> struct FftPlan<24, 1>  { static constexpr int E = 12; };
template <> struct FftPlan<32, 1>  { static constexpr int E = 8; };
template <> struct FftPlan<48, 1>  { static constexpr int E = 12; };
template <> struct FftPlan<64, 1>  { static constexpr int E = 8; };
template <> struct FftPlan<96, 1>  { static constexpr int E = 12; };
template <> struct FftPlan<128, 1> { static constexpr int E = 8; };
template <> struct FftPlan<192, 1> { static constexpr int E = 12; };
template <> struct FftPlan<256, 1> { static constexpr int E = 8; };
template <> struct FftPlan<384, 1> { static constexpr int E = 12; };
template <> struct FftPlan<512, 1> { static constexpr int E = 8; };
// variant 2: variant 1's transform shape (it differs only in lines per workgroup)
template <int L> struct FftPlan<L, 2> : FftPlan<L, 1> {};
// variant 3: 4 elements per thread (radix 4 and 2 only, so lengths 2^a):
// twice variant 1's threads per transform, for problems too small to keep
// enough waves in flight
template <int L> struct FftPlan<L, 3> { static constexpr int E = 4; };
// variant 4: variant 3's transform shape (it differs only in lines per workgroup)
template <int L> struct FftPlan<L, 4> : FftPlan<L, 3> {};
// (a transform then spans at most one wave, which the DST-I prefix sums need)
template <int L> constexpr bool fft_has_v3() { return (L & (L - 1)) == 0 && L >= 16 && L <= 256; }

// ---- cross-lane prefix sums over the NT lanes of one transform -------------
// Lane index mod NT is the position in the transform's group of threads.
// Groups of 16, 32 or 64 lanes use DPP row shifts (row_shr:1,2,4,8 within
// each row of 16 lanes, then row_bcast:15 / row_bcast:31 to carry row totals
// into the following rows): VALU work only, no LDS traffic.  Smaller groups
// use shuffles bounded to the group.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                              ROWMASK, 0xF, true));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWMASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int NT, typename T>
__device__ __forceinline__ T group_inclusive_scan(T x, int tid) {
  if constexpr (NT >= 16) {
    x += dpp_f<0x111, 0xF>(x);   // row_shr:1
    x += dpp_f<0x112, 0xF>(x);   // row_shr:2
    x += dpp_f<0x114, 0xF>(x);   // row_shr:4
    x += dpp_f<0x118, 0xF>(x);   // row_shr:8
    if constexpr (NT >= 32) x += dpp_f<0x142, 0xA>(x);   // row_bcast:15 into rows 1, 3
    if constexpr (NT >= 64) x += dpp_f<0x143, 0xC>(x);   // row_bcast:31 into rows 2, 3
  } else {
#pragma unroll
    for (int dd = 1; dd < NT; dd <<= 1) {
      const T u = __shfl_up(x, dd, NT);
      if (tid >= dd) x += u;
    }
  }
  return x;
}

// padded LDS index of FFT element k of a length-L transform: for power-of-two
// lengths one spare slot every 16 entries keeps the strided Stockham writes
// off a single bank; lengths with a factor 3 (radix-3 last stage) measured
// fastest unpadded.  The regions of consecutive transforms are staggered by 8
// elements so they start on different banks.
template <int L> constexpr bool fft_padded() { return L % 3 != 0; }
template <int L>
__device__ __forceinline__ int fpad(int k) { return fft_padded<L>() ? k + (k >> 4) : k; }
template <int L> constexpr int fft_region() { return L + (fft_padded<L>() ? L / 16 : 0) + 8; }

// One Stockham stage: reads, butterflies, barrier, writes.  FIRST: inputs
// come from ld(k, lo, k0, kh) instead of LDS, with lo = (k < L/2),
// k0 = (k == 0) and kh = (k == L/2) known per unrolled slot; LAST: outputs go
// to st(k, v) instead of LDS.  The barrier between a stage's reads and its
// writes lets `buf` alias whatever ld reads.
template <typename T, int L, int E, int NT, int NS, int R, bool FIRST, bool LAST, class LD,
          class ST>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, int tid, const cpx<T>* tw, LD& ld,
                                          ST& st) {
  constexpr int B = E / R;
  cpx<T> v[B][R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + NT * b;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = j + r * (L / R);
      // first stage: j < L/R, so k < L/2 exactly when r < R/2 (R is even for
      // every first radix), and k is 0 or L/2 only for j = 0
      if constexpr (FIRST) v[b][r] = ld(k, r < R / 2, j == 0 && r == 0, j == 0 && 2 * r == R);
      else v[b][r] = buf[fpad<L>(k)];
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + NT * b;
    const int k = j % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[b][r] = c_mul(v[b][r], tw[k * r * (L / (NS * R))]);
    }
    dft<T, R>(v[b]);
  }
  // every read of this stage precedes every write (the stages work in place);
  // the butterflies above overlap the other waves' reads
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + NT * b;
    const int o = (j / NS) * NS * R + j % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (LAST) st(o + r * NS, v[b][r]);
      else buf[fpad<L>(o + r * NS)] = v[b][r];
    }
  }
  if constexpr (!LAST) __syncthreads();
}

template <typename T, int L, int E, int NT, int NS, int R, int... Rest>
struct FftRun {
  template <class LD, class ST>
  __device__ __forceinline__ static void run(cpx<T>* buf, int tid, const cpx<T>* tw, LD& ld,
                                             ST& st) {
    constexpr bool first = (NS == 1);
    constexpr bool last = sizeof...(Rest) == 0;
    fft_stage<T, L, E, NT, NS, R, first, last>(buf, tid, tw, ld, st);
    if constexpr (!last) FftRun<T, L, E, NT, NS * R, Rest...>::run(buf, tid, tw, ld, st);
  }
};

// forward FFT of length L over NT = L/E threads; ld(k, lo, k0, kh) supplies input k,
// st(k, v) receives output k (natural order).  buf: this transform's LDS
// region of fft_region<L>() elements.  All threads of the block must call it.
template <typename T, int L, int V, class LD, class ST>
__device__ __forceinline__ void fft_forward(cpx<T>* buf, int tid, const cpx<T>* tw, LD& ld,
                                            ST& st) {
  constexpr int E = FftPlan<L, V>::E, NT = L / E;
  if constexpr (V == 0) {
    if constexpr (L == 16) FftRun<T, 16, E, NT, 1, 16>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 24) FftRun<T, 24, E, NT, 1, 8, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 32) FftRun<T, 32, E, NT, 1, 16, 2>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 48) FftRun<T, 48, E, NT, 1, 4, 4, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 64) FftRun<T, 64, E, NT, 1, 16, 4>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 96) FftRun<T, 96, E, NT, 1, 8, 4, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 128) FftRun<T, 128, E, NT, 1, 16, 8>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 192) FftRun<T, 192, E, NT, 1, 8, 8, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 256) FftRun<T, 256, E, NT, 1, 16, 16>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 384) FftRun<T, 384, E, NT, 1, 8, 8, 2, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 512) FftRun<T, 512, E, NT, 1, 16, 16, 2>::run(buf, tid, tw, ld, st);
  } else if constexpr (V == 3 || V == 4) {
    if constexpr (L == 16) FftRun<T, 16, E, NT, 1, 4, 4>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 32) FftRun<T, 32, E, NT, 1, 4, 4, 2>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 64) FftRun<T, 64, E, NT, 1, 4, 4, 4>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 128) FftRun<T, 128, E, NT, 1, 4, 4, 4, 2>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 256) FftRun<T, 256, E, NT, 1, 4, 4, 4, 4>::run(buf, tid, tw, ld, st);
    else static_assert(L == 16, "variant 3 needs a power-of-two length");
  } else {
    if constexpr (L == 16) FftRun<T, 16, E, NT, 1, 8, 2>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 24) FftRun<T, 24, E, NT, 1, 4, 2, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 32) FftRun<T, 32, E, NT, 1, 8, 4>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 48) FftRun<T, 48, E, NT, 1, 4, 4, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 64) FftRun<T, 64, E, NT, 1, 8, 8>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 96) FftRun<T, 96, E, NT, 1, 4, 4, 2, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 128) FftRun<T, 128, E, NT, 1, 8, 4, 4>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 192) FftRun<T, 192, E, NT, 1, 4, 4, 4, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 256) FftRun<T, 256, E, NT, 1, 8, 8, 4>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 384) FftRun<T, 384, E, NT, 1, 4, 4, 4, 2, 3>::run(buf, tid, tw, ld, st);
    else if constexpr (L == 512) FftRun<T, 512, E, NT, 1, 8, 8, 8>::run(buf, tid, tw, ld, st);
  }
}

}  // namespace iffd
