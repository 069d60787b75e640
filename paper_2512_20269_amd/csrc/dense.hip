// Classical Fast Diagonalization (Section 3, eq:exact_diagonalization) on
// gfx950: z = (Q x .. x Q) (sum_k Lambda_k)^{-1} (Q^T x .. x Q^T) r with the
// dense m x m eigenvector matrix Q of the pencil (K, M) (Q^T M Q = I,
// Q^T K Q = Lambda).  Q^T is applied first.  Every mode product is a GEMM on
// the matrix cores:
//   direction 1 (contiguous):  rows of the tensor times Q (forward) or Q^T
//                              (backward): C[M x m] = X[M x m] B
//   direction k > 1:           for each slab o, C_o = A X_o with A = Q^T
//                              (forward) or Q (backward), X_o an m x S slab
//                              (S = m^{k-1})
// The division by sum_k lambda_{j_k} is fused into the epilogue of the last
// forward product.  FP32 uses v_mfma_f32_16x16x4f32 with large workgroup
// tiles (gemm_f32_t16; small problems v_mfma_f32_32x32x2f32 with one 32 x 32
// tile per wave), FP64 v_mfma_f64_16x16x4f64 (16 x 16 per wave), FP16 and
// BF16 (IFFD_PREC_F16S / IFFD_PREC_BF16S) gfx950's v_mfma_f32_32x32x16_f16 /
// _bf16 with FP32 accumulation; four waves per workgroup, K staged through
// LDS in chunks.  In FP16 / BF16 every line along the transformed direction is
// first divided by its largest |value| and rounded (quant_lines), Q carries
// one scale s_Q, and the epilogue multiplies both back.
#include <type_traits>
#include <utility>

#include "launch.h"

namespace iffd {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct GemmArgs {
  int M, N, K;
  int lda, ldb, ldc;
  long long sA, sB, sC;   // element strides between batch entries
  int batch_per_rhs;      // batch entries per right-hand side
  const double* active;   // per-RHS flags or null
  int astride;
  // fused scaling (last forward product): C[i][j] /= lam[i] + lam[j % m] (+ lam[j / m])
  const void* lam;
  int scale_mode;          // 0 none, 2: 2D (lam[i] + lam[j]), 3: 3D (lam[i] + lam[j%m] + lam[j/m])
  int m;
  // FP16 operands: C[i][j] *= qs * ls[line], line = row i (ls_mode 1) or
  // batch entry * N + column j (ls_mode 2)
  const float* ls;
  int ls_mode;
  const float* qs;
};

template <typename T> struct MfmaCfg;
template <> struct MfmaCfg<float> { static constexpr int WT = 32, BK = 16; };   // wave tile
template <> struct MfmaCfg<double> { static constexpr int WT = 16, BK = 16; };
template <> struct MfmaCfg<_Float16> { static constexpr int WT = 32, BK = 16; };
template <> struct MfmaCfg<__bf16> { static constexpr int WT = 32, BK = 16; };

// C = A * B (all row-major), one workgroup of 4 waves per (2 WT) x (2 WT) tile
template <typename TA, typename TB, typename TC, typename T>
__global__ void __launch_bounds__(256) gemm_mfma(const TA* __restrict__ A, const TB* __restrict__ B,
                                                 TC* __restrict__ Cm, GemmArgs g) {
  constexpr int WT = MfmaCfg<T>::WT, BK = MfmaCfg<T>::BK;
  constexpr int BM = 2 * WT, BN = 2 * WT;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const int bat = blockIdx.z;
  const int rhs = bat / g.batch_per_rhs;
  if (g.active && g.active[(size_t)rhs * g.astride] == 0.0) return;
  const TA* Ab = A + bat * g.sA;
  const TB* Bb = B + bat * g.sB;
  TC* Cb = Cm + bat * g.sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * WT, wn = (w & 1) * WT;

  f32x16 accf = {};
  f64x4 accd = {};
  // T is the operand type; the accumulator is FP64 for FP64, else FP32
  using TE = std::conditional_t<sizeof(T) == 8, double, float>;

  // K chunks of the A (BM x BK) and B (BK x BN) tiles: the next chunk's loads
  // are issued into registers before the current chunk's products, so their
  // latency hides behind the matrix cores; entries outside the matrices read
  // 0 (buffer loads with a range check, no branches)
  constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
  const auto ra_ = buf_rsrc(Ab, (unsigned)(((long long)(g.M - 1) * g.lda + g.K) * sizeof(TA)));
  const auto rb_ = buf_rsrc(Bb, (unsigned)(((long long)(g.K - 1) * g.ldb + g.N) * sizeof(TB)));
  TA va[NA];
  TB vb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = t + 256 * u;
      const int i = e / BK, k = e - (e / BK) * BK;
      const int gi = m0 + i, gk = k0 + k;
      const unsigned off = (gi < g.M && gk < g.K)
                               ? (unsigned)(((long long)gi * g.lda + gk) * sizeof(TA)) : BUF_OOB;
      va[u] = buf_ld<TA>(ra_, off);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = t + 256 * u;
      const int k = e / BN, j = e - (e / BN) * BN;
      const int gk = k0 + k, gj = n0 + j;
      const unsigned off = (gk < g.K && gj < g.N)
                               ? (unsigned)(((long long)gk * g.ldb + gj) * sizeof(TB)) : BUF_OOB;
      vb[u] = buf_ld<TB>(rb_, off);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = t + 256 * u;
      As[e - (e / BK) * BK][e / BK] = (T)va[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = t + 256 * u;
      Bs[e / BN][e - (e / BN) * BN] = (T)vb[u];
    }
    __syncthreads();
    if (k0 + BK < g.K) fetch(k0 + BK);
    if constexpr (sizeof(T) == 2) {
      // gfx950 32x32x16 (FP16 or BF16): lane l supplies row (column) l%32,
      // k = 8(l/32) .. +7; one product per chunk of 16
      using V8 = std::conditional_t<std::is_same<T, __bf16>::value, bf16x8, f16x8>;
      V8 a, b;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = As[8 * (lane >> 5) + u][wm + (lane & 31)];
        b[u] = Bs[8 * (lane >> 5) + u][wn + (lane & 31)];
      }
      if constexpr (std::is_same<T, __bf16>::value)
        accf = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, accf, 0, 0, 0);
      else
        accf = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, accf, 0, 0, 0);
    } else if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        const float a = As[kk + (lane >> 5)][wm + (lane & 31)];
        const float b = Bs[kk + (lane >> 5)][wn + (lane & 31)];
        accf = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, accf, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const double a = As[kk + (lane >> 4)][wm + (lane & 15)];
        const double b = Bs[kk + (lane >> 4)][wn + (lane & 15)];
        accd = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, accd, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue
  const TE* lam = (const TE*)g.lam;
  auto put = [&](int i, int j, TE v) {
    if (i >= g.M || j >= g.N) return;
    if constexpr (sizeof(T) == 2) {
      const float ls = g.ls_mode == 1 ? g.ls[(long long)bat * g.M + i]
                                      : g.ls[(long long)bat * g.N + j];
      v *= g.qs[0] * ls;
    }
    if (g.scale_mode == 2) v /= lam[i] + lam[j];
    else if (g.scale_mode == 3) v /= lam[i] + lam[j % g.m] + lam[j / g.m];
    Cb[(long long)i * g.ldc + j] = (TC)v;
  };
  if constexpr (sizeof(T) != 8) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      // 32x32x2 f32: accumulator v of lane l holds row 8(v/4) + 4(l/32) + v%4, column l%32
      const int i = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int j = n0 + wn + (lane & 31);
      put(i, j, accf[v]);
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // 16x16x4 f64: accumulator v of lane l holds row l/16 + 4 v, column l%16
      const int i = m0 + wm + (lane >> 4) + 4 * v;
      const int j = n0 + wn + (lane & 15);
      put(i, j, accd[v]);
    }
  }
}

// FP32 mode products on v_mfma_f32_16x16x4f32 with large workgroup tiles.
// Four waves in a 2 x 2 grid, each owning a WM x WN tile of 16 x 16 blocks
// (one accumulator per block), so the workgroup tile is 2 WM x 2 WN and a
// dimension of size m pads only to the next multiple of the tile chosen for
// it (m = 257: 288 with 96-wide tiles, against 320 with 64-wide ones).  K runs
// in chunks of 16 staged in LDS, two buffers: the next chunk's loads are in
// flight in registers during the current chunk's products and land in the
// other buffer after them (one barrier per chunk); the K tail skips its empty
// k-steps.  LDS rows are padded to 17 mod 32 words, so the transposing stores
// and the fragment reads of two k rows per half-wave stay within two-way
// bank conflicts.
template <int WM, int WN>
struct Tile16 {
  static constexpr int BM = 2 * WM, BN = 2 * WN, BK = 16;
  static constexpr int PA = (17 - BM % 32 + 32) % 32, PB = (17 - BN % 32 + 32) % 32;
  static constexpr int LDA = BM + PA, LDB = BN + PB;   // LDS row strides, == 17 mod 32
  static constexpr int RB = WM / 16, CB = WN / 16;     // 16 x 16 blocks per wave
  static constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
};

template <typename TA, typename TB, typename TC, int WM, int WN>
__global__ void __launch_bounds__(256) gemm_f32_t16(const TA* __restrict__ A,
                                                    const TB* __restrict__ B,
                                                    TC* __restrict__ Cm, GemmArgs g) {
  using Tl = Tile16<WM, WN>;
  constexpr int BM = Tl::BM, BN = Tl::BN, BK = Tl::BK, LDA = Tl::LDA, LDB = Tl::LDB;
  constexpr int RB = Tl::RB, CB = Tl::CB, NA = Tl::NA, NB = Tl::NB;
  __shared__ float As[2][BK * LDA];
  __shared__ float Bs[2][BK * LDB];
  const int bat = blockIdx.z;
  const int rhs = bat / g.batch_per_rhs;
  if (g.active && g.active[(size_t)rhs * g.astride] == 0.0) return;
  const TA* Ab = A + bat * g.sA;
  const TB* Bb = B + bat * g.sB;
  TC* Cb = Cm + bat * g.sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * WM, wn = (w & 1) * WN;
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  f32x4 acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const auto ra_ = buf_rsrc(Ab, (unsigned)(((long long)(g.M - 1) * g.lda + g.K) * sizeof(TA)));
  const auto rb_ = buf_rsrc(Bb, (unsigned)(((long long)(g.K - 1) * g.ldb + g.N) * sizeof(TB)));
  TA va[NA];
  TB vb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = t + 256 * u;
      const int i = e / BK, k = e % BK;
      const int gi = m0 + i, gk = k0 + k;
      const unsigned off = (gi < g.M && gk < g.K)
                               ? (unsigned)(((long long)gi * g.lda + gk) * sizeof(TA)) : BUF_OOB;
      va[u] = buf_ld<TA>(ra_, off);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = t + 256 * u;
      const int k = e / BN, j = e % BN;
      const int gk = k0 + k, gj = n0 + j;
      const unsigned off = (gk < g.K && gj < g.N)
                               ? (unsigned)(((long long)gk * g.ldb + gj) * sizeof(TB)) : BUF_OOB;
      vb[u] = buf_ld<TB>(rb_, off);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = t + 256 * u;
      As[buf][(e % BK) * LDA + e / BK] = (float)va[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = t + 256 * u;
      Bs[buf][(e / BN) * LDB + e % BN] = (float)vb[u];
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    const bool more = k0 + BK < g.K;
    if (more) fetch(k0 + BK);
    const int ksteps = min(4, (g.K - k0 + 3) >> 2);   // k-steps of 4 that hold data
    const float* Ab_ = As[buf];
    const float* Bb_ = Bs[buf];
    for (int s = 0; s < 4; ++s) {
      if (s < ksteps) {
        const int kk = 4 * s + (lane >> 4);
        float a[RB], b[CB];
#pragma unroll
        for (int i = 0; i < RB; ++i) a[i] = Ab_[kk * LDA + wm + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < CB; ++j) b[j] = Bb_[kk * LDB + wn + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) {
      stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  const float* lam = (const float*)g.lam;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // 16x16x4 f32: register v of lane l holds row 4 (l / 16) + v, column l % 16
        const int gi = m0 + wm + 16 * i + 4 * (lane >> 4) + v;
        const int gj = n0 + wn + 16 * j + (lane & 15);
        if (gi < g.M && gj < g.N) {
          float x = acc[i][j][v];
          if (g.scale_mode == 2) x /= lam[gi] + lam[gj];
          else if (g.scale_mode == 3) x /= lam[gi] + lam[gj % g.m] + lam[gj / g.m];
          Cb[(long long)gi * g.ldc + gj] = (TC)x;
        }
      }
}

// FP16 operand of a mode product along a direction with stride S > 1: line q
// of a right-hand side (q = o S + j, entries o m S + i S + j, i < m) is
// divided by its largest |value| and rounded to FP16; scale[rhs][q] keeps
// that value (1 for an all-zero line).  A workgroup takes QL consecutive lines
// (neighbouring addresses) with QG threads per line, each on every QG-th
// entry; the partial maxima meet in LDS.
constexpr int QL = 32, QG = 256 / QL;
template <typename TI, typename TQ>
__global__ void __launch_bounds__(256)
quant_lines(const TI* __restrict__ in, TQ* __restrict__ out, float* __restrict__ scale,
            int m, int S, int lines, long long N, int nrhs, const double* __restrict__ active,
            int astride) {
  __shared__ float red[QG][QL];
  const int l = threadIdx.x % QL, gq = threadIdx.x / QL;
  const long long q = (long long)blockIdx.x * QL + l;
  bool ok = q < (long long)lines * nrhs;
  const int rhs = ok ? (int)(q / lines) : 0;
  if (ok && active && active[(size_t)rhs * astride] == 0.0) ok = false;
  const int ql = (int)(q - (long long)rhs * lines);
  const long long base = (long long)rhs * N + (long long)(ql / S) * m * S + (ql % S);
  float mx = 0.0f;
  if (ok)
    for (int i = gq; i < m; i += QG) mx = fmaxf(mx, fabsf((float)in[base + (long long)i * S]));
  red[gq][l] = mx;
  __syncthreads();   // every thread arrives (no early exit above)
  mx = red[0][l];
  for (int k = 1; k < QG; ++k) mx = fmaxf(mx, red[k][l]);
  if (!ok) return;
  const float sc = mx > 0.0f ? mx : 1.0f;
  const float inv = 1.0f / sc;
  for (int i = gq; i < m; i += QG)
    out[base + (long long)i * S] = (TQ)((float)in[base + (long long)i * S] * inv);
  if (gq == 0) scale[q] = sc;
}

// direction 1 (lines contiguous): one wave per line, lanes stride the line
template <typename TI, typename TQ>
__global__ void __launch_bounds__(256)
quant_rows(const TI* __restrict__ in, TQ* __restrict__ out, float* __restrict__ scale,
           int m, int lines, long long N, int nrhs, const double* __restrict__ active,
           int astride) {
  const long long q = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= (long long)lines * nrhs) return;   // uniform per wave
  const int rhs = (int)(q / lines);
  if (active && active[(size_t)rhs * astride] == 0.0) return;
  const int ql = (int)(q - (long long)rhs * lines);
  const long long base = (long long)rhs * N + (long long)ql * m;
  float mx = 0.0f;
  for (int i = lane; i < m; i += 64) mx = fmaxf(mx, fabsf((float)in[base + i]));
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  const float sc = mx > 0.0f ? mx : 1.0f;
  const float inv = 1.0f / sc;
  for (int i = lane; i < m; i += 64) out[base + i] = (TQ)((float)in[base + i] * inv);
  if (lane == 0) scale[q] = sc;
}

// workgroup tile (64, 96 or 128) for a GEMM dimension of size x: the least
// padding, the larger tile on ties
static int tile16_for(int x) {
  int best = 128, pad = ((x + 127) / 128) * 128;
  for (int tsz : {96, 64}) {
    const int pd = ((x + tsz - 1) / tsz) * tsz;
    if (pd < pad) { pad = pd; best = tsz; }
  }
  return best;
}

template <typename TA, typename TB, typename TC, int WM, int WN>
static hipError_t gemm_t16(const TA* A, const TB* B, TC* C, const GemmArgs& g, int batches,
                           hipStream_t s) {
  dim3 grid((g.N + 2 * WN - 1) / (2 * WN), (g.M + 2 * WM - 1) / (2 * WM), batches);
  hipLaunchKernelGGL((gemm_f32_t16<TA, TB, TC, WM, WN>), grid, dim3(256), 0, s, A, B, C, g);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC, int WM>
static hipError_t gemm_t16_n(int bn, const TA* A, const TB* B, TC* C, const GemmArgs& g,
                             int batches, hipStream_t s) {
  if (bn == 64) return gemm_t16<TA, TB, TC, WM, 32>(A, B, C, g, batches, s);
  if (bn == 96) return gemm_t16<TA, TB, TC, WM, 48>(A, B, C, g, batches, s);
  return gemm_t16<TA, TB, TC, WM, 64>(A, B, C, g, batches, s);
}

template <typename TA, typename TB, typename TC, typename T>
static hipError_t gemm(const TA* A, const TB* B, TC* C, GemmArgs g, int batches, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    // large tiles where both dimensions fill them (the small problems keep the
    // 64 x 64 kernel below)
    if (g.M >= 64 && g.N >= 64 && g.K >= 16) {
      const int bm = tile16_for(g.M), bn = tile16_for(g.N);
      if (bm == 64) return gemm_t16_n<TA, TB, TC, 32>(bn, A, B, C, g, batches, s);
      if (bm == 96) return gemm_t16_n<TA, TB, TC, 48>(bn, A, B, C, g, batches, s);
      return gemm_t16_n<TA, TB, TC, 64>(bn, A, B, C, g, batches, s);
    }
  }
  constexpr int BM = 2 * MfmaCfg<T>::WT, BN = BM;
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, batches);
  hipLaunchKernelGGL((gemm_mfma<TA, TB, TC, T>), grid, dim3(256), 0, s, A, B, C, g);
  return hipGetLastError();
}

// one mode product along `axis` (1-based).  fwd: apply Q^T, else Q.
template <typename TI, typename TO, typename T>
static hipError_t mode_product(const Plan& P, int axis, bool fwd, const TI* in, TO* out, int nrhs,
                               int scale, const double* act, int as, hipStream_t s) {
  const char* tb = P.d_tables;
  const bool f64 = sizeof(T) == 8;
  const T* Q = (const T*)(tb + (f64 ? P.lay.qfd64 : P.lay.qfd32));
  const T* QT = (const T*)(tb + (f64 ? P.lay.qtfd64 : P.lay.qtfd32));
  const T* lam = (const T*)(tb + (f64 ? P.lay.lamfd64 : P.lay.lamfd32));
  const int m = P.m;
  const long long N = P.N;
  GemmArgs g{};
  g.active = act;
  g.astride = as;
  g.lam = lam;
  g.scale_mode = scale;
  g.m = m;
  if (axis == 1) {
    // C[M x m] = X[M x m] * (Q or Q^T), M = m^{d-1} per right-hand side
    g.M = (int)(N / m); g.N = m; g.K = m;
    g.lda = m; g.ldb = m; g.ldc = m;
    g.sA = N; g.sB = 0; g.sC = N;
    g.batch_per_rhs = 1;
    return gemm<TI, T, TO, T>(in, fwd ? Q : QT, out, g, nrhs, s);
  }
  int S = 1;
  for (int k = 1; k < axis; ++k) S *= m;
  const int outer = (int)(N / ((long long)S * m));
  g.M = m; g.N = S; g.K = m;
  g.lda = m; g.ldb = S; g.ldc = S;
  g.sA = 0; g.sB = (long long)S * m; g.sC = (long long)S * m;
  g.batch_per_rhs = outer;
  return gemm<T, TI, TO, T>(fwd ? QT : Q, in, out, g, outer * nrhs, s);
}

template <typename T>
static hipError_t fd_apply_t(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                             const double* a, int as, hipStream_t s) {
  const int d = P.d;
  const size_t N = (size_t)P.N * nrhs;
  T* t1 = (T*)ws;
  T* t2 = sizeof(T) == 8 ? (T*)z : t1 + N;  // FP64: ping-pong with z
  hipError_t e;
  // forward: Q^T along every direction, scaling fused into the last one
  e = mode_product<double, T, T>(P, 1, true, r, t1, nrhs, 0, a, as, s);
  if (e != hipSuccess) return e;
  T* cur = t1;
  T* nxt = t2;
  for (int k = 2; k <= d; ++k) {
    e = mode_product<T, T, T>(P, k, true, cur, nxt, nrhs, k == d ? d : 0, a, as, s);
    if (e != hipSuccess) return e;
    std::swap(cur, nxt);
  }
  // backward: Q along directions d .. 2, then direction 1 into z (FP64)
  for (int k = d; k >= 2; --k) {
    e = mode_product<T, T, T>(P, k, false, cur, nxt, nrhs, 0, a, as, s);
    if (e != hipSuccess) return e;
    std::swap(cur, nxt);
  }
  return mode_product<T, double, T>(P, 1, false, cur, z, nrhs, 0, a, as, s);
}

// FP16 / BF16 (TQ) mode product along `axis`: in (TI) -> quantized lines -> GEMM ->
// out (TO), line scales and s_Q restored in the epilogue
template <typename TQ, typename TI, typename TO>
static hipError_t mode_product16(const Plan& P, int axis, bool fwd, const TI* in, TO* out,
                                 TQ* x16, float* ls, int nrhs, int scale, const double* act,
                                 int as, hipStream_t s) {
  const char* tb = P.d_tables;
  const TQ* Q = (const TQ*)(tb + P.lay.qfd16);
  const TQ* QT = (const TQ*)(tb + P.lay.qtfd16);
  const float* qs = (const float*)(tb + P.lay.qs16);
  const float* lam = (const float*)(tb + P.lay.lamfd32);
  const int m = P.m;
  const long long N = P.N;
  int S = 1;
  for (int k = 1; k < axis; ++k) S *= m;
  const int lines = (int)(N / m);
  const long long nq = (long long)lines * nrhs;
  if (S == 1)
    hipLaunchKernelGGL((quant_rows<TI, TQ>), dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, in, x16,
                       ls, m, lines, N, nrhs, act, as);
  else
    hipLaunchKernelGGL((quant_lines<TI, TQ>), dim3((unsigned)((nq + QL - 1) / QL)), dim3(256), 0, s, in,
                       x16, ls, m, S, lines, N, nrhs, act, as);
  GemmArgs g{};
  g.active = act;
  g.astride = as;
  g.lam = lam;
  g.scale_mode = scale;
  g.m = m;
  g.ls = ls;
  g.qs = qs;
  if (axis == 1) {
    g.M = lines; g.N = m; g.K = m;
    g.lda = m; g.ldb = m; g.ldc = m;
    g.sA = N; g.sB = 0; g.sC = N;
    g.batch_per_rhs = 1;
    g.ls_mode = 1;
    return gemm<TQ, TQ, TO, TQ>(x16, fwd ? Q : QT, out, g, nrhs, s);
  }
  const int outer = (int)(N / ((long long)S * m));
  g.M = m; g.N = S; g.K = m;
  g.lda = m; g.ldb = S; g.ldc = S;
  g.sA = 0; g.sB = (long long)S * m; g.sC = (long long)S * m;
  g.batch_per_rhs = outer;
  g.ls_mode = 2;
  return gemm<TQ, TQ, TO, TQ>(fwd ? QT : Q, x16, out, g, outer * nrhs, s);
}

template <typename TQ>
static hipError_t fd_apply_f16(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                               const double* a, int as, hipStream_t s) {
  const int d = P.d;
  const size_t N = (size_t)P.N * nrhs;
  const size_t b32 = (8 * N + 255) & ~(size_t)255, b16 = (2 * N + 255) & ~(size_t)255;
  float* t1 = (float*)ws;
  float* t2 = t1 + N;
  TQ* x16 = (TQ*)((char*)ws + b32);
  float* ls = (float*)((char*)ws + b32 + b16);
  hipError_t e = mode_product16<TQ, double, float>(P, 1, true, r, t1, x16, ls, nrhs, d == 1 ? d : 0,
                                               a, as, s);
  if (e != hipSuccess) return e;
  float* cur = t1;
  float* nxt = t2;
  for (int k = 2; k <= d; ++k) {
    e = mode_product16<TQ, float, float>(P, k, true, cur, nxt, x16, ls, nrhs, k == d ? d : 0, a, as, s);
    if (e != hipSuccess) return e;
    std::swap(cur, nxt);
  }
  for (int k = d; k >= 2; --k) {
    e = mode_product16<TQ, float, float>(P, k, false, cur, nxt, x16, ls, nrhs, 0, a, as, s);
    if (e != hipSuccess) return e;
    std::swap(cur, nxt);
  }
  return mode_product16<TQ, float, double>(P, 1, false, cur, z, x16, ls, nrhs, 0, a, as, s);
}

// ---- general plans: every direction its own m_k, Q_k and eigenvalues --------

// one mode product of a general plan along `axis` (1-based): the direction's
// own Q (or Q^T), lines of length m_k with stride S = m_1 .. m_{k-1}
template <typename TI, typename TO, typename T>
static hipError_t mode_product_gen(const Plan& P, int axis, bool fwd, const TI* in, TO* out,
                                   int nrhs, const double* act, int as, hipStream_t s) {
  const GDir& G = P.dirs[axis - 1];
  const bool f64 = sizeof(T) == 8;
  const T* Q = (const T*)(P.d_tables + (f64 ? G.fq64 : G.fq32));
  const T* QT = (const T*)(P.d_tables + (f64 ? G.fqt64 : G.fqt32));
  const int m = G.m;
  const long long N = P.N;
  GemmArgs g{};
  g.active = act;
  g.astride = as;
  g.scale_mode = 0;
  g.m = m;
  if (axis == 1) {
    g.M = (int)(N / m); g.N = m; g.K = m;
    g.lda = m; g.ldb = m; g.ldc = m;
    g.sA = N; g.sB = 0; g.sC = N;
    g.batch_per_rhs = 1;
    return gemm<TI, T, TO, T>(in, fwd ? Q : QT, out, g, nrhs, s);
  }
  int S = 1;
  for (int k = 0; k < axis - 1; ++k) S *= P.dirs[k].m;
  const int outer = (int)(N / ((long long)S * m));
  g.M = m; g.N = S; g.K = m;
  g.lda = m; g.ldb = S; g.ldc = S;
  g.sA = 0; g.sB = (long long)S * m; g.sC = (long long)S * m;
  g.batch_per_rhs = outer;
  return gemm<T, TI, TO, T>(fwd ? QT : Q, in, out, g, outer * nrhs, s);
}

// x[i1 + m1 (i2 + m2 i3)] /= l1[i1] + l2[i2] (+ l3[i3]): the Kronecker sum of
// the directions' eigenvalues (eq:exact_diagonalization)
template <typename T>
__global__ void __launch_bounds__(256)
fd_scale_gen(T* __restrict__ x, const T* __restrict__ l1, const T* __restrict__ l2,
             const T* __restrict__ l3, int m1, int m2, int N, int nrhs,
             const double* __restrict__ active, int astride) {
  const long long tot = (long long)N * nrhs;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
    const int rhs = (int)(e / N), i = (int)(e - (long long)rhs * N);
    if (active && active[(size_t)rhs * astride] == 0.0) continue;
    const int i1 = i % m1, rest = i / m1;
    const int i2 = rest % m2, i3 = rest / m2;
    T den = l1[i1] + l2[i2];
    if (l3) den += l3[i3];
    x[e] /= den;
  }
}

template <typename T>
static hipError_t fd_apply_gen(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                               const double* a, int as, hipStream_t s) {
  const int d = P.d;
  const size_t N = (size_t)P.N * nrhs;
  T* t1 = (T*)ws;
  T* t2 = sizeof(T) == 8 ? (T*)z : t1 + N;  // FP64: ping-pong with z
  hipError_t e = mode_product_gen<double, T, T>(P, 1, true, r, t1, nrhs, a, as, s);
  if (e != hipSuccess) return e;
  T* cur = t1;
  T* nxt = t2;
  for (int k = 2; k <= d; ++k) {
    e = mode_product_gen<T, T, T>(P, k, true, cur, nxt, nrhs, a, as, s);
    if (e != hipSuccess) return e;
    std::swap(cur, nxt);
  }
  {
    const bool f64 = sizeof(T) == 8;
    auto lam = [&](int k) { return (const T*)(P.d_tables + (f64 ? P.dirs[k].flam64 : P.dirs[k].flam32)); };
    const long long tot = (long long)N;
    const unsigned nb = (unsigned)std::min<long long>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(fd_scale_gen<T>, dim3(nb), dim3(256), 0, s, cur, lam(0), lam(1),
                       d == 3 ? lam(2) : (const T*)nullptr, P.dirs[0].m, P.dirs[1].m, (int)P.N,
                       nrhs, a, as);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int k = d; k >= 2; --k) {
    e = mode_product_gen<T, T, T>(P, k, false, cur, nxt, nrhs, a, as, s);
    if (e != hipSuccess) return e;
    std::swap(cur, nxt);
  }
  return mode_product_gen<T, double, T>(P, 1, false, cur, z, nrhs, a, as, s);
}

hipError_t launch_fd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                           const double* active, int astride, hipStream_t s) {
  if (P.method != IFFD_METHOD_DENSE_FD) return hipErrorInvalidValue;
  if (P.gen) {
    if (P.prec == IFFD_PREC_F64) return fd_apply_gen<double>(P, r, z, nrhs, ws, active, astride, s);
    if (P.prec == IFFD_PREC_F32) return fd_apply_gen<float>(P, r, z, nrhs, ws, active, astride, s);
    return hipErrorInvalidValue;
  }
  if (P.prec == IFFD_PREC_F16S) return fd_apply_f16<_Float16>(P, r, z, nrhs, ws, active, astride, s);
  if (P.prec == IFFD_PREC_BF16S) return fd_apply_f16<__bf16>(P, r, z, nrhs, ws, active, astride, s);
  if (P.prec == IFFD_PREC_F64) return fd_apply_t<double>(P, r, z, nrhs, ws, active, astride, s);
  return fd_apply_t<float>(P, r, z, nrhs, ws, active, astride, s);
}

}  // namespace iffd
