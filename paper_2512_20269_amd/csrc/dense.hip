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
// forward product.  FP32 uses v_mfma_f32_32x32x2f32 (a wave owns a 32 x 32
// tile), FP64 v_mfma_f64_16x16x4f64 (16 x 16 per wave); four waves per
// workgroup, K staged through LDS in chunks.
#include <utility>

#include "launch.h"

namespace iffd {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

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
};

template <typename T> struct MfmaCfg;
template <> struct MfmaCfg<float> { static constexpr int WT = 32, BK = 16; };   // wave tile
template <> struct MfmaCfg<double> { static constexpr int WT = 16, BK = 16; };

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

  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // stage A (BM x BK) and B (BK x BN) tiles, zero outside the matrices
    for (int e = t; e < BM * BK; e += 256) {
      const int i = e / BK, k = e - (e / BK) * BK;
      const int gi = m0 + i, gk = k0 + k;
      As[k][i] = (gi < g.M && gk < g.K) ? (T)Ab[(long long)gi * g.lda + gk] : T(0);
    }
    for (int e = t; e < BK * BN; e += 256) {
      const int k = e / BN, j = e - (e / BN) * BN;
      const int gk = k0 + k, gj = n0 + j;
      Bs[k][j] = (gk < g.K && gj < g.N) ? (T)Bb[(long long)gk * g.ldb + gj] : T(0);
    }
    __syncthreads();
    if constexpr (sizeof(T) == 4) {
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
  const T* lam = (const T*)g.lam;
  auto put = [&](int i, int j, T v) {
    if (i >= g.M || j >= g.N) return;
    if (g.scale_mode == 2) v /= lam[i] + lam[j];
    else if (g.scale_mode == 3) v /= lam[i] + lam[j % g.m] + lam[j / g.m];
    Cb[(long long)i * g.ldc + j] = (TC)v;
  };
  if constexpr (sizeof(T) == 4) {
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

template <typename TA, typename TB, typename TC, typename T>
static hipError_t gemm(const TA* A, const TB* B, TC* C, GemmArgs g, int batches, hipStream_t s) {
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

hipError_t launch_fd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                           const double* active, int astride, hipStream_t s) {
  if (P.method != IFFD_METHOD_DENSE_FD) return hipErrorInvalidValue;
  if (P.prec == IFFD_PREC_F64) return fd_apply_t<double>(P, r, z, nrhs, ws, active, astride, s);
  return fd_apply_t<float>(P, r, z, nrhs, ws, active, astride, s);
}

}  // namespace iffd
