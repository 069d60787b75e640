// The IFFD preconditioner of eq:preconditioner for small 2-D problems:
//   Z = Qt_1 W Qt_2^T,  W = (Qt_1^T R Qt_2) / (lam_1[a] + lam_2[b]),
// with R, Z the m_2 x m_1 coefficient arrays (direction 1 fastest) and Qt_k =
// [V_reg U Dt^{-1}, V_out Q_out] (Sections 4 and 6) held densely, one FP32
// m_k x m_k table per direction (row = dof, column = mode).  This is the same
// linear map as the line passes; at m <= 128 a dense product costs 2m flops
// per entry per direction instead of the transform's O(log m + p), but the
// whole apply is two launches whose workgroups never wait on one another,
// against three line passes whose FFT stages each end in a barrier.
//
//   launch A: each workgroup takes 8 modes a of direction 1 and one
//             right-hand side: T = Qt_1[:, a]^T R, W = T Qt_2 scaled,
//             V = W Qt_2^T, written as v[rhs][j][a] (FP32 workspace);
//   launch B: each workgroup takes 8 rows j of Z: Z[j][:] = V[:, j]^T Qt_1^T,
//             written in FP64.
// Every product runs from LDS: the left operand k-major with the 8 slice rows
// contiguous (a wave reads its row's entry as one broadcast), the right operand
// with an odd row stride so that the 64 lanes of a wave, one column each,
// read 64 different banks in either orientation.
#include "dense2d.h"

namespace iffd {

namespace {

constexpr int kSl = 8;     // slice rows per workgroup (8 waves x 1 row)
constexpr int kNt = 512;

// the k-major operands are read two floats at a time: their LDS regions start
// at an even float offset
__host__ __device__ constexpr int even(int x) { return x + (x & 1); }

struct D2Args {
  const double* r;
  float* v;
  double* z;
  const float* q1;   // Qt_1, m1 x m1, row = dof
  const float* q2;   // Qt_2, m2 x m2
  const float* l1;   // lam of direction 1 (m1), of direction 2 (m2)
  const float* l2;
  int m1, m2;
  float inv1, inv2;  // 1 / m1, 1 / m2
  const double* active;
  int astride;
};

// Copies n elements of one source into LDS: load(e) reads element e (its
// index clamped into the source, so every load is issued unconditionally),
// put(e, x) stores it for e < n.  Each thread issues kInflight loads before
// its first store, so a workgroup waits for about n / (kNt kInflight) load
// latencies instead of n / kNt.
constexpr int kInflight = 16;
template <typename Load, typename Put>
__device__ __forceinline__ void stage(int n, Load load, Put put) {
  for (int base = 0; base < n; base += kNt * kInflight) {
    float x[kInflight];
#pragma unroll
    for (int u = 0; u < kInflight; ++u) x[u] = load(min(base + u * kNt + (int)threadIdx.x, n - 1));
#pragma unroll
    for (int u = 0; u < kInflight; ++u) {
      const int e = base + u * kNt + (int)threadIdx.x;
      if (e < n) put(e, x[u]);
    }
  }
}

// e / m for 0 <= e < 129 m, m <= 128, with inv = 1/m rounded to FP32: the
// product is within a few ulps of (e + 1/2) / m, which is at least 1/(2m)
// away from an integer
__device__ __forceinline__ int div_small(int e, float inv) {
  return (int)(((float)e + 0.5f) * inv);
}

// C(a, c) = sum_k A[k kSl + a] B(c, k) for the 8 rows a of a slice and the
// columns c < nc <= 128, with B(c, k) = B[c ldb + k] (CK) or B[k ldb + c].
// Wave w computes row w, lane l the columns l and l + 64 (two waves per SIMD
// hide each other's LDS latency); out(a, c, value) receives each result once.
template <bool CK, typename F>
__device__ __forceinline__ void lds_product(const float* A, const float* B, int ldb, int K, int nc,
                                            F out) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c0 = lane, c1 = lane + 64;
  const int r0 = c0 < nc ? c0 : 0, r1 = c1 < nc ? c1 : 0;   // idle lanes read column 0
  float x0 = 0.f, x1 = 0.f;
  if (nc > 64) {
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
      const float a = A[k * kSl + w];
      const float b0 = CK ? B[r0 * ldb + k] : B[k * ldb + r0];
      const float b1 = CK ? B[r1 * ldb + k] : B[k * ldb + r1];
      x0 += a * b0;
      x1 += a * b1;
    }
  } else {   // one column per lane (the same branch for the whole workgroup)
#pragma unroll 4
    for (int k = 0; k < K; ++k) x0 += A[k * kSl + w] * (CK ? B[r0 * ldb + k] : B[k * ldb + r0]);
  }
  if (c0 < nc) out(w, c0, x0);
  if (c1 < nc) out(w, c1, x1);
}

__global__ void __launch_bounds__(kNt) dense2d_a(D2Args g) {
  extern __shared__ __align__(16) float sm[];
  const int rhs = blockIdx.y, a0 = blockIdx.x * kSl;
  if (g.active && g.active[(size_t)rhs * g.astride] == 0.0) return;
  const int m1 = g.m1, m2 = g.m2, s1 = m1 | 1, s2 = m2 | 1;
  float* R = sm;                  // R[j][i], stride s1
  float* Q2 = R + m2 * s1;        // Qt_2[j][b], stride s2
  float* A1 = Q2 + even(m2 * s2) + ((m2 * s1) & 1);   // Qt_1[i][a0 + a] at i kSl + a (8-byte aligned)
  float* T = A1 + m1 * kSl;       // T[a][j] at j kSl + a
  float* W = T + m2 * kSl;        // W[a][b] at b kSl + a
  const double* r = g.r + (size_t)rhs * m1 * m2;
  // R, Qt_2 and the slice's columns of Qt_1 (zero past m1)
  stage(m1 * m2, [&](int e) { return (float)r[e]; }, [&](int e, float x) {
    const int j = div_small(e, g.inv1);
    R[j * s1 + e - j * m1] = x;
  });
  stage(m2 * m2, [&](int e) { return g.q2[e]; }, [&](int e, float x) {
    const int j = div_small(e, g.inv2);
    Q2[j * s2 + e - j * m2] = x;
  });
  stage(m1 * kSl, [&](int e) { return g.q1[(size_t)(e >> 3) * m1 + min(a0 + (e & 7), m1 - 1)]; },
        [&](int e, float x) { A1[e] = a0 + (e & 7) < m1 ? x : 0.f; });
  __syncthreads();
  // T[a][j] = sum_i Qt_1[i][a0 + a] R[j][i]
  lds_product<true>(A1, R, s1, m1, m2, [&](int a, int j, float x) { T[j * kSl + a] = x; });
  __syncthreads();
  // W[a][b] = sum_j T[a][j] Qt_2[j][b] / (lam_1[a0 + a] + lam_2[b]); rows past
  // m1 are zero (their Qt_1 columns were) and stay zero
  lds_product<false>(T, Q2, s2, m2, m2, [&](int a, int b, float x) {
    const float la = a0 + a < m1 ? g.l1[a0 + a] : 1.f;
    W[b * kSl + a] = x * __builtin_amdgcn_rcpf(la + g.l2[b]);
  });
  __syncthreads();
  // V[a][j] = sum_b W[a][b] Qt_2[j][b]
  float* v = g.v + (size_t)rhs * m1 * m2;
  lds_product<true>(W, Q2, s2, m2, m2, [&](int a, int j, float x) {
    if (a0 + a < m1) v[(size_t)j * m1 + a0 + a] = x;
  });
}

__global__ void __launch_bounds__(kNt) dense2d_b(D2Args g) {
  extern __shared__ __align__(16) float sm[];
  const int rhs = blockIdx.y, j0 = blockIdx.x * kSl;
  if (g.active && g.active[(size_t)rhs * g.astride] == 0.0) return;
  const int m1 = g.m1, m2 = g.m2, s1 = m1 | 1;
  float* Q1 = sm;                 // Qt_1[i][a], stride s1
  float* A = Q1 + even(m1 * s1);  // V[a][j0 + jj] at a kSl + jj (8-byte aligned)
  const float* v = g.v + (size_t)rhs * m1 * m2;
  // Qt_1 and the slice's rows of V (zero past m2)
  stage(m1 * m1, [&](int e) { return g.q1[e]; }, [&](int e, float x) {
    const int i = div_small(e, g.inv1);
    Q1[i * s1 + e - i * m1] = x;
  });
  stage(kSl * m1,
        [&](int e) {
          const int jj = div_small(e, g.inv1);
          return v[(size_t)min(j0 + jj, m2 - 1) * m1 + e - jj * m1];
        },
        [&](int e, float x) {
          const int jj = div_small(e, g.inv1);
          A[(e - jj * m1) * kSl + jj] = j0 + jj < m2 ? x : 0.f;
        });
  __syncthreads();
  // Z[j0 + jj][i] = sum_a V[a][j0 + jj] Qt_1[i][a]
  double* z = g.z + (size_t)rhs * m1 * m2;
  lds_product<true>(A, Q1, s1, m1, m1, [&](int jj, int i, float x) {
    if (j0 + jj < m2) z[(size_t)(j0 + jj) * m1 + i] = (double)x;
  });
}

}  // namespace

size_t dense2d_lds_a(int m1, int m2) {
  const int r = m2 * (m1 | 1), q = m2 * (m2 | 1);
  return 4 * ((size_t)r + even(q) + (r & 1) + (size_t)(m1 + 2 * m2) * kSl);
}
size_t dense2d_lds_b(int m1) { return 4 * ((size_t)even(m1 * (m1 | 1)) + (size_t)m1 * kSl); }

hipError_t launch_dense2d(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                          const double* active, int astride, hipStream_t s) {
  if (!P.dense2d || !ws || nrhs < 1) return hipErrorInvalidValue;
  D2Args g{};
  const char* b = P.d_tables;
  if (P.gen) {
    g.m1 = P.dirs[0].m;
    g.m2 = P.dirs[1].m;
    g.q1 = (const float*)(b + P.dirs[0].dq32);
    g.q2 = (const float*)(b + P.dirs[1].dq32);
    g.l1 = (const float*)(b + P.dirs[0].dlam32);
    g.l2 = (const float*)(b + P.dirs[1].dlam32);
  } else {
    g.m1 = g.m2 = P.m;
    g.q1 = g.q2 = (const float*)(b + P.lay.dq32);
    g.l1 = g.l2 = (const float*)(b + P.lay.dlam32);
  }
  if (g.m1 < 1 || g.m2 < 1 || g.m1 > kDenseMax || g.m2 > kDenseMax) return hipErrorInvalidValue;
  g.inv1 = 1.0f / (float)g.m1;
  g.inv2 = 1.0f / (float)g.m2;
  g.r = r;
  g.z = z;
  g.v = (float*)ws;
  g.active = active;
  g.astride = astride;
  const size_t la = dense2d_lds_a(g.m1, g.m2), lb = dense2d_lds_b(g.m1);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)dense2d_a,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)dense2d_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(dense2d_a, dim3((unsigned)((g.m1 + kSl - 1) / kSl), (unsigned)nrhs), dim3(kNt),
                     la, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dense2d_b, dim3((unsigned)((g.m2 + kSl - 1) / kSl), (unsigned)nrhs), dim3(kNt),
                     lb, s, g);
  return hipGetLastError();
}

}  // namespace iffd
