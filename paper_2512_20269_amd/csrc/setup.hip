// Device-side completion of the IFFD tables: the generalized eigenproblem of
// the outlier block (eq:eigendecomposition_out)
//     Q_out^T (V_out^T K V_out) Q_out = Lambda_out,
//     Q_out^T (V_out^T M V_out) Q_out = I,
// solved in FP64 (n_out <= 8) by a Cholesky reduction and cyclic Jacobi, then
// Vt = (V_out Q_out)^T and the outlier eigenvalues are written into the
// tables in FP64 and FP32.  A status word reports a pencil whose mass block
// is not positive definite (the Cholesky pivot that failed, 1-based) or a
// non-finite or non-positive result (-1); the tables are then left unused.
#include "launch.h"

namespace iffd {

__global__ void setup_outliers_kernel(const double* Ao, const double* Bo, const double* Vout,
                                      int no, int m, int n_reg, double* lam64, float* lam32,
                                      double* vt64, float* vt32, double* stat) {
  __shared__ double Qs[64];
  __shared__ double ls[8];
  __shared__ int bad;
  if (threadIdx.x == 0) {
    double L[64], C[64], T[64], Z[64], w[8];
    for (int i = 0; i < 64; ++i) { L[i] = 0; C[i] = 0; Z[i] = 0; }
    // Cholesky Bo = L L^T; a non-positive pivot is reported, not clamped
    int bad_t = 0;
    for (int j = 0; j < no && !bad_t; ++j)
      for (int i = j; i < no; ++i) {
        double s = Bo[i * no + j];
        for (int k = 0; k < j; ++k) s -= L[i * 8 + k] * L[j * 8 + k];
        if (i == j) {
          if (!(s > 0.0)) { bad_t = j + 1; break; }
          L[j * 8 + j] = sqrt(s);
        } else {
          L[i * 8 + j] = s / L[j * 8 + j];
        }
      }
    if (!bad_t) {
      // T = L^{-1} Ao ; C = L^{-1} T^T = L^{-1} Ao L^{-T}
      for (int c = 0; c < no; ++c)
        for (int i = 0; i < no; ++i) {
          double s = Ao[i * no + c];
          for (int k = 0; k < i; ++k) s -= L[i * 8 + k] * T[k * 8 + c];
          T[i * 8 + c] = s / L[i * 8 + i];
        }
      for (int c = 0; c < no; ++c)
        for (int i = 0; i < no; ++i) {
          double s = T[c * 8 + i];
          for (int k = 0; k < i; ++k) s -= L[i * 8 + k] * C[k * 8 + c];
          C[i * 8 + c] = s / L[i * 8 + i];
        }
      for (int i = 0; i < no; ++i) {
        Z[i * 8 + i] = 1.0;
        for (int j = i + 1; j < no; ++j) {
          double a = 0.5 * (C[i * 8 + j] + C[j * 8 + i]);
          C[i * 8 + j] = C[j * 8 + i] = a;
        }
      }
      const double eps = 2.220446049250313e-16;
      for (int sweep = 0; sweep < 60; ++sweep) {
        bool rot = false;
        for (int p = 0; p < no - 1; ++p)
          for (int q = p + 1; q < no; ++q) {
            double apq = C[p * 8 + q], app = C[p * 8 + p], aqq = C[q * 8 + q];
            if (fabs(apq) <= fmax(eps * sqrt(fabs(app * aqq)), 1e-300)) continue;
            rot = true;
            double th = (aqq - app) / (2 * apq);
            double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1));
            double c = 1 / sqrt(t * t + 1), s = t * c;
            for (int k = 0; k < no; ++k) {
              double a = C[p * 8 + k], b = C[q * 8 + k];
              C[p * 8 + k] = c * a - s * b;
              C[q * 8 + k] = s * a + c * b;
            }
            for (int k = 0; k < no; ++k) {
              double a = C[k * 8 + p], b = C[k * 8 + q];
              C[k * 8 + p] = c * a - s * b;
              C[k * 8 + q] = s * a + c * b;
              double za = Z[k * 8 + p], zb = Z[k * 8 + q];
              Z[k * 8 + p] = c * za - s * zb;
              Z[k * 8 + q] = s * za + c * zb;
            }
          }
        if (!rot) break;
      }
      for (int i = 0; i < no; ++i) w[i] = C[i * 8 + i];
      // Q = L^{-T} Z
      for (int c = 0; c < no; ++c)
        for (int i = no - 1; i >= 0; --i) {
          double s = Z[i * 8 + c];
          for (int k = i + 1; k < no; ++k) s -= L[k * 8 + i] * T[k * 8 + c];
          T[i * 8 + c] = s / L[i * 8 + i];
        }
      // ascending order (selection sort on a handful of values)
      int ord[8];
      for (int i = 0; i < no; ++i) ord[i] = i;
      for (int i = 0; i < no; ++i)
        for (int j = i + 1; j < no; ++j)
          if (w[ord[j]] < w[ord[i]]) { int tmp = ord[i]; ord[i] = ord[j]; ord[j] = tmp; }
      bool finite = true;
      for (int j = 0; j < no; ++j) {
        ls[j] = w[ord[j]];
        finite = finite && isfinite(ls[j]) && ls[j] > 0.0;
        for (int i = 0; i < no; ++i) {
          Qs[i * 8 + j] = T[i * 8 + ord[j]];
          finite = finite && isfinite(Qs[i * 8 + j]);
        }
      }
      if (!finite) bad_t = -1;
    }
    bad = bad_t;
    stat[0] = (double)bad_t;
  }
  __syncthreads();
  if (bad) return;
  for (int idx = threadIdx.x; idx < no * m; idx += blockDim.x) {
    const int q = idx / m, i = idx - (idx / m) * m;
    double acc = 0;
    for (int k = 0; k < no; ++k) acc += Qs[k * 8 + q] * Vout[(size_t)k * m + i];
    vt64[idx] = acc;
    vt32[idx] = (float)acc;
  }
  if ((int)threadIdx.x < no) {
    lam64[n_reg + threadIdx.x] = ls[threadIdx.x];
    lam32[n_reg + threadIdx.x] = (float)ls[threadIdx.x];
  }
}

hipError_t launch_setup_outliers_at(const double* Ao, const double* Bo, const double* Vout, int no,
                                    int m, int n_reg, double* lam64, float* lam32, double* vt64,
                                    float* vt32, double* stat, hipStream_t s) {
  if (no == 0) return hipSuccess;
  hipLaunchKernelGGL(setup_outliers_kernel, dim3(1), dim3(256), 0, s, Ao, Bo, Vout, no, m, n_reg,
                     lam64, lam32, vt64, vt32, stat);
  return hipGetLastError();
}

hipError_t launch_setup_outliers(const Plan& P, hipStream_t s) {
  if (P.n_out == 0) return hipSuccess;
  char* b = P.d_tables;
  const TableLayout& t = P.lay;
  hipLaunchKernelGGL(setup_outliers_kernel, dim3(1), dim3(256), 0, s, (const double*)(b + t.ao64),
                     (const double*)(b + t.bo64), (const double*)(b + t.vout64), P.n_out, P.m,
                     P.n_reg, (double*)(b + t.lam64), (float*)(b + t.lam32),
                     (double*)(b + t.vt64), (float*)(b + t.vt32), (double*)(b + t.stat64));
  return hipGetLastError();
}

}  // namespace iffd
