// Classical Fast Diagonalization (Section 3, eq:exact_diagonalization) on
// gfx950: z = (Q x .. x Q) (sum_k Lambda_k)^{-1} (Q^T x .. x Q^T) r with the
// dense m x m eigenvector matrix Q of the pencil (K, M).  The mode products
// are GEMMs; they run on the matrix cores (MFMA).
#include "launch.h"

namespace iffd {

hipError_t launch_fd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                           const double* active, int astride, hipStream_t s) {
  (void)P; (void)r; (void)z; (void)nrhs; (void)ws; (void)active; (void)astride; (void)s;
  return hipErrorNotSupported;
}

}  // namespace iffd
