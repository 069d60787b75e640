// Instantiations of the IFFD line pass for FFT lengths 64, 96.
#include "apply_impl.h"

namespace iffd {

hipError_t line_pass_L64(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  return line_pass_for_L<64>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

hipError_t line_pass_L96(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  return line_pass_for_L<96>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

}  // namespace iffd
