// Instantiations of the IFFD line pass for FFT lengths 128.
#include "apply_impl.h"

namespace iffd {

hipError_t line_pass_L128(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  return line_pass_for_L<128>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

}  // namespace iffd
