// Instantiations of the IFFD line pass for FFT lengths 16, 24, 32, 48.
#include "apply_impl.h"

namespace iffd {

hipError_t line_pass_L16(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  return line_pass_for_L<16>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

hipError_t line_pass_L24(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  return line_pass_for_L<24>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

hipError_t line_pass_L32(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  return line_pass_for_L<32>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

hipError_t line_pass_L48(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  return line_pass_for_L<48>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

}  // namespace iffd
