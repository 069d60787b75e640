// IFFD apply: dispatch of the line passes (apply_impl.h) over FFT lengths and
// the sequence of passes that forms z = P^{-1} r.
#include "launch.h"

namespace iffd {

hipError_t line_pass_L16(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L24(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L32(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L48(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L64(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L96(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L128(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L192(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);
hipError_t line_pass_L256(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s);

hipError_t launch_line_pass(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                            void* out, int nrhs, const double* a, int as, hipStream_t s) {
  // pass index of (mode, axis) for the per-pass variant choice
  const int d = P.d;
  const int pass = mode == PASS_FWD ? axis - 1 : (mode == PASS_MID ? d - 1 : 2 * d - 1 - axis);
  const int var = P.variant[pass];
  switch (P.L) {
    case 16: return line_pass_L16(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 24: return line_pass_L24(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 32: return line_pass_L32(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 48: return line_pass_L48(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 64: return line_pass_L64(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 96: return line_pass_L96(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 128: return line_pass_L128(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 192: return line_pass_L192(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    case 256: return line_pass_L256(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_iffd_pass(const Plan& P, int pass, const double* r, double* z, int nrhs,
                            void* ws, const double* a, int as, hipStream_t s) {
  const int d = P.d;
  const bool f64 = P.prec == IFFD_PREC_F64;
  const int et = f64 ? ELEM_F64 : ELEM_F32;
  void* w = f64 ? (void*)z : ws;
  if (pass < d - 1) {
    const bool first = pass == 0;
    return launch_line_pass(P, PASS_FWD, pass + 1, first ? ELEM_F64 : et, first ? (const void*)r : w,
                            et, w, nrhs, a, as, s);
  }
  if (pass == d - 1) return launch_line_pass(P, PASS_MID, d, et, w, et, w, nrhs, a, as, s);
  if (pass < 2 * d - 1) {
    const int axis = 2 * d - 1 - pass;  // d-1 .. 1
    const bool last = axis == 1;
    return launch_line_pass(P, PASS_BWD, axis, et, w, last ? ELEM_F64 : et, last ? (void*)z : w,
                            nrhs, a, as, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_iffd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                             const double* a, int as, hipStream_t s) {
  for (int k = 0; k < 2 * P.d - 1; ++k) {
    hipError_t e = launch_iffd_pass(P, k, r, z, nrhs, ws, a, as, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace iffd
