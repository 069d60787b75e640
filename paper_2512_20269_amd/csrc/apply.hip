// IFFD apply: dispatch of the line passes (apply_impl.h) over FFT lengths and
// the sequence of passes that forms z = P^{-1} r.
#include "apply_impl.h"
#include "dense2d.h"

namespace iffd {

// each (L, mode) pair is compiled in its own translation unit (apply_l*_*.hip)
extern template IFFD_LINE_PASS_MODE(16, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(16, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(16, PASS_MID);
extern template IFFD_LINE_PASS_MODE(24, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(24, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(24, PASS_MID);
extern template IFFD_LINE_PASS_MODE(32, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(32, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(32, PASS_MID);
extern template IFFD_LINE_PASS_MODE(48, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(48, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(48, PASS_MID);
extern template IFFD_LINE_PASS_MODE(64, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(64, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(64, PASS_MID);
extern template IFFD_LINE_PASS_MODE(96, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(96, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(96, PASS_MID);
extern template IFFD_LINE_PASS_MODE(128, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(128, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(128, PASS_MID);
extern template IFFD_LINE_PASS_MODE(192, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(192, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(192, PASS_MID);
extern template IFFD_LINE_PASS_MODE(256, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(256, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(256, PASS_MID);
extern template IFFD_LINE_PASS_MODE(384, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(384, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(384, PASS_MID);
extern template IFFD_LINE_PASS_MODE(512, PASS_FWD);
extern template IFFD_LINE_PASS_MODE(512, PASS_BWD);
extern template IFFD_LINE_PASS_MODE(512, PASS_MID);

template <int L>
static hipError_t by_mode(const Plan& P, int mode, int var, int axis, int tin, const void* in,
                          int tout, void* out, int nrhs, const double* a, int as, hipStream_t s,
                          const PassHook* hk) {
  if (mode == PASS_FWD)
    return line_pass_mode<L, PASS_FWD>(P, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
  if (mode == PASS_BWD)
    return line_pass_mode<L, PASS_BWD>(P, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
  return line_pass_mode<L, PASS_MID>(P, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
}

hipError_t launch_line_pass(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                            void* out, int nrhs, const double* a, int as, hipStream_t s,
                            const PassHook* hk) {
  // pass index of (mode, axis) for the per-pass variant choice
  const int d = P.d;
  const int pass = mode == PASS_FWD ? axis - 1 : (mode == PASS_MID ? d - 1 : 2 * d - 1 - axis);
  const int var = P.variant[pass];
  switch (P.L) {
    case 16: return by_mode<16>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 24: return by_mode<24>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 32: return by_mode<32>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 48: return by_mode<48>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 64: return by_mode<64>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 96: return by_mode<96>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 128: return by_mode<128>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 192: return by_mode<192>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 256: return by_mode<256>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 384: return by_mode<384>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    case 512: return by_mode<512>(P, mode, var, axis, tin, in, tout, out, nrhs, a, as, s, hk);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_iffd_pass(const Plan& P, int pass, const double* r, double* z, int nrhs,
                            void* ws, const double* a, int as, hipStream_t s,
                            const PassHook* last, const PassHook* first) {
  if (P.gen) {
    if (last || first) return hipErrorInvalidValue;   // general plans fuse nothing
    return launch_gen_pass(P, pass, r, z, nrhs, ws, a, as, s);
  }
  const int d = P.d;
  const bool f64 = P.prec == IFFD_PREC_F64;
  const int et = f64 ? ELEM_F64 : ELEM_F32;
  void* w = f64 ? (void*)z : ws;
  if (pass < d - 1) {
    const bool p0 = pass == 0;
    return launch_line_pass(P, PASS_FWD, pass + 1, p0 ? ELEM_F64 : et, p0 ? (const void*)r : w,
                            et, w, nrhs, a, as, s, p0 ? first : nullptr);
  }
  if (pass == d - 1) return launch_line_pass(P, PASS_MID, d, et, w, et, w, nrhs, a, as, s);
  if (pass < 2 * d - 1) {
    const int axis = 2 * d - 1 - pass;  // d-1 .. 1
    return launch_line_pass(P, PASS_BWD, axis, et, w, axis == 1 ? ELEM_F64 : et,
                            axis == 1 ? (void*)z : w, nrhs, a, as, s, axis == 1 ? last : nullptr);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_iffd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                             const double* a, int as, hipStream_t s, const PassHook* last,
                             const PassHook* first) {
  if (!last && !first && dense2d_route(P, nrhs) == IFFD_ROUTE_DENSE2D)
    return launch_dense2d(P, r, z, nrhs, ws, a, as, s);
  for (int k = 0; k < 2 * P.d - 1; ++k) {
    hipError_t e = launch_iffd_pass(P, k, r, z, nrhs, ws, a, as, s, last, first);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// tiles per right-hand side of the direction-1 pass with the smallest tile
// of any variant (bounds the partials a PassHook receives)
template <typename T, int L>
static int tw_min() {
  int a = Cfg<T, L, 0>::TW, b = Cfg<T, L, 1>::TW, c = Cfg<T, L, 2>::TW;
  int w = a < b ? (a < c ? a : c) : (b < c ? b : c);
  if constexpr (fft_has_v3<L>()) {
    w = w < Cfg<T, L, 3>::TW ? w : Cfg<T, L, 3>::TW;
    w = w < Cfg<T, L, 4>::TW ? w : Cfg<T, L, 4>::TW;
  }
  return w;
}
template <int L>
static int tw_min_p(bool f64) {
  const int a = tw_min<double, L>(), b = tw_min<float, L>();
  return f64 ? a : (a < b ? a : b);   // FP32 plans may run their first pass in FP64
}

int apply_last_tiles_max(const Plan& P) {
  if (P.method != IFFD_METHOD_FFT || P.gen) return 1;
  const bool f64 = P.prec == IFFD_PREC_F64;
  int tw = 1;
  switch (P.L) {
    case 16: tw = tw_min_p<16>(f64); break;
    case 24: tw = tw_min_p<24>(f64); break;
    case 32: tw = tw_min_p<32>(f64); break;
    case 48: tw = tw_min_p<48>(f64); break;
    case 64: tw = tw_min_p<64>(f64); break;
    case 96: tw = tw_min_p<96>(f64); break;
    case 128: tw = tw_min_p<128>(f64); break;
    case 192: tw = tw_min_p<192>(f64); break;
    case 256: tw = tw_min_p<256>(f64); break;
    case 384: tw = tw_min_p<384>(f64); break;
    case 512: tw = tw_min_p<512>(f64); break;
    default: return 1;
  }
  const long long lpr = P.N / P.m;
  return (int)((lpr + tw - 1) / tw);
}

}  // namespace iffd
