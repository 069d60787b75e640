// General plans (per direction n, p and Dirichlet / Neumann ends): the
// sequence of line passes that forms z = P^{-1} r, the matrix-free operator
// and the device part of the setup.
#include <algorithm>

#include "gen_impl.h"

namespace iffd {

// each length's passes are compiled in their own translation unit (gen_l*.hip)
extern template IFFD_GEN_PASS_LEN(16);
extern template IFFD_GEN_PASS_LEN(24);
extern template IFFD_GEN_PASS_LEN(32);
extern template IFFD_GEN_PASS_LEN(48);
extern template IFFD_GEN_PASS_LEN(64);
extern template IFFD_GEN_PASS_LEN(96);
extern template IFFD_GEN_PASS_LEN(128);
extern template IFFD_GEN_PASS_LEN(192);
extern template IFFD_GEN_PASS_LEN(256);
extern template IFFD_GEN_PASS_LEN(384);
extern template IFFD_GEN_PASS_LEN(512);

static hipError_t gen_line(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                           void* out, int nrhs, const double* a, int as, hipStream_t s) {
  switch (P.dirs[axis - 1].L) {
    case 16: return gen_pass_len<16>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 24: return gen_pass_len<24>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 32: return gen_pass_len<32>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 48: return gen_pass_len<48>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 64: return gen_pass_len<64>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 96: return gen_pass_len<96>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 128: return gen_pass_len<128>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 192: return gen_pass_len<192>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 256: return gen_pass_len<256>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 384: return gen_pass_len<384>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    case 512: return gen_pass_len<512>(P, mode, axis, tin, in, tout, out, nrhs, a, as, s);
    default: return hipErrorInvalidValue;
  }
}

// pass k of the apply: forward along directions 1 .. d-1, the middle pass
// along d, backward along d-1 .. 1.  The FP64 apply works in place on z, the
// FP32 apply on the FP32 workspace; pass 0 reads r, the last pass writes z.
hipError_t launch_gen_pass(const Plan& P, int pass, const double* r, double* z, int nrhs, void* ws,
                           const double* a, int as, hipStream_t s) {
  const int d = P.d;
  const bool f64 = P.prec == IFFD_PREC_F64;
  const int et = f64 ? ELEM_F64 : ELEM_F32;
  void* w = f64 ? (void*)z : ws;
  if (pass < d - 1) {
    const bool p0 = pass == 0;
    return gen_line(P, PASS_FWD, pass + 1, p0 ? ELEM_F64 : et, p0 ? (const void*)r : w, et, w,
                    nrhs, a, as, s);
  }
  if (pass == d - 1) return gen_line(P, PASS_MID, d, et, w, et, w, nrhs, a, as, s);
  if (pass < 2 * d - 1) {
    const int axis = 2 * d - 1 - pass;
    return gen_line(P, PASS_BWD, axis, et, w, axis == 1 ? ELEM_F64 : et,
                    axis == 1 ? (void*)z : w, nrhs, a, as, s);
  }
  return hipErrorInvalidValue;
}

// ---- the operator y = Ahat x with per-direction banded K_k, M_k -------------
// one pass of mvroll.hip over band tables padded to the largest degree (a 2D
// plan adds the one-entry third direction M_3 = 1, K_3 = 0)

static RollBands gen_bands(const Plan& P) {
  RollBands B;
  int pm = 1;
  for (int k = 0; k < P.d; ++k) pm = std::max(pm, P.dirs[k].p);
  B.pm = pm;
  for (int k = 0; k < 3; ++k) {
    if (k < P.d) {
      const GDir& G = P.dirs[k];
      const double* b = (const double*)(P.d_tables + G.blob64);
      B.k[k] = b + G.o_kb;
      B.m[k] = b + G.o_mb;
      B.n[k] = G.m;
    } else {
      const double* u = (const double*)(P.d_tables + P.lay.unit64);
      B.k[k] = u;                 // zeros
      B.m[k] = u + (2 * pm + 1);  // e_pm
      B.n[k] = 1;
    }
  }
  return B;
}

int gen_matvec_blocks(const Plan& P) {
  RollBands B{};
  int pm = 1;
  for (int k = 0; k < P.d; ++k) pm = std::max(pm, P.dirs[k].p);
  B.pm = pm;
  for (int k = 0; k < 3; ++k) B.n[k] = k < P.d ? P.dirs[k].m : 1;
  return mv_roll_blocks(B);
}

size_t gen_matvec_ws_bytes(const Plan&, int) { return 0; }

hipError_t launch_gen_matvec(const Plan& P, const double* x, double* y, int nrhs, void*,
                             double* part, int npart, const double* act, int as, hipStream_t s,
                             const double* fres) {
  return launch_mv_roll(gen_bands(P), x, y, nrhs, (int)P.N, part, npart, act, as, s, fres);
}

}  // namespace iffd
