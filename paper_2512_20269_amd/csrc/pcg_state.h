// Per-slot scalar record of the stepped PCG (internal).
#pragma once

namespace iffd {

constexpr int kScal = 16;  // doubles per slot
enum ScalIndex {
  S_ACTIVE = 0,  // 1 while iterating
  S_CONV = 1,    // 1 once ||r|| <= rtol ||f||
  S_STATUS = 2,  // IFFD_* status of the solve
  S_IT = 3,      // iterations done
  S_MAXIT = 4,
  S_TOL = 5,     // rtol
  S_FF = 6,      // ||f||^2
  S_RELRES = 7,  // ||r_k|| / ||f||
  S_RZ0 = 8,     // r.z, by iteration parity (8, 9)
  S_RZ1 = 9,
  S_ALPHA = 10,
  S_BETA = 11,
  S_NEW = 12,    // 1 while being started by iffd_pcg_begin
  S_USED = 13,   // slot holds a solve (until taken)
  S_RUN = 14     // 1 if this iteration's alpha is valid (x += alpha p is due)
};

}  // namespace iffd
