// Launcher of the small 2-D route of the IFFD apply (dense2d.hip): the
// preconditioner of a 2-D plan with Plan::dense2d set, as two launches of LDS
// products with both directions' dense Qt (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace iffd {

// z = P^{-1} r for nrhs right-hand sides ([nrhs][m2][m1] FP64), ws: the FP32
// apply workspace (>= 4 m1 m2 nrhs bytes), active: optional per-RHS flags
// (stride astride doubles, 0 = skip).  hipErrorInvalidValue if the plan has
// no dense tables.
hipError_t launch_dense2d(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                          const double* active, int astride, hipStream_t s);

// dynamic LDS bytes of the two launches
size_t dense2d_lds_a(int m1, int m2);
size_t dense2d_lds_b(int m1);

// IFFD_ROUTE_AUTO takes the dense route when a full batch of the plan is at
// most this many multiply-adds per product pair (max_rhs m1 m2 (m1 + m2)):
// measured on the FP32 apply, the dense route wins up to about 160
// right-hand sides at m = 33, 70 at m = 65 and 35 at m = 97, where a batch
// of line passes starts to fill the chip; the bound keeps below all three.
constexpr double kDenseAutoWork = 16777216.0;   // 2^24

// the route an apply takes: IFFD_ROUTE_DENSE2D or IFFD_ROUTE_PASSES.  It is
// a property of the plan (its max_rhs), not of the batch size of a call, so
// a right-hand side gets the same bits alone and in any batch of the plan.
inline int dense2d_route(const Plan& P, int /*nrhs*/) {
  if (!P.dense2d || P.route == IFFD_ROUTE_PASSES) return IFFD_ROUTE_PASSES;
  if (P.route == IFFD_ROUTE_DENSE2D) return IFFD_ROUTE_DENSE2D;
  const double m1 = P.gen ? P.dirs[0].m : P.m, m2 = P.gen ? P.dirs[1].m : P.m;
  return (double)P.max_rhs * m1 * m2 * (m1 + m2) <= kDenseAutoWork ? IFFD_ROUTE_DENSE2D
                                                                    : IFFD_ROUTE_PASSES;
}

}  // namespace iffd
