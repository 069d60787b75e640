// Host-side launchers of the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace iffd {

enum PassMode { PASS_FWD = 0, PASS_BWD = 1, PASS_MID = 2 };

// Workgroups go to the 8 XCDs round-robin (block b to XCD b mod 8), each XCD
// with its own L2.  This bijection of [0, nblocks) gives every XCD one
// contiguous run of work items, so neighbouring items (which share cache
// lines or halos) meet in one L2.
__device__ __forceinline__ int xcd_linear(int b, int nblocks) {
  const int q8 = nblocks >> 3, r8 = nblocks & 7;
  const int x = b & 7, k = b >> 3;
  return x * q8 + (x < r8 ? x : r8) + k;
}
enum ElemType { ELEM_F32 = 0, ELEM_F64 = 1 };

// One IFFD line pass along `axis` (1-based; direction 1 = fastest) of the
// [nrhs][m]^d tensor.  Tin/Tout: ELEM_*; compute precision = plan.prec.
// active: optional per-RHS flags (stride `active_stride` doubles; 0 = skip).
hipError_t launch_line_pass(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                            void* out, int nrhs, const double* active, int active_stride,
                            hipStream_t s);

// Full IFFD apply z = P^{-1} r (FP64 in/out), ws = apply workspace.
hipError_t launch_iffd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                             const double* active, int active_stride, hipStream_t s);

// One pass of the IFFD apply (0 .. 2d-2), see iffd_apply_pass.
hipError_t launch_iffd_pass(const Plan& P, int pass, const double* r, double* z, int nrhs,
                            void* ws, const double* active, int active_stride, hipStream_t s);

// Dense FD apply (MFMA mode products).
hipError_t launch_fd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                           const double* active, int active_stride, hipStream_t s);

// Outlier pencil eigensolve + table completion (FP64, on device).
hipError_t launch_setup_outliers(const Plan& P, hipStream_t s);

// y = Ahat x; ws: matvec_ws_bytes(P, nrhs); optional fused partial dot sums
// part[b][blk] = sum x.y over a workgroup.
hipError_t launch_matvec(const Plan& P, const double* x, double* y, int nrhs, void* ws,
                         double* part, int npart, const double* active, int active_stride,
                         hipStream_t s);

}  // namespace iffd
