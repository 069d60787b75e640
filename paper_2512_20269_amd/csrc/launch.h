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
// Workgroup barrier that orders LDS only: LDS writes before it are visible to
// LDS reads after it, while global loads and stores stay in flight across it
// (__syncthreads also drains every outstanding global access).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Raw buffer access (gfx9 buffer resource, 32-bit data format): the hardware
// checks each lane's offset (`voff` plus the instruction's immediate offset)
// against `bytes`; a load beyond returns 0 and a store beyond is dropped, so
// tails and missing lines need no branches.  The whole offset goes in `voff`
// (the scalar offset field, not range-checked, stays 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
// an offset no resource reaches (resources cover under 2 GiB)
constexpr unsigned BUF_OOB = 0x80000000u;

template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff) {
  if constexpr (sizeof(T) == 2)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, 0, 0));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, 0, 0));
}
template <typename T>
__device__ __forceinline__ void buf_st(T v, __amdgpu_buffer_rsrc_t r, unsigned voff) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, (int)voff, 0, 0);
}
// 16 bytes
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
__device__ __forceinline__ u32x4 buf_ld16(__amdgpu_buffer_rsrc_t r, unsigned voff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0);
}

enum ElemType { ELEM_F32 = 0, ELEM_F64 = 1 };

// Work fused into an IFFD line pass along direction 1, reported as per-tile
// partial sums part[rhs][tile]; `tiles` receives the tile count per
// right-hand side of the launch (at most apply_last_tiles_max).
//  - backward pass with FP64 output z (dr set): part = sum over the tile of
//    dr . z, z as stored;
//  - forward pass with FP64 input r (q set, r_out = r): the PCG residual
//    update r <- r - alpha_b q (alpha_b = alpha[b * active_stride]) is applied
//    to each entry as it is loaded and written back to r, the transform takes
//    the updated r, and part = sum over the tile of the updated r^2.
struct PassHook {
  const double* dr;
  double* part;
  int npart;
  mutable int tiles;
  const double* q = nullptr;
  const double* alpha = nullptr;
  double* r_out = nullptr;
};

// One IFFD line pass along `axis` (1-based; direction 1 = fastest) of the
// [nrhs][m]^d tensor.  Tin/Tout: ELEM_*; compute precision = plan.prec.
// active: optional per-RHS flags (stride `active_stride` doubles; 0 = skip).
hipError_t launch_line_pass(const Plan& P, int mode, int axis, int tin, const void* in, int tout,
                            void* out, int nrhs, const double* active, int active_stride,
                            hipStream_t s, const PassHook* hk = nullptr);

// Full IFFD apply z = P^{-1} r (FP64 in/out), ws = apply workspace; `first`
// and `last` are fused into its first and last pass.
hipError_t launch_iffd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                             const double* active, int active_stride, hipStream_t s,
                             const PassHook* last = nullptr, const PassHook* first = nullptr);

// One pass of the IFFD apply (0 .. 2d-2), see iffd_apply_pass.
hipError_t launch_iffd_pass(const Plan& P, int pass, const double* r, double* z, int nrhs,
                            void* ws, const double* active, int active_stride, hipStream_t s,
                            const PassHook* last = nullptr, const PassHook* first = nullptr);

// Dense FD apply (MFMA mode products).
hipError_t launch_fd_apply(const Plan& P, const double* r, double* z, int nrhs, void* ws,
                           const double* active, int active_stride, hipStream_t s);

// Outlier pencil eigensolve + table completion (FP64, on device).
hipError_t launch_setup_outliers(const Plan& P, hipStream_t s);
// The same for one pencil given by pointers (n_out <= 8): writes the outlier
// eigenvalues at lam[n_reg ..], the rotated basis Vt (n_out x m) and a status
// word (0 = ok).
hipError_t launch_setup_outliers_at(const double* Ao, const double* Bo, const double* Vout, int no,
                                    int m, int n_reg, double* lam64, float* lam32, double* vt64,
                                    float* vt32, double* stat, hipStream_t s);

// General plans (gen.hip): one pass of the apply (as launch_iffd_pass) and the
// operator (as launch_matvec).
hipError_t launch_gen_pass(const Plan& P, int pass, const double* r, double* z, int nrhs, void* ws,
                           const double* active, int active_stride, hipStream_t s);
hipError_t launch_gen_matvec(const Plan& P, const double* x, double* y, int nrhs, void* ws,
                             double* part, int npart, const double* active, int active_stride,
                             hipStream_t s, const double* fres);
int gen_matvec_blocks(const Plan& P);

// The system matrix of a mapped domain (geo.hip), as launch_matvec.
hipError_t launch_geo_matvec(const Plan& P, const double* x, double* y, int nrhs, void* ws,
                             double* part, int npart, const double* active, int active_stride,
                             hipStream_t s, const double* fres);
int geo_matvec_blocks(const Plan& P);
size_t geo_matvec_ws_bytes(const Plan& P, int nrhs);
size_t gen_matvec_ws_bytes(const Plan& P, int nrhs);

// One-pass operator of mvroll.hip: per-direction band tables K_k, M_k of
// n[k] x (2 pm + 1) FP64 entries (row i holds columns i - pm .. i + pm;
// pm >= every direction's p, padded with zeros), direction 1 fastest; a 2D
// operator passes n[2] = 1 with M_3 = 1, K_3 = 0.
struct RollBands {
  const double* k[3];
  const double* m[3];
  int n[3];
  int pm;
};
int mv_roll_blocks(const RollBands& B);
hipError_t launch_mv_roll(const RollBands& B, const double* x, double* y, int nrhs, int N,
                          double* part, int npart, const double* active, int active_stride,
                          hipStream_t s, const double* fres);

// y = Ahat x; ws: matvec_ws_bytes(P, nrhs); optional fused partial sums per
// workgroup: part[b][blk] = sum x.y, or sum (f - y)^2 when fres (the true
// residual of a solution x for the right-hand side f) is given.
hipError_t launch_matvec(const Plan& P, const double* x, double* y, int nrhs, void* ws,
                         double* part, int npart, const double* active, int active_stride,
                         hipStream_t s, const double* fres = nullptr);

}  // namespace iffd
