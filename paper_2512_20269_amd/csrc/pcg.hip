// Preconditioned conjugate gradients on gfx950, FP64 (Section 3; protocol of
// Section 7: zero initial guess, stop at ||r_k|| <= rtol ||f||).
//
// Each slot is an independent solve.  Scalars live on the device in a record
// of 16 doubles per slot, so the iteration never waits for the host and can
// be captured in a HIP graph.  Inner products are reduced in two fixed-order
// steps (per-block partials, then one sum per slot), so a slot's arithmetic
// never depends on the other slots of the batch.
//
// One iteration, per active slot:
//   q = A p, pq = p.q (fused in the operator)      -> reduce pq
//   alpha = rz / pq; r -= alpha q; rr              -> reduce rr, test
//   z = P^{-1} r; rz' = r.z (fused in the IFFD apply's last pass)
//                                                  -> reduce rz'
// With IFFD the update of r and its rr are fused into the apply's first pass
// and the test runs between that pass and the rest.
//   beta = rz'/rz; x += alpha p; p = z + beta p
// x takes its update in the same sweep as p (it reads the old p anyway); a
// slot that stops in this iteration still gets it (flag S_RUN).
// rz alternates between two record entries by iteration parity so that no
// kernel reads a value another block of the same kernel overwrites.
#include "dense2d.h"
#include "launch.h"
#include "pcg_state.h"

namespace iffd {

constexpr int VT = 256;  // threads per block of the vector kernels
// The vector kernels take their chunk SU iterations at a time, with all
// loads of those iterations issued before the first use, so that each
// thread keeps several loads in flight (the sums keep their order).
constexpr int SU = 4;

// slot list of one begin call, passed by value (no device allocation)
constexpr int kBeginMax = 64;
struct BeginSlots {
  int count;
  int slot[kBeginMax];
};

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < VT / 64; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ void chunk(int N, int nblk, int blk, int& lo, int& hi) {
  const int c = (N + nblk - 1) / nblk;
  lo = min(N, blk * c);
  hi = min(N, lo + c);
}

// part[slot][blk] = sum a.b over the block's chunk; flags: slots to do
__global__ void __launch_bounds__(VT)
dot_partials(const double* __restrict__ a, const double* __restrict__ b, int N, int nblk,
             double* __restrict__ part, const double* __restrict__ scal, int flag) {
  __shared__ double red[VT / 64];
  const int slot = blockIdx.x / nblk, blk = blockIdx.x - slot * nblk;
  if (scal && scal[(size_t)slot * kScal + flag] == 0.0) return;
  int lo, hi;
  chunk(N, nblk, blk, lo, hi);
  const double* ar = a + (size_t)slot * N;
  const double* br = b + (size_t)slot * N;
  double s = 0.0;
  int i = lo + threadIdx.x;
  for (; i + (SU - 1) * VT < hi; i += SU * VT) {
    double av[SU], bv[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      av[u] = ar[i + u * VT];
      bv[u] = br[i + u * VT];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) s += av[u] * bv[u];
  }
  for (; i < hi; i += VT) s += ar[i] * br[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(size_t)slot * nblk + blk] = s;
}

// Sum of a slot's partials, computed by one block of VT threads in a fixed
// order (thread i adds entries i, i+VT, ... in turn; then a fixed butterfly
// across lanes and waves), so the result does not depend on the batch.  The
// total is returned in every thread.
__device__ __forceinline__ double block_psum(const double* __restrict__ p, int n, double* red) {
  double s = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * VT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * VT;
      v[u] = i < n ? p[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < VT / 64; ++w) tot += red[w];
  __syncthreads();
  return tot;
}

// one block per slot: pq = sum of partials; alpha = rz / pq; breakdown test
__global__ void __launch_bounds__(VT)
pcg_alpha(double* scal, const double* part, int npart_used, int npart, int nslots) {
  __shared__ double red[VT / 64];
  const int slot = blockIdx.x;
  double* sc = scal + (size_t)slot * kScal;
  if (sc[S_ACTIVE] == 0.0) {
    if (threadIdx.x == 0) sc[S_RUN] = 0.0;
    return;
  }
  const double pq = block_psum(part + (size_t)slot * npart, npart_used, red);
  if (threadIdx.x != 0) return;
  const int it = (int)sc[S_IT];
  const double rz = sc[S_RZ0 + (it & 1)];
  if (!(pq > 0.0) || !(rz > 0.0) || !isfinite(pq) || !isfinite(rz)) {
    sc[S_ACTIVE] = 0.0;
    sc[S_RUN] = 0.0;
    sc[S_STATUS] = (double)IFFD_E_BREAKDOWN;
    return;
  }
  sc[S_ALPHA] = rz / pq;
  sc[S_RUN] = 1.0;
}

// r -= alpha q; partial r.r
__global__ void __launch_bounds__(VT)
pcg_update_r(double* __restrict__ r, const double* __restrict__ q, int N, int nblk,
             const double* __restrict__ scal, double* __restrict__ part) {
  __shared__ double red[VT / 64];
  const int slot = blockIdx.x / nblk, blk = blockIdx.x - slot * nblk;
  const double* sc = scal + (size_t)slot * kScal;
  if (sc[S_ACTIVE] == 0.0) return;
  const double alpha = sc[S_ALPHA];
  int lo, hi;
  chunk(N, nblk, blk, lo, hi);
  const size_t o = (size_t)slot * N;
  double s = 0.0;
  int i = lo + threadIdx.x;
  for (; i + (SU - 1) * VT < hi; i += SU * VT) {
    double rv[SU], qv[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      rv[u] = r[o + i + u * VT];
      qv[u] = q[o + i + u * VT];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const double v = rv[u] - alpha * qv[u];
      r[o + i + u * VT] = v;
      s += v * v;
    }
  }
  for (; i < hi; i += VT) {
    const double rv = r[o + i] - alpha * q[o + i];
    r[o + i] = rv;
    s += rv * rv;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(size_t)slot * nblk + blk] = s;
}

// one block per slot: iteration count, residual test, history (r.r = the
// first nused of the slot's partials, stride apart per slot)
__global__ void __launch_bounds__(VT)
pcg_check(double* scal, double* hist, const double* part, int nused, int stride, int nslots) {
  __shared__ double red[VT / 64];
  const int slot = blockIdx.x;
  double* sc = scal + (size_t)slot * kScal;
  if (sc[S_ACTIVE] == 0.0) return;
  const double rr = block_psum(part + (size_t)slot * stride, nused, red);
  if (threadIdx.x != 0) return;
  const int it = (int)sc[S_IT] + 1;
  sc[S_IT] = it;
  if (it - 1 < kHist) hist[((size_t)slot * kHist + it - 1) * 2] = sc[S_ALPHA];
  const double rel = sqrt(rr / sc[S_FF]);
  sc[S_RELRES] = rel;
  if (!isfinite(rr)) {
    sc[S_ACTIVE] = 0.0;
    sc[S_STATUS] = (double)IFFD_E_BREAKDOWN;
  } else if (rel <= sc[S_TOL]) {
    sc[S_ACTIVE] = 0.0;
    sc[S_CONV] = 1.0;
    sc[S_STATUS] = (double)IFFD_OK;
  } else if (it >= (int)sc[S_MAXIT]) {
    sc[S_ACTIVE] = 0.0;
    sc[S_STATUS] = (double)IFFD_W_NOT_CONVERGED;
  }
}

// one block per slot: rz' = sum of the nused partials, beta = rz'/rz
__global__ void __launch_bounds__(VT)
pcg_beta(double* scal, double* hist, const double* part, int nused, int stride, int nslots) {
  __shared__ double red[VT / 64];
  const int slot = blockIdx.x;
  double* sc = scal + (size_t)slot * kScal;
  if (sc[S_ACTIVE] == 0.0) return;
  const double rzn = block_psum(part + (size_t)slot * stride, nused, red);
  if (threadIdx.x != 0) return;
  const int it = (int)sc[S_IT];  // already counts this iteration
  const double rzo = sc[S_RZ0 + ((it - 1) & 1)];
  if (!(rzn > 0.0) || !isfinite(rzn)) {
    sc[S_ACTIVE] = 0.0;
    sc[S_STATUS] = (double)IFFD_E_BREAKDOWN;
    return;
  }
  const double beta = rzn / rzo;
  sc[S_BETA] = beta;
  sc[S_RZ0 + (it & 1)] = rzn;
  if (it - 1 < kHist) hist[((size_t)slot * kHist + it - 1) * 2 + 1] = beta;
}

// x += alpha p (every slot whose alpha is valid); p = z + beta p (slots still
// iterating)
__global__ void __launch_bounds__(VT)
pcg_update_p(double* __restrict__ x, double* __restrict__ p, const double* __restrict__ z, int N,
             int nblk, const double* __restrict__ scal) {
  const int slot = blockIdx.x / nblk, blk = blockIdx.x - slot * nblk;
  const double* sc = scal + (size_t)slot * kScal;
  if (sc[S_RUN] == 0.0) return;
  const double alpha = sc[S_ALPHA], beta = sc[S_BETA];
  const bool act = sc[S_ACTIVE] != 0.0;
  int lo, hi;
  chunk(N, nblk, blk, lo, hi);
  const size_t o = (size_t)slot * N;
  int i = lo + threadIdx.x;
  if (act) {
    for (; i + (SU - 1) * VT < hi; i += SU * VT) {
      double pv[SU], xv[SU], zv[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        pv[u] = p[o + i + u * VT];
        xv[u] = x[o + i + u * VT];
        zv[u] = z[o + i + u * VT];
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        x[o + i + u * VT] = xv[u] + alpha * pv[u];
        p[o + i + u * VT] = zv[u] + beta * pv[u];
      }
    }
    for (; i < hi; i += VT) {
      const double pv = p[o + i];
      x[o + i] += alpha * pv;
      p[o + i] = z[o + i] + beta * pv;
    }
  } else {
    for (; i + (SU - 1) * VT < hi; i += SU * VT) {
      double pv[SU], xv[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        pv[u] = p[o + i + u * VT];
        xv[u] = x[o + i + u * VT];
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) x[o + i + u * VT] = xv[u] + alpha * pv[u];
    }
    for (; i < hi; i += VT) x[o + i] += alpha * p[o + i];
  }
}

// begin: x = 0, r = f (f packed [count][N], slot list), partial f.f
__global__ void __launch_bounds__(VT)
pcg_begin_copy(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ f,
               BeginSlots slots, int N, int nblk, double* __restrict__ part) {
  __shared__ double red[VT / 64];
  const int k = blockIdx.x / nblk, blk = blockIdx.x - k * nblk;
  const int slot = slots.slot[k];
  int lo, hi;
  chunk(N, nblk, blk, lo, hi);
  const size_t o = (size_t)slot * N;
  const double* fk = f + (size_t)k * N;
  double s = 0.0;
  int i = lo + threadIdx.x;
  for (; i + (SU - 1) * VT < hi; i += SU * VT) {
    double v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) v[u] = fk[i + u * VT];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      x[o + i + u * VT] = 0.0;
      r[o + i + u * VT] = v[u];
      s += v[u] * v[u];
    }
  }
  for (; i < hi; i += VT) {
    const double v = fk[i];
    x[o + i] = 0.0;
    r[o + i] = v;
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[(size_t)slot * nblk + blk] = s;
}

// begin scalars (one block per started slot)
__global__ void __launch_bounds__(VT)
pcg_begin_scal(double* scal, const double* part, int nblk, BeginSlots slots, double rtol,
               int maxit) {
  __shared__ double red[VT / 64];
  const int slot = slots.slot[blockIdx.x];
  double* sc = scal + (size_t)slot * kScal;
  const double ff = block_psum(part + (size_t)slot * nblk, nblk, red);
  if (threadIdx.x != 0) return;
  for (int i = 0; i < kScal; ++i) sc[i] = 0.0;
  sc[S_FF] = ff;
  sc[S_TOL] = rtol;
  sc[S_MAXIT] = maxit;
  sc[S_USED] = 1.0;
  sc[S_RELRES] = ff > 0 ? 1.0 : 0.0;
  if (!isfinite(ff)) {  // NaN / Inf right-hand side
    sc[S_STATUS] = (double)IFFD_E_BREAKDOWN;
    sc[S_RELRES] = ff;
  } else if (ff > 0.0 && maxit > 0) {
    sc[S_NEW] = 1.0;
  } else {
    sc[S_CONV] = ff > 0.0 ? 0.0 : 1.0;
    sc[S_STATUS] = ff > 0.0 ? (double)IFFD_W_NOT_CONVERGED : (double)IFFD_OK;
  }
}

__global__ void __launch_bounds__(VT)
pcg_begin_finish(double* scal, const double* part, int nused, int stride, int nslots) {
  __shared__ double red[VT / 64];
  const int slot = blockIdx.x;
  double* sc = scal + (size_t)slot * kScal;
  if (sc[S_NEW] == 0.0) return;
  const double rz = block_psum(part + (size_t)slot * stride, nused, red);
  if (threadIdx.x != 0) return;
  sc[S_NEW] = 0.0;
  if (!(rz > 0.0) || !isfinite(rz)) {
    sc[S_STATUS] = (double)IFFD_E_BREAKDOWN;
    return;
  }
  sc[S_RZ0] = rz;
  sc[S_ACTIVE] = 1.0;
}

// zero a byte range with a plain fill kernel (graph-safe, unlike memset nodes)
__global__ void fill_zero(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// u = x[slot]; mark the slot free
// copy slot `slot`'s iterate to u and free the slot; slot < 0: every slot
// (u holds nslots vectors back to back)
__global__ void pcg_take_kernel(const double* __restrict__ x, double* __restrict__ u, int N,
                                int slot, int nslots, double* scal) {
  const size_t o = slot < 0 ? 0 : (size_t)slot * N;
  const size_t cnt = slot < 0 ? (size_t)nslots * N : (size_t)N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (size_t)gridDim.x * blockDim.x)
    u[i] = x[o + i];
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < (slot < 0 ? nslots : 1); k += blockDim.x) {
      double* sc = scal + (size_t)(slot < 0 ? k : slot) * kScal;
      sc[S_USED] = 0.0;
      sc[S_ACTIVE] = 0.0;
    }
  }
}

// per-slot summary for asynchronous polling: out[4 k ..] = active, status
// (-100 for a free slot), iterations, relres
__global__ void pcg_status_kernel(const double* __restrict__ scal, double* __restrict__ out,
                                  int nslots) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nslots) return;
  const double* r = scal + (size_t)k * kScal;
  out[4 * k + 0] = r[S_ACTIVE];
  out[4 * k + 1] = r[S_USED] != 0.0 ? r[S_STATUS] : -100.0;
  out[4 * k + 2] = r[S_IT];
  out[4 * k + 3] = r[S_RELRES];
}

hipError_t pcg_status_dev(const Plan& P, const char* st, int nslots, double* out, hipStream_t s) {
  const StateLayout L = state_layout(P, nslots);
  hipLaunchKernelGGL(pcg_status_kernel, dim3((nslots + 63) / 64), dim3(64), 0, s,
                     (const double*)(st + L.scal), out, nslots);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// PCG steps fused into the apply's line passes: uniform plans of the FFT
// method, unless their applies take the small 2-D route (whose two launches
// carry no PCG work; such plans then run the unfused steps below)
static inline bool fused_steps(const Plan& P, int nslots) {
  return P.method == IFFD_METHOD_FFT && !P.gen &&
         dense2d_route(P, nslots) != IFFD_ROUTE_DENSE2D;
}

// the preconditioner without fused PCG steps: dense FD, the line passes of a
// general plan, or the small 2-D route (the r . z and residual updates then
// run as kernels of their own)
static hipError_t plain_apply(const Plan& P, const double* r, double* z, int nslots, void* ws,
                              const double* a, int as, hipStream_t s) {
  return P.method == IFFD_METHOD_FFT ? launch_iffd_apply(P, r, z, nslots, ws, a, as, s)
                                     : launch_fd_apply(P, r, z, nslots, ws, a, as, s);
}

hipError_t state_init(const Plan& P, char* st, int nslots, hipStream_t s) {
  const StateLayout L = state_layout(P, nslots);
  const size_t n = (L.part - L.scal) / 8;  // scalars + history
  hipLaunchKernelGGL(fill_zero, dim3(64), dim3(256), 0, s, (double*)(st + L.scal), n);
  return hipGetLastError();
}

hipError_t pcg_begin_dev(const Plan& P, char* st, int nslots, const int* h_slots, int count,
                         const double* f, double rtol, int maxit, hipStream_t s) {
  if (count > kBeginMax) {
    for (int c0 = 0; c0 < count; c0 += kBeginMax) {
      hipError_t e = pcg_begin_dev(P, st, nslots, h_slots + c0, count - c0 < kBeginMax ? count - c0 : kBeginMax,
                                   f + (size_t)c0 * P.N, rtol, maxit, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  BeginSlots bs;
  bs.count = count;
  for (int k = 0; k < kBeginMax; ++k) bs.slot[k] = k < count ? h_slots[k] : 0;
  const StateLayout L = state_layout(P, nslots);
  const int N = (int)P.N, nb = L.npart;
  double* scal = (double*)(st + L.scal);
  double* part = (double*)(st + L.part);
  double* x = (double*)(st + L.x);
  double* r = (double*)(st + L.r);
  double* p = (double*)(st + L.p);
  hipLaunchKernelGGL(pcg_begin_copy, dim3(count * nb), dim3(VT), 0, s, x, r, f, bs, N, nb, part);
  hipLaunchKernelGGL(pcg_begin_scal, dim3(count), dim3(VT), 0, s, scal, part, nb, bs, rtol, maxit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // p = z = P^{-1} r for the new slots only, written straight into p (IFFD:
  // r . z partials from its last pass)
  int nrz = nb;
  if (fused_steps(P, nslots)) {
    const PassHook hk{r, part, nb, 0};
    e = launch_iffd_apply(P, r, p, nslots, L.ws ? st + L.ws : nullptr, scal + S_NEW, kScal, s,
                          &hk);
    if (e != hipSuccess) return e;
    nrz = hk.tiles;
  } else {
    e = plain_apply(P, r, p, nslots, L.ws ? st + L.ws : nullptr, scal + S_NEW, kScal, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dot_partials, dim3(nslots * nb), dim3(VT), 0, s, r, p, N, nb, part, scal,
                       (int)S_NEW);
  }
  hipLaunchKernelGGL(pcg_begin_finish, dim3(nslots), dim3(VT), 0, s, scal, part, nrz, nb, nslots);
  return hipGetLastError();
}

hipError_t pcg_iterate_dev(const Plan& P, char* st, int nslots, int k, hipStream_t s) {
  const StateLayout L = state_layout(P, nslots);
  const int N = (int)P.N, nb = L.npart;
  double* scal = (double*)(st + L.scal);
  double* hist = (double*)(st + L.hist);
  double* part = (double*)(st + L.part);
  double* part2 = part + (size_t)nslots * nb;
  double* x = (double*)(st + L.x);
  double* r = (double*)(st + L.r);
  double* p = (double*)(st + L.p);
  double* qz = (double*)(st + L.qz);
  void* ws = L.ws ? st + L.ws : nullptr;
  void* mvws = L.mvws ? st + L.mvws : nullptr;
  const int nmv = matvec_blocks(P);
  for (int it = 0; it < k; ++it) {
    hipError_t e = launch_matvec(P, p, qz, nslots, mvws, part2, nb, scal + S_ACTIVE, kScal, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pcg_alpha, dim3(nslots), dim3(VT), 0, s, scal, part2, nmv, nb, nslots);
    int nrz = nb;
    if (fused_steps(P, nslots)) {
      // the apply's first pass takes r <- r - alpha q on its way in (r.r
      // partials), the residual test follows it, so the other passes skip the
      // slots that converged; r.z partials come from the last pass
      PassHook up{nullptr, part, nb, 0};
      up.q = qz;
      up.alpha = scal + S_ALPHA;
      up.r_out = r;
      e = launch_iffd_pass(P, 0, r, qz, nslots, ws, scal + S_ACTIVE, kScal, s, nullptr, &up);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(pcg_check, dim3(nslots), dim3(VT), 0, s, scal, hist, part, up.tiles, nb,
                         nslots);
      const PassHook hk{r, part, nb, 0};
      for (int k = 1; k < 2 * P.d - 1; ++k) {
        e = launch_iffd_pass(P, k, r, qz, nslots, ws, scal + S_ACTIVE, kScal, s, &hk);
        if (e != hipSuccess) return e;
      }
      nrz = hk.tiles;
    } else {
      hipLaunchKernelGGL(pcg_update_r, dim3(nslots * nb), dim3(VT), 0, s, r, qz, N, nb, scal,
                         part);
      hipLaunchKernelGGL(pcg_check, dim3(nslots), dim3(VT), 0, s, scal, hist, part, nb, nb, nslots);
      e = plain_apply(P, r, qz, nslots, ws, scal + S_ACTIVE, kScal, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(dot_partials, dim3(nslots * nb), dim3(VT), 0, s, r, qz, N, nb, part, scal,
                         (int)S_ACTIVE);
    }
    hipLaunchKernelGGL(pcg_beta, dim3(nslots), dim3(VT), 0, s, scal, hist, part, nrz, nb, nslots);
    hipLaunchKernelGGL(pcg_update_p, dim3(nslots * nb), dim3(VT), 0, s, x, p, qz, N, nb, scal);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t pcg_take_dev(const Plan& P, char* st, int nslots, int slot, double* u, hipStream_t s) {
  const StateLayout L = state_layout(P, nslots);
  hipLaunchKernelGGL(pcg_take_kernel, dim3(slot < 0 ? 2048 : 256), dim3(256), 0, s,
                     (const double*)(st + L.x), u, (int)P.N, slot, nslots, (double*)(st + L.scal));
  return hipGetLastError();
}

hipError_t dot_partials_dev(const Plan& P, const double* a, const double* b, double* part, int nrhs,
                            hipStream_t s) {
  const int N = (int)P.N, nb = pcg_blocks(P);
  hipLaunchKernelGGL(dot_partials, dim3(nrhs * nb), dim3(VT), 0, s, a, b, N, nb, part,
                     (const double*)nullptr, 0);
  return hipGetLastError();
}

}  // namespace iffd
