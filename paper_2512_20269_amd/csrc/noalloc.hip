// Allocation-free variant of iffd_precond_apply (iffd_precond_apply_noalloc
// in include/iffd.h).  The apply's workspace (the FP32 tensor between the
// IFFD line passes, or the dense-FD mode-product buffers) lives in one
// file-scope device array instead of a caller buffer, so callers that cannot
// allocate pass only the input and the output.
//
// Each device that runs the library holds its own copy of the array for the
// life of the process.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) on the entry point's first
// call there; the host-side name of the array is never passed to a kernel.
// Every call on a device shares that device's array: calls that overlap on
// one device (several streams or host threads) race on it.  The workspace is
// fully written by each apply before it is read, so nothing needs clearing.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "launch.h"
#include "plan.h"

namespace iffd {
namespace {

static __device__ __align__(256) unsigned char scratch[IFFD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return set_last_error(IFFD_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return set_last_error(IFFD_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return set_last_error(IFFD_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                            hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IFFD_OK;
}

}  // namespace
}  // namespace iffd

extern "C" int iffd_precond_apply_noalloc(const iffd_plan* plan, const double* d_r, double* d_z,
                                          int nrhs, void* stream) {
  using namespace iffd;
  if (!plan || !d_r || !d_z) return set_last_error(IFFD_E_INVAL, "null argument");
  const Plan& P = plan->P;
  if (!P.ready) return set_last_error(IFFD_E_STATE, "plan not set up");
  if (nrhs < 1 || nrhs > P.max_rhs) return set_last_error(IFFD_E_INVAL, "nrhs out of range");
  if ((const void*)d_r == (const void*)d_z)
    return set_last_error(IFFD_E_INVAL, "r and z must not alias");
  const size_t need = apply_ws_bytes(P, nrhs);
  if (need > (size_t)IFFD_NOALLOC_SCRATCH_BYTES)
    return set_last_error(IFFD_E_WORKSPACE,
                          "the apply needs " + std::to_string(need) +
                              " workspace bytes, more than the " +
                              std::to_string((size_t)IFFD_NOALLOC_SCRATCH_BYTES) +
                              "-byte scratch of the allocation-free entry point");
  void* ws = nullptr;
  if (need) {
    const int rc = scratch_address(&ws);
    if (rc != IFFD_OK) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = (P.method == IFFD_METHOD_FFT)
                     ? launch_iffd_apply(P, d_r, d_z, nrhs, ws, nullptr, 0, s)
                     : launch_fd_apply(P, d_r, d_z, nrhs, ws, nullptr, 0, s);
  if (e != hipSuccess)
    return set_last_error(IFFD_E_HIP, std::string("precond_apply_noalloc launch: ") +
                                          hipGetErrorString(e));
  return IFFD_OK;
}
