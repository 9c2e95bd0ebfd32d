// bcgs_qr_noalloc: the factorization of bcgs_qr_ex with its workspace in a
// fixed device array instead of caller or library allocations, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).
//
// The array `scratch` below is a file-scope __device__ object: every GPU the
// library runs on holds its own copy, at its own address, from the moment
// the code object is loaded on that device until the process ends.  In host
// code the name `scratch` is only a host-side stand-in, never a device
// address, so the host resolves each device's address once, with that
// device current, through hipGetSymbolAddress, and only that address is
// handed to kernels.
#include <mutex>

#include "common.h"

namespace bcgs {

static __device__ __align__(256) char scratch[BCGS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), resolved once.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

}  // namespace bcgs

using namespace bcgs;

extern "C" bcgs_status bcgs_qr_noalloc(const void* X, int64_t ldx, int64_t m,
                                       int64_t n, int64_t s,
                                       bcgs_variant variant,
                                       bcgs_precision precision, void* Q,
                                       int64_t ldq, double* R, int64_t ldr,
                                       bcgs_info* d_info,
                                       hipStream_t stream) {
  Plan p;
  const bcgs_status st = check_problem(X, ldx, m, n, s, variant, precision, Q,
                                       ldq, R, ldr, d_info, &p);
  if (st != BCGS_OK) return st;
  // the workspace of this problem must fit the fixed array
  if (p.bytes > (size_t)BCGS_NOALLOC_SCRATCH_BYTES) return BCGS_ERR_NOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BCGS_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return BCGS_ERR_UNSUPPORTED;
  void* ws = nullptr;
  if (scratch_address(dev, &ws) != hipSuccess) return BCGS_ERR_HIP;
  return run_problem(p, X, ldx, Q, ldq, R, ldr, ws, d_info, stream);
}
