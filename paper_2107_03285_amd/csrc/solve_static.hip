// sgn_solve_static: the refined solve of sgn_solve with all of its working memory in a static
// device array instead of the context's workspace, for callers that cannot allocate device memory
// at the time of the call (code under stream capture, tight serving loops).  The array is this
// file's `scratch`; each device holds its own copy for the life of the process.  Its address is
// looked up once per device, with that device current, on the first call there; the kernels
// receive that device address (the array's name is only a host-side handle for the lookup).
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

#include "../../include/sgn.h"

// The solve's working memory at most: 128 MiB per device.  The 100 x 25 x 25 cantilever
// (N = 718,100) needs 126 MB; the exact need is checked per call.
constexpr size_t kStaticScratchBytes = size_t(128) << 20;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Defined with the other drivers (api.cpp).
sgn_status solve_in_region(sgn_ctx c, const double* d_rhs, double* d_sol, sgn_solve_info* info, void* region,
                           size_t cap, hipError_t lookup);

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_addr[kMaxDevices] = {};
}  // namespace

extern "C" sgn_status sgn_solve_static(sgn_ctx ctx, const double* d_rhs, double* d_sol, sgn_solve_info* info) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  void* addr = nullptr;
  if (e == hipSuccess) {
    if (dev < 0 || dev >= kMaxDevices) {
      e = hipErrorInvalidDevice;
    } else {
      std::lock_guard<std::mutex> hold(g_lock);
      if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess) g_addr[dev] = p;
      }
      addr = g_addr[dev];
    }
  }
  return solve_in_region(ctx, d_rhs, d_sol, info, addr, kStaticScratchBytes, e);
}
