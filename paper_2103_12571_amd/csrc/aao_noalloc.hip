// Fixed device scratch for the allocation-free entry point
// (aao_residual_noalloc): partial sums and norms live in a file-scope device
// array instead of the caller's workspace.  Every GPU the library runs on
// holds its own copy of the array until the process ends.
#include <mutex>

#include "aao_noalloc.hpp"

namespace aao {

namespace {

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchMaxDevices] = {};

}  // namespace

// The device address of `scratch` on the current device, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in, so kernels get this address, never the name.
hipError_t noalloc_scratch(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace aao
