// The fixed device scratch of lbm_advance_noalloc: one static array per GPU,
// sized for the tables of one problem and a state that fits one workgroup's
// LDS, so that the entry point allocates nothing.  Host code reaches the array
// only through the device address hipGetSymbolAddress returns for the current
// device (the array's name is a host-side stand-in, not a device address).
#include <mutex>

#include "kernels.hpp"

namespace lbm {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ __launch_bounds__(64) void k_zero_ints(int* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += 64) p[i] = 0;
}
}  // namespace

hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  if (n < 0 || n > (1 << 20)) return hipErrorInvalidValue;
  k_zero_ints<<<1, 64, 0, s>>>(p, n);
  return hipGetLastError();
}

}  // namespace lbm
