// Statically allocated device scratch for the entry point that allocates nothing
// (die_te_matvec_noalloc): the FFT intermediate of its product lives in this array
// instead of a buffer the context allocates on demand.
//
// Each device that loads the library holds its own copy of the array until the process
// ends.  Host code never uses the array's name as an address: the device address of
// each device's copy is looked up once, with that device current, and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scratch.hpp"

static __device__ __align__(256) unsigned char scratch[die::kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[die::kScratchMaxDevices] = {};
}  // namespace

namespace die {

hipError_t scratch_init(int dev) {
  if (dev < 0 || dev >= kScratchMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != dev) return hipErrorInvalidDevice;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = p;
  return hipSuccess;
}

void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kScratchMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

}  // namespace die
