// The static device scratch of the allocation-free gradient apply: a
// file-scope array that every device holds from module load until the
// process ends, so the entry point never calls hipMalloc.  In host code the
// array's name stands for a host-side shadow, not a device address; the
// device address comes from hipGetSymbolAddress, looked up once per device
// (with that device current) and kept here.
#include "noalloc.hpp"
#include "common.hpp"

#include <hip/hip_runtime.h>

#include <mutex>

namespace lb {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {nullptr};
static std::mutex g_scratch_mu;

void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(LB_EINVAL, "device %d out of range for the static scratch", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) fail(LB_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace lb
