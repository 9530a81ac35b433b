// Static device scratch of the allocation-free apply (lb_apply_gradS_noalloc).
#pragma once
#include <cstddef>

namespace lb {

// Size of the per-device static scratch array: enough for the FP32
// gradient apply of one density on a 5120-patch order-6 surface (about
// 80 MB of strengths, expansions, derived leaf expansions and outputs).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

// Device address of the scratch array on device `dev`, which must be the
// current device.  The first call for a device looks the address up
// (hipGetSymbolAddress) and keeps it; later calls return the kept address.
void* noalloc_scratch(int dev);

}  // namespace lb
