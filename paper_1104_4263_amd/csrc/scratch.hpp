// Statically allocated device scratch (scratch.hip) for the entry point that allocates nothing.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace die {

// Size of the per-device scratch array: the FFT intermediate of die_te_matvec_noalloc,
// nrhs * 2 * px * ny complex values, must fit in it.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchMaxDevices = 64;

// Looks up the device address of the current device's copy of the scratch array (dev must be
// the current device) and keeps it; later calls for the same device return at once.
hipError_t scratch_init(int dev);

// The kept device address of device dev's copy, or nullptr if scratch_init has not run there.
void* scratch_ptr(int dev);

}  // namespace die
