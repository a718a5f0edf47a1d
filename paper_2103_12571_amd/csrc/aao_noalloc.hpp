// Fixed device scratch of the allocation-free entry point (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace aao {

// Layout of the scratch array (doubles): residual partial sums, the two
// finalized norms, then the (sum of squares, max) pairs of the w norms.
constexpr int kScratchResParts = 1024;
constexpr int kScratchOut = kScratchResParts;
constexpr int kScratchWParts = kScratchResParts + 256;
constexpr int kScratchWBlocks = 256;
constexpr int kScratchDoubles = kScratchWParts + 2 * kScratchWBlocks;  // 14 KiB
constexpr int kScratchMaxDevices = 64;

// Device address of the scratch array on the current device (looked up once
// per device).
hipError_t noalloc_scratch(double** out);

}  // namespace aao
