// Scratch memory of the entry point that allocates nothing (rl0_sketch_static).
#pragma once

#include <hip/hip_runtime.h>

namespace rl0 {

// Rows of the largest sketch rl0_sketch_static takes: its 64-bit fixed-point sums S [m]
// fill the front of the scratch array, the error flags sit right after them.
constexpr int kStaticSketchRows = 1 << 21;

// The calling device's copy of the scratch array, as a device address (looked up once per
// device with that device current, then cached).
hipError_t static_scratch(long long** out);

}  // namespace rl0
