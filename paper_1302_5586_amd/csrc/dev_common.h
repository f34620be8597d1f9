// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

// MI355X deals the workgroups of a launch round-robin over its 8 XCDs
// (workgroup b runs on XCD b mod 8), and each XCD has its own L2. The
// remap gives the workgroups of one XCD consecutive logical ids, so tiles
// with neighbouring logical ids (which share halo rows and cache lines)
// meet in the same L2. b: hardware workgroup id; g: workgroups in the grid.
__device__ __forceinline__ int xcd_remap(int b, int g) {
    const int xcd = b & 7, idx = b >> 3;
    const int per = g >> 3, rem = g & 7;
    return xcd * per + min(xcd, rem) + idx;
}

}  // namespace pf
