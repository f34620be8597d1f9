// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// A device address held as an integer (a descriptor field), as a pointer
// into global memory: cast through the global address space so that the
// compiler emits global accesses rather than flat ones.
template <class T>
__device__ __forceinline__ T *global_ptr(int64_t addr) {
    typedef __attribute__((address_space(1))) T gT;
    return (T *)(gT *)(uintptr_t)addr;
}

}  // namespace pf
