// XCD-aware workgroup order (device helper shared by the kernels).
#pragma once

#include <hip/hip_runtime.h>

namespace cdmt {

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical indices so that neighbouring work (the
// channels of one subband block, consecutive DM tiles) shares an L2.
__device__ __forceinline__ int xcd_remap(int w, int g) {
    const int q = g >> 3, r = g & 7;
    const int xcd = w & 7, i = w >> 3;
    return (xcd < r) ? xcd * (q + 1) + i : r * (q + 1) + (xcd - r) * q + i;
}

}  // namespace cdmt
