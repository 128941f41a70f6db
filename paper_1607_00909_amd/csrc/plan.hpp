// Internal definitions shared by the library's translation units: the plan
// object behind cdmt_plan_t, the dispersion constant and the XCD-aware
// workgroup order.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace cdmt {

// Sec. 2, text after Eq. 1: k_DM^{-1} = 2.41e-4 s MHz^2 (per unit DM).
constexpr double kKdm = 1.0 / 2.41e-4;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical indices so that neighbouring work (the
// channels of one subband block, consecutive DM tiles) shares an L2.
__device__ __forceinline__ int xcd_remap(int w, int g) {
    const int q = g >> 3, r = g & 7;
    const int xcd = w & 7, i = w >> 3;
    return (xcd < r) ? xcd * (q + 1) + i : r * (q + 1) + (xcd - r) * q + i;
}

}  // namespace cdmt

struct cdmt_plan_s {
    int nsub, nfft, noverlap, nchan, ndec;
    double f_centre, bw;
    int input_kind = 0, chirp_ref = 0, sign = -1, precision = 0, dm_tile = 16, chirp_exact = 0, lane_bins = 16;
    int out_layout = 0;     // 0: filterbanks [DM][t][ch], 1: [DM][ch][t]
    int m, nd, tblk, n1, n2;
};
