// nf_kernels.h -- host-side launch interfaces between the translation units
// of libnf.so (not part of the public ABI).
#pragma once

#include <algorithm>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nf_internal.h"

namespace nf {

// Sizes and scratch pointers of one binning call (all boxes together).
struct BinPlan {
    int64_t N = 0;          // sum of n_b
    int64_t C = 0;          // sum of K_b^3
    int64_t max_n = 0;      // largest n_b
    int64_t max_ncell = 0;  // largest K_b^3
    int64_t nblk = 0;       // radix tiles: ceil(N / kSortTile)
    int passes = 0;         // 8-bit radix passes covering keys 0..C-1
    BinScratch sc{};
    uint32_t *scan_scratch = nullptr;
};

int64_t scan_scratch_words(int64_t M);
hipError_t bin_launch(const DevBox *d_boxes, int nbox, const BinPlan &p, hipStream_t s);

// Force launches.  `items` and `nitems` describe the work list built on the
// host side of the call (see nf_accel.hip).
struct ForcePlan {
    int64_t max_n = 0;
    bool compensated = false;
    bool simple = false;
    float4 *cot_sorted = nullptr;   // vjp only: [N] cotangents in sorted order
    int64_t N = 0;
};

hipError_t accel_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s);
hipError_t vjp_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s);

}  // namespace nf
