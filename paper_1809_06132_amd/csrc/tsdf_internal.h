// Internal layout of the TSDF map shared by its host code and kernels.
// Nothing here is part of the C ABI.
#pragma once

#include <stdint.h>

namespace psw {

constexpr int kBlockVox = 512;      // 8 x 8 x 8 voxels per block

// Everything the TSDF kernels of one integration need (passed by value).
// World coordinates are taken relative to the box's first block, so that
// float positions stay small however far the vehicle drives: a box-relative
// point X maps to the camera as R X + t.
struct TsdfDev {
    float fx, fy, cx, cy, xi;
    int32_t w, h;
    float R[9], t[3];
    float voxel, block, mu, w_max;
    int32_t b0[3], nb[3];
    int32_t nslots, min_obs;
    const float *depth;
    int64_t pitch;
    unsigned long long *keys;   // packed block coordinates + valid bit, 0 = empty
    int32_t *count, *seen, *fresh, *list;
    int32_t *counters;          // [0] visible blocks, [1] allocated slots
    float *D, *W;               // [slot][512]
};

}  // namespace psw
