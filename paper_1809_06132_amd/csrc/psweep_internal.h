// Internal layout shared by the host side of the library and its kernels.
// Nothing here is part of the C ABI.
#pragma once

#include <stdint.h>

namespace psw {

constexpr int kMaxSrc = 4;
constexpr int kMaxLevels = 2;
constexpr int kMaxJobs = 64;          // frames x levels per psweep_run
constexpr int kWave = 64;

// One source camera of one level, as the sweep kernel reads it.
struct SrcDev {
    const uint32_t *tex;   // texels (4 x FP16 cell coefficients or 4 x float), row pitch = w texels
    int32_t w, h;
    float fx, fy, cx, cy, xi;
    float wm1, hm1;        // w - 1, h - 1 (inclusive sample bounds)
    int32_t pad;
};

// Everything the kernels need for one (frame, level).  Lives in device
// memory (the workspace); read through the scalar cache.
struct JobDev {
    // reference view of the level (downsampled copy or a view into the
    // frame); uint8_t, or float for the float-image kernels; pitch in elements
    const uint8_t *ref;
    int64_t ref_pitch;
    int32_t w, h;
    float fx, fy, cx, cy, xi;
    float inv_fx, inv_fy;
    int32_t n_src, n_fronto, n_ground, window, best_k, mode;
    float var_floor_n;     // N * tau
    float gn[3];
    float gd;
    float step_f, step_g;  // plane-parameter steps (inverse depth, height)
    float temperature;
    const float *htab;     // [P][S][9]: columns h1, h2, h3 of H = R + t n^T / d
    const float *theta;    // [P] plane parameter: rho (fronto) or h (ground)
    // level result maps (index < 0: invalid)
    int32_t *index;
    float *delta, *cost1, *cost2, *depth, *z;
    uint8_t *level_id;
    int64_t out_pitch;
    float *soft_rho, *soft_lse;
    int64_t soft_pitch;
    int32_t tiles_x, tiles_y, first_item, pad0;
    // tile shape used for this job by the grid launch (rows per wave, waves)
    int32_t rows, waves, pad1, pad2;
    // plane chunks: the fronto planes are cut into nch_f contiguous chunks and
    // the ground planes into nch_g; with more than one chunk every chunk of a
    // tile writes a partial state (kPartWords words per pixel) that
    // chunk_merge_kernel combines
    int32_t nch_f, nch_g, pad3, pad4;
    float *part;           // [chunk][word][h][w], pitch w
    // The job's (chunk, tile) items (chunk * tiles + tile) in eight queues,
    // one per XCD: order[0 .. 8] are the queues' starts in order + kQueueHead
    // (order[8]: the item count), each queue sorted largest item first;
    // queue_ctr: the eight queues' take counters (zeroed before the launch).
    const int32_t *order;
    int32_t *queue_ctr;
    float *volume;         // optional [P][h][w] aggregated costs (psweep_output::cost_volume)
    SrcDev src[kMaxSrc];
};

constexpr int kQueueHead = 16;   // ints before the items of an order table
constexpr int kQueues = 8;       // one item queue per XCD
constexpr int kPartWords = 7;   // c1, kb, c2, cm, cp, first, last (soft: max, sum, sum*theta)
constexpr int kMaxChunks = 8;

// plane range [kb, ke) of chunk c of a job (chunks never straddle families)
__host__ __device__ inline void chunk_range(int n_fronto, int n_ground, int nch_f, int nch_g, int c, int *kb,
                                            int *ke) {
    if (c < nch_f) {
        *kb = (int)((long long)c * n_fronto / nch_f);
        *ke = (int)((long long)(c + 1) * n_fronto / nch_f);
    } else {
        const int g = c - nch_f;
        *kb = n_fronto + (int)((long long)g * n_ground / nch_g);
        *ke = n_fronto + (int)((long long)(g + 1) * n_ground / nch_g);
    }
}

// FP64 description of one (frame, level) for the setup kernel.
struct SetupDev {
    double R[kMaxSrc][9];
    double t[kMaxSrc][3];
    double near_m, far_m, h_lo, h_hi;
    double gn[3];
    double gd;
    int32_t n_src, n_fronto, n_ground, pad;
    float *htab;
    float *theta;
};

// Level-image preparation for one (frame, level): downsampled reference (if
// any) and the source textures.
struct PrepDev {
    const uint8_t *ref_full;
    int64_t ref_pitch;
    int32_t ref_w, ref_h;          // full-resolution reference size
    uint8_t *ref_level;            // downsampled reference (downsample == 2), else null
    int32_t downsample, n_src;
    const void *src_full[kMaxSrc]; // uint8_t or float images (img)
    int64_t src_pitch[kMaxSrc];    // elements
    int32_t src_w[kMaxSrc], src_h[kMaxSrc];   // full-resolution sizes
    uint32_t *tex[kMaxSrc];        // level-size textures: 4 x FP16 cell coefficients or 4 floats per texel
    int32_t img, pad;
};

// Full-resolution merge of a frame's levels.
struct MergeDev {
    int32_t w, h;                  // full-resolution reference
    float fx, fy, cx, cy, xi;
    float gn[3];
    float gd;
    int32_t n_levels, ds0;
    int32_t low_w, low_h;
    const int32_t *low_index;
    const float *low_delta, *low_c1, *low_c2;
    int64_t low_pitch;
    const float *low_theta;
    int32_t low_nf;
    float low_step_f, low_step_g;
    int32_t crop_x, crop_y, crop_w, crop_h;
    const int32_t *crop_index;
    const float *crop_delta, *crop_c1, *crop_c2;
    int64_t crop_pitch;
    const float *crop_theta;
    int32_t crop_nf;
    float crop_step_f, crop_step_g;
    float crop_near;
    // merged outputs
    float *depth, *z, *delta, *cost1, *cost2;
    int32_t *index;
    uint8_t *level;
    int64_t out_pitch;
};

// Pixels outside the area where a window fits: written as invalid.
struct BorderDev {
    int32_t w, h, hw, pad;
    int32_t *index;
    float *delta, *cost1, *cost2, *depth, *z;
    uint8_t *level_id;
    int64_t out_pitch;
    float *soft_rho, *soft_lse;
    int64_t soft_pitch;
};

}  // namespace psw

namespace psw {

// Depth-map filtering of one full-resolution map.
struct FilterDev {
    int32_t w, h, win, pad;
    float fx, fy, cx, cy, xi;
    float gn[3];
    float alpha_upper, alpha_lower, ratio_min, gamma, min_count;
    const float *depth, *cost1, *cost2;
    int64_t in_pitch;
    float *out_depth;
    uint8_t *code;
    int64_t out_pitch;
};

// Box masking of a depth map: boxes passed by value, kMaxMaskBoxes per launch.
constexpr int kMaxMaskBoxes = 64;
struct MaskDev {
    float *depth;
    uint8_t *code;
    int64_t pitch;
    int32_t w, h, n, pad;
    int32_t box[kMaxMaskBoxes][4];   // clipped x0, y0, x1, y1
};

// One compiled variant of the sweep kernel.
struct KernelEntry {
    int win, rows, waves, n_src, store, soft, persistent;
    const void *fn;
    size_t lds;     // dynamic LDS bytes
    int img = 0;    // frame pixel type: 0 uint8, 1 float
};

}  // namespace psw

// Each instantiation unit exports its table through one of these.
extern "C" int psw_kernels_grid(const psw::KernelEntry **out);
extern "C" int psw_kernels_extra(const psw::KernelEntry **out);
extern "C" int psw_kernels_small(const psw::KernelEntry **out);
extern "C" int psw_kernels_grid8(const psw::KernelEntry **out);
extern "C" int psw_kernels_persistent(const psw::KernelEntry **out);
extern "C" int psw_kernels_f32img(const psw::KernelEntry **out);
