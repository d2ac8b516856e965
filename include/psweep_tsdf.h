/*
 * psweep_tsdf.h - C ABI of fisheye TSDF depth-map fusion on gfx950.
 *
 * Fuses the depth maps of the plane sweep into a truncated signed distance
 * map (Cui et al., Sec. III-C): voxel blocks are allocated along the segment
 * [d - mu, d + mu] of every valid pixel's Eq. (1) ray, the blocks in view are
 * listed, and every voxel of them takes the running average of Eq. (2) with a
 * capped weight.  The map is a box of blocks that follows a centre point (the
 * vehicle), like the paper's 60 m x 60 m x 3 m local map: blocks that leave
 * the box are dropped.  Blocks observed by fewer than min_observations depth
 * maps are left out of extraction (Sec. III-C).
 *
 * Conventions as in psweep.h: every call returns a psweep_status and never
 * aborts; device memory (workspace, depth maps, outputs) is owned by the
 * caller; calls taking a hip_stream are asynchronous on it.
 *
 * Layout on the device: the box holds blocks[0] x blocks[1] x blocks[2]
 * blocks of 8 x 8 x 8 voxels; a block with integer world block coordinates
 * (bx, by, bz) (it covers [b B, (b + 1) B) per axis, B = 8 voxel_m) lives in
 * slot ((bz mod nz) ny + (by mod ny)) nx + (bx mod nx), so a moving box wraps
 * around its storage and nothing is copied.  Per slot: the block's packed
 * coordinates, its observation count and 512 voxels of (TSDF, weight) as
 * floats.
 */
#ifndef PSWEEP_TSDF_H
#define PSWEEP_TSDF_H

#include <stddef.h>
#include <stdint.h>

#include "psweep.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psweep_tsdf psweep_tsdf;

typedef struct {
    double voxel_m;             /* voxel edge, metres; blocks are 8 x 8 x 8 voxels */
    double mu_m;                /* truncation distance mu, metres */
    int32_t blocks[3];          /* box of the local map in blocks along world x, y, z (each 1 .. 1024) */
    double w_max;               /* cap of the running-average weight (>= 1) */
    int32_t min_observations;   /* extraction leaves out blocks seen by fewer depth maps */
    int32_t max_width, max_height;  /* largest depth map */
} psweep_tsdf_config;

/* Create a map.  EINVAL for non-positive sizes, mu_m above 16 blocks
 * (128 voxel_m), blocks out of [1, 1024], a box of more than 2^24 blocks,
 * w_max < 1 or max sizes out of [8, 8192]. */
psweep_status psweep_tsdf_create(const psweep_tsdf_config *cfg, psweep_tsdf **out);

/* Bytes of device workspace the map needs (fixed by the config: 8 bytes per
 * slot key, 12 per slot of counts and flags, 4 per slot of visible list, and
 * 4096 per slot of voxels). */
psweep_status psweep_tsdf_workspace_size(const psweep_tsdf *ts, size_t *bytes);

/* Bind caller-allocated device memory (>= psweep_tsdf_workspace_size bytes,
 * 256-byte aligned).  The map must then be emptied with psweep_tsdf_reset
 * before its first integration. */
psweep_status psweep_tsdf_set_workspace(psweep_tsdf *ts, void *dev_ptr, size_t bytes);

/* Empty the map (kernels on hip_stream, no memset). */
psweep_status psweep_tsdf_reset(psweep_tsdf *ts, void *hip_stream);

/* Fuse one depth map.  cam: the unified-model camera of the map (its size is
 * the depth map's); world_to_cam: X_cam = R X_world + t (Sec. III-C's
 * (R_d, t_d)); centre: world point the box is centred on (block b0 = floor(c
 * / B) - blocks / 2 per axis); depth: device float range along the Eq. (1)
 * ray in metres (NaN or <= 0: invalid), row pitch in elements (0 = width).
 * Asynchronous.  EINVAL for NULL arguments, sizes above the maximum, a
 * non-finite camera or pose, a rotation that is not orthonormal, or a centre
 * whose block coordinates leave +-2^20; ESTATE before workspace and reset. */
psweep_status psweep_tsdf_integrate(psweep_tsdf *ts, const psweep_camera *cam, const psweep_pose *world_to_cam,
                                    const double centre[3], const float *depth, int64_t pitch, void *hip_stream);

/* Copy the box out in world order: tsdf and weight over its voxel grid,
 * [z][y][x] with (blocks[2] 8) x (blocks[1] 8) x (blocks[0] 8) floats, and the
 * observation count of every block, [z][y][x] int32; voxel 0 is the first
 * voxel of block b0 of the last integration.  tsdf is NaN where the voxel has
 * weight 0 or its block fewer than min_observations observations.  Any
 * pointer may be NULL.  Asynchronous.  ESTATE before the first integration. */
psweep_status psweep_tsdf_extract(psweep_tsdf *ts, float *d_tsdf, float *d_weight, int32_t *d_block_count,
                                  void *hip_stream);

/* Block coordinates b0 of the box's first block after the last integration
 * (host call, no device access). */
psweep_status psweep_tsdf_region(const psweep_tsdf *ts, int32_t first_block[3]);

/* Counters of the last integration copied to device memory d_stats[2]:
 * allocated slots, visible blocks.  Asynchronous. */
psweep_status psweep_tsdf_stats(psweep_tsdf *ts, int32_t *d_stats, void *hip_stream);

/* Message of the last failed call on `ts` (NULL: of the last failed create). */
const char *psweep_tsdf_last_error(const psweep_tsdf *ts);

void psweep_tsdf_destroy(psweep_tsdf *ts);

#ifdef __cplusplus
}
#endif

#endif /* PSWEEP_TSDF_H */
