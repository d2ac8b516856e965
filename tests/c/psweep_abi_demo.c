/*
 * The psweep C ABI used from plain C (no Python, no torch): device memory
 * from hipMalloc, one plane sweep, results checked against a case with a
 * known answer.
 *
 * Test infrastructure: built by the repository's build step, run by a GPU
 * test.  Exit status 0 when every check holds.
 *
 * Geometry: a pinhole camera (unified model with xi = 0), 256 x 128, fx = fy
 * = 100, and one source displaced by b = 0.2 m along x with the same
 * orientation (X_src = X_ref + (-0.2, 0, 0)).  A fronto-parallel wall at
 * depth Z is seen by the source shifted by fx b / Z pixels, so a source image
 * equal to the reference shifted left by 4 pixels is a wall at Z = 5 m.  With
 * 16 fronto planes uniform in inverse depth from 10 m to 2.5 m, plane k has
 * inverse depth 0.1 + 0.02 k: the wall is exactly plane 5, where the source
 * samples fall on whole pixels and ZNCC is 1.  Every pixel whose window and
 * samples lie inside both images must pick plane 5, with cost ~0 and z ~5 m.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "psweep.h"

#define W 256
#define H 128
#define SHIFT 4

#define CHECK_HIP(call)                                                         \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));  \
            return 2;                                                           \
        }                                                                       \
    } while (0)

#define CHECK_PS(call, ctx)                                                                  \
    do {                                                                                     \
        psweep_status s_ = (call);                                                           \
        if (s_ != PSWEEP_OK) {                                                               \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)s_, psweep_last_error(ctx)); \
            return 3;                                                                        \
        }                                                                                    \
    } while (0)

/* xorshift32: the texture of the wall */
static uint32_t rng_state = 2463534242u;
static uint32_t next_u32(void) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 17;
    rng_state ^= rng_state << 5;
    return rng_state;
}

int main(void) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        fprintf(stderr, "no GPU\n");
        return 2;
    }
    printf("%s\n", psweep_version());

    /* images: reference texture and the source = reference shifted left */
    static uint8_t ref[H * W], src[H * W];
    for (int i = 0; i < H * W; ++i) ref[i] = (uint8_t)(next_u32() >> 24);
    for (int v = 0; v < H; ++v)
        for (int x = 0; x < W; ++x) src[v * W + x] = x + SHIFT < W ? ref[v * W + x + SHIFT] : ref[v * W + x];

    psweep_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.n_levels = 1;
    cfg.level[0].n_fronto = 16;
    cfg.level[0].near_m = 2.5;
    cfg.level[0].far_m = 10.0;
    cfg.level[0].window = 7;
    cfg.level[0].downsample = 1;
    cfg.ground_n[1] = 1.0;
    cfg.ground_d = 1.5;
    cfg.best_k = 1;
    cfg.var_floor = 1.0;
    cfg.storage = PSWEEP_STORAGE_F32;
    cfg.mode = PSWEEP_MODE_WTA;
    cfg.launch = PSWEEP_LAUNCH_GRID;
    cfg.max_width = W;
    cfg.max_height = H;
    cfg.max_sources = 1;
    cfg.max_frames = 1;
    cfg.max_camera_sets = 1;
    cfg.image_format = PSWEEP_IMAGE_U8;

    psweep_ctx *ctx = NULL;
    CHECK_PS(psweep_create(&cfg, &ctx), NULL);
    size_t ws_bytes = 0;
    CHECK_PS(psweep_workspace_size(ctx, &ws_bytes), ctx);
    void *ws = NULL;
    CHECK_HIP(hipMalloc(&ws, ws_bytes));   /* hipMalloc returns 256-byte aligned memory */
    CHECK_PS(psweep_set_workspace(ctx, ws, ws_bytes), ctx);

    const psweep_camera cam = {0.0, 100.0, 100.0, 127.5, 63.5, W, H};
    psweep_pose pose;
    memset(&pose, 0, sizeof pose);
    pose.R[0] = pose.R[4] = pose.R[8] = 1.0;
    pose.t[0] = -0.2;
    CHECK_PS(psweep_set_cameras(ctx, 0, &cam, 1, &cam, &pose), ctx);

    uint8_t *d_ref = NULL, *d_src = NULL;
    CHECK_HIP(hipMalloc((void **)&d_ref, sizeof ref));
    CHECK_HIP(hipMalloc((void **)&d_src, sizeof src));
    CHECK_HIP(hipMemcpy(d_ref, ref, sizeof ref, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_src, src, sizeof src, hipMemcpyHostToDevice));
    float *d_z = NULL, *d_c1 = NULL;
    int32_t *d_idx = NULL;
    CHECK_HIP(hipMalloc((void **)&d_z, sizeof(float) * W * H));
    CHECK_HIP(hipMalloc((void **)&d_c1, sizeof(float) * W * H));
    CHECK_HIP(hipMalloc((void **)&d_idx, sizeof(int32_t) * W * H));

    psweep_frame frame;
    memset(&frame, 0, sizeof frame);
    frame.ref = d_ref;
    frame.ref_pitch = W;
    frame.src[0] = d_src;
    frame.src_pitch[0] = W;
    psweep_output out;
    memset(&out, 0, sizeof out);
    out.merged.z = d_z;
    out.merged.cost1 = d_c1;
    out.merged.index = d_idx;

    CHECK_PS(psweep_run(ctx, &frame, 1, &out, NULL), ctx);   /* NULL: the default stream */
    CHECK_HIP(hipDeviceSynchronize());

    static float z[H * W], c1[H * W];
    static int32_t idx[H * W];
    CHECK_HIP(hipMemcpy(z, d_z, sizeof z, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(c1, d_c1, sizeof c1, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(idx, d_idx, sizeof idx, hipMemcpyDeviceToHost));

    /* pixels whose window (3 px) and plane-5 samples (4 px to the left) lie
     * inside both images, away from the shifted-in right edge */
    int n = 0, right = 0, bad_cost = 0, bad_z = 0;
    for (int v = 3; v < H - 3; ++v)
        for (int u = 16; u < W - 16; ++u) {
            const int e = v * W + u;
            ++n;
            if (idx[e] == 5) ++right;
            if (!(c1[e] <= 1e-4f)) ++bad_cost;
            if (!(fabsf(z[e] - 5.0f) <= 0.1f)) ++bad_z;   /* the parabola moves z by a few cm */
        }
    /* the border frame is marked invalid in-band */
    int border_ok = idx[0] == -1 && idx[W * H - 1] == -1 && isnan(z[0]);
    printf("pixels %d, plane 5: %d, cost > 1e-4: %d, |z - 5| > 0.1: %d, border marks %s\n", n, right, bad_cost,
           bad_z, border_ok ? "ok" : "wrong");

    /* an out-of-order call is refused without aborting */
    psweep_status st = psweep_soft_depth_backward(ctx, d_z, NULL, (double *)d_c1, NULL);
    printf("backward after a WTA run: status %d (%s)\n", (int)st, psweep_last_error(ctx));

    psweep_destroy(ctx);
    hipFree(d_idx);
    hipFree(d_c1);
    hipFree(d_z);
    hipFree(d_src);
    hipFree(d_ref);
    hipFree(ws);
    const int ok = right == n && bad_cost == 0 && bad_z == 0 && border_ok && st == PSWEEP_ESTATE;
    printf("%s\n", ok ? "PASS" : "FAIL");
    return ok ? 0 : 1;
}
