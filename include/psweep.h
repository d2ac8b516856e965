/*
 * psweep.h -- C ABI of the MI355X (gfx950) fisheye plane-sweep stereo library.
 *
 * The library computes, for a reference fisheye image and up to four
 * supporting fisheye images with known relative poses, a depth map of the
 * reference view by plane-sweeping stereo (Cui et al., "Real-Time Dense
 * Mapping for Self-Driving Vehicles using Fisheye Cameras", Sec. III-A):
 *   - planes parallel to the reference image plane and planes parallel to the
 *     ground plane given by the extrinsic calibration (Sec. III-A);
 *   - every reference pixel's ray (unified camera model, Eq. (1), Sec. III-C)
 *     is intersected with each plane, projected into each source through the
 *     same model and bilinearly sampled;
 *   - the matching cost is negative ZNCC over a window, cost = (1 - ZNCC) / 2,
 *     so ZNCC -1 costs 1 and ZNCC +1 costs 0 (Sec. III-A);
 *   - the best plane per pixel with its first and second best costs (Sec.
 *     III-A, depth-map filtering), refined by a parabola through the winner
 *     and its two neighbours;
 *   - two resolution levels: a downsampled full field of view and a
 *     full-resolution centre crop, fused into one full-resolution map (Sec.
 *     III-A, multi-scale strategy);
 *   - optionally a soft-argmin over the planes (each standing for the
 *     inverse z-depth at which the pixel's ray meets it) with a gradient
 *     with respect to the source images and the source poses.
 *
 * Conventions shared by every call:
 *   - Pixel (i, j) has its centre at (u, v) = (i, j); normalized coordinates
 *     are x = (u - cx) / fx, y = (v - cy) / fy.
 *   - Reference frame: x right, y down, z forward, metres.  A source sees
 *     X_src = R X_ref + t (R row-major).
 *   - Images are 8-bit grey (or float, PSWEEP_IMAGE_F32), row-major, in
 *     device memory, with a row pitch in elements (pixels).  Output maps are
 *     row-major device arrays with a pitch in elements.
 *   - All device memory (images, outputs, workspace) is owned by the caller.
 *     The context owns host-side state only.
 *   - Every call returns a psweep_status and never aborts.  Launch errors are
 *     reported as PSWEEP_EHIP by the same or the next call.  Outputs are
 *     undefined after an error.  psweep_last_error() gives a message.
 *   - Work is enqueued asynchronously on the caller's HIP stream; only
 *     psweep_destroy() synchronises.  A context must not be used from two
 *     host threads at once.  Successive runs of one context reuse its
 *     workspace (job tables, level images, partial states): enqueue them on
 *     one stream, or order them with events.  Contexts are independent.
 *   - Invalid pixels are marked in-band: depth and z NaN, index -1, delta 0,
 *     cost1 and cost2 +inf, level 255.
 */
#ifndef PSWEEP_H
#define PSWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSWEEP_MAX_SOURCES 4
#define PSWEEP_MAX_LEVELS 2
#define PSWEEP_MAX_PLANES 1024   /* fronto + ground planes per level */

typedef enum {
    PSWEEP_OK = 0,
    PSWEEP_EINVAL = -1,        /* bad argument: NULL, size, range, layout */
    PSWEEP_ESTATE = -2,        /* call out of order */
    PSWEEP_ENOMEM = -3,        /* host allocation failed or workspace too small */
    PSWEEP_EHIP = -4,          /* HIP runtime or launch error */
    PSWEEP_EUNSUPPORTED = -5   /* valid request the library does not implement */
} psweep_status;

enum { PSWEEP_STORAGE_F32 = 0, PSWEEP_STORAGE_F16 = 1, PSWEEP_STORAGE_BF16 = 2 };
enum { PSWEEP_MODE_WTA = 0, PSWEEP_MODE_SOFT = 1 };
enum { PSWEEP_LAUNCH_GRID = 0, PSWEEP_LAUNCH_PERSISTENT = 1 };
/* Pixel type of the frame images: 8-bit grey levels, or 32-bit float grey
 * values (any real values; the cost is invariant to affine intensity changes
 * but the variance floor is in grey levels squared). */
enum { PSWEEP_IMAGE_U8 = 0, PSWEEP_IMAGE_F32 = 1 };

typedef struct psweep_ctx psweep_ctx;

/* Unified (Mei) fisheye camera, Sec. III-C Eq. (1): mirror parameter xi in
 * [0, 1] plus a pinhole part; no lens distortion. */
typedef struct {
    double xi, fx, fy, cx, cy;
    int32_t width, height;
} psweep_camera;

/* Rigid transform reference -> source: X_src = R X_ref + t (Sec. III-A,
 * "known relative poses"). */
typedef struct {
    double R[9];
    double t[3];
} psweep_pose;

/* One resolution level (Sec. III-A).  Fronto planes are uniform in inverse
 * depth from far_m (index 0) to near_m; ground-parallel planes follow,
 * uniform in height above the ground from h_lo to h_hi.  downsample 2 halves
 * every image with a 2x2 box filter (rounded integer mean).  A crop (crop_w >
 * 0) restricts the reference to a rectangle of the (possibly downsampled)
 * reference image; the sources stay whole. */
typedef struct {
    int32_t n_fronto;
    double near_m, far_m;
    int32_t n_ground;
    double h_lo, h_hi;
    int32_t window;                 /* odd, 3..15 */
    int32_t downsample;             /* 1 or 2 */
    int32_t crop_x, crop_y, crop_w, crop_h;
} psweep_level;

typedef struct {
    int32_t n_levels;               /* 1 or 2 (level 1 is the crop level) */
    psweep_level level[PSWEEP_MAX_LEVELS];
    double ground_n[3], ground_d;   /* ground plane n . X = ground_d, unit n, reference frame */
    int32_t best_k;                 /* per plane, mean of the best_k valid source costs */
    double var_floor;               /* windows with variance <= var_floor (grey^2) are unusable */
    int32_t storage;                /* PSWEEP_STORAGE_*: precision of staged warped samples */
    int32_t mode;                   /* PSWEEP_MODE_WTA or PSWEEP_MODE_SOFT */
    double temperature;             /* soft mode: softmax over -cost / temperature */
    int32_t launch;                 /* PSWEEP_LAUNCH_GRID or PSWEEP_LAUNCH_PERSISTENT */
    int32_t max_width, max_height;  /* largest reference / source image */
    int32_t max_sources;            /* <= PSWEEP_MAX_SOURCES */
    int32_t max_frames;             /* frames per psweep_run */
    int32_t max_camera_sets;
    int32_t image_format;           /* PSWEEP_IMAGE_U8 or PSWEEP_IMAGE_F32 (F32: one level, no
                                       downsample or crop, grid launch) */
} psweep_config;

/* One frame set: device images and the camera set describing them.  The
 * pointers are uint8_t or float images as the config's image_format says,
 * row-major; pitches in elements (pixels), not bytes. */
typedef struct {
    const void *ref;
    int64_t ref_pitch;
    const void *src[PSWEEP_MAX_SOURCES];
    int64_t src_pitch[PSWEEP_MAX_SOURCES];
    int32_t camera_set;
} psweep_frame;

/* Per-pixel maps; any pointer may be NULL (not written).  pitch in elements,
 * 0 = the map's width. */
typedef struct {
    float *depth;       /* range along the unit ray, metres */
    float *z;           /* camera-frame z, metres */
    int32_t *index;     /* winning plane of the level the pixel came from */
    float *delta;       /* parabolic subpixel offset, plane steps, [-0.5, 0.5] */
    float *cost1;       /* best aggregated cost */
    float *cost2;       /* best aggregated cost over all other planes */
    uint8_t *level;     /* merged maps only: 0 low level, 1 crop level, 255 invalid */
    int64_t pitch;
} psweep_maps;

typedef struct {
    psweep_maps merged;                       /* full reference resolution */
    psweep_maps level[PSWEEP_MAX_LEVELS];     /* per level, at the level's size (optional) */
    float *soft_invdepth;                     /* soft mode, full resolution: sum_k p_k rho_k, rho_k the
                                                 inverse z-depth of the pixel's ray at plane k */
    float *soft_lse;                          /* soft mode: log-sum-exp of -cost / T */
    int64_t soft_pitch;
    /* Optional (NULL = not written), winner-take-all mode with the grid
     * launch: per level, the aggregated cost of every (pixel, plane) of the
     * level (mean of the best_k source costs; +inf where no source window is
     * usable), device floats [P][h][w] at the level's size, plane k at
     * offset k * w * h.  Written only for pixels whose window lies inside the
     * level image, and not for a (pixel, plane family) the sweep skips (a
     * wave of pixels without a textured reference window or a ray that meets
     * the family): fill it with +inf beforehand.  For parity tests of every
     * cost; it costs one store per (pixel, plane). */
    float *cost_volume[PSWEEP_MAX_LEVELS];
} psweep_output;

/* Create a context for `cfg`.  EINVAL on inconsistent settings (even window,
 * fewer than 2 planes in a used family, non-positive plane distances, sizes
 * or counts out of range, best_k outside [1, max_sources], unknown
 * image_format); EUNSUPPORTED for soft mode with two levels, with a
 * downsampled or cropped level, with FP16/BF16 staging or with the
 * persistent launch,
 * and for float images with anything but one full-resolution level on the
 * grid launch.  *out receives the context. */
psweep_status psweep_create(const psweep_config *cfg, psweep_ctx **out);

/* Bytes of device workspace the context needs (fixed by the config). */
psweep_status psweep_workspace_size(const psweep_ctx *ctx, size_t *bytes);

/* Bind caller-allocated device memory (>= psweep_workspace_size bytes,
 * 256-byte aligned).  ENOMEM if smaller, EINVAL if misaligned or NULL. */
psweep_status psweep_set_workspace(psweep_ctx *ctx, void *dev_ptr, size_t bytes);

/* Define camera set `camera_set` (0 .. max_camera_sets-1): the reference
 * camera, n_src source cameras and the n_src poses reference -> source.
 * Sizes must not exceed max_width x max_height; n_src in [1, max_sources];
 * xi in [0, 1]; fx, fy > 0; R orthonormal to 1e-6.  Host pointers, copied. */
psweep_status psweep_set_cameras(psweep_ctx *ctx, int32_t camera_set, const psweep_camera *ref,
                                 int32_t n_src, const psweep_camera *src, const psweep_pose *ref_to_src);

/* Override the crop rectangle of level 1 for one camera set (frames of mixed
 * sizes need their own crop).  Full-resolution pixels of the reference. */
psweep_status psweep_set_crop(psweep_ctx *ctx, int32_t camera_set, int32_t x, int32_t y, int32_t w,
                              int32_t h);

/* Sweep n_frames frame sets (1 .. max_frames) and write out[i] for frames[i].
 * `frames` and `out` are host arrays of device pointers.  Enqueued on
 * hip_stream (a hipStream_t; NULL = default stream).  ESTATE before
 * psweep_set_workspace or for a camera set never defined; EINVAL for NULL
 * images, pitches below the width, or maps whose pitch is below their width.
 * Soft mode requires n_frames == 1.  The images must stay alive and unchanged
 * until a following psweep_soft_depth_backward has run. */
psweep_status psweep_run(psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                         const psweep_output *out, void *hip_stream);

/* psweep_run for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same maps, bitwise, with no workspace.  The run's scratch (job tables,
 * counters, level images, textures, level maps) lives in a static device
 * array of the library, 64 MiB per GPU, held until the process ends; each
 * tile sweeps all its planes in one pass (no plane chunks, which would need
 * partial-state room).  The caller passes only inputs and outputs; no
 * psweep_set_workspace is needed.  EINVAL (with the bytes the context needs)
 * when the context's limits (max_width x max_height, max_sources,
 * max_frames) need more than 64 MiB, e.g. one 1024 x 768 frame with three
 * sources needs about 31 MiB; EUNSUPPORTED in soft mode.  Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * (from any context) that overlap on one GPU race, so order them on one
 * stream; a call after psweep_run on the same context sets its tables up
 * again.  Calls no hipMalloc or hipFree. */
psweep_status psweep_run_noalloc(psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                                 const psweep_output *out, void *hip_stream);

/* Gradient of L = sum_p g_p * soft_invdepth_p (g = d_grad_invdepth, full
 * resolution, pitch soft_pitch of the last run) with respect to every source
 * image (d_grad_src[s]: float device array of the source's size, row-major,
 * overwritten; a NULL d_grad_src, or a NULL entry, skips that image gradient
 * and its atomics) and to every source pose as a left perturbation X_src ->
 * X_src + v + omega x X_src (d_grad_pose: device doubles [n_src][6] ordered
 * v, omega; overwritten).  Uses the images and soft outputs of the last
 * psweep_run, which must have been a soft run (ESTATE otherwise).  Both
 * plane families take part, as in the forward.  Warps are recomputed, not
 * stored.  The planes are split into chunks swept by separate
 * workgroups.  Image gradients are accumulated with atomics, so they vary in
 * the last bits from run to run.  The pose gradient is summed in a fixed
 * order, so it does not.  Its per-workgroup partial sums go to the context
 * workspace (the plane-chunk region of that soft run), so the call must be
 * ordered after the run and before the next run on the same workspace, like
 * every call on a context.  Windows 5, 7, 9 and up to four sources
 * (EUNSUPPORTED otherwise). */
psweep_status psweep_soft_depth_backward(psweep_ctx *ctx, const float *d_grad_invdepth,
                                         float *const *d_grad_src, double *d_grad_pose, void *hip_stream);

/* A source pose moved by the left perturbation xi = (v, omega) whose gradient
 * psweep_soft_depth_backward returns: R' = Exp(omega) R, t' = Exp(omega) t + v,
 * with Exp the rotation exponential (Rodrigues' formula, its series for
 * |omega| < 1e-4), i.e. X_src -> Exp(omega) X_src + v, which is
 * X_src + v + omega x X_src to first order.  Host memory, FP64: R and R_out
 * row-major 3x3, t and t_out 3-vectors, xi 6 values (v then omega); R_out may
 * alias R and t_out alias t.  No context or GPU needed.  EINVAL for a NULL
 * pointer or a non-finite xi. */
psweep_status psweep_perturb_pose(const double *R, const double *t, const double *xi, double *R_out,
                                  double *t_out);

/* Tile shape of the sweep kernel for one level: rows per wave (2, 4, 8 or
 * 16) and waves per workgroup (2, 4 or 8); 0, 0 restores the default.  Used
 * by the autotuner.  EINVAL for other values; psweep_run returns
 * EUNSUPPORTED when no kernel is built for the shape with the level's
 * window, source count and storage. */
psweep_status psweep_set_tile(psweep_ctx *ctx, int32_t level, int32_t rows_per_wave, int32_t waves);

/* Depth-map filtering parameters (Sec. III-A): the best-cost threshold for
 * pixels looking above the ground plane's horizon (alpha_upper, paper 0.05)
 * and below it (alpha_lower, paper 0.3); the minimum ratio cost2 / cost1
 * (the paper gives none); the continuity tolerance gamma_m (paper 0.5 m) and
 * the minimum fraction delta (paper 0.3) of the other pixels of an odd
 * window x window neighbourhood that must lie within gamma_m. */
typedef struct {
    double alpha_upper, alpha_lower, ratio_min, gamma_m, delta;
    int32_t window;
} psweep_filter_params;

/* Filter a full-resolution map of camera set `camera_set` (in: depth, cost1,
 * cost2 and pitch of a psweep_run output) in the paper's order: best cost,
 * uniqueness ratio, local continuity (on the pixels that passed the first
 * two).  Writes the kept range (NaN elsewhere) and a code per pixel: 0 kept,
 * 1 cost, 2 ratio, 3 continuity, 255 invalid before filtering.  Asynchronous
 * on hip_stream; EINVAL for bad parameters or pitches. */
psweep_status psweep_filter(psweep_ctx *ctx, int32_t camera_set, const psweep_maps *in,
                            const psweep_filter_params *params, float *out_depth, uint8_t *out_code,
                            int64_t out_pitch, void *hip_stream);

/* Remove potentially moving objects from a depth map (Sec. III overview and
 * Sec. IV-B: the detector's bounding boxes are masked out of the reference
 * depth map before fusion).  boxes: host array of n_boxes x 4 int32 (x0, y0,
 * x1, y1), the half-open pixel rectangle [x0, x1) x [y0, y1) of the camera
 * set's full-resolution reference image; parts outside the image are
 * ignored, empty boxes are allowed.  Every pixel inside a box gets depth NaN
 * and, if code is not NULL, code 4.  pitch in elements, 0 = the image width.
 * Asynchronous on hip_stream (the box list is copied before the call
 * returns).  EINVAL for NULL depth, NULL boxes with n_boxes > 0, or n_boxes <
 * 0; ESTATE for an undefined camera set. */
psweep_status psweep_mask_boxes(psweep_ctx *ctx, int32_t camera_set, float *depth, uint8_t *code, int64_t pitch,
                                int32_t n_boxes, const int32_t *boxes, void *hip_stream);

/* Plane chunks per tile for one level: each tile's planes are cut into
 * n_chunks contiguous ranges swept by separate workgroups (more parallelism
 * on small images) and combined exactly afterwards; 0 = automatic (about 28
 * waves per SIMD), 1 = one pass over all planes, at most 8.  Results do not
 * depend on the choice (bitwise, winner-take-all mode). */
psweep_status psweep_set_chunks(psweep_ctx *ctx, int32_t level, int32_t n_chunks);

/* Capture one psweep_run of these frames into a HIP graph owned by the
 * context (replacing any earlier graph).  The frame and output pointers are
 * baked in.  The capture runs on a stream of the context's own after a device
 * synchronisation (hip_stream is unused and may be NULL); this call blocks. */
psweep_status psweep_graph_capture(psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                                   const psweep_output *out, void *hip_stream);

/* Launch the captured graph on hip_stream.  ESTATE if none was captured.
 * The graph writes the same frame slots of the workspace as psweep_run (its
 * plane tables, level images and partial states), so graph launches and runs
 * must be ordered on one stream like any two runs; the next psweep_run sets
 * its plane tables up afresh. */
psweep_status psweep_graph_launch(psweep_ctx *ctx, void *hip_stream);

/* Record HIP events around every sweep-kernel launch of later runs (on = 1)
 * or stop (on = 0).  Off by default: events are outside the timed work. */
psweep_status psweep_set_timing(psweep_ctx *ctx, int32_t on);

/* Average duration in milliseconds of the sweep kernel launches enqueued by
 * the last psweep_run (measured with HIP events on the launch stream, read
 * after the stream has been synchronised by the caller).  ESTATE if no run
 * recorded events. */
psweep_status psweep_sweep_kernel_ms(psweep_ctx *ctx, double *ms, int32_t *n_launches);

/* Durations in milliseconds of each sweep kernel launch of the last run, in
 * launch order (one per (frame, level) with the grid launch, one for the
 * persistent launch); at most `capacity` values, *n receives the count. */
psweep_status psweep_sweep_kernel_times(psweep_ctx *ctx, double *ms, int32_t capacity, int32_t *n);

/* Plane-pixel evaluations (pixels x planes, all levels, all frames) of one
 * psweep_run with these frames, for throughput accounting. */
psweep_status psweep_plane_pixels(const psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                                  int64_t *count);

/* The (pixel, plane) pairs of the same run that take part in the method:
 * pixels whose whole window lies inside their level's reference image and
 * whose Eq. (1) ray meets the plane in front of the camera (z > 0 for a
 * fronto plane, n . r > 0 for a ground plane; computed in FP64 on the host,
 * O(pixels) per call).  Pairs left out have no cost at all: the ray never
 * reaches the plane, or the pixel has no window.  For throughput accounting
 * against the algorithmic work. */
psweep_status psweep_plane_pixels_met(const psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                                      int64_t *count);

/* Wait for the context's work, free its host state and events. */
void psweep_destroy(psweep_ctx *ctx);

/* Message of the last error on this context (or of the last failed create
 * when ctx is NULL); never NULL. */
const char *psweep_last_error(const psweep_ctx *ctx);

/* Library version string. */
const char *psweep_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSWEEP_H */
