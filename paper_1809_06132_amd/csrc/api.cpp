// Host side of the psweep C ABI (include/psweep.h): argument checks, the
// workspace layout, FP64 level cameras, the per-run job tables and the launch
// sequence
//   table upload -> FP64 plane setup -> level images and border marks ->
//   sweep (one grid per level, or one persistent launch) -> level merge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/psweep.h"
#include "psweep_internal.h"

using namespace psw;

extern "C" const void *psw_setup_kernel();
extern "C" const void *psw_prep_kernel();
extern "C" const void *psw_reset_kernel();
extern "C" const void *psw_merge_kernel();
extern "C" const void *psw_chunk_merge_kernel();
extern "C" const void *psw_filter_kernel();
extern "C" const void *psw_mask_kernel();
extern "C" const void *psw_backward_kernel(int win, int n_src, int img, int image_grads, int ground);
extern "C" size_t psw_backward_lds(int win, int n_src, int image_grads);
extern "C" int psw_backward_tile_rows();
extern "C" int psw_backward_threads(int image_grads);
extern "C" const void *psw_zero_kernel();
extern "C" const void *psw_pose_reduce_kernel();
extern "C" hipError_t psw_static_scratch(void **ptr, size_t *bytes);

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

thread_local std::string g_create_error;

struct CamSet {
    bool defined = false;
    psweep_camera ref{};
    int n_src = 0;
    psweep_camera src[PSWEEP_MAX_SOURCES]{};
    psweep_pose pose[PSWEEP_MAX_SOURCES]{};
    bool crop_set = false;
    int crop[4] = {0, 0, 0, 0};
};

struct LevelCam {
    double xi, fx, fy, cx, cy;
    int w, h;
};

// intrinsics of a level: 2x2 downsampling puts a level pixel's centre at the
// centre of its 2x2 block (2 i + 0.5); a crop shifts the principal point
LevelCam level_cam(const psweep_camera &c, int ds, int cx0, int cy0, int cw, int ch) {
    LevelCam o{c.xi, c.fx, c.fy, c.cx, c.cy, c.width, c.height};
    if (ds == 2) {
        o.fx = c.fx / 2.0; o.fy = c.fy / 2.0;
        o.cx = (c.cx - 0.5) / 2.0; o.cy = (c.cy - 0.5) / 2.0;
        o.w = c.width / 2; o.h = c.height / 2;
    }
    if (cw > 0) {
        o.cx -= cx0; o.cy -= cy0;
        o.w = cw; o.h = ch;
    }
    return o;
}

// every kernel instance of the library, gathered once (thread-safe static
// initialisation)
const std::vector<KernelEntry> &all_kernels() {
    static const std::vector<KernelEntry> all = [] {
        std::vector<KernelEntry> v;
        int (*const tables[])(const KernelEntry **) = {psw_kernels_grid, psw_kernels_extra, psw_kernels_small,
                                                      psw_kernels_grid8, psw_kernels_f32img, psw_kernels_persistent};
        for (auto tab : tables) {
            const KernelEntry *t;
            const int n = tab(&t);
            v.insert(v.end(), t, t + n);
        }
        return v;
    }();
    return all;
}

const KernelEntry *find_kernel(int win, int rows, int waves, int n_src, int store, int soft, int persistent,
                               int img) {
    for (const KernelEntry &e : all_kernels()) {
        if (e.persistent == persistent && e.rows == rows && e.waves == waves && e.n_src == n_src &&
            e.store == store && e.soft == soft && e.img == img && (persistent || e.win == win))
            return &e;
    }
    return nullptr;
}

}  // namespace

namespace {
// Where a run's scratch lives inside its device memory (the bound workspace,
// or the library's static scratch array): two job-table regions (direct
// runs, graph), two counter regions, then one slot per frame with the level
// images, textures, level maps, plane tables and plane-chunk partial states.
struct Layout {
    size_t table_bytes = 0, off_table[2] = {0, 0}, off_counter[2] = {0, 0}, off_slots = 0, slot_bytes = 0;
    size_t s_ref[PSWEEP_MAX_LEVELS] = {0, 0}, s_tex[PSWEEP_MAX_LEVELS] = {0, 0}, s_maps[PSWEEP_MAX_LEVELS] = {0, 0},
           s_htab[PSWEEP_MAX_LEVELS] = {0, 0}, s_theta[PSWEEP_MAX_LEVELS] = {0, 0}, s_part[PSWEEP_MAX_LEVELS] = {0, 0};
    size_t need = 0;
    bool parts = true;   // room for plane-chunk partial states
};
}  // namespace

struct psweep_ctx {
    psweep_config cfg{};
    std::vector<CamSet> sets;
    int P[PSWEEP_MAX_LEVELS] = {0, 0};
    // level size bounds for the workspace
    int ref_w[PSWEEP_MAX_LEVELS] = {0, 0}, ref_h[PSWEEP_MAX_LEVELS] = {0, 0};
    int src_w[PSWEEP_MAX_LEVELS] = {0, 0}, src_h[PSWEEP_MAX_LEVELS] = {0, 0};
    // workspace (bound by the caller) and the memory the current call uses:
    // the workspace with `full`, or the static scratch with `lean`
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Layout full, lean;
    const Layout *lay = &full;
    char *base = nullptr;
    const char *last_base = nullptr;   // memory the device tables were uploaded to
    // pinned staging of the job tables (double buffered)
    char *staging[2] = {nullptr, nullptr};
    hipEvent_t staging_ev[2] = {nullptr, nullptr};
    bool staging_pending[2] = {false, false};
    int staging_idx = 0;
    std::vector<char> last_table;
    uint64_t cam_version = 1, setup_version = 0;
    // item orders by level geometry and launch shape (see item_order)
    std::map<std::vector<double>, std::vector<int32_t>> order_cache;
    int tile_rows[PSWEEP_MAX_LEVELS] = {4, 4}, tile_waves[PSWEEP_MAX_LEVELS] = {4, 4};
    int chunks[PSWEEP_MAX_LEVELS] = {0, 0};   // plane chunks per tile; 0 = automatic
    int n_cu = 256;
    // timing of sweep launches
    bool timing = false;
    std::vector<hipEvent_t> ev0, ev1;
    int n_timed = 0;
    // soft-mode state for the backward pass
    bool soft_ready = false;
    psweep_frame soft_frame{};
    float *soft_rho = nullptr, *soft_lse = nullptr;
    int64_t soft_pitch = 0;
    size_t soft_job_off = 0;   // device address of the job used by the backward
    char *soft_part = nullptr;   // that job's plane-chunk region, free once its run is merged
    // graph (captured on a stream of the context's own: the default stream
    // cannot be captured)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t capture_stream = nullptr;
    // grid launches of consecutive jobs alternate between the caller's stream
    // and this one (default priority), forked and joined with events
    hipStream_t side_stream = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    std::string err;
};

namespace {

psweep_status fail(psweep_ctx *c, psweep_status st, const std::string &msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return st;
}

psweep_status hip_fail(psweep_ctx *c, hipError_t e, const char *what) {
    return fail(c, PSWEEP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define PSW_HIP(call, what)                               \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

// bytes of one source texel: 4 x FP16 bilinear coefficients (u8 images), or
// the 2x2 cell as 4 x float
size_t texel_bytes(const psweep_config &c) { return c.image_format == PSWEEP_IMAGE_F32 ? 16 : 8; }

bool single_full(const psweep_config &c) {
    return c.n_levels == 1 && c.level[0].downsample == 1 && c.level[0].crop_w == 0;
}

psweep_status check_config(const psweep_config *c) {
    auto bad = [](const std::string &m) { return fail(nullptr, PSWEEP_EINVAL, m); };
    if (c->n_levels < 1 || c->n_levels > PSWEEP_MAX_LEVELS) return bad("n_levels must be 1 or 2");
    if (c->max_width < 8 || c->max_height < 8 || c->max_width > 8192 || c->max_height > 8192)
        return bad("max_width/max_height out of [8, 8192]");
    if (c->max_sources < 1 || c->max_sources > PSWEEP_MAX_SOURCES) return bad("max_sources out of [1, 4]");
    if (c->max_frames < 1 || c->max_frames * c->n_levels > kMaxJobs) return bad("max_frames out of range");
    if (c->max_camera_sets < 1 || c->max_camera_sets > 4096) return bad("max_camera_sets out of range");
    if (c->best_k < 1 || c->best_k > c->max_sources) return bad("best_k out of [1, max_sources]");
    if (!(c->var_floor >= 0.0)) return bad("var_floor must be >= 0");
    if (c->storage < 0 || c->storage > 2) return bad("storage must be F32, F16 or BF16");
    if (c->mode != PSWEEP_MODE_WTA && c->mode != PSWEEP_MODE_SOFT) return bad("mode must be WTA or SOFT");
    if (c->launch != PSWEEP_LAUNCH_GRID && c->launch != PSWEEP_LAUNCH_PERSISTENT) return bad("bad launch kind");
    if (c->image_format != PSWEEP_IMAGE_U8 && c->image_format != PSWEEP_IMAGE_F32) return bad("bad image_format");
    const double gn = std::sqrt(c->ground_n[0] * c->ground_n[0] + c->ground_n[1] * c->ground_n[1] +
                                c->ground_n[2] * c->ground_n[2]);
    for (int l = 0; l < c->n_levels; ++l) {
        const psweep_level &L = c->level[l];
        if (L.window < 3 || L.window > 15 || (L.window & 1) == 0) return bad("window must be odd in [3, 15]");
        if (L.downsample != 1 && L.downsample != 2) return bad("downsample must be 1 or 2");
        if (L.n_fronto < 0 || L.n_ground < 0 || L.n_fronto + L.n_ground < 1 ||
            L.n_fronto + L.n_ground > PSWEEP_MAX_PLANES)
            return bad("plane counts out of range");
        if (L.n_fronto == 1 || L.n_ground == 1) return bad("a used plane family needs >= 2 planes");
        if (L.n_fronto > 0 && !(L.near_m > 0.0 && L.far_m > L.near_m)) return bad("need 0 < near_m < far_m");
        if (L.n_ground > 0) {
            if (!(L.h_hi > L.h_lo)) return bad("need h_lo < h_hi");
            if (!(std::fabs(gn - 1.0) < 1e-6)) return bad("ground_n must be a unit vector");
            if (!(c->ground_d - L.h_hi > 0.0)) return bad("ground planes must stay below the camera (ground_d > h_hi)");
        }
        if (L.crop_w < 0 || L.crop_h < 0 || (L.crop_w > 0) != (L.crop_h > 0) ||
            (L.crop_w > 0 && (L.crop_x < 0 || L.crop_y < 0)))
            return bad("bad crop rectangle");
    }
    if (c->n_levels == 2) {
        if (c->level[0].crop_w != 0) return fail(nullptr, PSWEEP_EUNSUPPORTED, "level 0 must not be cropped");
        if (c->level[1].downsample != 1) return fail(nullptr, PSWEEP_EUNSUPPORTED, "the crop level must be full resolution");
        if (c->level[1].n_fronto < 1) return bad("the crop level needs fronto planes");
    } else if (c->level[0].crop_w != 0) {
        return fail(nullptr, PSWEEP_EUNSUPPORTED, "a single level cannot be cropped");
    }
    if (c->mode == PSWEEP_MODE_SOFT) {
        if (!single_full(*c)) return fail(nullptr, PSWEEP_EUNSUPPORTED, "soft mode needs one full-resolution level");
        if (c->launch != PSWEEP_LAUNCH_GRID) return fail(nullptr, PSWEEP_EUNSUPPORTED, "soft mode uses the grid launch");
        if (c->storage != PSWEEP_STORAGE_F32) return fail(nullptr, PSWEEP_EUNSUPPORTED, "soft mode stages in FP32");
        if (!(c->temperature > 0.0)) return bad("temperature must be > 0");
    }
    if (c->image_format == PSWEEP_IMAGE_F32) {
        if (!single_full(*c))
            return fail(nullptr, PSWEEP_EUNSUPPORTED, "float images need one full-resolution level");
        if (c->launch != PSWEEP_LAUNCH_GRID) return fail(nullptr, PSWEEP_EUNSUPPORTED, "float images use the grid launch");
        if (c->storage != PSWEEP_STORAGE_F32) return fail(nullptr, PSWEEP_EUNSUPPORTED, "float images stage in FP32");
    }
    if (c->launch == PSWEEP_LAUNCH_PERSISTENT) {
        for (int l = 0; l < c->n_levels; ++l)
            if (c->level[l].window != 7 && c->level[l].window != 9)
                return fail(nullptr, PSWEEP_EUNSUPPORTED, "the persistent launch supports windows 7 and 9");
    }
    return PSWEEP_OK;
}

struct Blob {
    std::vector<char> bytes;
    size_t jobs = 0, setups = 0, preps = 0, borders = 0, merges = 0, orders = 0;
    int nj = 0, nm = 0;
};

// Largest number of (chunk, tile) items of one job on level l of a config:
// the level's largest image, the smallest tile (4 output rows, 64 - 2 h
// columns) and the most chunks.
size_t max_items(const psweep_config &c, int l, int w, int h) {
    const int hw = c.level[l].window / 2;
    const int txo = kWave - 2 * hw;
    const size_t tx = (size_t)std::max(0, (w - 2 * hw + txo - 1) / txo);
    const size_t ty = (size_t)std::max(0, (h - 2 * hw + 3) / 4);
    return tx * ty * kMaxChunks;
}

Layout make_layout(const psweep_config &cfg, const int *P, const int *ref_w, const int *ref_h, const int *src_w,
                   const int *src_h, bool parts) {
    Layout L;
    L.parts = parts;
    // table region: every kind of record for kMaxJobs jobs, and the item queues
    size_t order_bytes = 0;
    for (int l = 0; l < cfg.n_levels; ++l)
        order_bytes += align_up(sizeof(int32_t) * (kQueueHead + max_items(cfg, l, ref_w[l], ref_h[l]))) *
                       (size_t)cfg.max_frames;
    L.table_bytes = align_up(sizeof(JobDev) * kMaxJobs) + align_up(sizeof(SetupDev) * kMaxJobs) +
                    align_up(sizeof(PrepDev) * kMaxJobs) + align_up(sizeof(BorderDev) * kMaxJobs) +
                    align_up(sizeof(MergeDev) * kMaxJobs) + order_bytes;
    size_t off = 0;
    for (int g = 0; g < 2; ++g) { L.off_table[g] = off; off += L.table_bytes; }
    for (int g = 0; g < 2; ++g) { L.off_counter[g] = off; off += align_up(sizeof(int) * (kQueueHead + kQueues * kMaxJobs)); }
    L.off_slots = off;
    size_t so = 0;
    const int S = cfg.max_sources;
    for (int l = 0; l < cfg.n_levels; ++l) {
        const size_t rpx = (size_t)ref_w[l] * ref_h[l];
        const size_t spx = (size_t)src_w[l] * src_h[l];
        L.s_ref[l] = so;   so += align_up(rpx);
        L.s_tex[l] = so;   so += align_up(spx * texel_bytes(cfg)) * S;
        L.s_maps[l] = so;  so += align_up(rpx * 4) * 4;
        L.s_htab[l] = so;  so += align_up((size_t)P[l] * S * 9 * 4);
        L.s_theta[l] = so; so += align_up((size_t)P[l] * 4);
        L.s_part[l] = so;  so += parts ? align_up(rpx * 4 * kPartWords * kMaxChunks) : 0;
    }
    L.slot_bytes = align_up(so);
    L.need = L.off_slots + L.slot_bytes * cfg.max_frames;
    return L;
}

}  // namespace

extern "C" {

const char *psweep_version(void) { return "psweep-gfx950 1.0"; }

const char *psweep_last_error(const psweep_ctx *ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

psweep_status psweep_create(const psweep_config *cfg, psweep_ctx **out) {
    if (!cfg || !out) return fail(nullptr, PSWEEP_EINVAL, "NULL argument");
    *out = nullptr;
    psweep_status st = check_config(cfg);
    if (st != PSWEEP_OK) return st;
    psweep_ctx *ctx = new (std::nothrow) psweep_ctx();
    if (!ctx) return fail(nullptr, PSWEEP_ENOMEM, "host allocation failed");
    ctx->cfg = *cfg;
    ctx->sets.resize(cfg->max_camera_sets);
    const int W = cfg->max_width, H = cfg->max_height;
    for (int l = 0; l < cfg->n_levels; ++l) {
        const psweep_level &L = cfg->level[l];
        ctx->P[l] = L.n_fronto + L.n_ground;
        ctx->src_w[l] = W / L.downsample;
        ctx->src_h[l] = H / L.downsample;
        ctx->ref_w[l] = ctx->src_w[l];
        ctx->ref_h[l] = ctx->src_h[l];
    }
    ctx->full = make_layout(*cfg, ctx->P, ctx->ref_w, ctx->ref_h, ctx->src_w, ctx->src_h, true);
    ctx->lean = make_layout(*cfg, ctx->P, ctx->ref_w, ctx->ref_h, ctx->src_w, ctx->src_h, false);
    for (int b = 0; b < 2; ++b) {
        if (hipHostMalloc((void **)&ctx->staging[b], ctx->full.table_bytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->staging_ev[b], hipEventDisableTiming) != hipSuccess) {
            psweep_destroy(ctx);
            return fail(nullptr, PSWEEP_EHIP, "pinned staging allocation failed");
        }
    }
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            ctx->n_cu = prop.multiProcessorCount;
    }
    if (hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming) != hipSuccess) {
        psweep_destroy(ctx);
        return fail(nullptr, PSWEEP_EHIP, "stream or event creation failed");
    }
    // kernels with more than 64 KB of dynamic LDS need the limit raised
    for (const KernelEntry &e : all_kernels())
        if (e.lds > 65536) (void)hipFuncSetAttribute(e.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)e.lds);
    *out = ctx;
    return PSWEEP_OK;
}

psweep_status psweep_workspace_size(const psweep_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return PSWEEP_EINVAL;
    *bytes = ctx->full.need;
    return PSWEEP_OK;
}

psweep_status psweep_set_workspace(psweep_ctx *ctx, void *dev_ptr, size_t bytes) {
    if (!ctx) return PSWEEP_EINVAL;
    if (!dev_ptr) return fail(ctx, PSWEEP_EINVAL, "NULL workspace");
    if (((uintptr_t)dev_ptr) % kAlign) return fail(ctx, PSWEEP_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < ctx->full.need) return fail(ctx, PSWEEP_ENOMEM, "workspace smaller than psweep_workspace_size");
    ctx->ws = (char *)dev_ptr;
    ctx->ws_bytes = bytes;
    ctx->last_table.clear();
    ctx->setup_version = 0;
    return PSWEEP_OK;
}

psweep_status psweep_set_cameras(psweep_ctx *ctx, int32_t camera_set, const psweep_camera *ref, int32_t n_src,
                                 const psweep_camera *src, const psweep_pose *ref_to_src) {
    if (!ctx) return PSWEEP_EINVAL;
    if (camera_set < 0 || camera_set >= (int)ctx->sets.size()) return fail(ctx, PSWEEP_EINVAL, "camera_set out of range");
    if (!ref || !src || !ref_to_src) return fail(ctx, PSWEEP_EINVAL, "NULL camera or pose");
    if (n_src < 1 || n_src > ctx->cfg.max_sources) return fail(ctx, PSWEEP_EINVAL, "n_src out of [1, max_sources]");
    if (ctx->cfg.best_k > n_src) return fail(ctx, PSWEEP_EINVAL, "best_k exceeds n_src");
    auto cam_ok = [&](const psweep_camera &c) {
        return c.xi >= 0.0 && c.xi <= 1.0 && c.fx > 0.0 && c.fy > 0.0 && c.width >= 8 && c.height >= 8 &&
               c.width <= ctx->cfg.max_width && c.height <= ctx->cfg.max_height && std::isfinite(c.cx) &&
               std::isfinite(c.cy);
    };
    if (!cam_ok(*ref)) return fail(ctx, PSWEEP_EINVAL, "bad reference camera (xi in [0,1], f > 0, size <= max)");
    for (int s = 0; s < n_src; ++s) {
        if (!cam_ok(src[s])) return fail(ctx, PSWEEP_EINVAL, "bad source camera");
        const double *t = ref_to_src[s].t;
        if (!(std::isfinite(t[0]) && std::isfinite(t[1]) && std::isfinite(t[2])))
            return fail(ctx, PSWEEP_EINVAL, "pose translation not finite");
        const double *R = ref_to_src[s].R;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double d = 0;
                for (int k = 0; k < 3; ++k) d += R[3 * a + k] * R[3 * b + k];
                if (!(std::fabs(d - (a == b ? 1.0 : 0.0)) <= 1e-6)) return fail(ctx, PSWEEP_EINVAL, "R not orthonormal");
            }
    }
    CamSet &cs = ctx->sets[camera_set];
    cs.defined = true;
    cs.ref = *ref;
    cs.n_src = n_src;
    for (int s = 0; s < n_src; ++s) { cs.src[s] = src[s]; cs.pose[s] = ref_to_src[s]; }
    ctx->cam_version++;
    return PSWEEP_OK;
}

psweep_status psweep_set_crop(psweep_ctx *ctx, int32_t camera_set, int32_t x, int32_t y, int32_t w, int32_t h) {
    if (!ctx) return PSWEEP_EINVAL;
    if (camera_set < 0 || camera_set >= (int)ctx->sets.size()) return fail(ctx, PSWEEP_EINVAL, "camera_set out of range");
    if (ctx->cfg.n_levels != 2) return fail(ctx, PSWEEP_ESTATE, "only a two-level config has a crop level");
    if (x < 0 || y < 0 || w < 8 || h < 8) return fail(ctx, PSWEEP_EINVAL, "bad crop rectangle");
    CamSet &cs = ctx->sets[camera_set];
    cs.crop_set = true;
    cs.crop[0] = x; cs.crop[1] = y; cs.crop[2] = w; cs.crop[3] = h;
    return PSWEEP_OK;
}

psweep_status psweep_set_tile(psweep_ctx *ctx, int32_t level, int32_t rows_per_wave, int32_t waves) {
    if (!ctx) return PSWEEP_EINVAL;
    if (level < 0 || level >= ctx->cfg.n_levels) return fail(ctx, PSWEEP_EINVAL, "level out of range");
    if (rows_per_wave == 0 && waves == 0) { rows_per_wave = 4; waves = 4; }
    const bool rows_ok = rows_per_wave == 2 || rows_per_wave == 4 || rows_per_wave == 8 || rows_per_wave == 16;
    if (!rows_ok || (waves != 2 && waves != 4 && waves != 8))
        return fail(ctx, PSWEEP_EINVAL, "rows_per_wave must be 2, 4, 8 or 16 and waves 2, 4 or 8");
    ctx->tile_rows[level] = rows_per_wave;
    ctx->tile_waves[level] = waves;
    return PSWEEP_OK;
}

psweep_status psweep_set_chunks(psweep_ctx *ctx, int32_t level, int32_t n_chunks) {
    if (!ctx) return PSWEEP_EINVAL;
    if (level < 0 || level >= ctx->cfg.n_levels) return fail(ctx, PSWEEP_EINVAL, "level out of range");
    if (n_chunks < 0 || n_chunks > kMaxChunks) return fail(ctx, PSWEEP_EINVAL, "n_chunks out of [0, 8]");
    ctx->chunks[level] = n_chunks;
    return PSWEEP_OK;
}

psweep_status psweep_set_timing(psweep_ctx *ctx, int32_t on) {
    if (!ctx) return PSWEEP_EINVAL;
    ctx->timing = on != 0;
    return PSWEEP_OK;
}

psweep_status psweep_plane_pixels(const psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames, int64_t *count) {
    if (!ctx || !frames || !count || n_frames < 1) return PSWEEP_EINVAL;
    int64_t n = 0;
    for (int f = 0; f < n_frames; ++f) {
        const int cs = frames[f].camera_set;
        if (cs < 0 || cs >= (int)ctx->sets.size() || !ctx->sets[cs].defined) return PSWEEP_ESTATE;
        const CamSet &C = ctx->sets[cs];
        for (int l = 0; l < ctx->cfg.n_levels; ++l) {
            const psweep_level &L = ctx->cfg.level[l];
            int cw = L.crop_w, ch = L.crop_h;
            if (l == 1 && C.crop_set) { cw = C.crop[2]; ch = C.crop[3]; }
            const LevelCam lc = level_cam(C.ref, L.downsample, 0, 0, cw, ch);
            n += (int64_t)lc.w * lc.h * (L.n_fronto + L.n_ground);
        }
    }
    *count = n;
    return PSWEEP_OK;
}

psweep_status psweep_perturb_pose(const double *R, const double *t, const double *xi, double *R_out,
                                  double *t_out) {
    if (!R || !t || !xi || !R_out || !t_out) return PSWEEP_EINVAL;
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(xi[i])) return PSWEEP_EINVAL;
    // Exp(omega) = I + a K + b K^2, K = [omega]x, a = sin(th) / th,
    // b = (1 - cos(th)) / th^2 (their series below 1e-4, exact to FP64 there)
    const double w0 = xi[3], w1 = xi[4], w2 = xi[5];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = std::sqrt(th2);
    double a, b;
    if (th < 1e-4) {
        a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    } else {
        a = std::sin(th) / th;
        b = (1.0 - std::cos(th)) / th2;
    }
    const double K[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    double E[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double kk = 0.0;
            for (int m = 0; m < 3; ++m) kk += K[i * 3 + m] * K[m * 3 + j];
            E[i * 3 + j] = (i == j ? 1.0 : 0.0) + a * K[i * 3 + j] + b * kk;
        }
    double Rn[9], tn[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            Rn[i * 3 + j] = E[i * 3 + 0] * R[0 * 3 + j] + E[i * 3 + 1] * R[1 * 3 + j] + E[i * 3 + 2] * R[2 * 3 + j];
        tn[i] = E[i * 3 + 0] * t[0] + E[i * 3 + 1] * t[1] + E[i * 3 + 2] * t[2] + xi[i];
    }
    for (int i = 0; i < 9; ++i) R_out[i] = Rn[i];
    for (int i = 0; i < 3; ++i) t_out[i] = tn[i];
    return PSWEEP_OK;
}

psweep_status psweep_plane_pixels_met(const psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                                      int64_t *count) {
    if (!ctx || !frames || !count || n_frames < 1) return PSWEEP_EINVAL;
    const psweep_config &cfg = ctx->cfg;
    int64_t n = 0;
    for (int f = 0; f < n_frames; ++f) {
        const int cs = frames[f].camera_set;
        if (cs < 0 || cs >= (int)ctx->sets.size() || !ctx->sets[cs].defined) return PSWEEP_ESTATE;
        const CamSet &C = ctx->sets[cs];
        for (int l = 0; l < cfg.n_levels; ++l) {
            const psweep_level &L = cfg.level[l];
            int cx0 = L.crop_x, cy0 = L.crop_y, cw = L.crop_w, ch = L.crop_h;
            if (l == 1 && C.crop_set) { cx0 = C.crop[0]; cy0 = C.crop[1]; cw = C.crop[2]; ch = C.crop[3]; }
            const LevelCam lc = level_cam(C.ref, L.downsample, cx0, cy0, cw, ch);
            const int hw = L.window / 2;
            // Eq. (1): the unit ray is eta (x, y, 1 - xi / eta), so its z is
            // eta - xi; a fronto plane (z = 1 / rho > 0) is met when that is
            // positive, a ground plane (n . X = ground_d - h > 0) when n . r is
            int64_t met_f = 0, met_g = 0;
            for (int j = hw; j < lc.h - hw; ++j) {
                const double y = (j - lc.cy) / lc.fy;
                for (int i = hw; i < lc.w - hw; ++i) {
                    const double x = (i - lc.cx) / lc.fx;
                    const double q = x * x + y * y;
                    const double eta = (lc.xi + std::sqrt(1.0 + (1.0 - lc.xi * lc.xi) * q)) / (q + 1.0);
                    const double rz = eta - lc.xi;
                    met_f += rz > 0.0;
                    met_g += cfg.ground_n[0] * eta * x + cfg.ground_n[1] * eta * y + cfg.ground_n[2] * rz > 0.0;
                }
            }
            n += met_f * L.n_fronto + met_g * L.n_ground;
        }
    }
    *count = n;
    return PSWEEP_OK;
}

}  // extern "C"

namespace {

// The item queues of one job (see JobDev::order): tile row y goes to queue
// y mod 8, one queue per XCD, so that an XCD's L2 holds the source texels of
// its rows; each queue is sorted largest item first, the size of an item
// being its (pixel, plane) pairs that meet their plane (the pixels of its
// tile whose Eq. (1) ray meets the chunk's family, times the chunk's planes;
// FP64 on the host).  Long items then start first and short ones fill the
// end of the launch, instead of a long one starting last; ties keep the
// chunk-major order.  Depends only on the level's geometry and the launch
// shape: cached.
const std::vector<int32_t> &item_order(psweep_ctx *ctx, const LevelCam &rc, const psweep_level &L,
                                       const JobDev &J) {
    const psweep_config &cfg = ctx->cfg;
    const std::vector<double> key = {rc.xi, rc.fx, rc.fy, rc.cx, rc.cy, (double)rc.w, (double)rc.h,
                                     (double)L.window, (double)L.n_fronto, (double)L.n_ground,
                                     cfg.ground_n[0], cfg.ground_n[1], cfg.ground_n[2], (double)J.rows,
                                     (double)J.waves, (double)J.nch_f, (double)J.nch_g};
    auto it = ctx->order_cache.find(key);
    if (it != ctx->order_cache.end()) return it->second;
    const int hw = L.window / 2, txo = kWave - 2 * hw, tyo = J.rows * J.waves;
    const int ntile = J.tiles_x * J.tiles_y;
    std::vector<int64_t> met_f(ntile, 0), met_g(ntile, 0);
    for (int j = hw; j < rc.h - hw; ++j) {
        const double y = (j - rc.cy) / rc.fy;
        const int trow = ((j - hw) / tyo) * J.tiles_x;
        for (int i = hw; i < rc.w - hw; ++i) {
            const double x = (i - rc.cx) / rc.fx;
            const double q = x * x + y * y;
            const double eta = (rc.xi + std::sqrt(1.0 + (1.0 - rc.xi * rc.xi) * q)) / (q + 1.0);
            const double rz = eta - rc.xi;
            const int t = trow + (i - hw) / txo;
            met_f[t] += rz > 0.0;
            met_g[t] += cfg.ground_n[0] * eta * x + cfg.ground_n[1] * eta * y + cfg.ground_n[2] * rz > 0.0;
        }
    }
    const int nch = std::max(1, J.nch_f + J.nch_g);
    std::vector<int64_t> weight((size_t)nch * ntile);
    for (int c = 0; c < nch; ++c) {
        int kb = 0, ke = L.n_fronto + L.n_ground;
        if (nch > 1) chunk_range(L.n_fronto, L.n_ground, J.nch_f, J.nch_g, c, &kb, &ke);
        const int64_t pf = std::max(0, std::min(ke, L.n_fronto) - kb);
        const int64_t pg = std::max(0, ke - std::max(kb, L.n_fronto));
        for (int t = 0; t < ntile; ++t) weight[(size_t)c * ntile + t] = met_f[t] * pf + met_g[t] * pg;
    }
    // Grid launch: each queue largest item first, which shortens the launch's
    // tail.  Persistent launch: each queue row by row, every chunk of a tile
    // row before the next row, so that the workgroups resident on an XCD work
    // on neighbouring source footprints that its L2 holds (measured faster on
    // one-level, two-level and batched workloads alike).
    const bool by_row = cfg.launch == PSWEEP_LAUNCH_PERSISTENT;
    std::vector<int32_t> order(kQueueHead, 0);
    for (int q = 0; q < kQueues; ++q) {
        order[q] = (int32_t)(order.size() - kQueueHead);
        const size_t lo = order.size();
        if (by_row) {
            for (int y = q; y < J.tiles_y; y += kQueues)
                for (int c = 0; c < nch; ++c)
                    for (int x = 0; x < J.tiles_x; ++x) order.push_back(c * ntile + y * J.tiles_x + x);
        } else {
            for (int c = 0; c < nch; ++c)
                for (int y = q; y < J.tiles_y; y += kQueues)
                    for (int x = 0; x < J.tiles_x; ++x) order.push_back(c * ntile + y * J.tiles_x + x);
            std::stable_sort(order.begin() + lo, order.end(),
                             [&](int32_t a, int32_t b) { return weight[a] > weight[b]; });
        }
    }
    order[kQueues] = (int32_t)(order.size() - kQueueHead);
    return ctx->order_cache.emplace(key, std::move(order)).first->second;
}

// Build the per-run tables (host side) for `frames`: job, setup, prep,
// border and merge records and the jobs' item orders, packed at fixed
// offsets of one blob that is uploaded to device address `tb`.
psweep_status build_tables(psweep_ctx *ctx, const psweep_frame *frames, int nf, const psweep_output *out,
                           char *tb, int *counters, Blob &blob, std::vector<int> &job_frame) {
    const psweep_config &cfg = ctx->cfg;
    const int NL = cfg.n_levels;
    const bool sf = single_full(cfg);
    std::vector<JobDev> jobs;
    std::vector<SetupDev> setups;
    std::vector<PrepDev> preps;
    std::vector<BorderDev> borders;
    std::vector<MergeDev> merges;
    std::vector<const std::vector<int32_t> *> orders;   // map nodes: stable while the run is built
    if (ctx->order_cache.size() > 192) ctx->order_cache.clear();   // one run adds at most kMaxJobs
    int first_item = 0;
    for (int f = 0; f < nf; ++f) {
        const psweep_frame &fr = frames[f];
        const int csi = fr.camera_set;
        if (csi < 0 || csi >= (int)ctx->sets.size() || !ctx->sets[csi].defined)
            return fail(ctx, PSWEEP_ESTATE, "frame uses an undefined camera set");
        const CamSet &C = ctx->sets[csi];
        if (!fr.ref || fr.ref_pitch < C.ref.width) return fail(ctx, PSWEEP_EINVAL, "bad reference image or pitch");
        for (int s = 0; s < C.n_src; ++s)
            if (!fr.src[s] || fr.src_pitch[s] < C.src[s].width)
                return fail(ctx, PSWEEP_EINVAL, "bad source image or pitch");
        const Layout &Y = *ctx->lay;
        char *slot = ctx->base + Y.off_slots + (size_t)f * Y.slot_bytes;
        const psweep_output &O = out[f];
        int crop_x = 0, crop_y = 0, crop_w = 0, crop_h = 0;
        if (NL == 2) {
            crop_x = cfg.level[1].crop_x; crop_y = cfg.level[1].crop_y;
            crop_w = cfg.level[1].crop_w; crop_h = cfg.level[1].crop_h;
            if (C.crop_set) { crop_x = C.crop[0]; crop_y = C.crop[1]; crop_w = C.crop[2]; crop_h = C.crop[3]; }
            if (crop_w <= 0 || crop_h <= 0 || crop_x + crop_w > C.ref.width || crop_y + crop_h > C.ref.height)
                return fail(ctx, PSWEEP_EINVAL, "crop rectangle outside the reference image");
        }
        if (sf) {
            if (cfg.mode == PSWEEP_MODE_SOFT) {
                if (!O.soft_invdepth || !O.soft_lse) return fail(ctx, PSWEEP_EINVAL, "soft mode needs soft outputs");
                if (O.soft_pitch != 0 && O.soft_pitch < C.ref.width) return fail(ctx, PSWEEP_EINVAL, "soft pitch");
            } else if (O.merged.pitch != 0 && O.merged.pitch < C.ref.width) {
                return fail(ctx, PSWEEP_EINVAL, "output pitch below width");
            }
        } else if (O.merged.pitch != 0 && O.merged.pitch < C.ref.width) {
            return fail(ctx, PSWEEP_EINVAL, "output pitch below width");
        }
        int lvl_job[PSWEEP_MAX_LEVELS] = {-1, -1};
        for (int l = 0; l < NL; ++l) {
            const psweep_level &L = cfg.level[l];
            const int ds = L.downsample;
            const LevelCam rc = level_cam(C.ref, ds, l == 1 ? crop_x : 0, l == 1 ? crop_y : 0, l == 1 ? crop_w : 0,
                                          l == 1 ? crop_h : 0);
            const int P = L.n_fronto + L.n_ground;
            const int hw = L.window / 2;
            JobDev J;
            std::memset(&J, 0, sizeof J);
            if (ds == 2) {
                J.ref = (const uint8_t *)(slot + Y.s_ref[l]);
                J.ref_pitch = C.ref.width / 2;
            } else {
                J.ref = (const uint8_t *)fr.ref + (l == 1 ? (int64_t)crop_y * fr.ref_pitch + crop_x : 0);
                J.ref_pitch = fr.ref_pitch;
            }
            J.w = rc.w; J.h = rc.h;
            J.fx = (float)rc.fx; J.fy = (float)rc.fy; J.cx = (float)rc.cx; J.cy = (float)rc.cy; J.xi = (float)rc.xi;
            J.inv_fx = (float)(1.0 / rc.fx); J.inv_fy = (float)(1.0 / rc.fy);
            J.n_src = C.n_src; J.n_fronto = L.n_fronto; J.n_ground = L.n_ground; J.window = L.window;
            J.best_k = cfg.best_k; J.mode = cfg.mode;
            J.var_floor_n = (float)(cfg.var_floor * L.window * L.window);
            for (int a = 0; a < 3; ++a) J.gn[a] = (float)cfg.ground_n[a];
            J.gd = (float)cfg.ground_d;
            J.step_f = L.n_fronto > 1 ? (float)((1.0 / L.near_m - 1.0 / L.far_m) / (L.n_fronto - 1)) : 0.0f;
            J.step_g = L.n_ground > 1 ? (float)((L.h_hi - L.h_lo) / (L.n_ground - 1)) : 0.0f;
            J.temperature = (float)cfg.temperature;
            if (O.cost_volume[l]) {
                if (cfg.mode != PSWEEP_MODE_WTA || cfg.launch != PSWEEP_LAUNCH_GRID)
                    return fail(ctx, PSWEEP_EUNSUPPORTED, "cost volumes come from winner-take-all grid launches");
                J.volume = O.cost_volume[l];
            }
            J.htab = (const float *)(slot + Y.s_htab[l]);
            J.theta = (const float *)(slot + Y.s_theta[l]);
            // outputs
            if (sf) {
                if (cfg.mode == PSWEEP_MODE_SOFT) {
                    J.soft_rho = O.soft_invdepth; J.soft_lse = O.soft_lse;
                    J.soft_pitch = O.soft_pitch ? O.soft_pitch : C.ref.width;
                } else {
                    const psweep_maps &M = O.merged;
                    J.index = M.index; J.delta = M.delta; J.cost1 = M.cost1; J.cost2 = M.cost2;
                    J.depth = M.depth; J.z = M.z; J.level_id = M.level;
                    J.out_pitch = M.pitch ? M.pitch : C.ref.width;
                }
            } else {
                const psweep_maps &M = O.level[l];
                if (M.index || M.delta || M.cost1 || M.cost2) {
                    if (!(M.index && M.delta && M.cost1 && M.cost2))
                        return fail(ctx, PSWEEP_EINVAL, "level maps need index, delta, cost1 and cost2 together");
                    if (M.pitch != 0 && M.pitch < rc.w) return fail(ctx, PSWEEP_EINVAL, "level map pitch below width");
                    J.index = M.index; J.delta = M.delta; J.cost1 = M.cost1; J.cost2 = M.cost2;
                    J.out_pitch = M.pitch ? M.pitch : rc.w;
                } else {
                    const size_t plane = align_up((size_t)ctx->ref_w[l] * ctx->ref_h[l] * 4);
                    char *m = slot + Y.s_maps[l];
                    J.index = (int32_t *)m; J.delta = (float *)(m + plane);
                    J.cost1 = (float *)(m + 2 * plane); J.cost2 = (float *)(m + 3 * plane);
                    J.out_pitch = rc.w;
                }
                J.depth = M.depth; J.z = M.z;
            }
            const int TXO = kWave - 2 * hw;
            const int rows = ctx->tile_rows[l], waves = ctx->tile_waves[l];
            const int TYO = rows * waves;
            J.tiles_x = rc.w > 2 * hw ? (rc.w - 2 * hw + TXO - 1) / TXO : 0;
            J.tiles_y = rc.h > 2 * hw ? (rc.h - 2 * hw + TYO - 1) / TYO : 0;
            J.rows = rows; J.waves = waves;
            // plane chunks: enough workgroups for about 28 waves per SIMD
            // over the launch, so that uneven tiles still balance
            {
                const int ntile = J.tiles_x * J.tiles_y;
                int nch = ctx->lay->parts ? ctx->chunks[l] : 1;   // no partial-state room: one pass
                if (nch == 0) {
                    const long long target = 28LL * ctx->n_cu * 4;
                    const long long have = (long long)ntile * waves * (cfg.launch == PSWEEP_LAUNCH_PERSISTENT ? nf : 1);
                    nch = have > 0 ? (int)((target + have - 1) / have) : 1;
                    nch = std::max(1, std::min(nch, kMaxChunks));
                }
                if (cfg.mode == PSWEEP_MODE_SOFT && nch > 1) nch = std::min(nch, std::max(1, L.n_fronto / 2));
                J.nch_f = 0; J.nch_g = 0;
                if (nch > 1) {
                    const int cs = (P + nch - 1) / nch;
                    J.nch_f = L.n_fronto > 0 ? (L.n_fronto + cs - 1) / cs : 0;
                    J.nch_g = L.n_ground > 0 ? (L.n_ground + cs - 1) / cs : 0;
                    while (J.nch_f + J.nch_g > kMaxChunks) { if (J.nch_f >= J.nch_g) --J.nch_f; else --J.nch_g; }
                    if (J.nch_f + J.nch_g <= 1) { J.nch_f = 0; J.nch_g = 0; }
                }
                J.part = (float *)(slot + Y.s_part[l]);
                const int items = ntile * std::max(1, J.nch_f + J.nch_g);
                J.first_item = first_item;
                first_item += items;
                orders.push_back(&item_order(ctx, rc, L, J));
                J.queue_ctr = counters + kQueueHead + kQueues * (int)orders.size() - kQueues;
            }
            for (int s = 0; s < C.n_src; ++s) {
                const LevelCam sc = level_cam(C.src[s], ds, 0, 0, 0, 0);
                SrcDev &D = J.src[s];
                D.tex = (const uint32_t *)(slot + Y.s_tex[l] +
                                           align_up((size_t)ctx->src_w[l] * ctx->src_h[l] * texel_bytes(cfg)) * s);
                D.w = sc.w; D.h = sc.h;
                D.fx = (float)sc.fx; D.fy = (float)sc.fy; D.cx = (float)sc.cx; D.cy = (float)sc.cy; D.xi = (float)sc.xi;
                D.wm1 = (float)(sc.w - 1); D.hm1 = (float)(sc.h - 1);
            }
            // FP64 setup
            SetupDev Sd;
            std::memset(&Sd, 0, sizeof Sd);
            for (int s = 0; s < C.n_src; ++s) {
                std::memcpy(Sd.R[s], C.pose[s].R, sizeof(double) * 9);
                std::memcpy(Sd.t[s], C.pose[s].t, sizeof(double) * 3);
            }
            Sd.near_m = L.near_m; Sd.far_m = L.far_m; Sd.h_lo = L.h_lo; Sd.h_hi = L.h_hi;
            for (int a = 0; a < 3; ++a) Sd.gn[a] = cfg.ground_n[a];
            Sd.gd = cfg.ground_d;
            Sd.n_src = C.n_src; Sd.n_fronto = L.n_fronto; Sd.n_ground = L.n_ground;
            Sd.htab = (float *)(slot + Y.s_htab[l]);
            Sd.theta = (float *)(slot + Y.s_theta[l]);
            // level images
            PrepDev Pd;
            std::memset(&Pd, 0, sizeof Pd);
            Pd.ref_full = (const uint8_t *)fr.ref; Pd.ref_pitch = fr.ref_pitch;
            Pd.img = cfg.image_format;
            Pd.ref_w = C.ref.width; Pd.ref_h = C.ref.height;
            Pd.ref_level = ds == 2 ? (uint8_t *)(slot + Y.s_ref[l]) : nullptr;
            Pd.downsample = ds; Pd.n_src = C.n_src;
            for (int s = 0; s < C.n_src; ++s) {
                Pd.src_full[s] = fr.src[s]; Pd.src_pitch[s] = fr.src_pitch[s];
                Pd.src_w[s] = C.src[s].width; Pd.src_h[s] = C.src[s].height;
                Pd.tex[s] = (uint32_t *)J.src[s].tex;
            }
            // border marks
            BorderDev Bd;
            std::memset(&Bd, 0, sizeof Bd);
            Bd.w = rc.w; Bd.h = rc.h; Bd.hw = hw;
            Bd.index = J.index; Bd.delta = J.delta; Bd.cost1 = J.cost1; Bd.cost2 = J.cost2;
            Bd.depth = J.depth; Bd.z = J.z; Bd.level_id = J.level_id; Bd.out_pitch = J.out_pitch;
            Bd.soft_rho = J.soft_rho; Bd.soft_lse = J.soft_lse; Bd.soft_pitch = J.soft_pitch;
            lvl_job[l] = (int)jobs.size();
            jobs.push_back(J);
            setups.push_back(Sd);
            preps.push_back(Pd);
            borders.push_back(Bd);
            job_frame.push_back(f);
        }
        if (!sf) {
            const psweep_maps &M = O.merged;
            MergeDev Md;
            std::memset(&Md, 0, sizeof Md);
            Md.w = C.ref.width; Md.h = C.ref.height;
            Md.fx = (float)C.ref.fx; Md.fy = (float)C.ref.fy; Md.cx = (float)C.ref.cx; Md.cy = (float)C.ref.cy;
            Md.xi = (float)C.ref.xi;
            for (int a = 0; a < 3; ++a) Md.gn[a] = (float)cfg.ground_n[a];
            Md.gd = (float)cfg.ground_d;
            Md.n_levels = NL; Md.ds0 = cfg.level[0].downsample;
            const JobDev &J0 = jobs[lvl_job[0]];
            Md.low_w = J0.w; Md.low_h = J0.h;
            Md.low_index = J0.index; Md.low_delta = J0.delta; Md.low_c1 = J0.cost1; Md.low_c2 = J0.cost2;
            Md.low_pitch = J0.out_pitch; Md.low_theta = J0.theta; Md.low_nf = J0.n_fronto;
            Md.low_step_f = J0.step_f; Md.low_step_g = J0.step_g;
            if (NL == 2) {
                const JobDev &J1 = jobs[lvl_job[1]];
                Md.crop_x = crop_x; Md.crop_y = crop_y; Md.crop_w = crop_w; Md.crop_h = crop_h;
                Md.crop_index = J1.index; Md.crop_delta = J1.delta; Md.crop_c1 = J1.cost1; Md.crop_c2 = J1.cost2;
                Md.crop_pitch = J1.out_pitch; Md.crop_theta = J1.theta; Md.crop_nf = J1.n_fronto;
                Md.crop_step_f = J1.step_f; Md.crop_step_g = J1.step_g;
                Md.crop_near = (float)cfg.level[1].near_m;
            }
            Md.depth = M.depth; Md.z = M.z; Md.delta = M.delta; Md.cost1 = M.cost1; Md.cost2 = M.cost2;
            Md.index = M.index; Md.level = M.level;
            Md.out_pitch = M.pitch ? M.pitch : C.ref.width;
            merges.push_back(Md);
        }
    }
    // compact blob: records at fixed offsets of the table region
    const int nj = (int)jobs.size(), nm = (int)merges.size();
    blob.nj = nj; blob.nm = nm;
    blob.jobs = 0;
    blob.setups = align_up(sizeof(JobDev) * nj);
    blob.preps = blob.setups + align_up(sizeof(SetupDev) * nj);
    blob.borders = blob.preps + align_up(sizeof(PrepDev) * nj);
    blob.merges = blob.borders + align_up(sizeof(BorderDev) * nj);
    blob.orders = blob.merges + align_up(sizeof(MergeDev) * (nm > 0 ? nm : 1));
    size_t total = blob.orders;
    for (int j = 0; j < nj; ++j) {
        jobs[j].order = (const int32_t *)(tb + total);
        total += align_up(sizeof(int32_t) * orders[j]->size());
    }
    if (total > ctx->lay->table_bytes) return fail(ctx, PSWEEP_EINVAL, "too many frames for the table region");
    blob.bytes.assign(total, 0);
    for (int j = 0; j < nj; ++j)
        std::memcpy(blob.bytes.data() + ((const char *)jobs[j].order - tb), orders[j]->data(),
                    sizeof(int32_t) * orders[j]->size());
    std::memcpy(blob.bytes.data() + blob.jobs, jobs.data(), sizeof(JobDev) * nj);
    std::memcpy(blob.bytes.data() + blob.setups, setups.data(), sizeof(SetupDev) * nj);
    std::memcpy(blob.bytes.data() + blob.preps, preps.data(), sizeof(PrepDev) * nj);
    std::memcpy(blob.bytes.data() + blob.borders, borders.data(), sizeof(BorderDev) * nj);
    if (nm) std::memcpy(blob.bytes.data() + blob.merges, merges.data(), sizeof(MergeDev) * nm);
    return PSWEEP_OK;
}

// Enqueue the kernels of one run whose tables sit at device address `tb`.
psweep_status enqueue(psweep_ctx *ctx, const Blob &blob, char *tb, int which, hipStream_t stream, bool do_setup,
                      bool timed, const std::vector<JobDev> *host_jobs) {
    const psweep_config &cfg = ctx->cfg;
    const int nj = blob.nj;
    JobDev *dj = (JobDev *)(tb + blob.jobs);
    SetupDev *dsu = (SetupDev *)(tb + blob.setups);
    PrepDev *dp = (PrepDev *)(tb + blob.preps);
    BorderDev *db = (BorderDev *)(tb + blob.borders);
    MergeDev *dm = (MergeDev *)(tb + blob.merges);
    int maxPS = 1, maxS = 1;
    for (int j = 0; j < nj; ++j) {
        const JobDev &J = (*host_jobs)[j];
        maxPS = std::max(maxPS, (J.n_fronto + J.n_ground) * J.n_src);
        maxS = std::max(maxS, J.n_src);
    }
    if (do_setup) {
        void *a[] = {&dsu};
        PSW_HIP(hipLaunchKernel(psw_setup_kernel(), dim3((maxPS + 255) / 256, nj), dim3(256), a, 0, stream), "setup");
    }
    {
        // level images and the border marks of every job
        void *a[] = {&dp, &db};
        PSW_HIP(hipLaunchKernel(psw_prep_kernel(), dim3(256, 1 + maxS, nj), dim3(256), a, 0, stream), "prep");
    }
    const int store = cfg.storage, soft = cfg.mode == PSWEEP_MODE_SOFT ? 1 : 0;
    {
        // the item queues' take counters of every job start at zero (a kernel,
        // not a memset: the run may be captured into a graph)
        int *counter = (int *)(ctx->base + ctx->lay->off_counter[which]);
        int n = kQueueHead + kQueues * nj;
        void *a[] = {&counter, &n};
        PSW_HIP(hipLaunchKernel(psw_reset_kernel(), dim3(1), dim3(256), a, 0, stream), "reset");
    }
    if (timed) {
        const size_t need = cfg.launch == PSWEEP_LAUNCH_PERSISTENT ? 1 : (size_t)nj;
        while (ctx->ev0.size() < need) {
            hipEvent_t e0, e1;
            PSW_HIP(hipEventCreate(&e0), "event");
            PSW_HIP(hipEventCreate(&e1), "event");
            ctx->ev0.push_back(e0);
            ctx->ev1.push_back(e1);
        }
        ctx->n_timed = 0;
    }
    if (cfg.launch == PSWEEP_LAUNCH_GRID) {
        std::vector<const KernelEntry *> kern(nj, nullptr);
        int n_launch = 0;
        for (int j = 0; j < nj; ++j) {
            const JobDev &J = (*host_jobs)[j];
            if (J.tiles_x * J.tiles_y == 0) continue;
            kern[j] = find_kernel(J.window, J.rows, J.waves, J.n_src, store, soft, 0, cfg.image_format);
            if (!kern[j]) return fail(ctx, PSWEEP_EUNSUPPORTED, "no kernel for this window/tile/sources/storage");
            ++n_launch;
        }
        // Jobs share nothing they write (maps, partial states, queue
        // counters are per job), so consecutive ones go to the caller's
        // stream and the side stream in turn: a job's tail then overlaps the
        // next job's start.  Both streams join the caller's before the merges.
        const bool two = n_launch > 1 && ctx->side_stream;
        if (two) {
            PSW_HIP(hipEventRecord(ctx->fork_ev, stream), "fork event");
            PSW_HIP(hipStreamWaitEvent(ctx->side_stream, ctx->fork_ev, 0), "fork wait");
        }
        int turn = 0;
        for (int j = 0; j < nj; ++j) {
            const JobDev &J = (*host_jobs)[j];
            const KernelEntry *e = kern[j];
            if (!e) continue;
            const hipStream_t s = two && (turn++ & 1) ? ctx->side_stream : stream;
            JobDev *jp = dj + j;
            void *a[] = {&jp};
            // one block per (chunk, tile) item
            const int grid = J.tiles_x * J.tiles_y * std::max(1, J.nch_f + J.nch_g);
            if (timed) PSW_HIP(hipEventRecord(ctx->ev0[ctx->n_timed], s), "event record");
            PSW_HIP(hipLaunchKernel(e->fn, dim3(grid), dim3(kWave * J.waves), a, e->lds, s), "sweep");
            if (timed) PSW_HIP(hipEventRecord(ctx->ev1[ctx->n_timed++], s), "event record");
        }
        if (two) {
            PSW_HIP(hipEventRecord(ctx->join_ev, ctx->side_stream), "join event");
            PSW_HIP(hipStreamWaitEvent(stream, ctx->join_ev, 0), "join wait");
        }
    } else {
        int n_items = 0, n_src = (*host_jobs)[0].n_src;
        for (int j = 0; j < nj; ++j) {
            const JobDev &J = (*host_jobs)[j];
            n_items += J.tiles_x * J.tiles_y * std::max(1, J.nch_f + J.nch_g);
            if (J.n_src != n_src) return fail(ctx, PSWEEP_EUNSUPPORTED, "persistent launch needs one source count");
            if (J.rows != ctx->tile_rows[0] || J.waves != ctx->tile_waves[0])
                return fail(ctx, PSWEEP_EUNSUPPORTED, "persistent launch needs one tile shape");
        }
        const KernelEntry *e = find_kernel(0, ctx->tile_rows[0], ctx->tile_waves[0], n_src, store, 0, 1, 0);
        if (!e) return fail(ctx, PSWEEP_EUNSUPPORTED, "no persistent kernel for this tile/sources/storage");
        int *counter = (int *)(ctx->base + ctx->lay->off_counter[which]);
        int dev = 0, n_cu = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n_cu = prop.multiProcessorCount;
        }
        int per_cu = 1;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, e->fn, kWave * ctx->tile_waves[0], e->lds);
        if (per_cu < 1) per_cu = 1;
        const int grid = std::min(n_items, n_cu * per_cu);
        if (grid > 0) {
            void *a[] = {&dj, (void *)&nj, &n_items, &counter};
            int nj_v = nj;
            a[1] = &nj_v;
            if (timed) PSW_HIP(hipEventRecord(ctx->ev0[0], stream), "event record");
            PSW_HIP(hipLaunchKernel(e->fn, dim3(grid), dim3(kWave * ctx->tile_waves[0]), a, e->lds, stream), "sweep");
            if (timed) { PSW_HIP(hipEventRecord(ctx->ev1[0], stream), "event record"); ctx->n_timed = 1; }
        }
    }
    // the merges run one thread per pixel (their loads depend on each other,
    // so they need the parallelism), up to 8192 workgroups per job
    auto blocks_for = [](int64_t px) { return (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (px + 255) / 256)); };
    int64_t chunk_px = 0;
    for (int j = 0; j < nj; ++j) {
        const JobDev &J = (*host_jobs)[j];
        if (J.nch_f + J.nch_g > 1) chunk_px = std::max<int64_t>(chunk_px, (int64_t)J.w * J.h);
    }
    if (chunk_px > 0) {
        void *a[] = {&dj};
        PSW_HIP(hipLaunchKernel(psw_chunk_merge_kernel(), dim3(blocks_for(chunk_px), nj), dim3(256), a, 0, stream),
                "chunk merge");
    }
    if (blob.nm > 0) {
        const MergeDev *hm = reinterpret_cast<const MergeDev *>(blob.bytes.data() + blob.merges);
        int64_t merge_px = 0;
        for (int m = 0; m < blob.nm; ++m) merge_px = std::max<int64_t>(merge_px, (int64_t)hm[m].w * hm[m].h);
        void *a[] = {&dm};
        PSW_HIP(hipLaunchKernel(psw_merge_kernel(), dim3(blocks_for(merge_px), blob.nm), dim3(256), a, 0, stream),
                "merge");
    }
    return PSWEEP_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// One run on device memory `base` laid out as `lay` (the bound workspace, or
// the static scratch of psweep_run_noalloc).
psweep_status run_on(psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames, const psweep_output *out,
                     void *hip_stream, char *base, const Layout *lay) {
    if (!frames || !out) return fail(ctx, PSWEEP_EINVAL, "NULL frames or outputs");
    if (n_frames < 1 || n_frames > ctx->cfg.max_frames) return fail(ctx, PSWEEP_EINVAL, "n_frames out of range");
    if (ctx->cfg.mode == PSWEEP_MODE_SOFT && n_frames != 1) return fail(ctx, PSWEEP_EINVAL, "soft mode runs one frame");
    hipStream_t stream = (hipStream_t)hip_stream;
    ctx->base = base;
    ctx->lay = lay;
    if (base != ctx->last_base) {
        // the device tables and plane setup of the other memory do not apply here
        ctx->last_table.clear();
        ctx->setup_version = 0;
        ctx->last_base = base;
    }
    Blob blob;
    std::vector<int> job_frame;
    char *tb = base + lay->off_table[0];
    psweep_status st = build_tables(ctx, frames, n_frames, out, tb, (int *)(base + lay->off_counter[0]), blob, job_frame);
    if (st != PSWEEP_OK) return st;
    std::vector<JobDev> hj(blob.nj);
    std::memcpy(hj.data(), blob.bytes.data() + blob.jobs, sizeof(JobDev) * blob.nj);
    // upload the tables when they changed (the device copy stays valid: only
    // runs on this memory write this region)
    const bool changed = blob.bytes != ctx->last_table;
    if (changed) {
        const int b = ctx->staging_idx;
        if (ctx->staging_pending[b]) {
            PSW_HIP(hipEventSynchronize(ctx->staging_ev[b]), "staging wait");
            ctx->staging_pending[b] = false;
        }
        std::memcpy(ctx->staging[b], blob.bytes.data(), blob.bytes.size());
        PSW_HIP(hipMemcpyAsync(tb, ctx->staging[b], blob.bytes.size(), hipMemcpyHostToDevice, stream), "table upload");
        PSW_HIP(hipEventRecord(ctx->staging_ev[b], stream), "staging event");
        ctx->staging_pending[b] = true;
        ctx->staging_idx ^= 1;
        ctx->last_table = blob.bytes;
    }
    const bool do_setup = changed || ctx->setup_version != ctx->cam_version;
    st = enqueue(ctx, blob, tb, 0, stream, do_setup, ctx->timing, &hj);
    if (st != PSWEEP_OK) { ctx->last_table.clear(); return st; }
    ctx->setup_version = ctx->cam_version;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "launch");
    if (ctx->cfg.mode == PSWEEP_MODE_SOFT) {
        ctx->soft_ready = true;
        ctx->soft_frame = frames[0];
        ctx->soft_rho = out[0].soft_invdepth;
        ctx->soft_lse = out[0].soft_lse;
        ctx->soft_pitch = out[0].soft_pitch ? out[0].soft_pitch : hj[0].w;
        ctx->soft_job_off = lay->off_table[0] + blob.jobs;
        ctx->soft_part = reinterpret_cast<char *>(hj[0].part);
    } else {
        ctx->soft_ready = false;
    }
    return PSWEEP_OK;
}

}  // namespace

extern "C" {

psweep_status psweep_run(psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames, const psweep_output *out,
                         void *hip_stream) {
    if (!ctx) return PSWEEP_EINVAL;
    if (!ctx->ws) return fail(ctx, PSWEEP_ESTATE, "psweep_set_workspace has not been called");
    return run_on(ctx, frames, n_frames, out, hip_stream, ctx->ws, &ctx->full);
}

psweep_status psweep_run_noalloc(psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                                 const psweep_output *out, void *hip_stream) {
    if (!ctx) return PSWEEP_EINVAL;
    if (ctx->cfg.mode == PSWEEP_MODE_SOFT)
        return fail(ctx, PSWEEP_EUNSUPPORTED, "psweep_run_noalloc sweeps in winner-take-all mode only");
    void *scratch = nullptr;
    size_t bytes = 0;
    const hipError_t e = psw_static_scratch(&scratch, &bytes);
    if (e != hipSuccess) return hip_fail(ctx, e, "static scratch address");
    if (ctx->lean.need > bytes)
        return fail(ctx, PSWEEP_EINVAL,
                    "psweep_run_noalloc: this context needs " + std::to_string(ctx->lean.need) +
                        " bytes of scratch, more than the library's static " + std::to_string(bytes) +
                        " (smaller max_width / max_height / max_sources / max_frames)");
    return run_on(ctx, frames, n_frames, out, hip_stream, (char *)scratch, &ctx->lean);
}

psweep_status psweep_sweep_kernel_ms(psweep_ctx *ctx, double *ms, int32_t *n_launches) {
    if (!ctx || !ms) return PSWEEP_EINVAL;
    if (ctx->n_timed == 0) return fail(ctx, PSWEEP_ESTATE, "no timed sweep launches (enable timing first)");
    double sum = 0;
    for (int i = 0; i < ctx->n_timed; ++i) {
        float t = 0;
        hipError_t e = hipEventElapsedTime(&t, ctx->ev0[i], ctx->ev1[i]);
        if (e != hipSuccess) return hip_fail(ctx, e, "event elapsed");
        sum += t;
    }
    *ms = sum / ctx->n_timed;
    if (n_launches) *n_launches = ctx->n_timed;
    return PSWEEP_OK;
}

psweep_status psweep_sweep_kernel_times(psweep_ctx *ctx, double *ms, int32_t capacity, int32_t *n) {
    if (!ctx || !ms || !n || capacity < 0) return PSWEEP_EINVAL;
    if (ctx->n_timed == 0) return fail(ctx, PSWEEP_ESTATE, "no timed sweep launches (enable timing first)");
    const int m = std::min(capacity, ctx->n_timed);
    for (int i = 0; i < m; ++i) {
        float t = 0;
        hipError_t e = hipEventElapsedTime(&t, ctx->ev0[i], ctx->ev1[i]);
        if (e != hipSuccess) return hip_fail(ctx, e, "event elapsed");
        ms[i] = t;
    }
    *n = ctx->n_timed;
    return PSWEEP_OK;
}

psweep_status psweep_graph_capture(psweep_ctx *ctx, const psweep_frame *frames, int32_t n_frames,
                                   const psweep_output *out, void *hip_stream) {
    if (!ctx) return PSWEEP_EINVAL;
    if (!ctx->ws) return fail(ctx, PSWEEP_ESTATE, "psweep_set_workspace has not been called");
    if (!frames || !out || n_frames < 1 || n_frames > ctx->cfg.max_frames)
        return fail(ctx, PSWEEP_EINVAL, "bad frames");
    if (ctx->cfg.mode == PSWEEP_MODE_SOFT) return fail(ctx, PSWEEP_EUNSUPPORTED, "graphs are for the WTA sweep");
    (void)hip_stream;
    if (!ctx->capture_stream)
        PSW_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking), "capture stream");
    hipStream_t stream = ctx->capture_stream;
    // work already enqueued by the caller must finish before the tables change
    PSW_HIP(hipDeviceSynchronize(), "synchronise before capture");
    Blob blob;
    std::vector<int> job_frame;
    ctx->base = ctx->ws;
    ctx->lay = &ctx->full;
    char *tb = ctx->ws + ctx->full.off_table[1];
    psweep_status st =
        build_tables(ctx, frames, n_frames, out, tb, (int *)(ctx->ws + ctx->full.off_counter[1]), blob, job_frame);
    if (st != PSWEEP_OK) return st;
    std::vector<JobDev> hj(blob.nj);
    std::memcpy(hj.data(), blob.bytes.data() + blob.jobs, sizeof(JobDev) * blob.nj);
    // the graph's own table region is filled once, outside the graph
    PSW_HIP(hipMemcpy(tb, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice), "graph table upload");
    if (ctx->gexec) { (void)hipGraphExecDestroy(ctx->gexec); ctx->gexec = nullptr; }
    if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
    PSW_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture");
    st = enqueue(ctx, blob, tb, 1, stream, true, false, &hj);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &g);
    if (st != PSWEEP_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
    ctx->graph = g;
    PSW_HIP(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0), "graph instantiate");
    ctx->soft_ready = false;
    ctx->setup_version = 0;
    return PSWEEP_OK;
}

psweep_status psweep_graph_launch(psweep_ctx *ctx, void *hip_stream) {
    if (!ctx) return PSWEEP_EINVAL;
    if (!ctx->gexec) return fail(ctx, PSWEEP_ESTATE, "no captured graph");
    PSW_HIP(hipGraphLaunch(ctx->gexec, (hipStream_t)hip_stream), "graph launch");
    // the graph's setup kernel rewrote the frame slots' plane tables with the
    // graph's own camera sets: the next psweep_run must set them up again
    ctx->setup_version = 0;
    return PSWEEP_OK;
}

psweep_status psweep_soft_depth_backward(psweep_ctx *ctx, const float *d_grad_invdepth, float *const *d_grad_src,
                                         double *d_grad_pose, void *hip_stream) {
    if (!ctx) return PSWEEP_EINVAL;
    if (!ctx->soft_ready) return fail(ctx, PSWEEP_ESTATE, "backward needs a preceding soft-mode psweep_run");
    if (!d_grad_invdepth || !d_grad_pose) return fail(ctx, PSWEEP_EINVAL, "NULL gradient buffer");
    hipStream_t stream = (hipStream_t)hip_stream;
    const JobDev *job = (const JobDev *)(ctx->ws + ctx->soft_job_off);
    const CamSet &C = ctx->sets[ctx->soft_frame.camera_set];
    // source image gradients are optional: a NULL array or entry skips them
    float *gsrc[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int s = 0; s < C.n_src; ++s) gsrc[s] = d_grad_src ? d_grad_src[s] : nullptr;
    const void *zk = psw_zero_kernel();
    for (int s = 0; s < C.n_src; ++s) {
        float *p = gsrc[s];
        if (!p) continue;
        int64_t n = (int64_t)C.src[s].width * C.src[s].height;
        void *a[] = {&p, &n};
        PSW_HIP(hipLaunchKernel(zk, dim3(256), dim3(256), a, 0, stream), "zero");
    }
    const int win = ctx->cfg.level[0].window;
    bool any_image = false;
    for (int s = 0; s < C.n_src; ++s) any_image |= gsrc[s] != nullptr;
    const void *bk = psw_backward_kernel(win, C.n_src, ctx->cfg.image_format, any_image ? 1 : 0,
                                         ctx->cfg.level[0].n_ground > 0 ? 1 : 0);
    if (!bk) return fail(ctx, PSWEEP_EUNSUPPORTED, "no backward kernel for this window / source count");
    const size_t lds = psw_backward_lds(win, C.n_src, any_image ? 1 : 0);
    if (lds > 65536) PSW_HIP(hipFuncSetAttribute(bk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds), "lds limit");
    const int hw = win / 2;
    const int w = C.ref.width, h = C.ref.height;
    const int tyo = psw_backward_tile_rows();
    const int tx = (w - 2 * hw + (kWave - 2 * hw) - 1) / (kWave - 2 * hw);
    const int ty = (h - 2 * hw + tyo - 1) / tyo;
    const int tiles = tx > 0 && ty > 0 ? tx * ty : 0;
    // planes in chunks swept by separate workgroups (each plane's share of the
    // gradient is independent given rho_hat and lse): about 14 waves per
    // SIMD, at least two planes per chunk.  Fewer, longer chunks repeat less
    // of the per-tile set-up and share each image-gradient patch over more
    // planes (C4: 0.56 ms with 6 chunks, 0.58 ms with 10, 0.61 ms with 16)
    const int nf = ctx->cfg.level[0].n_fronto + ctx->cfg.level[0].n_ground;   // every plane
    const long long wpg = psw_backward_threads(any_image ? 1 : 0) / kWave;   // waves per workgroup
    int nch = tiles ? (int)((14LL * ctx->n_cu * 4 + wpg * tiles - 1) / (wpg * tiles)) : 1;
    nch = std::max(1, std::min(std::min(nch, 16), std::max(1, nf / 2)));
    // the pose gradient: one partial row of 6 S doubles per workgroup, in the
    // plane-chunk region of the soft run (merged by then), summed in order
    double *gpart = reinterpret_cast<double *>(ctx->soft_part);
    const int n_rows = tiles * nch, n_pose = 6 * C.n_src;
    const size_t part_bytes = align_up((size_t)ctx->ref_w[0] * ctx->ref_h[0] * 4 * kPartWords * kMaxChunks);
    if ((size_t)n_rows * n_pose * sizeof(double) > part_bytes)
        return fail(ctx, PSWEEP_EUNSUPPORTED, "backward partial sums exceed the workspace region");
    if (tiles) {
        float *g0 = gsrc[0], *g1 = gsrc[1], *g2 = gsrc[2], *g3 = gsrc[3];
        const float *rho = ctx->soft_rho, *lse = ctx->soft_lse;
        int64_t sp = ctx->soft_pitch;
        void *a[] = {(void *)&job, (void *)&d_grad_invdepth, (void *)&rho, (void *)&lse, &sp,
                     &g0, &g1, &g2, &g3, &gpart};
        PSW_HIP(hipLaunchKernel(bk, dim3(tx, ty, nch), dim3(psw_backward_threads(any_image ? 1 : 0)), a, lds, stream),
                "backward");
    }
    {
        int nr = n_rows, np = n_pose;
        void *a[] = {&gpart, &nr, &np, &d_grad_pose};
        PSW_HIP(hipLaunchKernel(psw_pose_reduce_kernel(), dim3(n_pose), dim3(256), a, 0, stream), "pose reduce");
    }
    return PSWEEP_OK;
}

psweep_status psweep_filter(psweep_ctx *ctx, int32_t camera_set, const psweep_maps *in,
                            const psweep_filter_params *prm, float *out_depth, uint8_t *out_code, int64_t out_pitch,
                            void *hip_stream) {
    if (!ctx) return PSWEEP_EINVAL;
    if (camera_set < 0 || camera_set >= (int)ctx->sets.size() || !ctx->sets[camera_set].defined)
        return fail(ctx, PSWEEP_ESTATE, "undefined camera set");
    if (!in || !prm || !in->depth || !in->cost1 || !in->cost2 || !out_depth || !out_code)
        return fail(ctx, PSWEEP_EINVAL, "NULL map");
    if (prm->window < 3 || prm->window > 15 || (prm->window & 1) == 0)
        return fail(ctx, PSWEEP_EINVAL, "filter window must be odd in [3, 15]");
    if (!(prm->gamma_m > 0.0) || !(prm->delta >= 0.0 && prm->delta <= 1.0) || !(prm->ratio_min >= 1.0))
        return fail(ctx, PSWEEP_EINVAL, "need gamma > 0, 0 <= delta <= 1, ratio_min >= 1");
    const psweep_camera &c = ctx->sets[camera_set].ref;
    if ((in->pitch != 0 && in->pitch < c.width) || (out_pitch != 0 && out_pitch < c.width))
        return fail(ctx, PSWEEP_EINVAL, "pitch below width");
    if (!ctx->ws) return fail(ctx, PSWEEP_ESTATE, "psweep_set_workspace has not been called");
    FilterDev F;
    std::memset(&F, 0, sizeof F);
    F.w = c.width; F.h = c.height; F.win = prm->window;
    F.fx = (float)c.fx; F.fy = (float)c.fy; F.cx = (float)c.cx; F.cy = (float)c.cy; F.xi = (float)c.xi;
    for (int a = 0; a < 3; ++a) F.gn[a] = (float)ctx->cfg.ground_n[a];
    F.alpha_upper = (float)prm->alpha_upper; F.alpha_lower = (float)prm->alpha_lower;
    F.ratio_min = (float)prm->ratio_min; F.gamma = (float)prm->gamma_m;
    F.min_count = (float)(prm->delta * (prm->window * prm->window - 1));
    F.depth = in->depth; F.cost1 = in->cost1; F.cost2 = in->cost2;
    F.in_pitch = in->pitch ? in->pitch : c.width;
    F.out_depth = out_depth; F.code = out_code;
    F.out_pitch = out_pitch ? out_pitch : c.width;
    hipStream_t stream = (hipStream_t)hip_stream;
    void *a[] = {&F};
    PSW_HIP(hipLaunchKernel(psw_filter_kernel(), dim3((c.width + 15) / 16, (c.height + 15) / 16), dim3(16, 16), a, 0,
                            stream), "filter");
    return PSWEEP_OK;
}

psweep_status psweep_mask_boxes(psweep_ctx *ctx, int32_t camera_set, float *depth, uint8_t *code, int64_t pitch,
                                int32_t n_boxes, const int32_t *boxes, void *hip_stream) {
    if (!ctx) return PSWEEP_EINVAL;
    if (camera_set < 0 || camera_set >= (int)ctx->sets.size() || !ctx->sets[camera_set].defined)
        return fail(ctx, PSWEEP_ESTATE, "undefined camera set");
    if (!depth || n_boxes < 0 || (n_boxes > 0 && !boxes)) return fail(ctx, PSWEEP_EINVAL, "NULL depth or boxes");
    const psweep_camera &c = ctx->sets[camera_set].ref;
    if (pitch != 0 && pitch < c.width) return fail(ctx, PSWEEP_EINVAL, "pitch below width");
    hipStream_t stream = (hipStream_t)hip_stream;
    MaskDev M;
    std::memset(&M, 0, sizeof M);
    M.depth = depth; M.code = code; M.pitch = pitch ? pitch : c.width;
    M.w = c.width; M.h = c.height;
    auto flush = [&]() -> psweep_status {
        if (M.n == 0) return PSWEEP_OK;
        void *a[] = {&M};
        PSW_HIP(hipLaunchKernel(psw_mask_kernel(), dim3(64, M.n), dim3(256), a, 0, stream), "mask");
        M.n = 0;
        return PSWEEP_OK;
    };
    for (int b = 0; b < n_boxes; ++b) {
        // clip to the image; boxes left empty are dropped
        const int x0 = std::max(boxes[4 * b + 0], 0), y0 = std::max(boxes[4 * b + 1], 0);
        const int x1 = std::min(boxes[4 * b + 2], c.width), y1 = std::min(boxes[4 * b + 3], c.height);
        if (x1 <= x0 || y1 <= y0) continue;
        M.box[M.n][0] = x0; M.box[M.n][1] = y0; M.box[M.n][2] = x1; M.box[M.n][3] = y1;
        if (++M.n == kMaxMaskBoxes) {
            const psweep_status st = flush();
            if (st != PSWEEP_OK) return st;
        }
    }
    return flush();
}

void psweep_destroy(psweep_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->side_stream) (void)hipStreamDestroy(ctx->side_stream);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    for (int b = 0; b < 2; ++b) {
        if (ctx->staging[b]) (void)hipHostFree(ctx->staging[b]);
        if (ctx->staging_ev[b]) (void)hipEventDestroy(ctx->staging_ev[b]);
    }
    for (auto e : ctx->ev0) (void)hipEventDestroy(e);
    for (auto e : ctx->ev1) (void)hipEventDestroy(e);
    delete ctx;
}

}  // extern "C"
