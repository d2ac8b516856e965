// Host side of the TSDF map: validation, workspace layout, and the launch
// sequence of one integration (recentre -> allocate -> initialise new blocks
// -> count and list visible blocks -> integrate).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/psweep_tsdf.h"
#include "tsdf_internal.h"

using psw::TsdfDev;

extern "C" const void *psw_tsdf_kernel(int which);

namespace {

thread_local std::string g_tsdf_create_error;
constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct psweep_tsdf {
    psweep_tsdf_config cfg{};
    int32_t nslots = 0;
    char *ws = nullptr;
    size_t ws_need = 0;
    size_t off_keys = 0, off_count = 0, off_seen = 0, off_fresh = 0, off_list = 0, off_counters = 0, off_d = 0,
           off_w = 0;
    bool reset_done = false, integrated = false;
    int32_t b0[3] = {0, 0, 0};
    TsdfDev last{};
    std::string err;
};

namespace {

psweep_status tfail(psweep_tsdf *ts, psweep_status st, const std::string &m) {
    if (ts) ts->err = m;
    else g_tsdf_create_error = m;
    return st;
}

#define TSDF_HIP(call, what)                                                        \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return tfail(ts, PSWEEP_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

TsdfDev base_dev(const psweep_tsdf *ts) {
    TsdfDev T;
    std::memset(&T, 0, sizeof T);
    const psweep_tsdf_config &c = ts->cfg;
    T.voxel = (float)c.voxel_m;
    T.block = (float)(8.0 * c.voxel_m);
    T.mu = (float)c.mu_m;
    T.w_max = (float)c.w_max;
    for (int a = 0; a < 3; ++a) { T.nb[a] = c.blocks[a]; T.b0[a] = ts->b0[a]; }
    T.nslots = ts->nslots;
    T.min_obs = c.min_observations;
    char *w = ts->ws;
    T.keys = (unsigned long long *)(w + ts->off_keys);
    T.count = (int32_t *)(w + ts->off_count);
    T.seen = (int32_t *)(w + ts->off_seen);
    T.fresh = (int32_t *)(w + ts->off_fresh);
    T.list = (int32_t *)(w + ts->off_list);
    T.counters = (int32_t *)(w + ts->off_counters);
    T.D = (float *)(w + ts->off_d);
    T.W = (float *)(w + ts->off_w);
    return T;
}

psweep_status launch(psweep_tsdf *ts, int which, dim3 grid, dim3 block, void **args, hipStream_t stream,
                     const char *what) {
    TSDF_HIP(hipLaunchKernel(psw_tsdf_kernel(which), grid, block, args, 0, stream), what);
    return PSWEEP_OK;
}

}  // namespace

extern "C" {

const char *psweep_tsdf_last_error(const psweep_tsdf *ts) {
    return ts ? ts->err.c_str() : g_tsdf_create_error.c_str();
}

psweep_status psweep_tsdf_create(const psweep_tsdf_config *cfg, psweep_tsdf **out) {
    psweep_tsdf *ts = nullptr;
    if (!cfg || !out) return tfail(ts, PSWEEP_EINVAL, "NULL argument");
    *out = nullptr;
    if (!(cfg->voxel_m > 0.0) || !(cfg->mu_m > 0.0)) return tfail(ts, PSWEEP_EINVAL, "voxel_m and mu_m must be > 0");
    // the allocation walks at most 64 blocks per pixel: a segment of 2 mu
    // crosses at most 2 sqrt(3) mu / B + 3 block faces
    if (!(cfg->mu_m <= 16.0 * 8.0 * cfg->voxel_m)) return tfail(ts, PSWEEP_EINVAL, "mu_m above 16 blocks");
    long long n = 1;
    for (int a = 0; a < 3; ++a) {
        if (cfg->blocks[a] < 1 || cfg->blocks[a] > 1024) return tfail(ts, PSWEEP_EINVAL, "blocks out of [1, 1024]");
        n *= cfg->blocks[a];
    }
    if (n > (1ll << 24)) return tfail(ts, PSWEEP_EINVAL, "more than 2^24 blocks");
    if (!(cfg->w_max >= 1.0)) return tfail(ts, PSWEEP_EINVAL, "w_max must be >= 1");
    if (cfg->min_observations < 0) return tfail(ts, PSWEEP_EINVAL, "min_observations must be >= 0");
    if (cfg->max_width < 8 || cfg->max_height < 8 || cfg->max_width > 8192 || cfg->max_height > 8192)
        return tfail(ts, PSWEEP_EINVAL, "max_width/max_height out of [8, 8192]");
    ts = new (std::nothrow) psweep_tsdf();
    if (!ts) return tfail(nullptr, PSWEEP_ENOMEM, "host allocation failed");
    ts->cfg = *cfg;
    ts->nslots = (int32_t)n;
    const size_t s = (size_t)n;
    size_t off = 0;
    ts->off_keys = off; off += align_up(s * 8);
    ts->off_count = off; off += align_up(s * 4);
    ts->off_seen = off; off += align_up(s * 4);
    ts->off_fresh = off; off += align_up(s * 4);
    ts->off_list = off; off += align_up(s * 4);
    ts->off_counters = off; off += kAlign;
    ts->off_d = off; off += align_up(s * psw::kBlockVox * 4);
    ts->off_w = off; off += align_up(s * psw::kBlockVox * 4);
    ts->ws_need = off;
    *out = ts;
    return PSWEEP_OK;
}

psweep_status psweep_tsdf_workspace_size(const psweep_tsdf *ts, size_t *bytes) {
    if (!ts || !bytes) return PSWEEP_EINVAL;
    *bytes = ts->ws_need;
    return PSWEEP_OK;
}

psweep_status psweep_tsdf_set_workspace(psweep_tsdf *ts, void *dev_ptr, size_t bytes) {
    if (!ts) return PSWEEP_EINVAL;
    if (!dev_ptr || ((uintptr_t)dev_ptr & (kAlign - 1))) return tfail(ts, PSWEEP_EINVAL, "workspace NULL or misaligned");
    if (bytes < ts->ws_need) return tfail(ts, PSWEEP_ENOMEM, "workspace too small");
    ts->ws = (char *)dev_ptr;
    ts->reset_done = false;
    ts->integrated = false;
    return PSWEEP_OK;
}

psweep_status psweep_tsdf_reset(psweep_tsdf *ts, void *hip_stream) {
    if (!ts) return PSWEEP_EINVAL;
    if (!ts->ws) return tfail(ts, PSWEEP_ESTATE, "psweep_tsdf_set_workspace has not been called");
    TsdfDev T = base_dev(ts);
    void *a[] = {&T};
    const int g = (ts->nslots + 255) / 256;
    psweep_status st = launch(ts, 0, dim3(g < 4096 ? g : 4096), dim3(256), a, (hipStream_t)hip_stream, "tsdf reset");
    if (st != PSWEEP_OK) return st;
    ts->reset_done = true;
    ts->integrated = false;
    return PSWEEP_OK;
}

psweep_status psweep_tsdf_integrate(psweep_tsdf *ts, const psweep_camera *cam, const psweep_pose *pose,
                                    const double centre[3], const float *depth, int64_t pitch, void *hip_stream) {
    if (!ts) return PSWEEP_EINVAL;
    if (!cam || !pose || !centre || !depth) return tfail(ts, PSWEEP_EINVAL, "NULL argument");
    if (cam->width < 1 || cam->height < 1 || cam->width > ts->cfg.max_width || cam->height > ts->cfg.max_height)
        return tfail(ts, PSWEEP_EINVAL, "depth map size out of range");
    if (!(cam->fx > 0.0) || !(cam->fy > 0.0) || !(cam->xi >= 0.0 && cam->xi <= 1.0) || !std::isfinite(cam->cx) ||
        !std::isfinite(cam->cy))
        return tfail(ts, PSWEEP_EINVAL, "bad camera");
    for (int i = 0; i < 3; ++i) {
        if (!std::isfinite(pose->t[i])) return tfail(ts, PSWEEP_EINVAL, "pose translation not finite");
        for (int j = 0; j < 3; ++j) {
            double d = 0.0;
            for (int k = 0; k < 3; ++k) d += pose->R[3 * i + k] * pose->R[3 * j + k];
            if (!(std::fabs(d - (i == j ? 1.0 : 0.0)) <= 1e-6)) return tfail(ts, PSWEEP_EINVAL, "R not orthonormal");
        }
    }
    if (pitch != 0 && pitch < cam->width) return tfail(ts, PSWEEP_EINVAL, "pitch below width");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(centre[a]) || std::fabs(centre[a]) > 1e6) return tfail(ts, PSWEEP_EINVAL, "bad centre");
    const double B = 8.0 * ts->cfg.voxel_m;
    // block coordinates are packed in 21 bits each, biased by 2^20
    for (int a = 0; a < 3; ++a)
        if (!(std::fabs(std::floor(centre[a] / B)) + ts->cfg.blocks[a] < (double)(1 << 20) - 2))
            return tfail(ts, PSWEEP_EINVAL, "centre too far from the origin for the voxel size");
    if (!ts->ws || !ts->reset_done) return tfail(ts, PSWEEP_ESTATE, "workspace not set or map never reset");
    for (int a = 0; a < 3; ++a) ts->b0[a] = (int32_t)std::floor(centre[a] / B) - ts->cfg.blocks[a] / 2;
    TsdfDev T = base_dev(ts);
    T.fx = (float)cam->fx; T.fy = (float)cam->fy; T.cx = (float)cam->cx; T.cy = (float)cam->cy;
    T.xi = (float)cam->xi;
    T.w = cam->width; T.h = cam->height;
    // box-relative world: X = O + X_rel with O = b0 B, so X_cam = R X_rel + (R O + t)
    const double O[3] = {ts->b0[0] * B, ts->b0[1] * B, ts->b0[2] * B};
    for (int i = 0; i < 3; ++i) {
        double ti = pose->t[i];
        for (int j = 0; j < 3; ++j) { T.R[i * 3 + j] = (float)pose->R[i * 3 + j]; ti += pose->R[i * 3 + j] * O[j]; }
        T.t[i] = (float)ti;
    }
    T.depth = depth;
    T.pitch = pitch ? pitch : cam->width;
    hipStream_t stream = (hipStream_t)hip_stream;
    void *a[] = {&T};
    const int gs = (ts->nslots + 255) / 256;
    psweep_status st;
    if ((st = launch(ts, 1, dim3(gs < 4096 ? gs : 4096), dim3(256), a, stream, "tsdf recentre")) != PSWEEP_OK) return st;
    if ((st = launch(ts, 2, dim3((T.w + 15) / 16, (T.h + 15) / 16), dim3(16, 16), a, stream, "tsdf alloc")) != PSWEEP_OK)
        return st;
    if ((st = launch(ts, 3, dim3(ts->nslots), dim3(256), a, stream, "tsdf init")) != PSWEEP_OK) return st;
    if ((st = launch(ts, 4, dim3(gs), dim3(256), a, stream, "tsdf blocks")) != PSWEEP_OK) return st;
    if ((st = launch(ts, 5, dim3(ts->nslots), dim3(256), a, stream, "tsdf integrate")) != PSWEEP_OK) return st;
    ts->last = T;
    ts->integrated = true;
    return PSWEEP_OK;
}

psweep_status psweep_tsdf_extract(psweep_tsdf *ts, float *d_tsdf, float *d_weight, int32_t *d_block_count,
                                  void *hip_stream) {
    if (!ts) return PSWEEP_EINVAL;
    if (!ts->integrated) return tfail(ts, PSWEEP_ESTATE, "nothing integrated yet");
    TsdfDev T = ts->last;
    void *a[] = {&T, &d_tsdf, &d_weight, &d_block_count};
    const long long nvox = (long long)ts->nslots * psw::kBlockVox;
    const long long g = (nvox + 255) / 256;
    return launch(ts, 6, dim3(g < 65536 ? (unsigned)g : 65536u), dim3(256), a, (hipStream_t)hip_stream, "tsdf extract");
}

psweep_status psweep_tsdf_region(const psweep_tsdf *ts, int32_t first_block[3]) {
    if (!ts || !first_block) return PSWEEP_EINVAL;
    for (int a = 0; a < 3; ++a) first_block[a] = ts->b0[a];
    return PSWEEP_OK;
}

psweep_status psweep_tsdf_stats(psweep_tsdf *ts, int32_t *d_stats, void *hip_stream) {
    if (!ts || !d_stats) return PSWEEP_EINVAL;
    if (!ts->integrated) return tfail(ts, PSWEEP_ESTATE, "nothing integrated yet");
    TsdfDev T = ts->last;
    void *a[] = {&T, &d_stats};
    return launch(ts, 7, dim3(1), dim3(64), a, (hipStream_t)hip_stream, "tsdf stats");
}

void psweep_tsdf_destroy(psweep_tsdf *ts) {
    if (!ts) return;
    (void)hipDeviceSynchronize();
    delete ts;
}

}  // extern "C"
