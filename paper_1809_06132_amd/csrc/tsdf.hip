// Fisheye TSDF fusion kernels (Sec. III-C): allocation of voxel blocks along
// the truncation segment of every depth pixel's Eq. (1) ray, the list of
// blocks in view, and the running average of Eq. (2) over their voxels.
//
// The map is a box of nx x ny x nz blocks stored in as many slots; block
// (bx, by, bz) lives in slot ((bz mod nz) ny + (by mod ny)) nx + (bx mod nx).
// Inside the box no two blocks share a slot, so a block is allocated with one
// compare-and-swap of its packed coordinates into an empty slot key, and a
// box that moves only has to empty the slots whose blocks it left.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsdf_internal.h"

namespace psw {

namespace {

constexpr unsigned long long kValid = 1ull << 63;
constexpr int kCoordBias = 1 << 20;

__device__ __forceinline__ unsigned long long pack_block(int bx, int by, int bz) {
    return kValid | (unsigned long long)(bx + kCoordBias) | ((unsigned long long)(by + kCoordBias) << 21) |
           ((unsigned long long)(bz + kCoordBias) << 42);
}
__device__ __forceinline__ void unpack_block(unsigned long long k, int *bx, int *by, int *bz) {
    *bx = (int)(k & 0x1fffffull) - kCoordBias;
    *by = (int)((k >> 21) & 0x1fffffull) - kCoordBias;
    *bz = (int)((k >> 42) & 0x1fffffull) - kCoordBias;
}
__device__ __forceinline__ int wrap(int b, int n) {
    const int r = b % n;
    return r < 0 ? r + n : r;
}
__device__ __forceinline__ int slot_of(const TsdfDev &T, int bx, int by, int bz) {
    return (wrap(bz, T.nb[2]) * T.nb[1] + wrap(by, T.nb[1])) * T.nb[0] + wrap(bx, T.nb[0]);
}
// camera point of a box-relative world point
__device__ __forceinline__ void to_cam(const TsdfDev &T, float x, float y, float z, float *c) {
    c[0] = fmaf(T.R[0], x, fmaf(T.R[1], y, fmaf(T.R[2], z, T.t[0])));
    c[1] = fmaf(T.R[3], x, fmaf(T.R[4], y, fmaf(T.R[5], z, T.t[1])));
    c[2] = fmaf(T.R[6], x, fmaf(T.R[7], y, fmaf(T.R[8], z, T.t[2])));
}
// unified-model projection; false behind the model's viewpoint
__device__ __forceinline__ bool project(const TsdfDev &T, const float *c, float *u, float *v, float *range) {
    const float m = sqrtf(fmaf(c[0], c[0], fmaf(c[1], c[1], c[2] * c[2])));
    const float den = fmaf(T.xi, m, c[2]);
    *range = m;
    if (!(den > 0.0f)) return false;
    *u = fmaf(T.fx, c[0] / den, T.cx);
    *v = fmaf(T.fy, c[1] / den, T.cy);
    return true;
}

}  // namespace

__global__ void tsdf_reset_kernel(TsdfDev T) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < T.nslots; s += gridDim.x * blockDim.x) {
        T.keys[s] = 0ull;
        T.count[s] = 0;
        T.seen[s] = 0;
        T.fresh[s] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) T.counters[threadIdx.x] = 0;
}

// empty the slots whose blocks lie outside the box; clear the counters
__global__ void tsdf_recentre_kernel(TsdfDev T) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < T.nslots; s += gridDim.x * blockDim.x) {
        const unsigned long long k = T.keys[s];
        if (!k) continue;
        int bx, by, bz;
        unpack_block(k, &bx, &by, &bz);
        const bool in = bx >= T.b0[0] && bx < T.b0[0] + T.nb[0] && by >= T.b0[1] && by < T.b0[1] + T.nb[1] &&
                        bz >= T.b0[2] && bz < T.b0[2] + T.nb[2];
        if (!in) {
            T.keys[s] = 0ull;
            T.count[s] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) T.counters[threadIdx.x] = 0;
}

// one thread per depth pixel: walk the blocks its truncation segment crosses
// (a 3-D digital differential analyser in block units) and allocate them
__global__ void tsdf_alloc_kernel(TsdfDev T) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= T.w || v >= T.h) return;
    const float d = T.depth[(int64_t)v * T.pitch + u];
    if (!(d > 0.0f) || !(d < 3.0e38f)) return;
    // Eq. (1): unit ray of the pixel
    const float x = ((float)u - T.cx) / T.fx, y = ((float)v - T.cy) / T.fy;
    const float q = fmaf(x, x, y * y);
    const float disc = fmaf(1.0f - T.xi * T.xi, q, 1.0f);
    if (disc < 0.0f) return;
    const float eta = (T.xi + sqrtf(disc)) / (q + 1.0f);
    const float r[3] = {eta * x, eta * y, eta - T.xi};
    const float l0 = fmaxf(d - T.mu, 0.0f), l1 = d + T.mu;
    // segment ends in box-relative world coordinates: R^T (l r - t), in blocks
    const float c0 = l0 * r[0] - T.t[0], c1 = l0 * r[1] - T.t[1], c2 = l0 * r[2] - T.t[2];
    const float d0 = l1 * r[0] - T.t[0], d1 = l1 * r[1] - T.t[1], d2 = l1 * r[2] - T.t[2];
    float a[3], e[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = fmaf(T.R[0 * 3 + i], c0, fmaf(T.R[1 * 3 + i], c1, T.R[2 * 3 + i] * c2)) / T.block;
        e[i] = fmaf(T.R[0 * 3 + i], d0, fmaf(T.R[1 * 3 + i], d1, T.R[2 * 3 + i] * d2)) / T.block;
    }
    int cur[3], step[3];
    float tmax[3], tdel[3];
    for (int i = 0; i < 3; ++i) {
        cur[i] = (int)floorf(a[i]);
        const float dir = e[i] - a[i];
        if (dir > 0.0f) {
            step[i] = 1; tmax[i] = ((float)(cur[i] + 1) - a[i]) / dir; tdel[i] = 1.0f / dir;
        } else if (dir < 0.0f) {
            step[i] = -1; tmax[i] = ((float)cur[i] - a[i]) / dir; tdel[i] = -1.0f / dir;
        } else {
            step[i] = 0; tmax[i] = 3.0e38f; tdel[i] = 3.0e38f;
        }
    }
    // a segment of length L blocks crosses at most L + 3 block faces
    for (int it = 0; it < 64; ++it) {
        if (cur[0] >= 0 && cur[0] < T.nb[0] && cur[1] >= 0 && cur[1] < T.nb[1] && cur[2] >= 0 && cur[2] < T.nb[2]) {
            const int bx = T.b0[0] + cur[0], by = T.b0[1] + cur[1], bz = T.b0[2] + cur[2];
            const int s = slot_of(T, bx, by, bz);
            const unsigned long long key = pack_block(bx, by, bz);
            // most pixels meet blocks that are already allocated and marked:
            // read first, so that only the first visits contend for the
            // atomic (the compare-and-swap still decides who allocates)
            if (__atomic_load_n(T.keys + s, __ATOMIC_RELAXED) != key) {
                const unsigned long long old = atomicCAS(T.keys + s, 0ull, key);
                if (old == 0ull) T.fresh[s] = 1;
            }
            if (!__atomic_load_n(T.seen + s, __ATOMIC_RELAXED)) T.seen[s] = 1;
        }
        const int ax = tmax[0] <= tmax[1] ? (tmax[0] <= tmax[2] ? 0 : 2) : (tmax[1] <= tmax[2] ? 1 : 2);
        if (tmax[ax] > 1.0f) break;
        cur[ax] += step[ax];
        tmax[ax] += tdel[ax];
    }
}

// new blocks start with D = 1, w = 0
__global__ void tsdf_init_kernel(TsdfDev T) {
    const int s = blockIdx.x;
    if (!T.fresh[s]) return;
    for (int e = threadIdx.x; e < kBlockVox; e += blockDim.x) {
        T.D[(int64_t)s * kBlockVox + e] = 1.0f;
        T.W[(int64_t)s * kBlockVox + e] = 0.0f;
    }
    __syncthreads();
    if (threadIdx.x == 0) T.fresh[s] = 0;
}

// per slot: observation count, then the list of allocated blocks with a
// corner in view
__global__ void tsdf_blocks_kernel(TsdfDev T) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T.nslots) return;
    if (T.seen[s]) {
        T.count[s] += 1;
        T.seen[s] = 0;
    }
    const unsigned long long k = T.keys[s];
    if (!k) return;
    atomicAdd(T.counters + 1, 1);
    int bx, by, bz;
    unpack_block(k, &bx, &by, &bz);
    const float ox = (float)(bx - T.b0[0]) * T.block, oy = (float)(by - T.b0[1]) * T.block;
    const float oz = (float)(bz - T.b0[2]) * T.block;
    bool vis = false;
    for (int c = 0; c < 8; ++c) {
        float cc[3], u, v, rg;
        to_cam(T, ox + ((c & 1) ? T.block : 0.0f), oy + ((c & 2) ? T.block : 0.0f), oz + ((c & 4) ? T.block : 0.0f),
               cc);
        if (project(T, cc, &u, &v, &rg) && u >= 0.0f && v >= 0.0f && u <= (float)(T.w - 1) && v <= (float)(T.h - 1))
            vis = true;
    }
    if (vis) T.list[atomicAdd(T.counters + 0, 1)] = s;
}

// one workgroup per visible block, two voxels per thread: Eq. (2)
__global__ void tsdf_integrate_kernel(TsdfDev T) {
    if ((int)blockIdx.x >= T.counters[0]) return;
    const int s = T.list[blockIdx.x];
    int bx, by, bz;
    unpack_block(T.keys[s], &bx, &by, &bz);
    const int rx = (bx - T.b0[0]) * 8, ry = (by - T.b0[1]) * 8, rz = (bz - T.b0[2]) * 8;
    for (int e = threadIdx.x; e < kBlockVox; e += blockDim.x) {
        const float X = ((float)(rx + (e & 7)) + 0.5f) * T.voxel;
        const float Y = ((float)(ry + ((e >> 3) & 7)) + 0.5f) * T.voxel;
        const float Z = ((float)(rz + (e >> 6)) + 0.5f) * T.voxel;
        float c[3], u, v, range;
        to_cam(T, X, Y, Z, c);
        if (!project(T, c, &u, &v, &range)) continue;
        const float fu = floorf(u + 0.5f), fv = floorf(v + 0.5f);   // nearest pixel
        if (!(fu >= 0.0f && fv >= 0.0f && fu <= (float)(T.w - 1) && fv <= (float)(T.h - 1))) continue;
        const float d_obs = T.depth[(int64_t)fv * T.pitch + (int64_t)fu];
        if (!(d_obs > 0.0f) || !(d_obs < 3.0e38f)) continue;
        const float eta = d_obs - range;
        if (eta < -T.mu) continue;
        const int64_t o = (int64_t)s * kBlockVox + e;
        const float w = T.W[o];
        T.D[o] = (w * T.D[o] + fminf(1.0f, eta / T.mu)) / (w + 1.0f);
        T.W[o] = fminf(w + 1.0f, T.w_max);
    }
}

// dense copy of the box in world order
__global__ void tsdf_extract_kernel(TsdfDev T, float *out_d, float *out_w, int32_t *out_count) {
    const int nx = T.nb[0] * 8, ny = T.nb[1] * 8, nz = T.nb[2] * 8;
    const int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < nvox; o += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(o % nx), y = (int)((o / nx) % ny), z = (int)(o / ((int64_t)nx * ny));
        const int bx = T.b0[0] + (x >> 3), by = T.b0[1] + (y >> 3), bz = T.b0[2] + (z >> 3);
        const int s = slot_of(T, bx, by, bz);
        const bool here = T.keys[s] == pack_block(bx, by, bz);
        const int64_t v = (int64_t)s * kBlockVox + (((z & 7) * 8 + (y & 7)) * 8 + (x & 7));
        const float w = here ? T.W[v] : 0.0f;
        if (out_w) out_w[o] = w;
        if (out_d) out_d[o] = (here && w > 0.0f && T.count[s] >= T.min_obs) ? T.D[v] : __builtin_nanf("");
        if (out_count && (x & 7) == 0 && (y & 7) == 0 && (z & 7) == 0)
            out_count[((int64_t)(z >> 3) * T.nb[1] + (y >> 3)) * T.nb[0] + (x >> 3)] = here ? T.count[s] : 0;
    }
}

__global__ void tsdf_stats_kernel(TsdfDev T, int32_t *out) {
    if (threadIdx.x == 0) {
        out[0] = T.counters[1];
        out[1] = T.counters[0];
    }
}

}  // namespace psw

extern "C" {
const void *psw_tsdf_kernel(int which) {
    switch (which) {
    case 0: return (const void *)&psw::tsdf_reset_kernel;
    case 1: return (const void *)&psw::tsdf_recentre_kernel;
    case 2: return (const void *)&psw::tsdf_alloc_kernel;
    case 3: return (const void *)&psw::tsdf_init_kernel;
    case 4: return (const void *)&psw::tsdf_blocks_kernel;
    case 5: return (const void *)&psw::tsdf_integrate_kernel;
    case 6: return (const void *)&psw::tsdf_extract_kernel;
    case 7: return (const void *)&psw::tsdf_stats_kernel;
    }
    return nullptr;
}
}
