// Small kernels around the sweep: FP64 per-plane setup, level images,
// border marks, the work counter reset and the level merge; and the static
// scratch array of psweep_run_noalloc.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "sweep_common.h"

namespace psw {

// ---------------------------------------------------------------------------
// per-plane parameters in FP64 (H = R + t n^T / d rounded to float)
// ---------------------------------------------------------------------------
__global__ void setup_kernel(const SetupDev *__restrict__ jobs) {
    const SetupDev &J = jobs[blockIdx.y];
    const int P = J.n_fronto + J.n_ground, S = J.n_src;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < P * S; e += gridDim.x * blockDim.x) {
        const int k = e / S, s = e % S;
        double n[3], d, theta;
        if (k < J.n_fronto) {
            double rho = 1.0 / J.far_m;
            if (J.n_fronto > 1) rho += k * (1.0 / J.near_m - 1.0 / J.far_m) / (J.n_fronto - 1);
            n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
            d = 1.0 / rho;
            theta = rho;
        } else {
            const int g = k - J.n_fronto;
            double h = J.h_lo;
            if (J.n_ground > 1) h += g * (J.h_hi - J.h_lo) / (J.n_ground - 1);
            n[0] = J.gn[0]; n[1] = J.gn[1]; n[2] = J.gn[2];
            d = J.gd - h;
            theta = h;
        }
        float *out = J.htab + (size_t)(k * S + s) * 9;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int r = 0; r < 3; ++r) out[c * 3 + r] = (float)(J.R[s][r * 3 + c] + J.t[s][r] * n[c] / d);
        if (s == 0) J.theta[k] = (float)theta;
    }
}

// ---------------------------------------------------------------------------
// level images: 2x2 box-downsampled reference, source textures of bilinear
// cell coefficients
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t level_pix(const uint8_t *img, int64_t pitch, int x, int y, int ds) {
    if (ds == 1) return img[(int64_t)y * pitch + x];
    const uint8_t *p = img + (int64_t)(2 * y) * pitch + 2 * x;
    return ((uint32_t)p[0] + p[1] + p[pitch] + p[pitch + 1] + 2u) >> 2;
}

// bilinear coefficients of a 2x2 cell as the sweep reads them: FP16 c0 =
// p00 - 128, c1 = p10 - p00, c2 = p01 - p00, c3 = p11 - p10 - p01 + p00
// (integers of magnitude <= 510, exact in FP16), packed (c0 | c1 << 16,
// c2 | c3 << 16)
__device__ __forceinline__ uint32_t half_bits(int c) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)c);
}
__device__ __forceinline__ uint2 coef_texel(uint32_t p00, uint32_t p10, uint32_t p01, uint32_t p11) {
    const int a = (int)p00, b = (int)p10, c = (int)p01, d = (int)p11;
    return make_uint2(half_bits(a - 128) | (half_bits(b - a) << 16), half_bits(c - a) | (half_bits(d - b - c + a) << 16));
}

// invalid marks on the frame of pixels whose window leaves the image
// (threads t, t + stride, ... of the frame's pixels)
__device__ void border_marks(const BorderDev &B, int t, int stride) {
    const int w = B.w, h = B.h, hw = B.hw;
    const int band = min(hw, h);             // rows at top and at bottom
    const int top = band * w;
    const int side_rows = max(h - 2 * band, 0);
    const int total = 2 * top + side_rows * 2 * min(hw, w);
    for (int e = t; e < total; e += stride) {
        int x, y;
        if (e < 2 * top) {
            const int r = e / w;
            x = e % w;
            y = r < band ? r : h - 2 * band + r;
        } else {
            const int q = e - 2 * top, cw = min(hw, w);
            const int r = q / (2 * cw), c = q % (2 * cw);
            y = band + r;
            x = c < cw ? c : w - 2 * cw + c;
        }
        if (x < 0 || x >= w || y < 0 || y >= h) continue;
        const int64_t o = (int64_t)y * B.out_pitch + x;
        if (B.index) B.index[o] = -1;
        if (B.delta) B.delta[o] = 0.0f;
        if (B.cost1) B.cost1[o] = PSW_INF;
        if (B.cost2) B.cost2[o] = PSW_INF;
        if (B.depth) B.depth[o] = __builtin_nanf("");
        if (B.z) B.z[o] = __builtin_nanf("");
        if (B.level_id) B.level_id[o] = 255;
        if (B.soft_rho) {
            const int64_t so = (int64_t)y * B.soft_pitch + x;
            B.soft_rho[so] = __builtin_nanf("");
            B.soft_lse[so] = -PSW_INF;
        }
    }
}

// blockIdx.z: job; blockIdx.y: 0 = reference level and the job's border
// marks, 1 + s = source s
__global__ void prep_kernel(const PrepDev *__restrict__ preps, const BorderDev *__restrict__ borders) {
    const PrepDev &P = preps[blockIdx.z];
    const int which = blockIdx.y;
    const int ds = P.downsample;
    if (which == 0) {
        border_marks(borders[blockIdx.z], blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
        if (!P.ref_level) return;
        const int lw = P.ref_w / ds, lh = P.ref_h / ds;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < lw * lh; e += gridDim.x * blockDim.x) {
            const int x = e % lw, y = e / lw;
            P.ref_level[e] = (uint8_t)level_pix(P.ref_full, P.ref_pitch, x, y, ds);
        }
        return;
    }
    const int s = which - 1;
    if (s >= P.n_src) return;
    const int lw = P.src_w[s] / ds, lh = P.src_h[s] / ds;
    const int64_t pitch = P.src_pitch[s];
    if (P.img == 1) {
        // float images (full resolution only): four floats per texel
        const float *img = static_cast<const float *>(P.src_full[s]);
        float4 *tex = reinterpret_cast<float4 *>(P.tex[s]);
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < lw * lh; e += gridDim.x * blockDim.x) {
            const int x = e % lw, y = e / lw;
            const int x1 = min(x + 1, lw - 1), y1 = min(y + 1, lh - 1);
            tex[e] = make_float4(img[(int64_t)y * pitch + x], img[(int64_t)y * pitch + x1],
                                 img[(int64_t)y1 * pitch + x], img[(int64_t)y1 * pitch + x1]);
        }
        return;
    }
    const uint8_t *img = static_cast<const uint8_t *>(P.src_full[s]);
    uint2 *tex = reinterpret_cast<uint2 *>(P.tex[s]);
    if (ds == 1 && (lw & 3) == 0 && (pitch & 3) == 0 && ((uintptr_t)img & 3) == 0) {
        // four texels per thread: two aligned words and one byte per row, two
        // 16-byte stores (rows of the texture start 32-byte aligned: lw % 4 == 0)
        const int qw = lw >> 2;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < qw * lh; e += gridDim.x * blockDim.x) {
            const int x = (e % qw) << 2, y = e / qw;
            const int y1 = min(y + 1, lh - 1);
            const uint8_t *r0 = img + (int64_t)y * pitch + x, *r1 = img + (int64_t)y1 * pitch + x;
            const uint32_t a = *reinterpret_cast<const uint32_t *>(r0), b = *reinterpret_cast<const uint32_t *>(r1);
            // the texel right of the group, clamped at the last column
            const uint32_t a4 = x + 4 < lw ? r0[4] : (a >> 24), b4 = x + 4 < lw ? r1[4] : (b >> 24);
            const uint64_t ra = a | ((uint64_t)a4 << 32), rb = b | ((uint64_t)b4 << 32);
            uint2 q[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t p00 = (uint32_t)(ra >> (8 * t)) & 0xffu, p10 = (uint32_t)(ra >> (8 * t + 8)) & 0xffu;
                const uint32_t p01 = (uint32_t)(rb >> (8 * t)) & 0xffu, p11 = (uint32_t)(rb >> (8 * t + 8)) & 0xffu;
                q[t] = coef_texel(p00, p10, p01, p11);
            }
            uint4 *dst = reinterpret_cast<uint4 *>(tex + (int64_t)y * lw + x);
            dst[0] = make_uint4(q[0].x, q[0].y, q[1].x, q[1].y);
            dst[1] = make_uint4(q[2].x, q[2].y, q[3].x, q[3].y);
        }
        return;
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < lw * lh; e += gridDim.x * blockDim.x) {
        const int x = e % lw, y = e / lw;
        const int x1 = min(x + 1, lw - 1), y1 = min(y + 1, lh - 1);
        const uint32_t p00 = level_pix(img, pitch, x, y, ds), p10 = level_pix(img, pitch, x1, y, ds);
        const uint32_t p01 = level_pix(img, pitch, x, y1, ds), p11 = level_pix(img, pitch, x1, y1, ds);
        tex[e] = coef_texel(p00, p10, p01, p11);
    }
}

__global__ void reset_counter_kernel(int *counter, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counter[i] = 0;
}

// ---------------------------------------------------------------------------
// level merge (Sec. III-A multi-scale strategy; reading: nearest-neighbour
// plane from the low level with the range recomputed on the full-resolution
// ray, replaced inside the crop by the crop result when that is valid and the
// low result is invalid or at least as far as the crop's nearest plane)
// ---------------------------------------------------------------------------
__global__ void merge_kernel(const MergeDev *__restrict__ ms) {
    const MergeDev &M = ms[blockIdx.y];
    const int n = M.w * M.h;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int i = e % M.w, j = e / M.w;
        const float x = ((float)i - M.cx) / M.fx, y = ((float)j - M.cy) / M.fy;
        float eta;
        const float t = ray_tau(x, y, M.xi, &eta);
        const float rz = eta * t;
        const float ng = eta * fmaf(M.gn[0], x, fmaf(M.gn[1], y, M.gn[2] * t));
        float lam_lo = __builtin_nanf("");
        int64_t src_lo = -1;
        const int il = i / M.ds0, jl = j / M.ds0;
        if (il < M.low_w && jl < M.low_h) {
            const int64_t le = (int64_t)jl * M.low_pitch + il;
            const int k = M.low_index[le];
            if (k >= 0) {
                const bool fr = k < M.low_nf;
                const float th = M.low_theta[k] + M.low_delta[le] * (fr ? M.low_step_f : M.low_step_g);
                if (fr) { if (rz > 0.0f) lam_lo = 1.0f / (th * rz); }
                else if (ng > 0.0f) lam_lo = (M.gd - th) / ng;
                if (!__builtin_isnan(lam_lo)) src_lo = le;
            }
        }
        float lam_c = __builtin_nanf("");
        int64_t src_c = -1;
        if (M.n_levels > 1 && i >= M.crop_x && i < M.crop_x + M.crop_w && j >= M.crop_y && j < M.crop_y + M.crop_h) {
            const int64_t ce = (int64_t)(j - M.crop_y) * M.crop_pitch + (i - M.crop_x);
            const int k = M.crop_index[ce];
            if (k >= 0) {
                const bool fr = k < M.crop_nf;
                const float th = M.crop_theta[k] + M.crop_delta[ce] * (fr ? M.crop_step_f : M.crop_step_g);
                lam_c = fr ? 1.0f / (th * rz) : (M.gd - th) / ng;
                src_c = ce;
            }
        }
        const float z_lo = lam_lo * rz;
        const int64_t o = (int64_t)j * M.out_pitch + i;
        int lev = 255;
        float lam = __builtin_nanf("");
        if (src_c >= 0 && (src_lo < 0 || z_lo >= M.crop_near)) { lev = 1; lam = lam_c; }
        else if (src_lo >= 0) { lev = 0; lam = lam_lo; }
        if (M.depth) M.depth[o] = lam;
        if (M.z) M.z[o] = lam * rz;
        if (M.level) M.level[o] = (uint8_t)lev;
        if (M.index) M.index[o] = lev == 1 ? M.crop_index[src_c] : (lev == 0 ? M.low_index[src_lo] : -1);
        if (M.delta) M.delta[o] = lev == 1 ? M.crop_delta[src_c] : (lev == 0 ? M.low_delta[src_lo] : 0.0f);
        if (M.cost1) M.cost1[o] = lev == 1 ? M.crop_c1[src_c] : (lev == 0 ? M.low_c1[src_lo] : PSW_INF);
        if (M.cost2) M.cost2[o] = lev == 1 ? M.crop_c2[src_c] : (lev == 0 ? M.low_c2[src_lo] : PSW_INF);
    }
}

// Combine the partial states of a tile's plane chunks, in plane order: the
// winner is the lowest-index minimum, the second best the minimum over every
// other plane, and a winner at a chunk edge takes its neighbour's cost from
// the adjacent chunk of the same family.  Soft mode merges running
// log-sum-exp states.
__global__ void chunk_merge_kernel(const JobDev *__restrict__ jobs) {
    const JobDev &J = jobs[blockIdx.y];
    const int nch = J.nch_f + J.nch_g;
    if (nch <= 1) return;
    const int hw = J.window / 2;
    const int iw = J.w - 2 * hw, ih = J.h - 2 * hw;
    if (iw <= 0 || ih <= 0) return;
    const size_t plane = (size_t)J.h * J.w;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < iw * ih; e += gridDim.x * blockDim.x) {
        const int col = hw + e % iw, row = hw + e / iw;
        const float *p = J.part + (size_t)row * J.w + col;
        if (J.mode == 1) {
            float mx = -PSW_INF;
            for (int c = 0; c < nch; ++c) mx = fmaxf(mx, p[(size_t)c * kPartWords * plane]);
            float se = 0.0f, sr = 0.0f;
            if (mx > -PSW_INF) {
                for (int c = 0; c < nch; ++c) {
                    const float m = p[(size_t)c * kPartWords * plane];
                    if (m > -PSW_INF) {
                        const float f = __expf(m - mx);
                        se = fmaf(p[((size_t)c * kPartWords + 1) * plane], f, se);
                        sr = fmaf(p[((size_t)c * kPartWords + 2) * plane], f, sr);
                    }
                }
            }
            finish_soft(J, row, col, mx, se, sr);
            continue;
        }
        float best = PSW_INF;
        int win = -1;
        for (int c = 0; c < nch; ++c) {
            const float v = p[(size_t)c * kPartWords * plane];
            if (v < best) { best = v; win = c; }
        }
        const float x = ((float)col - J.cx) * J.inv_fx;
        if (win < 0) {
            finish_pixel(J, x, row, col, -1, PSW_INF, PSW_INF, PSW_INF, PSW_INF);
            continue;
        }
        const float *q = p + (size_t)win * kPartWords * plane;
        const int k = __float_as_int(q[plane]);
        float c2 = q[2 * plane], cm = q[3 * plane], cp = q[4 * plane];
        for (int c = 0; c < nch; ++c)
            if (c != win) c2 = fminf(c2, p[(size_t)c * kPartWords * plane]);
        int a, b;
        chunk_range(J.n_fronto, J.n_ground, J.nch_f, J.nch_g, win, &a, &b);
        const bool fam = win < J.nch_f;
        if (k == a && win > 0 && ((win - 1 < J.nch_f) == fam))
            cm = p[((size_t)(win - 1) * kPartWords + 6) * plane];
        if (k == b - 1 && win + 1 < nch && ((win + 1 < J.nch_f) == fam))
            cp = p[((size_t)(win + 1) * kPartWords + 5) * plane];
        finish_pixel(J, x, row, col, k, best, c2, cm, cp);
    }
}

// Depth-map filtering (Sec. III-A): best-cost threshold per image part
// (above / below the ground plane's horizon), second-to-best cost ratio,
// then local continuity over a window of the pixels that passed.  16x16
// output pixels per workgroup; the first two tests are evaluated once per
// pixel of the tile and its halo into LDS, then every thread counts its
// consistent neighbours there.
constexpr int kFT = 16;
constexpr int kFMaxHalo = 7;
__global__ __launch_bounds__(256) void filter_kernel(const FilterDev F) {
    __shared__ float d1[(kFT + 2 * kFMaxHalo) * (kFT + 2 * kFMaxHalo)];
    __shared__ uint8_t c1code[(kFT + 2 * kFMaxHalo) * (kFT + 2 * kFMaxHalo)];
    const int hw = F.win / 2;
    const int tw = kFT + 2 * hw;
    const int x0 = blockIdx.x * kFT - hw, y0 = blockIdx.y * kFT - hw;
    const int tid = threadIdx.y * kFT + threadIdx.x;
    for (int e = tid; e < tw * tw; e += kFT * kFT) {
        const int x = x0 + e % tw, y = y0 + e / tw;
        float v = __builtin_nanf("");
        uint8_t code = 255;
        if (x >= 0 && y >= 0 && x < F.w && y < F.h) {
            const int64_t o = (int64_t)y * F.in_pitch + x;
            const float d = F.depth[o];
            if (!__builtin_isnan(d)) {
                const float xn = ((float)x - F.cx) / F.fx, yn = ((float)y - F.cy) / F.fy;
                const float t = ray_tau(xn, yn, F.xi, nullptr);
                const float up = fmaf(F.gn[0], xn, fmaf(F.gn[1], yn, F.gn[2] * t));
                const float alpha = up <= 0.0f ? F.alpha_upper : F.alpha_lower;
                const float a = F.cost1[o], b = F.cost2[o];
                if (a > alpha) code = 1;
                else if (!(b >= F.ratio_min * a)) code = 2;
                else { code = 0; v = d; }
            }
        }
        d1[e] = v;
        c1code[e] = code;
    }
    __syncthreads();
    const int x = blockIdx.x * kFT + threadIdx.x, y = blockIdx.y * kFT + threadIdx.y;
    if (x >= F.w || y >= F.h) return;
    const int le = (threadIdx.y + hw) * tw + threadIdx.x + hw;
    uint8_t code = c1code[le];
    float out = __builtin_nanf("");
    if (code == 0) {
        const float d = d1[le];
        int cons = 0;
        for (int dj = -hw; dj <= hw; ++dj)
            for (int di = -hw; di <= hw; ++di) {
                if (di == 0 && dj == 0) continue;
                const float q = d1[le + dj * tw + di];
                cons += __builtin_fabsf(q - d) < F.gamma ? 1 : 0;   // NaN compares false
            }
        if ((float)cons < F.min_count) code = 3;
        else out = d;
    }
    const int64_t o = (int64_t)y * F.out_pitch + x;
    F.out_depth[o] = out;
    F.code[o] = code;
}

}  // namespace psw

namespace psw {

// blockIdx.y: box; the block's threads cover the box's pixels row by row
__global__ void mask_kernel(MaskDev M) {
    const int b = blockIdx.y;
    const int x0 = M.box[b][0], y0 = M.box[b][1], x1 = M.box[b][2], y1 = M.box[b][3];
    const int bw = x1 - x0, n = bw * (y1 - y0);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int64_t o = (int64_t)(y0 + e / bw) * M.pitch + x0 + e % bw;
        M.depth[o] = __builtin_nanf("");
        if (M.code) M.code[o] = 4;
    }
}

}  // namespace psw

// Scratch of psweep_run_noalloc: job tables, counters, level images,
// textures and level maps of one run, for callers that cannot allocate.
// Every GPU the library runs on holds one copy until the process ends; host
// code uses its device address (from hipGetSymbolAddress, taken once per
// device with that device current), never the array's name.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

extern "C" hipError_t psw_static_scratch(void **ptr, size_t *bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

extern "C" {
const void *psw_filter_kernel() { return (const void *)&psw::filter_kernel; }
const void *psw_mask_kernel() { return (const void *)&psw::mask_kernel; }
const void *psw_chunk_merge_kernel() { return (const void *)&psw::chunk_merge_kernel; }
const void *psw_setup_kernel() { return (const void *)&psw::setup_kernel; }
const void *psw_prep_kernel() { return (const void *)&psw::prep_kernel; }
const void *psw_reset_kernel() { return (const void *)&psw::reset_counter_kernel; }
const void *psw_merge_kernel() { return (const void *)&psw::merge_kernel; }
}
