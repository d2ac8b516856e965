// Soft-argmin backward pass: gradient of L = sum_p g_p rho_hat_p with respect
// to every source image and every source pose (left perturbation
// X_s -> X_s + v + omega x X_s).
//
// Chain per (pixel p, plane k, source s), recomputed from scratch (nothing of
// the forward cost volume is stored):
//   rho_hat = sum_k p_k theta_k(p), p = softmax(-C / T), theta_k(p) the
//   inverse z-depth of the pixel's ray at plane k (a fronto plane's parameter;
//   (n . r) / ((d - h) r_z) for a ground plane n . X = d - h):
//       dL/dC_k = g_p * (-1/T) * p_k * (theta_k(p) - rho_hat_p)
//   C_k = mean of the best K' source costs:   dC/dc_s = 1/K' (chosen s)
//   c_s = (1 - Z) / 2:                        dc/dZ = -1/2
//   Z = sum (a-abar)(b-bbar) / sqrt(s_aa s_bb):
//       dZ/db_q = (a_q - abar)/D - Z (b_q - bbar)/s_bb   for q in the window
// so that, with G = dL/dZ per window, the gradient at sample q is a window
// (transposed box) sum over the pixels whose window holds q:
//   dL/db_q = a_q sum(G/D) - sum(G abar/D) - b_q sum(G Z/s_bb) + sum(G Z bbar/s_bb).
// Each sample's gradient then goes through the bilinear interpolant to the
// four source texels and through the projection to the pose.
//
// Image gradient: a workgroup sweeps one chunk of consecutive planes, and
// between neighbouring planes its tile's footprint in a source moves only by
// the parallax of one plane step.  Each source gets an LDS patch of the source
// image placed over the footprint of the whole chunk (from a few probe
// samples warped at the chunk's first and last plane); the taps land there as
// LDS atomics, and at the end the patch goes to the gradient image with one
// global atomic per touched texel.  A sample whose taps fall outside the
// patch adds them to the gradient image directly.
//
// The patch holds 64-bit fixed-point sums: LDS float atomics are slow next
// to the rest of the loop (about one lane every two clocks per CU), integer
// ones are not.  The workgroup's scale 2^F follows from a bound on every tap:
// with |a_q - abar| <= sqrt(s_aa), |b_q - bbar| <= sqrt(s_bb), |Z| < 1 and
// s_bb above the variance floor, |dL/db_q| <= N max|g| (theta range) /
// (T sqrt(floor)), and a texel takes at most 4 taps of each sample of the
// tile on each plane of the chunk; F leaves that total below 2^61 (times a
// safety factor of 4 for FP32 rounding).  Below a floor of 1/16 grey^2 per
// pixel FP32 cancellation in s_bb can exceed the bound, so there (and for a
// bound that is not finite) every tap goes to the gradient image directly.
// Before the atomics, the taps neighbouring samples share are folded
// together in registers: a lane's bottom taps with the same lane's top taps
// of the next sample row, and a lane's right taps with the left taps of the
// lane to its right, about one atomic per sample at unit scale instead of
// four.
//
// Tile layout: 16 output rows, lane = sample column, 8 waves of 2 output
// rows.  Per output pixel the channels G/D,
// G Z/s_bb and G Z bbar/s_bb of every source and the reference mean abar
// (shared by the sources; sum(G abar/D) is formed from G/D and abar while
// summing) take 28 KB of LDS for two sources.  Every wave owns a contiguous
// block of the tile's sample rows: it warps them into LDS, and after the
// channels are written it walks down the block keeping running sums of the
// channels over the output rows whose window holds the current sample row
// (one row added, one dropped per step).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sweep_common.h"

namespace psw {

// lane l gets v of lane l - 1 (wave_shr:1) or of lane l + 1 (wave_shl:1);
// the lane with no neighbour gets `fill`
__device__ __forceinline__ int lane_shr1_i(int v, int fill) {
    return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int lane_shl1_i(int v, int fill) {
    return __builtin_amdgcn_update_dpp(fill, v, 0x130, 0xf, 0xf, false);
}

// atomic add of v to the float at byte offset off of a buffer (no return)
__device__ __forceinline__ void gadd(__amdgpu_buffer_rsrc_t rs, int off, float v) {
    __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(v, rs, off, 0, 0);
}

// fixed-point atomic add to a 64-bit sum in LDS (no return): v times the
// scale, truncated (|v * scale| < 2^61)
__device__ __forceinline__ void ladd(unsigned long long *p, float v, float scale) {
    __hip_atomic_fetch_add(p, (unsigned long long)(long long)(v * scale), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// minimum over the wave
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

// GI: whether any source's image gradient is wanted (false: pose only).
// GND: whether the level has ground planes (false: fronto planes only, and
// none of the ground family's per-pixel values is kept).
// Tiles of 16 output rows, 8 waves of 2 output rows: two workgroups with
// their patches fill a CU with 16 waves.  The pose-only form has the same
// shape, so that its pose gradient is summed in the same order, bit for bit
// the one of the full form.
template <int WIN, int S, int IMG, bool GI, bool GND>
struct Backward {
    static constexpr int NW = 8, R = 2;
    static constexpr int HW = WIN / 2;
    static constexpr int TXO = kWave - 2 * HW;
    static constexpr int TYO = NW * R;
    static constexpr int T = TYO + 2 * HW;
    static constexpr int RS = (T + NW - 1) / NW;   // contiguous sample rows per wave
    static constexpr int VR = R + 2 * HW;
    static constexpr int NCH = 3;   // channels per source; plus one plane of abar

    // image-gradient patch of each source: PH rows of PW texels (the tile's
    // 64 x T samples, plus the parallax of a chunk's planes and a margin)
    static constexpr int PW = 80, PH = T + 8;

    static constexpr size_t lds_tile() { return (size_t)S * T * kWave * 4; }
    static constexpr size_t lds_patch() { return GI ? (size_t)S * PH * PW * 8 : 0; }
    static constexpr size_t lds_bytes() {
        return lds_tile() + (size_t)(NCH * S + 1) * TYO * kWave * 4 + lds_patch();
    }
    // Occupancy hint: the pose-only form of one or two sources leaves LDS for
    // three workgroups per CU (6 waves per SIMD), which its registers reach
    // when held to 80 (a few spills outside the hottest loops; C4's pose-only
    // backward 0.40 -> 0.36 ms).  Elsewhere LDS holds the CU to two
    // workgroups, and the hint would only add spills (1: no hint); so would it
    // in the ground form, whose per-row values of both families need about
    // 100 registers.
    static constexpr int waves_per_eu() {
        return !GI && !GND && 3 * (lds_bytes() + 1024) <= 160 * 1024 ? 6 : 1;
    }

    __device__ static void run(const JobDev *__restrict__ Jp, const float *__restrict__ gin,
                               const float *__restrict__ rho_hat, const float *__restrict__ lse, int64_t spitch,
                               float *const gsrc[4], double *__restrict__ gpart, char *smem) {
        const JobDev &J = *Jp;
        float *tile = reinterpret_cast<float *>(smem);
        float *chan = tile + (size_t)S * T * kWave;   // [s][c][output row][lane]
        float *abar = chan + (size_t)NCH * S * TYO * kWave;   // [output row][lane]
        // [s][PH][PW] fixed-point sums (GI); 8-byte aligned (the regions
        // before it are multiples of 256 bytes)
        unsigned long long *patch = reinterpret_cast<unsigned long long *>(abar + (size_t)TYO * kWave);
        __shared__ int porg[2 * kMaxSrc];                      // patch origin (column, row) per source
        __shared__ float gmax_w[NW], rng_lo[NW], rng_hi[NW];  // per-wave max |g|, hypothesis range
        const int lane = threadIdx.x & (kWave - 1);
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        const int W = J.w, H = J.h;
        const int sc = blockIdx.x * TXO + lane;
        const int sr0 = blockIdx.y * TYO;
        const int or0 = sr0 + wave * R + HW;
        const float xi = J.xi;
        const float x = ((float)sc - J.cx) * J.inv_fx;
        const float invT = 1.0f / J.temperature;
        const float invN = 1.0f / (float)(WIN * WIN);
        Shifts sh;
        sh.init(lane);

        // sample rows this wave warps (and later scatters): j0 .. j0 + RS - 1
        const int j0 = wave * RS;
        float yw[RS], aw[RS];
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            const int v = sr0 + j0 + i;
            yw[i] = ((float)v - J.cy) * J.inv_fy;
            aw[i] = (sc < W && v < H) ? Texel<IMG>::ref(J.ref, (int64_t)v * J.ref_pitch + sc) - 128.0f : 0.0f;
        }
        // rows this wave runs down (forward recompute of the window sums)
        float av[VR];
#pragma unroll
        for (int m = 0; m < VR; ++m) {
            const int v = sr0 + wave * R + m;
            av[m] = (sc < W && v < H) ? Texel<IMG>::ref(J.ref, (int64_t)v * J.ref_pitch + sc) - 128.0f : 0.0f;
        }
        float mean_a[R], isd_a[R], gp[R], rh[R], ls[R];
        uint32_t ref_ok = 0;
        {
            // reference window sums: exact integers for 8-bit images, FP64 for float images
            using Acc = typename std::conditional<IMG == 1, double, int>::type;
            const float N = (float)(WIN * WIN);
            Acc va = 0, vaa = 0;
#pragma unroll
            for (int m = 0; m < VR; ++m) {
                const Acc a = (Acc)av[m];
                va += a;
                if constexpr (IMG == 1) vaa = fma(a, a, vaa); else vaa += a * a;
                if (m >= WIN) {
                    const Acc ao = (Acc)av[m - WIN];
                    va -= ao;
                    if constexpr (IMG == 1) vaa = fma(-ao, ao, vaa); else vaa -= ao * ao;
                }
                if (m >= WIN - 1) {
                    const int i = m - (WIN - 1);
                    Acc sa, saa;
                    if constexpr (IMG == 1) { sa = wsum_d<WIN>(va, sh); saa = wsum_d<WIN>(vaa, sh); }
                    else { sa = wsum_i<WIN>(va, sh); saa = wsum_i<WIN>(vaa, sh); }
                    float var_a;
                    // the same expressions as the forward sweep, so the costs agree bit for bit
                    if constexpr (IMG == 1) var_a = (float)fma(-sa / (double)(WIN * WIN), sa, saa);
                    else var_a = (float)(WIN * WIN * saa - sa * sa) / N;
                    const int orow = or0 + i;
                    const bool p = lane >= HW && lane < kWave - HW && sc <= W - 1 - HW && orow <= H - 1 - HW;
                    float g = 0.f, r = 0.f, l = -__builtin_huge_valf();
                    if (p) {
                        const int64_t so = (int64_t)orow * spitch + sc;
                        g = gin[so]; r = rho_hat[so]; l = lse[so];
                    }
                    const bool ok = p && var_a > J.var_floor_n && g != 0.0f && l > -__builtin_huge_valf() &&
                                    !__builtin_isnan(r);
                    ref_ok |= (ok ? 1u : 0u) << i;
                    if constexpr (IMG == 1) mean_a[i] = (float)(sa / (double)(WIN * WIN));
                    else mean_a[i] = (float)sa / N;
                    isd_a[i] = ok ? __builtin_amdgcn_rsqf(var_a) : 0.0f;
                    gp[i] = g; rh[i] = r; ls[i] = l;
                }
            }
        }
        if constexpr (GI) {
            float gm = 0.0f;
#pragma unroll
            for (int i = 0; i < R; ++i) gm = fmaxf(gm, __builtin_fabsf(gp[i]));
            gm = -wave_min(-gm);
            if (lane == 0) gmax_w[wave] = gm;
        }
        // the reference means of this wave's output rows, for every plane
#pragma unroll
        for (int i = 0; i < R; ++i) abar[(size_t)(wave * R + i) * kWave + lane] = mean_a[i];
        // pose terms: FP32 per lane over this chunk's planes, FP64 from the
        // wave reduction on
        float acc[S][6];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int a = 0; a < 6; ++a) acc[s][a] = 0.0f;
        const int K = J.best_k;

        // this workgroup's planes: chunk blockIdx.z of gridDim.z even ranges
        // (each plane's contribution is independent given rho_hat and lse)
        const int nchunk = (int)gridDim.z, chunk = (int)blockIdx.z;
        const int nf = J.n_fronto, n_planes = GND ? J.n_fronto + J.n_ground : J.n_fronto;
        const int k_lo = (int)((int64_t)chunk * n_planes / nchunk);
        const int k_hi = (int)((int64_t)(chunk + 1) * n_planes / nchunk);
        if constexpr (GI) {
            for (int t = threadIdx.x; t < S * PH * PW; t += NW * kWave) patch[t] = 0ull;
            {
                // range of the hypothesis values over the tile's pixels (every
                // rho_hat lies within it): the fronto planes' parameters, and
                // each pixel's ground values at the lowest and highest plane
                float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
                for (int k = lane; k < nf; k += kWave) {
                    const float th = J.theta[k];
                    lo = fminf(lo, th); hi = fmaxf(hi, th);
                }
                if constexpr (GND) {
                    const float e0 = 1.0f / (J.gd - J.theta[nf]), e1 = 1.0f / (J.gd - J.theta[n_planes - 1]);
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        if (!((ref_ok >> i) & 1u)) continue;
                        const float yo = ((float)(or0 + i) - J.cy) * J.inv_fy;
                        const float t = ray_tau(x, yo, xi, nullptr);
                        const float g = fmaf(J.gn[0], x, fmaf(J.gn[1], yo, J.gn[2] * t));
                        if (!(g > 0.0f)) continue;
                        const float a = g / t * e0, b = g / t * e1;
                        lo = fminf(lo, fminf(a, b)); hi = fmaxf(hi, fmaxf(a, b));
                    }
                }
                lo = wave_min(lo); hi = -wave_min(-hi);
                if (lane == 0) { rng_lo[wave] = lo; rng_hi[wave] = hi; }
            }
            if (wave == 0) {
                // probes: 3 x 3 sample positions of the tile (without the
                // centre for four sources, so that they fit the wave) at the
                // chunk's first and last plane: 2 NP lanes per source
                constexpr int NP = S <= 3 ? 9 : 8;
                const int s = lane / (2 * NP), p = lane - 2 * NP * (lane / (2 * NP));
                const int q = (p % NP) + (NP == 8 && p % NP >= 4 ? 1 : 0);
                float u = __builtin_nanf(""), v = __builtin_nanf("");
                if (s < S && k_hi > k_lo) {
                    const int k = p < NP ? k_lo : k_hi - 1;
                    const int pc = blockIdx.x * TXO + (q % 3) * (kWave / 2 - 1) + (q % 3) / 2;   // 0, 31, 63
                    const int pr = sr0 + (q / 3) * ((T - 1) / 2) + (q / 3) / 2 * ((T - 1) % 2);
                    const float px_ = ((float)pc - J.cx) * J.inv_fx, py_ = ((float)pr - J.cy) * J.inv_fy;
                    const float t = ray_tau(px_, py_, xi, nullptr);
                    const float *hm = J.htab + (k * S + s) * 9;
                    const float X = fmaf(hm[6], t, fmaf(hm[3], py_, hm[0] * px_));
                    const float Y = fmaf(hm[7], t, fmaf(hm[4], py_, hm[1] * px_));
                    const float Z = fmaf(hm[8], t, fmaf(hm[5], py_, hm[2] * px_));
                    const SrcDev &sd = J.src[s];
                    const float den = fmaf(sd.xi, __builtin_amdgcn_sqrtf(fmaf(X, X, fmaf(Y, Y, Z * Z))), Z);
                    if (t > 0.0f && den > 0.0f) {
                        u = fmaf(X / den, sd.fx, sd.cx);
                        v = fmaf(Y / den, sd.fy, sd.cy);
                    }
                }
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) {
                    const bool mine = s == s2 && u == u && v == v;
                    const float inf = __builtin_huge_valf();
                    const float u0 = wave_min(mine ? u : inf), u1 = -wave_min(mine ? -u : inf);
                    const float v0 = wave_min(mine ? v : inf), v1 = -wave_min(mine ? -v : inf);
                    int ox = 0, oy = 0;
                    if (u0 < inf) {
                        // the taps of the probes span columns floor(u0) .. floor(u1) + 1;
                        // centre that span (clamped to the float range of ints) in the patch
                        const float cu = fminf(fmaxf(0.5f * (u0 + u1), -1.0e9f), 1.0e9f);
                        const float cv = fminf(fmaxf(0.5f * (v0 + v1), -1.0e9f), 1.0e9f);
                        ox = (int)floorf(cu) - PW / 2;
                        oy = (int)floorf(cv) - PH / 2;
                    }
                    if (lane == 0) { porg[2 * s2] = ox; porg[2 * s2 + 1] = oy; }
                }
            }
        }
        float scale = 0.0f;   // 2^F of the fixed-point patch sums; 0: no patch
        if constexpr (GI) {
            __syncthreads();
            float gm = 0.0f, lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                gm = fmaxf(gm, gmax_w[w]);
                lo = fminf(lo, rng_lo[w]); hi = fmaxf(hi, rng_hi[w]);
            }
            const float theta_rng = hi > lo ? hi - lo : 0.0f;
            // bound on the sum of one texel's taps (times 4), then F so that
            // it stays below 2^61
            const float per_tap = (float)(WIN * WIN) * gm * theta_rng /
                                  (J.temperature * __builtin_sqrtf(J.var_floor_n));
            const float total = 4.0f * per_tap * (float)(4 * (k_hi - k_lo) * T * kWave);
            const bool ok = J.var_floor_n >= (float)(WIN * WIN) * 0.0625f && total < 1.0e30f;
            if (ok) {
                int e;
                (void)frexpf(fmaxf(total, 1.0e-30f), &e);   // total < 2^e
                scale = ldexpf(1.0f, min(61 - e, 126));
            }
        }
        // Per plane family, at each sample row: tq = tau where the ray meets
        // the family's planes (NaN elsewhere: the sample is then invalid) and
        // tw = the weight of the translation part of the pose gradient, tau
        // (fronto) or n . (x, y, tau) (ground); at each output row (ground
        // form) hq, with the pixel's hypothesis hq * pf: 1 (fronto) or
        // (n . (x, y, tau)) / tau (ground; NaN where the ray misses it).  Set
        // for the fronto family here, and rebuilt where the plane range
        // crosses into the ground family (wave-uniform).
        float tq[RS], tw[GND ? RS : 1], hq[GND ? R : 1];
        const auto set_family = [&](bool ground) {
#pragma unroll
            for (int i = 0; i < RS; ++i) {
                const float t = ray_tau(x, yw[i], xi, nullptr);
                const float g = ground ? fmaf(J.gn[0], x, fmaf(J.gn[1], yw[i], J.gn[2] * t)) : t;
                tq[i] = g > 0.0f ? t : __builtin_nanf("");
                if constexpr (GND) tw[i] = g;
            }
            if constexpr (GND) {
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const float yo = ((float)(or0 + i) - J.cy) * J.inv_fy;
                    const float t = ray_tau(x, yo, xi, nullptr);
                    const float g = fmaf(J.gn[0], x, fmaf(J.gn[1], yo, J.gn[2] * t));
                    hq[i] = !ground ? 1.0f : g > 0.0f ? g / t : __builtin_nanf("");
                }
            }
        };
        set_family(false);
        bool fam_cur = false;
        for (int k = k_lo; k < k_hi; ++k) {
            const float theta = cptr(J.theta)[k];
            const bool fam = GND && k >= nf;   // ground plane (wave-uniform)
            if (GND && fam != fam_cur) {
                fam_cur = fam;
                set_family(true);
            }
            // the translation part of the pose gradient scales by theta tau
            // (fronto) or (n . (x, y, tau)) / (d - h) (ground): per-plane factor
            const float pf = fam ? 1.0f / (J.gd - theta) : theta;
            // ---- forward recompute: warped rows of every source into LDS ----
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const PSW_CONST float *hm = cptr(J.htab) + (k * S + s) * 9;
                const float h1x = hm[0], h1y = hm[1], h1z = hm[2], h2x = hm[3], h2y = hm[4], h2z = hm[5];
                const float h3x = hm[6], h3y = hm[7], h3z = hm[8];
                const SrcDev &sd = J.src[s];
                const uint32_t row_bytes = (uint32_t)sd.w * Texel<IMG>::bytes;
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)sd.tex, (short)0, (int)(row_bytes * (uint32_t)sd.h), 0x00020000);
                const float px = h1x * x, py = h1y * x, pz = h1z * x;
#pragma unroll
                for (int i = 0; i < RS; ++i) {
                    const int j = j0 + i;
                    if (j >= T) break;   // the last wave's block is shorter
                    const float X = fmaf(h3x, tq[i], fmaf(h2x, yw[i], px));
                    const float Y = fmaf(h3y, tq[i], fmaf(h2y, yw[i], py));
                    const float Z = fmaf(h3z, tq[i], fmaf(h2z, yw[i], pz));
                    const float m = __builtin_amdgcn_sqrtf(fmaf(X, X, fmaf(Y, Y, Z * Z)));
                    const float den = fmaf(sd.xi, m, Z);
                    const float inv = __builtin_amdgcn_rcpf(den);
                    const float u = fmaf(X * inv, sd.fx, sd.cx);
                    const float v = fmaf(Y * inv, sd.fy, sd.cy);
                    // the sweep's validity test (bit patterns: 0 <= u <= wm1)
                    const bool ok = (den > 0.0f) & (__float_as_uint(u) <= __float_as_uint(sd.wm1)) &
                                    (__float_as_uint(v) <= __float_as_uint(sd.hm1));
                    const uint32_t off = __umul24((uint32_t)(int)v, row_bytes) + (uint32_t)(int)u * Texel<IMG>::bytes;
                    const float al = __builtin_amdgcn_fractf(u), be = __builtin_amdgcn_fractf(v);
                    const float b = Texel<IMG>::sample(rs, off, al, be);
                    tile[((size_t)s * T + j) * kWave + lane] = ok ? b : -0.0f;
                }
            }
            __syncthreads();

            // ---- per output pixel: costs, softmax weight, window channels ----
            {
                float vb[S], vbb[S], vab[S];
                int last_bad[S];
#pragma unroll
                for (int s = 0; s < S; ++s) { vb[s] = 0.f; vbb[s] = 0.f; vab[s] = 0.f; last_bad[s] = -1000; }
#pragma unroll
                for (int m = 0; m < VR; ++m) {
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const float *cs = tile + ((size_t)s * T + wave * R) * kWave + lane;
                        const float b = cs[(size_t)m * kWave];
                        last_bad[s] = is_neg_zero(b) ? m : last_bad[s];
                        vb[s] += b; vbb[s] = fmaf(b, b, vbb[s]); vab[s] = fmaf(av[m], b, vab[s]);
                        if (m >= WIN) {
                            const float bo = cs[(size_t)(m - WIN) * kWave];
                            vb[s] -= bo; vbb[s] = fmaf(-bo, bo, vbb[s]); vab[s] = fmaf(-av[m - WIN], bo, vab[s]);
                        }
                    }
                    if (m >= WIN - 1) {
                        const int i = m - (WIN - 1);
                        float c4[4] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf(),
                                       __builtin_huge_valf()};
                        float zs[S], rsb[S], hbs[S];
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            const float hb = wsum<WIN>(vb[s], sh), hbb = wsum<WIN>(vbb[s], sh);
                            const float hab = wsum<WIN>(vab[s], sh);
                            const uint64_t bm = __builtin_amdgcn_ballot_w64(last_bad[s] > m - WIN);
                            const bool bad = bm != 0 && __builtin_amdgcn_inverse_ballot_w64(dilate<WIN>(bm));
                            const float cov = fmaf(-mean_a[i], hb, hab);
                            const float varb = fmaf(-hb * invN, hb, hbb);
                            const float rv = __builtin_amdgcn_rsqf(varb);
                            const float zn = cov * isd_a[i] * rv;
                            const float c = fmaf(-0.5f, __builtin_amdgcn_fmed3f(zn, -1.0f, 1.0f), 0.5f);
                            c4[s] = (!bad && varb > J.var_floor_n) ? c : __builtin_huge_valf();
                            zs[s] = zn; rsb[s] = rv; hbs[s] = hb;
                        }
                        const float C = aggregate<S>(c4, K);
                        const bool live = ((ref_ok >> i) & 1u) && C < __builtin_huge_valf();
                        // dL/dC_k, then the share of every chosen source
                        float dC = 0.0f;
                        if (live) {
                            const float pk = __expf(-C * invT - ls[i]);
                            const float th = GND ? hq[i] * pf : theta;   // the pixel's hypothesis
                            dC = gp[i] * (-invT) * pk * (th - rh[i]);
                        }
                        int nvalid = 0;
#pragma unroll
                        for (int s = 0; s < S; ++s) nvalid += c4[s] < __builtin_huge_valf() ? 1 : 0;
                        const int kk = K < nvalid ? K : nvalid;
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            int rank = 0;
#pragma unroll
                            for (int t = 0; t < S; ++t)
                                rank += (c4[t] < c4[s] || (c4[t] == c4[s] && t < s)) ? 1 : 0;
                            const bool chosen = live && c4[s] < __builtin_huge_valf() && rank < kk &&
                                                __builtin_fabsf(zs[s]) < 1.0f;
                            const float G = -0.5f * dC / (float)kk;   // dL/dZ of a chosen window
                            const float invD = isd_a[i] * rsb[s];
                            const float varb_inv = rsb[s] * rsb[s];
                            const float bbar = hbs[s] * invN;
                            // unusable windows hold NaN/inf statistics: select, never multiply by 0
                            float *ch = chan + (((size_t)s * NCH) * TYO + wave * R + i) * kWave + lane;
                            ch[0] = chosen ? G * invD : 0.0f;
                            ch[(size_t)TYO * kWave] = chosen ? G * zs[s] * varb_inv : 0.0f;
                            ch[(size_t)2 * TYO * kWave] = chosen ? G * zs[s] * bbar * varb_inv : 0.0f;
                        }
                    }
                }
            }
            __syncthreads();

            // ---- transposed window sums at every sample, then scatter ----
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const PSW_CONST float *hm = cptr(J.htab) + (k * S + s) * 9;
                const float h1x = hm[0], h1y = hm[1], h1z = hm[2], h2x = hm[3], h2y = hm[4], h2z = hm[5];
                const float h3x = hm[6], h3y = hm[7], h3z = hm[8];
                const SrcDev &sd = J.src[s];
                const uint32_t row_bytes = (uint32_t)sd.w * Texel<IMG>::bytes;
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)sd.tex, (short)0, (int)(row_bytes * (uint32_t)sd.h), 0x00020000);
                const float px = h1x * x, py = h1y * x, pz = h1z * x;
                float *gimg = GI ? gsrc[s] : nullptr;
                // the gradient image as a buffer: taps are byte offsets into it
                const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
                    gimg, (short)0, (int)((uint32_t)sd.w * (uint32_t)sd.h * 4u), 0x00020000);
                const uint32_t grow = (uint32_t)sd.w * 4u;
                // running sums of the channels over the output rows whose
                // window holds sample row j: rows [j - 2 HW, j] within the tile
                const float *chs = chan + ((size_t)s * NCH) * TYO * kWave + lane;
                const float *abs_ = abar + lane;
                float rA = 0.f, rB = 0.f, rC = 0.f, rE = 0.f;
                for (int r = j0 - 1 - 2 * HW < 0 ? 0 : j0 - 1 - 2 * HW; r <= j0 - 1 && r < TYO; ++r) {
                    const float *ch = chs + (size_t)r * kWave;
                    const float a = ch[0];
                    rA += a; rB = fmaf(a, abs_[(size_t)r * kWave], rB);
                    rC += ch[(size_t)TYO * kWave]; rE += ch[(size_t)2 * TYO * kWave];
                }
                // pose terms of this plane in FP32 (at most RS per lane), then FP64
                float ps[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                int pox = 0, poy = 0;
                unsigned long long *pat = patch + (size_t)s * PH * PW;
                if (GI) { pox = porg[2 * s]; poy = porg[2 * s + 1]; }
                if (GI && scale == 0.0f) { pox = -(1 << 30); poy = -(1 << 30); }   // every tap direct
                // patch taps carried down from the previous sample row of this
                // lane: patch index (-1: none) and value of (v1, i0) and (v1, i1)
                int ca0 = -1, ca1 = -1;
                float cv0 = 0.f, cv1 = 0.f;
#pragma unroll
                for (int i = 0; i < RS; ++i) {
                    const int j = j0 + i;
                    if (j >= T) break;
                    if (j < TYO) {
                        const float *ch = chs + (size_t)j * kWave;
                        const float a = ch[0];
                        rA += a; rB = fmaf(a, abs_[(size_t)j * kWave], rB);
                        rC += ch[(size_t)TYO * kWave]; rE += ch[(size_t)2 * TYO * kWave];
                    }
                    if (j - 2 * HW - 1 >= 0) {
                        const int jo = j - 2 * HW - 1;
                        const float *ch = chs + (size_t)jo * kWave;
                        const float a = ch[0];
                        rA -= a; rB = fmaf(-a, abs_[(size_t)jo * kWave], rB);
                        rC -= ch[(size_t)TYO * kWave]; rE -= ch[(size_t)2 * TYO * kWave];
                    }
                    const float sA = wsum<WIN>(rA, sh), sB = wsum<WIN>(rB, sh);
                    const float sC = wsum<WIN>(rC, sh), sE = wsum<WIN>(rE, sh);
                    const float b = tile[((size_t)s * T + j) * kWave + lane];
                    const float gb = fmaf(aw[i], sA, -sB) + fmaf(-b, sC, sE);
                    // this sample's patch taps (v0, i0), (v0, i1), (v1, i0), (v1, i1):
                    // patch index (-1: none) and gradient
                    int a00 = -1, a10 = -1, a01 = -1, a11 = -1;
                    float c00 = 0.f, c10 = 0.f, c01 = 0.f, c11 = 0.f;
                    if ((gb != 0.0f) & !is_neg_zero(b)) {
                        // recompute the warp of this sample with its derivatives
                        const float X = fmaf(h3x, tq[i], fmaf(h2x, yw[i], px));
                        const float Y = fmaf(h3y, tq[i], fmaf(h2y, yw[i], py));
                        const float Z = fmaf(h3z, tq[i], fmaf(h2z, yw[i], pz));
                        const float m = __builtin_amdgcn_sqrtf(fmaf(X, X, fmaf(Y, Y, Z * Z)));
                        const float den = fmaf(sd.xi, m, Z);
                        const float inv = __builtin_amdgcn_rcpf(den);
                        const float u = fmaf(X * inv, sd.fx, sd.cx);
                        const float v = fmaf(Y * inv, sd.fy, sd.cy);
                        const int i0 = (int)u, v0 = (int)v;
                        const int i1 = i0 + 1 < sd.w ? i0 + 1 : sd.w - 1;
                        const int v1 = v0 + 1 < sd.h ? v0 + 1 : sd.h - 1;
                        const float al = u - (float)i0, be = v - (float)v0;
                        float dbu, dbv;
                        Texel<IMG>::slope(rs, __umul24((uint32_t)v0, row_bytes) + (uint32_t)i0 * Texel<IMG>::bytes, al, be,
                                          &dbu, &dbv);
                        if (GI && gimg) {
                            c00 = gb * (1.0f - al) * (1.0f - be); c10 = gb * al * (1.0f - be);
                            c01 = gb * (1.0f - al) * be; c11 = gb * al * be;
                            const int pi = i0 - pox, pj = v0 - poy;
                            if ((uint32_t)pi < (uint32_t)(PW - 1) && (uint32_t)pj < (uint32_t)(PH - 1)) {
                                a00 = pj * PW + pi;
                                a10 = a00 + (i1 - i0);
                                a01 = a00 + (v1 - v0) * PW;
                                a11 = a01 + (i1 - i0);
                            } else {
                                gadd(grs, (int)(__umul24((uint32_t)v0, grow) + (uint32_t)i0 * 4u), c00);
                                gadd(grs, (int)(__umul24((uint32_t)v0, grow) + (uint32_t)i1 * 4u), c10);
                                gadd(grs, (int)(__umul24((uint32_t)v1, grow) + (uint32_t)i0 * 4u), c01);
                                gadd(grs, (int)(__umul24((uint32_t)v1, grow) + (uint32_t)i1 * 4u), c11);
                            }
                        }
                        // (X, Y, Z) = H (x, y, tau) is the source point P divided by
                        // sigma = 1 / (theta tau) (fronto planes; for a ground plane
                        // sigma = (d - h) / (n . (x, y, tau))).  With
                        // xu = X / den, yv = Y / den, Au = dbu fx / den,
                        // Av = dbv fy / den, Q = Au xu + Av yv and
                        // Qm = xi Q / |(X, Y, Z)|, the sample's gradient along P is
                        // (gb / sigma) g' with g' = (Au - X Qm, Av - Y Qm, -(Q + Z Qm)),
                        // so the translation part is gb g' / sigma and the
                        // rotation part P x (gb / sigma) g' = gb (X, Y, Z) x g'.
                        const float xu = X * inv, yv = Y * inv;
                        const float Au = dbu * (sd.fx * inv), Av = dbv * (sd.fy * inv);
                        const float Q = fmaf(Au, xu, Av * yv);
                        const float Qm = Q * (sd.xi * __builtin_amdgcn_rcpf(m));
                        const float e0 = fmaf(-X, Qm, Au), e1 = fmaf(-Y, Qm, Av), e2 = -fmaf(Z, Qm, Q);
                        const float gt = gb * (GND ? tw[i] : tq[i]);   // times pf once per plane
                        ps[0] = fmaf(gt, e0, ps[0]);
                        ps[1] = fmaf(gt, e1, ps[1]);
                        ps[2] = fmaf(gt, e2, ps[2]);
                        ps[3] = fmaf(gb, fmaf(Y, e2, -Z * e1), ps[3]);
                        ps[4] = fmaf(gb, fmaf(Z, e0, -X * e2), ps[4]);
                        ps[5] = fmaf(gb, fmaf(X, e1, -Y * e0), ps[5]);
                    }
                    if (GI && gimg) {
                        // (a) this lane's bottom taps of the previous row are this
                        // row's top taps (same texel row and columns)
                        if (ca0 >= 0 && ca0 == a00) {
                            c00 += cv0;
                            c10 += cv1;   // ca1 is a10, or was handed on (cv1 = 0)
                        } else {
                            if (ca0 >= 0) ladd(pat + ca0, cv0, scale);
                            if (ca1 >= 0) ladd(pat + ca1, cv1, scale);
                        }
                        // (b) the left lane's right taps are this lane's left taps;
                        // the left lane then drops them
                        const int l10 = lane_shr1_i(a10, -1);
                        const float l10v = shr1(c10), l11v = shr1(c11);
                        if (a00 >= 0 && l10 == a00) { c00 += l10v; c01 += l11v; }
                        const bool handed = a10 >= 0 && lane_shl1_i(a00, -1) == a10;
                        if (a00 >= 0) ladd(pat + a00, c00, scale);
                        if (a10 >= 0 && !handed) ladd(pat + a10, c10, scale);
                        ca0 = a01; cv0 = c01;
                        ca1 = handed ? -1 : a11; cv1 = handed ? 0.f : c11;
                    }
                }
                if (GI && gimg) {
                    if (ca0 >= 0) ladd(pat + ca0, cv0, scale);
                    if (ca1 >= 0) ladd(pat + ca1, cv1, scale);
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) acc[s][a] = fmaf(ps[a], pf, acc[s][a]);
#pragma unroll
                for (int a = 3; a < 6; ++a) acc[s][a] += ps[a];
            }
            __syncthreads();
        }
        // ---- image gradient: the patches to the gradient images, one atomic
        // per touched texel (a texel is touched only by in-image taps) ----
        if constexpr (GI) {
            __syncthreads();
#pragma unroll
            for (int s = 0; s < S; ++s) {
                float *gimg = gsrc[s];
                if (!gimg) continue;
                const SrcDev &sd = J.src[s];
                const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
                    gimg, (short)0, (int)((uint32_t)sd.w * (uint32_t)sd.h * 4u), 0x00020000);
                const int pox = porg[2 * s], poy = porg[2 * s + 1];
                const unsigned long long *pat = patch + (size_t)s * PH * PW;
                const float inv_scale = scale > 0.0f ? 1.0f / scale : 0.0f;   // a power of two
                for (int t = threadIdx.x; t < PH * PW; t += NW * kWave) {
                    const long long q = (long long)pat[t];
                    if (q != 0) {
                        const int pj = t / PW, pi = t - pj * PW;
                        gadd(grs, ((poy + pj) * sd.w + pox + pi) * 4, (float)q * inv_scale);
                    }
                }
            }
        }
        // ---- pose gradient: wave reduction, then the workgroup's partial sum
        // (one row of gpart per workgroup; a second kernel adds the rows in a
        // fixed order).  The LDS tile is free: the plane loop ended on a barrier.
        double *red = reinterpret_cast<double *>(smem);   // [wave][6 S]
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                double v = (double)acc[s][a];
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
                if (lane == 0) red[wave * 6 * S + s * 6 + a] = v;
            }
        __syncthreads();
        if (wave == 0 && lane < 6 * S) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) t += red[w * 6 * S + lane];
            const int64_t wg = (int64_t)blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
            gpart[wg * 6 * S + lane] = t;
        }
    }
};

template <int WIN, int S, int IMG, bool GI, bool GND>
__global__ __launch_bounds__((Backward<WIN, S, IMG, GI, GND>::NW * kWave))
__attribute__((amdgpu_waves_per_eu(Backward<WIN, S, IMG, GI, GND>::waves_per_eu()))) void backward_kernel(const JobDev *__restrict__ job, const float *__restrict__ gin,
                                                        const float *__restrict__ rho, const float *__restrict__ lse,
                                                        int64_t spitch, float *g0, float *g1, float *g2, float *g3,
                                                        double *gpart) {
    extern __shared__ __attribute__((aligned(16))) char smem[];   // after the static LDS, 16-byte aligned
    float *gs[4] = {g0, g1, g2, g3};
    Backward<WIN, S, IMG, GI, GND>::run(job, gin, rho, lse, spitch, gs, gpart, smem);
}

}  // namespace psw
