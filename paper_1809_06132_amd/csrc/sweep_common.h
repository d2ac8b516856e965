#pragma once
// Sweep kernel templates of the fisheye plane-sweep library (gfx950).
//
// Method (Cui et al., Sec. III-A; camera model Sec. III-C Eq. (1)): every
// reference pixel's ray is cut with each plane hypothesis, the point is
// projected into each source with the unified model and sampled bilinearly;
// the cost of a (pixel, plane, source) is (1 - ZNCC) / 2 over a square
// window; the best few source costs are averaged; the best plane per pixel
// wins, refined by a parabola through its neighbours.
//
// Layout on the chip (one workgroup = NW waves = one tile):
//   * a wave owns 64 consecutive sample columns (lane = column) and R output
//     rows; the tile's 64 - (W-1) output columns are the lanes whose whole
//     window lies inside the 64;
//   * per plane, the NW waves warp the tile's NW*R + W - 1 sample rows of
//     every source (rows interleaved across waves) into LDS; the LDS tile is
//     double-buffered, so the warp of the next plane overlaps the rows of
//     this one and one barrier per plane suffices;
//   * each wave then runs down its R + W - 1 rows with per-lane running
//     vertical sums of b, b^2 and a*b (one set per source, in registers) and
//     forms horizontal window sums across lanes with ds_bpermute/DPP shifts;
//   * ZNCC, best-K aggregation and the winner-take-all (or soft-argmin)
//     state of the wave's R pixels per lane stay in registers for the whole
//     sweep.  Nothing per-plane ever leaves the chip.
// Invalid samples (plane missed, point behind the model's viewpoint, outside
// the source) are staged as -0.0: they add nothing to the sums and a lane
// keeps the row of its last invalid sample, so a window is unusable when
// that row is inside it (vertical), dilated across lanes on the wave's
// 64-bit ballot (horizontal).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psweep_internal.h"

namespace psw {

#define PSW_INF __builtin_huge_valf()

// ---------------------------------------------------------------------------
// staging precision of warped samples (centred: b - 128)
// ---------------------------------------------------------------------------
// put() stages a usable sample and never yields -0.0, the marker of an
// unusable one (bad()).
template <int STORE> struct Stage;
template <> struct Stage<0> {
    using T = float;
    // a bilinear blend of integer coefficients is never -0.0 in FP32
    static __device__ __forceinline__ T put(float v) { return v; }
    static __device__ __forceinline__ T bad() { return -0.0f; }
    static __device__ __forceinline__ float get(T v) { return v; }
};
template <> struct Stage<1> {
    using T = _Float16;
    // a tiny negative rounding residue (|v| < 2^-25) rounds to -0.0 in FP16;
    // + 0 turns it into +0 and leaves every other value as it is
    static __device__ __forceinline__ T put(float v) { return (_Float16)v + (_Float16)0.0f; }
    static __device__ __forceinline__ T bad() { return (_Float16)-0.0f; }
    // one conversion, kept apart from the FMAs that use it: folded into them
    // as mixed-precision FMAs, the row loop schedules with stalls on the
    // window sums' lane shifts (about 10% slower than the BF16 form)
    static __device__ __forceinline__ float get(T v) {
        float f = (float)v;
        asm("" : "+v"(f));
        return f;
    }
};
template <> struct Stage<2> {
    using T = uint16_t;   // bfloat16 bits, round to nearest even
    // BF16 keeps FP32's exponent range: a nonzero value stays nonzero
    static __device__ __forceinline__ T put(float v) {
        uint32_t u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
    static __device__ __forceinline__ T bad() { return (uint16_t)0x8000u; }
    static __device__ __forceinline__ float get(T v) { return __uint_as_float(((uint32_t)v) << 16); }
};

#define PSW_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ PSW_GLOBAL T *gptr(T *p) { return (PSW_GLOBAL T *)p; }
template <typename T> __device__ __forceinline__ const PSW_GLOBAL T *gptr(const T *p) { return (const PSW_GLOBAL T *)p; }
// read-only tables written before the launch: scalar loads
#define PSW_CONST __attribute__((address_space(4)))
template <typename T> __device__ __forceinline__ const PSW_CONST T *cptr(const T *p) { return (const PSW_CONST T *)p; }

__device__ __forceinline__ bool is_neg_zero(float v) { return __float_as_uint(v) == 0x80000000u; }
// Lane selects on a scalar lane mask (lane in m ? t : f), one v_cndmask
// each.  Written as instructions because the compiler turns a group of
// selects on one condition into an exec-masked branch with register copies.
__device__ __forceinline__ float vsel(uint64_t m, float t, float f) {
    return __builtin_amdgcn_inverse_ballot_w64(m) ? t : f;
}
__device__ __forceinline__ int vsel_i(uint64_t m, int t, int f) {
    return __builtin_amdgcn_inverse_ballot_w64(m) ? t : f;
}
// lanes where a < b (ordered), as a scalar lane mask
__device__ __forceinline__ uint64_t lanes_lt(float a, float b) {
    return __builtin_amdgcn_fcmpf(a, b, 4 /* ordered less than */);
}
// the wave's lanes holding -0.0, as one compare into a scalar register pair
// (a ballot of is_neg_zero would first be widened into a vector register)
__device__ __forceinline__ uint64_t neg_zero_mask(float v) {
    return __builtin_amdgcn_uicmp(__float_as_uint(v), 0x80000000u, 32 /* equal */);
}

// value of v held by lane (lane - d); lanes wrap (only interior lanes are used)
__device__ __forceinline__ float lane_from(float v, int addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ int lane_from_i(int v, int addr) { return __builtin_amdgcn_ds_bpermute(addr, v); }
// lane l gets v[l-1], lane 0 gets 0 (bound_ctrl: a lane with no source lane
// reads 0, so no register has to be cleared first)
__device__ __forceinline__ float shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ int shr1_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }

// Byte addresses for ds_bpermute: lane (lane - d) for the shifts a window
// sum of side WIN needs (d = 2, 4 for the block sums, then the final
// placements, which are all in [-7, 7]).
struct Shifts {
    int a[16];   // a[d + 7] = ((lane - d) & 63) * 4
    __device__ __forceinline__ void init(int lane) {
#pragma unroll
        for (int d = -7; d <= 8; ++d) a[d + 7] = ((lane - d) & 63) << 2;
    }
    __device__ __forceinline__ int at(int d) const { return a[d + 7]; }
};

// Sum of v over lanes [l - h, l + h] (W = 2h + 1), built from power-of-two
// block sums B_n[l] = sum v[l-n+1 .. l] placed at the window's right end.
template <int WIN, typename T, typename SHR1, typename FROM>
__device__ __forceinline__ T window_sum(T v, const Shifts &sh, SHR1 s1, FROM from) {
    // Windows 5, 7 and 9: the same operand pairs added in the same order as
    // the general form below (so the same result bit for bit on the interior
    // lanes: a + b == b + a), with two lane permutes fewer.  A block needed at
    // one place only is added from its two halves there, shifts by one lane
    // are DPP operands, and B4 takes B2[l-2] through two of them (lanes 0 and 1
    // then get 0 instead of a wrapped value; no output reads them).  The
    // ds_bpermute round trips sit on the critical path of the row loop: two
    // fewer per sum took C2's kernel from 0.99 to 0.85 ms, although the DPP
    // form of B4 costs two more VALU instructions.
    if constexpr (WIN == 5) {
        const T b2 = v + s1(v);
        return (from(b2, sh.at(-2)) + b2) + from(v, sh.at(2));          // B4[l+2] + v[l-2]
    } else if constexpr (WIN == 7) {
        const T b2 = v + s1(v);
        const T b4 = b2 + s1(s1(b2));
        return (from(b4, sh.at(-3)) + s1(b2)) + from(v, sh.at(3));      // B4[l+3] + B2[l-1] + v[l-3]
    } else if constexpr (WIN == 9) {
        const T b2 = v + s1(v);
        const T b4 = b2 + s1(s1(b2));
        return (from(b4, sh.at(-4)) + b4) + from(v, sh.at(4));          // B8[l+4] + v[l-4]
    }
    // Other windows: blocks B_n[l] = sum v[l-n+1 .. l] placed at the window's
    // right end; B4 takes B2[l-2] through two DPP shifts (lanes 0 and 1 get 0,
    // and no output reads B4 or B8 there), a placement one lane to the left is
    // a DPP shift, the others are lane permutes.
    constexpr int h = WIN / 2;
    T b1 = v;
    T b2 = v + s1(v);
    T b4 = (WIN >= 5) ? b2 + s1(s1(b2)) : b2;
    T b8 = (WIN >= 9) ? b4 + from(b4, sh.at(4)) : b4;
    // the first block placed starts the sum (0 + x is not free: it turns -0
    // into +0, so the compiler keeps the add)
    T acc;
    bool first = true;
    int pos = h;   // right end of the uncovered part, relative to l
    auto put = [&](T blk) {
        acc = first ? blk : acc + blk;
        first = false;
    };
    // the block's value at lane l + p
    auto at_offset = [&](T blk, int p) { return p == 0 ? blk : (p == -1 ? s1(blk) : from(blk, sh.at(-p))); };
    if (WIN & 8) { put(at_offset(b8, pos)); pos -= 8; }
    if (WIN & 4) { put(at_offset(b4, pos)); pos -= 4; }
    if (WIN & 2) { put(at_offset(b2, pos)); pos -= 2; }
    if (WIN & 1) { put(at_offset(b1, pos)); }
    return acc;
}
template <int WIN>
__device__ __forceinline__ float wsum(float v, const Shifts &sh) {
    return window_sum<WIN>(v, sh, shr1, lane_from);
}
template <int WIN>
__device__ __forceinline__ int wsum_i(int v, const Shifts &sh) {
    return window_sum<WIN>(v, sh, shr1_i, lane_from_i);
}
// doubles move between lanes as two 32-bit halves
__device__ __forceinline__ double shr1_d(double v) {
    return __hiloint2double(shr1_i(__double2hiint(v)), shr1_i(__double2loint(v)));
}
__device__ __forceinline__ double lane_from_d(double v, int addr) {
    return __hiloint2double(lane_from_i(__double2hiint(v), addr), lane_from_i(__double2loint(v), addr));
}
template <int WIN>
__device__ __forceinline__ double wsum_d(double v, const Shifts &sh) {
    return window_sum<WIN>(v, sh, shr1_d, lane_from_d);
}

// Bilinear sampling of a source texture at texel (iu, iv) with weights
// (al, be), value centred (minus 128), and its slopes along u and v.
// IMG 0: a texel holds the bilinear coefficients of its 2x2 cell as four
// FP16 integers, c0 = p00 - 128, c1 = p10 - p00, c2 = p01 - p00,
// c3 = p11 - p10 - p01 + p00 (exact: |c| <= 510), so that
// b = c0 + al c1 + be (c2 + al c3), three mixed-precision FMAs with FP32
// rounding; IMG 1: four floats p00, p10, p01, p11.  Reads outside the buffer
// return 0.
// Indexed buffer loads (the buffer's stride in the resource, the element
// index in a register): address = base + index * stride.  An index at or past
// the resource's record count reads 0.
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));
__device__ U32x2 buffer_load_index_b64(__amdgpu_buffer_rsrc_t rsrc, int index, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");
__device__ U32x4 buffer_load_index_b128(__amdgpu_buffer_rsrc_t rsrc, int index, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");
struct Half2 { _Float16 lo, hi; };
__device__ __forceinline__ float half_lo(uint32_t w) { return (float)__builtin_bit_cast(Half2, w).lo; }
__device__ __forceinline__ float half_hi(uint32_t w) { return (float)__builtin_bit_cast(Half2, w).hi; }
template <int IMG>
struct Texel;
template <>
struct Texel<0> {
    static constexpr uint32_t bytes = 8;
    typedef unsigned int Raw __attribute__((ext_vector_type(2)));
    __device__ static Raw raw(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        return __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    }
    // texel `index` of a resource whose stride is `bytes`
    __device__ static Raw at(__amdgpu_buffer_rsrc_t rs, uint32_t index) {
        return buffer_load_index_b64(rs, (int)index, 0, 0, 0);
    }
    __device__ static float blend(Raw q, float al, float be) {
        const float t = fmaf(al, half_hi(q[1]), half_lo(q[1]));
        return fmaf(al, half_hi(q[0]), fmaf(be, t, half_lo(q[0])));
    }
    __device__ static float sample(__amdgpu_buffer_rsrc_t rs, uint32_t off, float al, float be) {
        return blend(raw(rs, off), al, be);
    }
    __device__ static void slope(__amdgpu_buffer_rsrc_t rs, uint32_t off, float al, float be, float *du, float *dv) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
        *du = fmaf(be, half_hi(q[1]), half_hi(q[0]));
        *dv = fmaf(al, half_hi(q[1]), half_lo(q[1]));
    }
    __device__ static float ref(const uint8_t *p, int64_t i) { return (float)gptr(p)[i]; }
};
template <>
struct Texel<1> {
    static constexpr uint32_t bytes = 16;
    struct Quad { float p00, p10, p01, p11; };
    typedef unsigned int Raw __attribute__((ext_vector_type(4)));
    __device__ static Raw raw(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        return __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    }
    // texel `index` of a resource whose stride is `bytes`
    __device__ static Raw at(__amdgpu_buffer_rsrc_t rs, uint32_t index) {
        return buffer_load_index_b128(rs, (int)index, 0, 0, 0);
    }
    __device__ static Quad load(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        const Raw q = raw(rs, off);
        return {__uint_as_float(q[0]), __uint_as_float(q[1]), __uint_as_float(q[2]), __uint_as_float(q[3])};
    }
    __device__ static float blend(Raw r, float al, float be) {
        const Quad q = {__uint_as_float(r[0]), __uint_as_float(r[1]), __uint_as_float(r[2]), __uint_as_float(r[3])};
        const float top = fmaf(al, q.p10 - q.p00, q.p00);
        const float bot = fmaf(al, q.p11 - q.p01, q.p01);
        return fmaf(be, bot - top, top - 128.0f);
    }
    __device__ static float sample(__amdgpu_buffer_rsrc_t rs, uint32_t off, float al, float be) {
        return blend(raw(rs, off), al, be);
    }
    __device__ static void slope(__amdgpu_buffer_rsrc_t rs, uint32_t off, float al, float be, float *du, float *dv) {
        const Quad q = load(rs, off);
        *du = fmaf(be, q.p11 - q.p01, (1.0f - be) * (q.p10 - q.p00));
        *dv = fmaf(al, q.p11 - q.p10, (1.0f - al) * (q.p01 - q.p00));
    }
    __device__ static float ref(const uint8_t *p, int64_t i) {
        return gptr(reinterpret_cast<const float *>(p))[i];
    }
};

// lanes whose window [l-h, l+h] contains a lane with bit set in m (scalar
// work): the reach grows 0 -> 1 -> 3 -> 7 by shifts of 1, 2, 4, capped at h,
// so h = 4 takes three steps instead of four
template <int WIN>
__device__ __forceinline__ uint64_t dilate(uint64_t m) {
    uint64_t d = m;
    int reach = 0;
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const int k = (reach + 1 < WIN / 2 - reach) ? reach + 1 : WIN / 2 - reach;
        if (k > 0) { d |= (d << k) | (d >> k); reach += k; }
    }
    return d;
}

// Scale-free ray (x, y, tau) of a normalized point: Eq. (1) gives the unit
// ray eta * (x, y, 1 - xi / eta); tau = 1 - xi / eta = (sq - xi q) / (xi + sq)
// with q = x^2 + y^2, sq = sqrt(1 + (1 - xi^2) q).  Also eta.
__device__ __forceinline__ float ray_tau(float x, float y, float xi, float *eta) {
    float q = fmaf(x, x, y * y);
    float sq = __builtin_amdgcn_sqrtf(fmaf(1.0f - xi * xi, q, 1.0f));
    if (eta) *eta = (xi + sq) / (q + 1.0f);
    return (sq - xi * q) / (xi + sq);
}

// Mean of the K smallest valid costs (invalid = +inf) of S <= 4 sources,
// summed in ascending order; +inf if none is valid.
template <int S>
__device__ __forceinline__ float aggregate(const float c[4], int K) {
    float m0, m1, m2, m3;
    if (S == 1) {
        return c[0];
    } else if (S == 2) {
        m0 = fminf(c[0], c[1]); m1 = fmaxf(c[0], c[1]); m2 = PSW_INF; m3 = PSW_INF;
    } else if (S == 3) {
        m0 = __builtin_fminf(c[0], __builtin_fminf(c[1], c[2]));
        m1 = __builtin_amdgcn_fmed3f(c[0], c[1], c[2]);
        m2 = __builtin_fmaxf(c[0], __builtin_fmaxf(c[1], c[2]));
        m3 = PSW_INF;
    } else {
        const float a0 = fminf(c[0], c[1]), a1 = fmaxf(c[0], c[1]);
        const float a2 = fminf(c[2], c[3]), a3 = fmaxf(c[2], c[3]);
        const float t0 = fmaxf(a0, a2), t1 = fminf(a1, a3);
        m0 = fminf(a0, a2); m3 = fmaxf(a1, a3);
        m1 = fminf(t0, t1); m2 = fmaxf(t0, t1);
    }
    // branch-free for a runtime K: the valid ones among the K best are a
    // prefix of the sorted costs, so the weight is that of the last one
    // added; an invalid best gives +inf by itself (inf + 0 and inf * w)
    float acc = m0, w = 1.0f;
    { const bool f = (K >= 2) & (m1 < PSW_INF); acc += f ? m1 : 0.f; w = f ? 0.5f : w; }
    if (S >= 3) { const bool f = (K >= 3) & (m2 < PSW_INF); acc += f ? m2 : 0.f; w = f ? (1.0f / 3.0f) : w; }
    if (S >= 4) { const bool f = (K >= 4) & (m3 < PSW_INF); acc += f ? m3 : 0.f; w = f ? 0.25f : w; }
    return acc * w;
}

// Mean of the two smallest valid costs (the smallest alone if only one is
// valid), +inf if none is: aggregate<S>(c, 2) with fewer instructions and
// the same result (the same sum, times 0.5 or 1).
template <int S>
__device__ __forceinline__ float aggregate2(const float c[4]) {
    float m0, m1;
    if (S == 1) {
        return c[0];
    } else if (S == 2) {
        m0 = fminf(c[0], c[1]); m1 = fmaxf(c[0], c[1]);
    } else if (S == 3) {
        m0 = __builtin_fminf(c[0], __builtin_fminf(c[1], c[2]));
        m1 = __builtin_amdgcn_fmed3f(c[0], c[1], c[2]);
    } else {
        const float a0 = fminf(c[0], c[1]), a1 = fmaxf(c[0], c[1]);
        const float a2 = fminf(c[2], c[3]), a3 = fmaxf(c[2], c[3]);
        m0 = fminf(a0, a2);
        m1 = fminf(fmaxf(a0, a2), fminf(a1, a3));
    }
    return m1 < PSW_INF ? (m0 + m1) * 0.5f : m0;
}

// Winner-take-all result of one pixel: parabolic subpixel step through the
// winner and its two same-family neighbours (missing neighbour = +inf), the
// refined plane parameter, the range along the Eq. (1) ray and z.
__device__ __forceinline__ void finish_pixel(const JobDev &J, float x, int orow, int col, int k, float c1, float c2,
                                             float cm, float cp) {
    const int64_t o = (int64_t)orow * J.out_pitch + col;
    float dl = 0.0f, depth = __builtin_nanf(""), zz = __builtin_nanf("");
    if (k >= 0) {
        if (cm < PSW_INF && cp < PSW_INF) {
            const float den = cm - 2.0f * c1 + cp;
            if (den > 0.0f) dl = __builtin_amdgcn_fmed3f((cm - cp) / (2.0f * den), -0.5f, 0.5f);
        }
        const bool fr = k < J.n_fronto;
        const float th = cptr(J.theta)[k] + dl * (fr ? J.step_f : J.step_g);
        const float y = ((float)orow - J.cy) * J.inv_fy;
        float eta;
        const float t = ray_tau(x, y, J.xi, &eta);
        const float rz = eta * t;
        if (fr) {
            depth = 1.0f / (th * rz);
        } else {
            const float nr = eta * fmaf(J.gn[0], x, fmaf(J.gn[1], y, J.gn[2] * t));
            depth = (J.gd - th) / nr;
        }
        zz = depth * rz;
    }
    if (J.index) gptr(J.index)[o] = k;
    if (J.delta) gptr(J.delta)[o] = dl;
    if (J.cost1) gptr(J.cost1)[o] = k >= 0 ? c1 : PSW_INF;
    if (J.cost2) gptr(J.cost2)[o] = k >= 0 ? c2 : PSW_INF;
    if (J.depth) gptr(J.depth)[o] = depth;
    if (J.z) gptr(J.z)[o] = zz;
    if (J.level_id) gptr(J.level_id)[o] = k >= 0 ? 0 : 255;
}

__device__ __forceinline__ void finish_soft(const JobDev &J, int orow, int col, float mx, float se, float sr) {
    const bool ok = mx > -PSW_INF;
    const int64_t so = (int64_t)orow * J.soft_pitch + col;
    gptr(J.soft_rho)[so] = ok ? sr / se : __builtin_nanf("");
    gptr(J.soft_lse)[so] = ok ? mx + __logf(se) : -PSW_INF;
}

// ---------------------------------------------------------------------------
// the sweep of one tile
// ---------------------------------------------------------------------------
template <int WIN, int R, int NW, int S, int STORE, bool SOFT, int IMG = 0, bool K2 = false, bool VOL = false>
struct Tile {
    static constexpr int HW = WIN / 2;
    static constexpr int TXO = kWave - 2 * HW;       // output columns per tile
    static constexpr int TYO = NW * R;               // output rows per tile
    static constexpr int T = TYO + 2 * HW;           // sample rows per tile
    static constexpr int NWR = (T + NW - 1) / NW;    // warp rows per wave
    // rows whose texel loads the warp issues together: all of them where the
    // registers they hold (two per load in flight) keep the occupancy that
    // LDS allows (three or four sources, 8-bit images, FP32 staging, windows
    // up to 9), else two
    static constexpr int LG = (IMG == 0 && STORE == 0 && S >= 3 && R == 4 && WIN <= 9) ? NWR : 2;
    // texel loads by index into a texel-strided resource (no address shift,
    // one instruction per sample less), except for the one tile that it takes
    // past 128 VGPRs (two sources, window 9, 8-bit images, FP32 staging on the
    // default tile: 129, i.e. three waves per SIMD), which keeps byte offsets
    static constexpr bool kIndexed = !(IMG == 0 && STORE == 0 && S == 2 && WIN == 9 && R == 4 && NW == 4);
    static constexpr int VR = R + 2 * HW;            // rows each wave runs down
    using St = Stage<STORE>;
    using ST = typename St::T;

    static constexpr size_t lds_bytes() { return 2 * (size_t)S * T * kWave * sizeof(ST); }

    // lane = threadIdx.x % 64 (passed in: see the persistent kernel)
    __device__ static void run(const JobDev *__restrict__ Jp, int tile_x, int tile_y, int chunk, char *smem,
                               const int lane) {
        const JobDev &J = *Jp;
        ST *tile = reinterpret_cast<ST *>(smem);
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        __builtin_assume(wave >= 0 && wave < NW);   // lets the warp rows' loads issue as one batch
        const int W = J.w, H = J.h;
        const int sc = tile_x * TXO + lane;            // sample column of this lane
        const int sr0 = tile_y * TYO;                  // first sample row of the tile
        const int or0 = sr0 + wave * R + HW;           // first output row of this wave
        const float xi = J.xi;
        const float x = ((float)sc - J.cx) * J.inv_fx;

        Shifts sh;
        sh.init(lane);

        // --- plane-independent per-lane state -------------------------------
        float yw[NWR];   // wave-uniform
#pragma unroll
        for (int i = 0; i < NWR; ++i) {
            const int v = sr0 + wave + NW * i;
            yw[i] = ((float)v - J.cy) * J.inv_fy;
        }
        float av[VR];          // centred reference intensities of the rows this wave runs down
        {
            const bool col_in = sc < W;
#pragma unroll
            for (int m = 0; m < VR; ++m) {
                const int v = sr0 + wave * R + m;
                av[m] = (col_in && v < H) ? Texel<IMG>::ref(J.ref, (int64_t)v * J.ref_pitch + sc) - 128.0f : 0.0f;
            }
        }
        float mean_a[R], nis_a[R];   // reference window mean and -1/(2 sqrt(S_aa))
        uint32_t pos_ok = 0, ref_ok = 0;
        if constexpr (IMG == 1) {
            // float images: window sums in FP64 (products of floats are exact)
            const double N = (double)(WIN * WIN);
            double va = 0.0, vaa = 0.0;
#pragma unroll
            for (int m = 0; m < VR; ++m) {
                const double a = av[m];
                va += a; vaa = fma(a, a, vaa);
                if (m >= WIN) {
                    const double ao = av[m - WIN];
                    va -= ao; vaa = fma(-ao, ao, vaa);
                }
                if (m >= WIN - 1) {
                    const int i = m - (WIN - 1);
                    const double sa = wsum_d<WIN>(va, sh), saa = wsum_d<WIN>(vaa, sh);
                    const float var_a = (float)fma(-sa / N, sa, saa);   // sum of squared deviations
                    const int orow = or0 + i;
                    const bool p = lane >= HW && lane < kWave - HW && sc <= W - 1 - HW && orow <= H - 1 - HW;
                    const bool r = p && var_a > J.var_floor_n;
                    pos_ok |= (p ? 1u : 0u) << i;
                    ref_ok |= (r ? 1u : 0u) << i;
                    mean_a[i] = (float)(sa / N);
                    nis_a[i] = r ? -0.5f * __builtin_amdgcn_rsqf(var_a) : 0.0f;
                }
            }
        } else {
            // 8-bit images: exact in integers (|a'| <= 128, window sums of a'^2 < 2^24)
            const float N = (float)(WIN * WIN);
            int va = 0, vaa = 0;
#pragma unroll
            for (int m = 0; m < VR; ++m) {
                const int a = (int)av[m];
                va += a; vaa += a * a;
                if (m >= WIN) {
                    const int ao = (int)av[m - WIN];
                    va -= ao; vaa -= ao * ao;
                }
                if (m >= WIN - 1) {
                    const int i = m - (WIN - 1);
                    const int sa = wsum_i<WIN>(va, sh), saa = wsum_i<WIN>(vaa, sh);
                    const int nvar = WIN * WIN * saa - sa * sa;          // N^2 * variance, exact
                    const float var_a = (float)nvar / N;                 // sum of squared deviations
                    const int orow = or0 + i;
                    const bool p = lane >= HW && lane < kWave - HW && sc <= W - 1 - HW && orow <= H - 1 - HW;
                    const bool r = p && var_a > J.var_floor_n;
                    pos_ok |= (p ? 1u : 0u) << i;
                    ref_ok |= (r ? 1u : 0u) << i;
                    mean_a[i] = (float)sa / N;
                    nis_a[i] = r ? -0.5f * __builtin_amdgcn_rsqf(var_a) : 0.0f;
                }
            }
        }

        // lanes of each output row without a usable reference window (outside
        // the image, or textureless): a scalar mask, ORed into every source's
        // unusable-window mask
        // (Four sources leave no scalar registers for these masks: there the
        // test is a select on the aggregated cost, and the previous plane's
        // win is a compare of the winning index.)
        constexpr bool kScalarMasks = S <= 3;
        uint64_t ref_bad[R];
#pragma unroll
        for (int i = 0; i < R; ++i) ref_bad[i] = kScalarMasks ? __builtin_amdgcn_ballot_w64(!((ref_ok >> i) & 1u)) : 0;

        // --- per-pixel sweep state -------------------------------------------
        float c1[R], c2[R], cm[R], cp[R], cprev[R];
        int kb[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            c1[i] = PSW_INF; c2[i] = PSW_INF; cm[i] = PSW_INF; cp[i] = PSW_INF; cprev[i] = PSW_INF;
            kb[i] = -1;
        }
        const float invT = SOFT ? 1.0f / J.temperature : 0.0f;
        // soft state reuses c1 (running max of -C/T), c2 (sum exp), cm (sum exp * rho)
        if (SOFT) {
#pragma unroll
            for (int i = 0; i < R; ++i) { c1[i] = -PSW_INF; c2[i] = 0.0f; cm[i] = 0.0f; }
        }

        const int K = J.best_k;
        const float inf = PSW_INF;
        const float invN = 1.0f / (float)(WIN * WIN);
        const float vfn = J.var_floor_n;

        // planes this workgroup sweeps: every plane, or one chunk of them
        const int nch = J.nch_f + J.nch_g;
        int k_lo[2] = {0, J.n_fronto}, k_hi[2] = {J.n_fronto, J.n_fronto + J.n_ground};
        if (nch > 1) {
            int a, b;
            chunk_range(J.n_fronto, J.n_ground, J.nch_f, J.nch_g, chunk, &a, &b);
            const int f = a >= J.n_fronto ? 1 : 0;
            k_lo[f] = a; k_hi[f] = b;
            k_lo[1 - f] = 0; k_hi[1 - f] = 0;
        }
        float cfirst[R];
#pragma unroll
        for (int i = 0; i < R; ++i) cfirst[i] = PSW_INF;

        for (int fam = 0; fam < 2; ++fam) {
            const int np = k_hi[fam] - k_lo[fam];
            if (np <= 0) continue;
            const int k0 = k_lo[fam];
            // family ray parameter: tau where the family's planes are hit in
            // front of the camera, NaN elsewhere (NaN fails every later test)
            float tf[NWR];
#pragma unroll
            for (int i = 0; i < NWR; ++i) {
                float t = ray_tau(x, yw[i], xi, nullptr);
                const float g = fam ? fmaf(J.gn[0], x, fmaf(J.gn[1], yw[i], J.gn[2] * t)) : t;
                tf[i] = g > 0.0f ? t : __builtin_nanf("");
            }
            // A wave whose output pixels all lack a usable reference window or
            // a ray that meets this family's planes has nothing to compute: its
            // costs would all be unusable and leave its state as it is.  It
            // still warps its share of the tile's rows for the others, unless
            // no wave of the tile is live, when the tile skips the family.
            bool live = false;
            // soft mode, ground planes: a plane's value at an output pixel is
            // the inverse z-depth of the ray's cut, (n . r) / ((d - h) r_z) =
            // gfac / (d - h) with gfac = (n . (x, y, tau)) / tau
            float gfac[SOFT ? R : 1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const float yo = ((float)(or0 + i) - J.cy) * J.inv_fy;
                const float t = ray_tau(x, yo, xi, nullptr);
                const float g = fam ? fmaf(J.gn[0], x, fmaf(J.gn[1], yo, J.gn[2] * t)) : t;
                live |= ((ref_ok >> i) & 1u) && g > 0.0f;
                if constexpr (SOFT) gfac[i] = fam ? g / t : 1.0f;
            }
            const bool wave_live = __builtin_amdgcn_ballot_w64(live) != 0;
            if (!__syncthreads_or(wave_live)) continue;
            uint64_t won[R];
#pragma unroll
            for (int i = 0; i < R; ++i) { cprev[i] = PSW_INF; won[i] = 0; }

            // double-buffered tile: the warp of plane k + 1 goes to the other
            // buffer while the rows of plane k are read; one barrier per plane
            auto warp_plane = [&](const int k, ST *buf) {
                // ---- warp all sources' sample rows of this plane into LDS ----
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const PSW_CONST float *hm = cptr(J.htab) + (k * S + s) * 9;
                    const float h1x = hm[0], h1y = hm[1], h1z = hm[2];
                    const float h2x = hm[3], h2y = hm[4], h2z = hm[5];
                    const float h3x = hm[6], h3y = hm[7], h3z = hm[8];
                    const float sxi = J.src[s].xi, sfx = J.src[s].fx, sfy = J.src[s].fy;
                    const float scx = J.src[s].cx, scy = J.src[s].cy;
                    const float wm1 = J.src[s].wm1, hm1 = J.src[s].hm1;
                    const uint32_t sw = (uint32_t)J.src[s].w;
                    const uint32_t row_bytes = sw * Texel<IMG>::bytes;
                    // the texture as an array of texels (stride Texel::bytes,
                    // w h records), or as bytes: reads past it return 0, so
                    // even the address of an invalid sample cannot fault
                    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                        (void *)J.src[s].tex, (short)(kIndexed ? Texel<IMG>::bytes : 0),
                        (int)(kIndexed ? sw * (uint32_t)J.src[s].h : row_bytes * (uint32_t)J.src[s].h), 0x00020000);
                    const float px = h1x * x, py = h1y * x, pz = h1z * x;
                    ST *dst = buf + (size_t)s * T * kWave + lane;
                    // the texel loads of LG rows are issued before the first of
                    // them is blended, so that they overlap instead of each
                    // waiting in turn
#pragma unroll
                    for (int i0 = 0; i0 < NWR; i0 += LG) {
                        float al[LG], be[LG];
                        bool ok[LG], have[LG];
                        typename Texel<IMG>::Raw q[LG];
#pragma unroll
                        for (int d = 0; d < LG; ++d) {
                            const int i = i0 + d;
                            // the last row may be past the tile
                            have[d] = i < NWR && !(i == NWR - 1 && wave + NW * i >= T);
                            if (!have[d]) continue;
                            const float X = fmaf(h3x, tf[i], fmaf(h2x, yw[i], px));
                            const float Y = fmaf(h3y, tf[i], fmaf(h2y, yw[i], py));
                            const float Z = fmaf(h3z, tf[i], fmaf(h2z, yw[i], pz));
                            const float m = __builtin_amdgcn_sqrtf(fmaf(X, X, fmaf(Y, Y, Z * Z)));
                            const float den = fmaf(sxi, m, Z);
                            const float inv = __builtin_amdgcn_rcpf(den);
                            const float u = fmaf(X * inv, sfx, scx);
                            const float v = fmaf(Y * inv, sfy, scy);
                            // 0 <= u <= wm1 as one unsigned compare of the bit patterns
                            // (non-negative floats order like their bits; negative
                            // values and NaN compare above wm1; u is never -0 here)
                            ok[d] = (den > 0.0f) & (__float_as_uint(u) <= __float_as_uint(wm1)) &
                                    (__float_as_uint(v) <= __float_as_uint(hm1));
                            al[d] = __builtin_amdgcn_fractf(u);
                            be[d] = __builtin_amdgcn_fractf(v);
                            if constexpr (kIndexed)
                                q[d] = Texel<IMG>::at(rs, __umul24((uint32_t)(int)v, sw) + (uint32_t)(int)u);
                            else
                                q[d] = Texel<IMG>::raw(rs, __umul24((uint32_t)(int)v, row_bytes) +
                                                               (uint32_t)(int)u * Texel<IMG>::bytes);
                        }
#pragma unroll
                        for (int d = 0; d < LG; ++d) {
                            if (!have[d]) continue;
                            const float b = Texel<IMG>::blend(q[d], al[d], be[d]);
                            dst[(size_t)(wave + NW * (i0 + d)) * kWave] = ok[d] ? St::put(b) : St::bad();
                        }
                    }
                }
            };
            warp_plane(k0, tile);
            __syncthreads();
            for (int kk = 0; kk < np; ++kk) {
                const int k = k0 + kk;
                // soft mode: plane k's value at a pixel is gfac * pf, pf = theta_k
                // (fronto, gfac = 1) or 1 / (d - h_k) (ground) (wave-uniform)
                const float pf = !SOFT ? 0.0f : fam ? 1.0f / (J.gd - cptr(J.theta)[k]) : cptr(J.theta)[k];
                const ST *cur = tile + (size_t)(kk & 1) * S * T * kWave;
                if (kk + 1 < np) warp_plane(k + 1, tile + (size_t)((kk + 1) & 1) * S * T * kWave);
                if (wave_live) {
                // ---- run down the rows: vertical sums, then window sums ----
                // Unusable samples: the compare of each row gives the wave's
                // 64-bit mask of them (scalar registers); the rows of an output
                // row's window are ORed on the scalar unit.  With R <= WIN the
                // windows of the wave's R output rows share the rows R-1 ..
                // WIN-1 (core); output i adds the rows i .. R-2 above them
                // (head) and WIN .. i+WIN-1 below them (tail).
                float vb[S], vbb[S], vab[S];
                uint64_t rbad[S][VR], head[S][R], core[S], tail[S];
#pragma unroll
                for (int s = 0; s < S; ++s) { vb[s] = 0.f; vbb[s] = 0.f; vab[s] = 0.f; core[s] = 0; tail[s] = 0; }
                const ST *col = cur + (size_t)(wave * R) * kWave + lane;
#pragma unroll
                for (int m = 0; m < VR; ++m) {
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const ST *cs = col + (size_t)s * T * kWave;
                        const float b = St::get(cs[(size_t)m * kWave]);
                        rbad[s][m] = neg_zero_mask(b);
                        if (R <= WIN) {
                            if (m == R - 2) {
                                head[s][m] = rbad[s][m];
#pragma unroll
                                for (int r = R - 3; r >= 0; --r) head[s][r] = rbad[s][r] | head[s][r + 1];
                            }
                            if (m == R - 1) core[s] = rbad[s][m];
                            else if (m > R - 1 && m < WIN) core[s] |= rbad[s][m];
                            if (m == WIN) tail[s] = rbad[s][m];
                            else if (m > WIN) tail[s] |= rbad[s][m];
                        }
                        if (m == 0) {   // start the sums with the first row (no 0 + x)
                            vb[s] = b; vbb[s] = b * b; vab[s] = av[m] * b;
                        } else {
                            vb[s] += b;
                            vbb[s] = fmaf(b, b, vbb[s]);
                            vab[s] = fmaf(av[m], b, vab[s]);
                        }
                        if (m >= WIN) {
                            const float bo = St::get(cs[(size_t)(m - WIN) * kWave]);
                            vb[s] -= bo;
                            vbb[s] = fmaf(-bo, bo, vbb[s]);
                            vab[s] = fmaf(-av[m - WIN], bo, vab[s]);
                        }
                    }
                    if (m >= WIN - 1) {
                        const int i = m - (WIN - 1);
                        float cs4[4];
#pragma unroll
                        for (int s = 0; s < 4; ++s) cs4[s] = PSW_INF;
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            const float hb = wsum<WIN>(vb[s], sh);
                            const float hbb = wsum<WIN>(vbb[s], sh);
                            const float hab = wsum<WIN>(vab[s], sh);
                            // scalar work only, no branch: an empty mask dilates to 0
                            uint64_t bm;
                            if (R <= WIN) {
                                bm = core[s];
                                if (i <= R - 2) bm |= head[s][i];
                                if (i >= 1) bm |= tail[s];
                            } else {
                                bm = rbad[s][i];
#pragma unroll
                                for (int r = 1; r < WIN; ++r) bm |= rbad[s][i + r];
                            }
                            if (kScalarMasks) bm = dilate<WIN>(bm) | ref_bad[i];
                            else bm = dilate<WIN>(bm);
                            const bool bad = __builtin_amdgcn_inverse_ballot_w64(bm);
                            const float cov = fmaf(-mean_a[i], hb, hab);
                            const float varb = fmaf(-hb * invN, hb, hbb);
                            // (1 - ZNCC) / 2 with ZNCC = cov / sqrt(S_aa S_bb), clamped to [0, 1]
                            const float c = __builtin_amdgcn_fmed3f(
                                fmaf(cov * nis_a[i], __builtin_amdgcn_rsqf(varb), 0.5f), 0.0f, 1.0f);
                            cs4[s] = (!bad && varb > vfn) ? c : PSW_INF;   // the reference window's test is in bm
                        }
                        // mean of the best K (K2: K is 2, the short form with the
                        // same result)
                        float C = K2 ? aggregate2<S>(cs4) : aggregate<S>(cs4, K);
                        if (!kScalarMasks) C = ((ref_ok >> i) & 1u) ? C : PSW_INF;
                        if (kk == 0) cfirst[i] = C;
                        if (VOL && ((pos_ok >> i) & 1u))
                            gptr(J.volume)[((int64_t)k * H + or0 + i) * W + sc] = C;
                        if (!SOFT) {
                            // branch-free: with c1 <= c2 (no NaN reaches here) the new
                            // second best is med3(c1, c2, C) and the new best min(c1, C);
                            // won[i] (a lane mask) says the best is the previous plane,
                            // whose neighbour cost on the right is this plane's
                            const uint64_t nb = lanes_lt(C, c1[i]);
                            const uint64_t prev_won =
                                kScalarMasks ? won[i] : (kk > 0 ? __builtin_amdgcn_ballot_w64(kb[i] == k - 1) : 0);
                            cp[i] = vsel(nb, inf, vsel(prev_won, C, cp[i]));
                            c2[i] = __builtin_amdgcn_fmed3f(c1[i], c2[i], C);
                            cm[i] = vsel(nb, cprev[i], cm[i]);
                            kb[i] = vsel_i(nb, k, kb[i]);
                            c1[i] = fminf(c1[i], C);
                            cprev[i] = C;
                            if (kScalarMasks) won[i] = nb;
                        } else if (C < PSW_INF) {
                            const float l = -C * invT;
                            const float nm = fmaxf(c1[i], l);
                            const float ea = __expf(c1[i] - nm), eb = __expf(l - nm);
                            const float th = gfac[i] * pf;
                            c2[i] = fmaf(c2[i], ea, eb);
                            cm[i] = fmaf(cm[i], ea, eb * th);
                            c1[i] = nm;
                        }
                    }
                }
                }   // wave_live
                __syncthreads();
            }
        }

        // --- epilogue --------------------------------------------------------
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (!((pos_ok >> i) & 1u)) continue;
            const int orow = or0 + i;
            if (nch > 1) {
                // partial state of this chunk, combined by chunk_merge_kernel
                const size_t plane = (size_t)H * W;
                float *pp = J.part + (size_t)chunk * kPartWords * plane + (size_t)orow * W + sc;
                PSW_GLOBAL float *g = gptr(pp);
                g[0] = c1[i];
                g[plane] = SOFT ? c2[i] : __int_as_float(kb[i]);
                g[2 * plane] = SOFT ? cm[i] : c2[i];
                if (!SOFT) {
                    g[3 * plane] = cm[i];
                    g[4 * plane] = cp[i];
                    g[5 * plane] = cfirst[i];
                    g[6 * plane] = cprev[i];
                }
                continue;
            }
            if (SOFT) finish_soft(J, orow, sc, c1[i], c2[i], cm[i]);
            else finish_pixel(J, x, orow, sc, kb[i], c1[i], c2[i], cm[i], cp[i]);
        }
    }
};

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
// One grid per (frame, level), one workgroup per (chunk, tile) item, in the
// job's item order (largest first).
// FP16 staging on the default tile (4 waves of 4 rows) with windows up to 9:
// held to 128 VGPRs, four waves per SIMD, without spills (left alone, the
// compiler takes a register more for some and settles for three waves).
// The other kernels keep the compiler's choice: a cap changes their schedule
// for the worse (measured on the persistent launch).
template <int WIN, int R, int NW, int S, int STORE>
constexpr int sweep_waves_per_eu() { return R == 4 && NW == 4 && WIN <= 9 && STORE == 1 ? 4 : 1; }

template <int WIN, int R, int NW, int S, int STORE, bool SOFT, int IMG = 0>
__global__ __launch_bounds__(kWave *NW) __attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu<WIN, R, NW, S, STORE>())))
void sweep_grid_kernel(const JobDev *__restrict__ job) {
    extern __shared__ __attribute__((aligned(16))) char smem[];   // after the static LDS, 16-byte aligned
    const int tx = job->tiles_x;
    // Blocks go to the eight XCDs round-robin (block b to XCD b % 8), and
    // every XCD has a queue of items (its share of the tile rows, so that
    // its L2 holds the source texels those rows reach; largest item first).
    // A block takes the next item of its XCD's queue, or of the next queue
    // that has items left when its own is empty, so the XCDs finish together.
    // There are as many blocks as items: every block takes exactly one.
    __shared__ int item_s;
    if (threadIdx.x == 0) {
        const PSW_CONST int32_t *hd = cptr(job->order);
        int it = -1;
        for (int a = 0; a < kQueues && it < 0; ++a) {
            const int q = (blockIdx.x + a) & (kQueues - 1);
            const int lo = hd[q], n = hd[q + 1] - lo;
            if (n <= 0) continue;
            const int c = atomicAdd(job->queue_ctr + q, 1);
            if (c < n) it = hd[kQueueHead + lo + c];
        }
        item_s = it;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_s);   // uniform: the tile stays scalar
    if (item < 0) return;
    const int ntile = tx * job->tiles_y;
    const int chunk = item / ntile;
    const int tile = item - chunk * ntile;
    const int tile_y = tile / tx;
    const int r = tile - tile_y * tx;
    // the mean of the best two sources (the usual setting) has a short form;
    // the cost volume output has kernels of its own
    const int lane = threadIdx.x & (kWave - 1);
    if (!SOFT && job->volume) {
        if (S >= 2 && job->best_k == 2)
            Tile<WIN, R, NW, S, STORE, SOFT, IMG, true, true>::run(job, r % tx, tile_y, chunk, smem, lane);
        else
            Tile<WIN, R, NW, S, STORE, SOFT, IMG, false, true>::run(job, r % tx, tile_y, chunk, smem, lane);
    } else if (!SOFT && S >= 2 && job->best_k == 2) {
        Tile<WIN, R, NW, S, STORE, SOFT, IMG, true>::run(job, r % tx, tile_y, chunk, smem, lane);
    } else {
        Tile<WIN, R, NW, S, STORE, SOFT, IMG>::run(job, r % tx, tile_y, chunk, smem, lane);
    }
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
// threadIdx.x % 64 from an instruction the compiler may not hoist or merge
__device__ __forceinline__ int opaque_lane() {
    int lane;
    asm volatile("v_and_b32 %0, 63, %1" : "=v"(lane) : "v"((int)threadIdx.x));
    return lane;
}

// One persistent launch for every (frame, level, tile) of a run: workgroups
// take (chunk, tile) items job after job, from their XCD's queue of the job
// (or the next queue with items left), until every job is exhausted; every
// workgroup then leaves.
template <int R, int NW, int S, int STORE>
__global__ __launch_bounds__(kWave *NW) void sweep_persistent_kernel(const JobDev *__restrict__ jobs, int n_jobs,
                                                                     int n_items, int *counter) {
    extern __shared__ __attribute__((aligned(16))) char smem[];   // after the static LDS, 16-byte aligned
    __shared__ int item_s, job_s;
    (void)n_items;
    (void)counter;
    int j = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int it = -1;
            while (j < n_jobs && it < 0) {
                const PSW_CONST int32_t *hd = cptr(jobs[j].order);
                for (int a = 0; a < kQueues && it < 0; ++a) {
                    const int q = (blockIdx.x + a) & (kQueues - 1);
                    const int lo = hd[q], n = hd[q + 1] - lo;
                    if (n <= 0) continue;
                    const int c = atomicAdd(jobs[j].queue_ctr + q, 1);
                    if (c < n) it = hd[kQueueHead + lo + c];
                }
                if (it < 0) ++j;
            }
            item_s = it;
            job_s = j;
        }
        __syncthreads();
        // the same for every lane: uniform, so the tile's values stay scalar
        const int t = __builtin_amdgcn_readfirstlane(item_s);
        j = __builtin_amdgcn_readfirstlane(job_s);
        __syncthreads();
        if (t < 0) break;
        const JobDev *J = jobs + j;
        const int ntile = J->tiles_x * J->tiles_y;
        const int tile = t % ntile, chunk = t / ntile;
        const int tx = tile % J->tiles_x, ty = tile / J->tiles_x;
        // The compiler hoists the per-lane constants of both windows' sweeps
        // (lane-shift addresses and the like) out of this loop, where they stay
        // live across it: about 17 VGPRs more than either sweep needs.  An
        // opaque lane index in each branch prevents that.  It is used where it
        // brings the kernel to 4 waves per SIMD (three sources FP32: 129 -> 125
        // VGPRs; four sources FP16: 145 -> 128, BF16: 144 -> 126).  Elsewhere
        // it gains no wave, and for four sources FP32 (146 -> 129, still 3
        // waves) the batch ran 25 % slower with it.
        constexpr bool opaque = (S == 3 && STORE == 0) || (S == 4 && STORE != 0);
        const bool k2 = S >= 2 && J->best_k == 2;
        if (J->window == 7) {
            if (k2) Tile<7, R, NW, S, STORE, false, 0, true>::run(J, tx, ty, chunk, smem, opaque ? opaque_lane() : lane_id());
            else Tile<7, R, NW, S, STORE, false>::run(J, tx, ty, chunk, smem, opaque ? opaque_lane() : lane_id());
        } else {
            if (k2) Tile<9, R, NW, S, STORE, false, 0, true>::run(J, tx, ty, chunk, smem, opaque ? opaque_lane() : lane_id());
            else Tile<9, R, NW, S, STORE, false>::run(J, tx, ty, chunk, smem, opaque ? opaque_lane() : lane_id());
        }
    }
}

}  // namespace psw
