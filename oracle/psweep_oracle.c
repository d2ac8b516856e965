/*
 * FP64 CPU oracle for fisheye plane-sweep stereo.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library: plain, slow, direct evaluation of the definitions.
 *
 * What it computes, and where each step comes from (Cui et al., "Real-Time
 * Dense Mapping for Self-Driving Vehicles using Fisheye Cameras"):
 *   - Unified camera model, back-projection of a pixel to a unit ray: Eq. (1),
 *     Sec. III-C; projection of a point: the model of Mei and Rives that
 *     Sec. III-C cites (the inverse of Eq. (1)).
 *   - Plane-sweep stereo with fronto-parallel and ground-parallel planes, each
 *     plane giving one depth hypothesis per pixel: Sec. III-A.
 *   - Matching cost: negative ZNCC over a local window, cost 1 for ZNCC -1 and
 *     cost 0 for ZNCC +1, i.e. (1 - ZNCC) / 2: Sec. III-A.
 *   - Best depth candidate per pixel and first/second best costs: Sec. III-A
 *     (depth map filtering paragraph).
 *   - Two resolution levels (downsampled full view + full-resolution centre
 *     crop) and their fusion: Sec. III-A (multi-scale strategy).
 * Points the paper leaves open are fixed by the readings documented beside
 * the code (pixel centres, plane spacing, aggregation over sources, subpixel
 * parabola, downsampling filter, level merge, soft-argmin).
 *
 * Every window is evaluated from scratch: each sample is warped on its own and
 * the ZNCC is the textbook two-pass formula (means first, then centred sums).
 */
#include <omp.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double xi, fx, fy, cx, cy; int32_t width, height; } or_camera;
typedef struct { double R[9]; double t[3]; } or_pose;      /* X_src = R X_ref + t */
typedef struct { int32_t width, height; const double *data; } or_image;  /* row-major */

typedef struct {
    int32_t n_fronto; double near_m, far_m;   /* fronto planes, uniform in inverse depth */
    int32_t n_ground; double h_lo, h_hi;      /* ground-parallel planes, heights above ground */
    int32_t window;                           /* odd window side */
    int32_t best_k;                           /* sources averaged per plane */
    double var_floor;                         /* tau: grey-level^2 per sample */
    double ground_n[3], ground_d;             /* ground plane n . X = ground_d, reference frame */
    double temperature;                       /* soft-argmin temperature */
} or_params;

/* ------------------------------------------------------------------------ */
/* camera model                                                             */
/* ------------------------------------------------------------------------ */

/* Eq. (1): unit ray of pixel (u, v).  Normalized coordinates x = (u - cx)/fx,
 * y = (v - cy)/fy (pixel centres at integer coordinates).  Returns 0 where the
 * square root is not real. */
int or_unproject(const or_camera *c, double u, double v, double r[3])
{
    double x = (u - c->cx) / c->fx, y = (v - c->cy) / c->fy;
    double q = x * x + y * y;
    double disc = 1.0 + (1.0 - c->xi * c->xi) * q;
    if (disc < 0.0) return 0;
    double eta = (c->xi + sqrt(disc)) / (q + 1.0);
    r[0] = eta * x;
    r[1] = eta * y;
    r[2] = eta - c->xi;
    return 1;
}

/* Unified-model projection of a camera-frame point: normalise onto the unit
 * sphere, shift the centre by xi along z, then the pinhole part.  Returns 0
 * where the point is behind the model's viewpoint (Z + xi |X| <= 0). */
int or_project(const or_camera *c, const double X[3], double *u, double *v)
{
    double m = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    double den = X[2] + c->xi * m;
    if (!(den > 1e-12 * m)) return 0;
    *u = c->fx * X[0] / den + c->cx;
    *v = c->fy * X[1] / den + c->cy;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* planes                                                                   */
/* ------------------------------------------------------------------------ */
static int n_planes(const or_params *p) { return p->n_fronto + p->n_ground; }

/* Plane k as n . X = d in the reference frame.  Fronto planes come first, far
 * to near, uniform in inverse depth rho; then ground-parallel planes, low to
 * high, uniform in height h above the ground plane. */
static void plane_of(const or_params *p, int k, double n[3], double *d)
{
    if (k < p->n_fronto) {
        double rho = 1.0 / p->far_m;
        if (p->n_fronto > 1) rho += k * (1.0 / p->near_m - 1.0 / p->far_m) / (p->n_fronto - 1);
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
        *d = 1.0 / rho;
    } else {
        int j = k - p->n_fronto;
        double h = p->h_lo;
        if (p->n_ground > 1) h += j * (p->h_hi - p->h_lo) / (p->n_ground - 1);
        n[0] = p->ground_n[0]; n[1] = p->ground_n[1]; n[2] = p->ground_n[2];
        *d = p->ground_d - h;
    }
}

/* plane parameter (rho for fronto planes, h for ground planes) and its step */
double or_plane_param(const or_params *p, int k, double *step)
{
    if (k < p->n_fronto) {
        double dr = p->n_fronto > 1 ? (1.0 / p->near_m - 1.0 / p->far_m) / (p->n_fronto - 1) : 0.0;
        if (step) *step = dr;
        return 1.0 / p->far_m + k * dr;
    }
    double dh = p->n_ground > 1 ? (p->h_hi - p->h_lo) / (p->n_ground - 1) : 0.0;
    if (step) *step = dh;
    return p->h_lo + (k - p->n_fronto) * dh;
}

/* ------------------------------------------------------------------------ */
/* warp of one reference pixel under one plane into one source              */
/* ------------------------------------------------------------------------ */

/* Intersect the ray of reference pixel (u, v) with plane k and project the
 * point into source s.  Returns 1 and (us, vs) if the plane is hit in front of
 * the reference camera and the point projects; the caller checks bounds. */
int or_warp(const or_params *p, const or_camera *ref, const or_camera *src, const or_pose *pose,
            int k, double u, double v, double *us, double *vs, double Xs_out[3])
{
    double r[3], n[3], d;
    if (!or_unproject(ref, u, v, r)) return 0;
    plane_of(p, k, n, &d);
    double t = n[0] * r[0] + n[1] * r[1] + n[2] * r[2];
    if (!(t > 0.0)) return 0;
    double lam = d / t;
    double X[3] = {lam * r[0], lam * r[1], lam * r[2]};
    double Xs[3];
    for (int a = 0; a < 3; ++a)
        Xs[a] = pose->R[3 * a] * X[0] + pose->R[3 * a + 1] * X[1] + pose->R[3 * a + 2] * X[2] + pose->t[a];
    if (Xs_out) { Xs_out[0] = Xs[0]; Xs_out[1] = Xs[1]; Xs_out[2] = Xs[2]; }
    return or_project(src, Xs, us, vs);
}

/* Bilinear sample with edge taps clamped; valid iff 0 <= u <= W-1 and
 * 0 <= v <= H-1.  Optionally the four tap indices/weights and the derivatives
 * of the interpolant with respect to u and v. */
static int bilinear(const or_image *im, double u, double v, double *val,
                    int64_t idx[4], double w[4], double *dbdu, double *dbdv)
{
    if (!(u >= 0.0 && u <= im->width - 1 && v >= 0.0 && v <= im->height - 1)) return 0;
    int i0 = (int)floor(u), j0 = (int)floor(v);
    double al = u - i0, be = v - j0;
    int i1 = i0 + 1 < im->width ? i0 + 1 : im->width - 1;
    int j1 = j0 + 1 < im->height ? j0 + 1 : im->height - 1;
    const double *D = im->data;
    double p00 = D[(int64_t)j0 * im->width + i0], p10 = D[(int64_t)j0 * im->width + i1];
    double p01 = D[(int64_t)j1 * im->width + i0], p11 = D[(int64_t)j1 * im->width + i1];
    *val = (1 - al) * (1 - be) * p00 + al * (1 - be) * p10 + (1 - al) * be * p01 + al * be * p11;
    if (idx) {
        idx[0] = (int64_t)j0 * im->width + i0; w[0] = (1 - al) * (1 - be);
        idx[1] = (int64_t)j0 * im->width + i1; w[1] = al * (1 - be);
        idx[2] = (int64_t)j1 * im->width + i0; w[2] = (1 - al) * be;
        idx[3] = (int64_t)j1 * im->width + i1; w[3] = al * be;
    }
    if (dbdu) *dbdu = (1 - be) * (p10 - p00) + be * (p11 - p01);
    if (dbdv) *dbdv = (1 - al) * (p01 - p00) + al * (p11 - p10);
    return 1;
}

/* ------------------------------------------------------------------------ */
/* matching cost of one (pixel, plane, source)                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int valid;
    int sampled;   /* every window sample usable: the window statistics are set */
    double zncc, cost;
    double mean_a, mean_b, s_aa, s_bb, s_ab;
} win_stats;

static int window_inside(const or_image *ref, int w, int i, int j)
{
    int h = w / 2;
    return i - h >= 0 && j - h >= 0 && i + h <= ref->width - 1 && j + h <= ref->height - 1;
}

/* Negative-ZNCC cost of pixel (i, j) for plane k and source s, two-pass.
 * A window is unusable (valid = 0) if any of its samples misses the plane or
 * the source image, or if either patch is flatter than the variance floor. */
static win_stats pixel_cost(const or_params *p, const or_camera *rc, const or_image *ref,
                            const or_camera *sc, const or_image *src, const or_pose *pose,
                            int k, int i, int j, double *bbuf)
{
    win_stats st;
    memset(&st, 0, sizeof st);
    const int w = p->window, h = w / 2, N = w * w;
    if (!window_inside(ref, w, i, j)) return st;
    int n = 0;
    for (int dj = -h; dj <= h; ++dj)
        for (int di = -h; di <= h; ++di) {
            double us, vs, b;
            if (!or_warp(p, rc, sc, pose, k, i + di, j + dj, &us, &vs, NULL)) return st;
            if (!bilinear(src, us, vs, &b, NULL, NULL, NULL, NULL)) return st;
            bbuf[n++] = b;
        }
    double ma = 0, mb = 0;
    n = 0;
    for (int dj = -h; dj <= h; ++dj)
        for (int di = -h; di <= h; ++di) {
            ma += ref->data[(int64_t)(j + dj) * ref->width + i + di];
            mb += bbuf[n++];
        }
    ma /= N; mb /= N;
    double saa = 0, sbb = 0, sab = 0;
    n = 0;
    for (int dj = -h; dj <= h; ++dj)
        for (int di = -h; di <= h; ++di) {
            double a = ref->data[(int64_t)(j + dj) * ref->width + i + di] - ma;
            double b = bbuf[n++] - mb;
            saa += a * a; sbb += b * b; sab += a * b;
        }
    st.mean_a = ma; st.mean_b = mb; st.s_aa = saa; st.s_bb = sbb; st.s_ab = sab;
    st.sampled = 1;
    if (saa <= N * p->var_floor || sbb <= N * p->var_floor) return st;
    double z = sab / sqrt(saa * sbb);
    if (z > 1.0) z = 1.0;
    if (z < -1.0) z = -1.0;
    st.zncc = z;
    st.cost = 0.5 * (1.0 - z);
    st.valid = 1;
    return st;
}

/* Mean of the best K valid source costs (fewer if fewer are valid).  Returns
 * NaN if no source is valid. */
static double aggregate(int S, int K, const double *c, const int *valid, int *chosen)
{
    double v[64];
    int id[64], m = 0;
    for (int s = 0; s < S; ++s)
        if (valid[s]) { v[m] = c[s]; id[m] = s; ++m; }
    if (m == 0) return NAN;
    /* insertion sort, ascending, ties by source index */
    for (int a = 1; a < m; ++a)
        for (int b = a; b > 0 && v[b] < v[b - 1]; --b) {
            double tv = v[b]; v[b] = v[b - 1]; v[b - 1] = tv;
            int ti = id[b]; id[b] = id[b - 1]; id[b - 1] = ti;
        }
    int kk = K < m ? K : m;
    double sum = 0;
    for (int a = 0; a < kk; ++a) sum += v[a];
    if (chosen) {
        for (int s = 0; s < S; ++s) chosen[s] = 0;
        for (int a = 0; a < kk; ++a) chosen[id[a]] = 1;
    }
    return sum / kk;
}

/* Aggregated cost of pixel (i, j) for every plane (NaN = invalid) and,
 * optionally, every per-source cost (NaN = invalid) and the standard
 * deviation of every source window's samples, sqrt(s_bb / N) (NaN where a
 * sample is unusable; set also below the variance floor). */
static void pixel_costs(const or_params *p, const or_camera *rc, const or_image *ref, int S,
                        const or_camera *scs, const or_image *srcs, const or_pose *poses,
                        int i, int j, double *C, double *Cs, double *Sig)
{
    const int P = n_planes(p);
    double cs[64];
    int vs[64];
    double *bbuf = (double *)malloc(sizeof(double) * p->window * p->window);
    for (int k = 0; k < P; ++k) {
        for (int s = 0; s < S; ++s) {
            win_stats st = pixel_cost(p, rc, ref, &scs[s], &srcs[s], &poses[s], k, i, j, bbuf);
            vs[s] = st.valid;
            cs[s] = st.cost;
            if (Cs) Cs[(int64_t)k * S + s] = st.valid ? st.cost : NAN;
            if (Sig) Sig[(int64_t)k * S + s] = st.sampled ? sqrt(st.s_bb / (p->window * p->window)) : NAN;
        }
        C[k] = aggregate(S, p->best_k, cs, vs, NULL);
    }
    free(bbuf);
}

/* ------------------------------------------------------------------------ */
/* winner-take-all sweep of one level                                       */
/* ------------------------------------------------------------------------ */

/* Vertex of the parabola through (-1, cm), (0, c0), (+1, cp), in plane steps,
 * clamped to [-0.5, 0.5]; 0 if the parabola does not open upwards.  (The
 * paper names no subpixel step; this is the reading used throughout.) */
double or_parabola(double cm, double c0, double cp)
{
    double den = cm - 2.0 * c0 + cp;
    if (!(den > 0.0)) return 0.0;
    double dl = (cm - cp) / (2.0 * den);
    if (dl > 0.5) dl = 0.5;
    if (dl < -0.5) dl = -0.5;
    return dl;
}

/*
 * Evaluate n_pix reference pixels (pix = interleaved x, y; NULL = every pixel
 * in row-major order, n_pix = W * H).  Outputs per evaluated pixel (any may be
 * NULL):
 *   depth  range along the unit ray (metres), NaN if no plane is valid
 *   z      camera-frame z of the point, NaN if invalid
 *   index  winning plane (lowest index among equal costs), -1 if invalid
 *   delta  parabolic subpixel offset in plane steps, in [-0.5, 0.5]
 *   c1     best aggregated cost (+inf if invalid)
 *   c2     best aggregated cost over the other planes (+inf if none)
 *   c2na   best aggregated cost over planes not adjacent to the winner
 *   param  refined plane parameter (rho or h), NaN if invalid
 *   volume aggregated cost per plane [n_pix][P] (NaN = invalid)
 *   srcvol per-source cost [n_pix][P][S] (NaN = invalid)
 *   srcsig per-source standard deviation of the window's samples [n_pix][P][S]
 *          (NaN where a sample is unusable; set also for windows below the
 *          variance floor)
 */
void or_sweep(const or_params *p, const or_camera *rc, const or_image *ref, int32_t S,
              const or_camera *scs, const or_image *srcs, const or_pose *poses,
              int64_t n_pix, const int32_t *pix,
              double *depth, double *z, int32_t *index, double *delta, double *c1, double *c2,
              double *c2na, double *param, double *volume, double *srcvol, double *srcsig)
{
    const int P = n_planes(p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < n_pix; ++e) {
        int i = pix ? pix[2 * e] : (int)(e % ref->width);
        int j = pix ? pix[2 * e + 1] : (int)(e / ref->width);
        double *C = (double *)malloc(sizeof(double) * P);
        pixel_costs(p, rc, ref, S, scs, srcs, poses, i, j, C, srcvol ? srcvol + e * P * S : NULL,
                    srcsig ? srcsig + e * P * S : NULL);
        if (volume) memcpy(volume + e * P, C, sizeof(double) * P);
        int kb = -1;
        double b1 = INFINITY, b2 = INFINITY, bna = INFINITY;
        for (int k = 0; k < P; ++k) {
            if (isnan(C[k])) continue;
            if (C[k] < b1) { kb = k; b1 = C[k]; }
        }
        for (int k = 0; k < P; ++k) {
            if (isnan(C[k]) || k == kb) continue;
            if (C[k] < b2) b2 = C[k];
            if (abs(k - kb) > 1 && C[k] < bna) bna = C[k];
        }
        double dl = 0.0, lam = NAN, zz = NAN, prm = NAN;
        if (kb >= 0) {
            /* parabola through the winner and its two neighbours of the same
             * family, in plane-parameter space */
            int fam = kb < p->n_fronto ? 0 : 1;
            int lo = fam == 0 ? 0 : p->n_fronto, hi = fam == 0 ? p->n_fronto - 1 : P - 1;
            if (kb - 1 >= lo && kb + 1 <= hi && !isnan(C[kb - 1]) && !isnan(C[kb + 1]))
                dl = or_parabola(C[kb - 1], C[kb], C[kb + 1]);
            double step;
            prm = or_plane_param(p, kb, &step) + dl * step;
            double r[3];
            or_unproject(rc, i, j, r);
            if (fam == 0) lam = 1.0 / (prm * r[2]);
            else lam = (p->ground_d - prm) / (p->ground_n[0] * r[0] + p->ground_n[1] * r[1] + p->ground_n[2] * r[2]);
            zz = lam * r[2];
        }
        if (depth) depth[e] = lam;
        if (z) z[e] = zz;
        if (index) index[e] = kb;
        if (delta) delta[e] = dl;
        if (c1) c1[e] = b1;
        if (c2) c2[e] = b2;
        if (c2na) c2na[e] = bna;
        if (param) param[e] = prm;
        free(C);
    }
}

/* Negative-ZNCC cost and statistics of a single (pixel, plane, source), for
 * checks of individual windows.  out: valid, zncc, cost, mean_a, mean_b,
 * s_aa, s_bb, s_ab. */
void or_window_cost(const or_params *p, const or_camera *rc, const or_image *ref,
                    const or_camera *sc, const or_image *src, const or_pose *pose,
                    int32_t k, int32_t i, int32_t j, double out[8])
{
    double *bbuf = (double *)malloc(sizeof(double) * p->window * p->window);
    win_stats st = pixel_cost(p, rc, ref, sc, src, pose, k, i, j, bbuf);
    free(bbuf);
    out[0] = st.valid; out[1] = st.zncc; out[2] = st.cost; out[3] = st.mean_a;
    out[4] = st.mean_b; out[5] = st.s_aa; out[6] = st.s_bb; out[7] = st.s_ab;
}

/* ------------------------------------------------------------------------ */
/* resolution levels (Sec. III-A, multi-scale strategy)                     */
/* ------------------------------------------------------------------------ */

/* 2x2 box downsampling with round-half-up integer arithmetic:
 * out = (s00 + s01 + s10 + s11 + 2) >> 2, out size floor(W/2) x floor(H/2). */
void or_downsample2(const uint8_t *in, int32_t w, int32_t h, uint8_t *out)
{
    int wo = w / 2, ho = h / 2;
    for (int j = 0; j < ho; ++j)
        for (int i = 0; i < wo; ++i) {
            int s = in[(2 * j) * w + 2 * i] + in[(2 * j) * w + 2 * i + 1] +
                    in[(2 * j + 1) * w + 2 * i] + in[(2 * j + 1) * w + 2 * i + 1];
            out[j * wo + i] = (uint8_t)((s + 2) >> 2);
        }
}

/* Camera of a level: a 2x2-downsampled pixel (i, j) covers full-resolution
 * pixel centres 2i .. 2i+1, so its centre is at 2i + 0.5; a crop shifts the
 * principal point by the crop offset. */
void or_level_camera(const or_camera *full, int32_t downsample, int32_t crop_x, int32_t crop_y,
                     int32_t crop_w, int32_t crop_h, or_camera *out)
{
    *out = *full;
    if (downsample == 2) {
        out->fx = full->fx / 2.0; out->fy = full->fy / 2.0;
        out->cx = (full->cx - 0.5) / 2.0; out->cy = (full->cy - 0.5) / 2.0;
        out->width = full->width / 2; out->height = full->height / 2;
    }
    if (crop_w > 0) {
        out->cx -= crop_x; out->cy -= crop_y;
        out->width = crop_w; out->height = crop_h;
    }
}

/*
 * Fuse the low level (whole field of view, downsample factor `ds0`) and the
 * crop level into full-resolution maps.  Reading of the paper's "up-sample
 * the depth estimates" and "fuse the two depth maps": the low result is taken
 * by nearest neighbour (full pixel (i, j) -> low pixel (i/ds0, j/ds0)) as a
 * plane (family + refined parameter), whose range is recomputed along the
 * full-resolution ray; inside the crop the crop result replaces it when the
 * crop result is valid and the low result is either invalid or at least as
 * far as the crop level's nearest plane (z_low >= crop_near).
 * low_param/crop_param: refined plane parameter per level pixel (NaN invalid);
 * low_index/crop_index: winning plane index (-1 invalid), used for the family.
 * Outputs full resolution: depth, z, level (0 low, 1 crop, 255 invalid),
 * source index into the chosen level's maps (-1 if invalid).
 */
void or_merge(const or_camera *full, const or_params *p0, const or_params *p1,
              int32_t ds0, int32_t low_w, int32_t low_h,
              const double *low_param, const int32_t *low_index,
              int32_t crop_x, int32_t crop_y, int32_t crop_w, int32_t crop_h,
              const double *crop_param, const int32_t *crop_index,
              double *depth, double *z, uint8_t *level, int64_t *src_pix)
{
    const int W = full->width, H = full->height;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t e = (int64_t)j * W + i;
            double r[3];
            or_unproject(full, i, j, r);
            double lam_lo = NAN, z_lo = NAN;
            int64_t src_lo = -1;
            int il = i / ds0, jl = j / ds0;
            if (il < low_w && jl < low_h) {
                int64_t le = (int64_t)jl * low_w + il;
                int k = low_index[le];
                if (k >= 0) {
                    double prm = low_param[le];
                    if (k < p0->n_fronto) {
                        if (r[2] > 0.0) lam_lo = 1.0 / (prm * r[2]);
                    } else {
                        double t = p0->ground_n[0] * r[0] + p0->ground_n[1] * r[1] + p0->ground_n[2] * r[2];
                        if (t > 0.0) lam_lo = (p0->ground_d - prm) / t;
                    }
                    if (!isnan(lam_lo)) { z_lo = lam_lo * r[2]; src_lo = le; }
                }
            }
            double lam_c = NAN, z_c = NAN;
            int64_t src_c = -1;
            if (p1 && crop_w > 0 && i >= crop_x && i < crop_x + crop_w && j >= crop_y && j < crop_y + crop_h) {
                int64_t ce = (int64_t)(j - crop_y) * crop_w + (i - crop_x);
                int k = crop_index[ce];
                if (k >= 0) {
                    double prm = crop_param[ce];
                    if (k < p1->n_fronto) {
                        lam_c = 1.0 / (prm * r[2]);
                    } else {
                        double t = p1->ground_n[0] * r[0] + p1->ground_n[1] * r[1] + p1->ground_n[2] * r[2];
                        lam_c = (p1->ground_d - prm) / t;
                    }
                    z_c = lam_c * r[2];
                    src_c = ce;
                }
            }
            if (src_c >= 0 && (src_lo < 0 || z_lo >= p1->near_m)) {
                depth[e] = lam_c; z[e] = z_c; level[e] = 1; src_pix[e] = src_c;
            } else if (src_lo >= 0) {
                depth[e] = lam_lo; z[e] = z_lo; level[e] = 0; src_pix[e] = src_lo;
            } else {
                depth[e] = NAN; z[e] = NAN; level[e] = 255; src_pix[e] = -1;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* soft-argmin over the planes and its analytic gradient                   */
/* ------------------------------------------------------------------------ */

/*
 * Hypothesis value of plane k at reference pixel (i, j) for the soft-argmin:
 * the inverse z-depth of the point where the pixel's Eq. (1) ray meets the
 * plane.  A fronto plane's is its parameter rho_k; along the unit ray r a
 * ground plane n_g . X = d_g - h is met at range (d_g - h) / (n_g . r), so its
 * value is (n_g . r) / ((d_g - h) r_z).  (The soft-argmin has no counterpart
 * in the paper; the planes are the paper's.)
 */
double or_soft_hypothesis(const or_params *p, const or_camera *rc, int k, int i, int j)
{
    const double prm = or_plane_param(p, k, NULL);
    if (k < p->n_fronto) return prm;
    double r[3];
    or_unproject(rc, i, j, r);
    const double nr = p->ground_n[0] * r[0] + p->ground_n[1] * r[1] + p->ground_n[2] * r[2];
    return nr / ((p->ground_d - prm) * r[2]);
}

/*
 * Soft-argmin of one pixel (no counterpart in the paper; the hypotheses are
 * the paper's planes): with l_k = -C_k / T over the valid planes (C_k
 * not NaN), p = softmax(l) and rho_hat = sum_k p_k rho_k, lse = log sum_k
 * exp(l_k), both computed with the largest l_k taken out.  No valid plane:
 * rho_hat = NaN and lse = -inf.
 */
void or_soft_argmin(const double *C, const double *rho, int32_t P, double T, double *rho_hat, double *lse)
{
    double m = -INFINITY;
    for (int k = 0; k < P; ++k)
        if (!isnan(C[k]) && -C[k] / T > m) m = -C[k] / T;
    if (isinf(m)) {
        *rho_hat = NAN; *lse = -INFINITY;
        return;
    }
    double se = 0, sr = 0;
    for (int k = 0; k < P; ++k) {
        if (isnan(C[k])) continue;
        double ex = exp(-C[k] / T - m);
        se += ex;
        sr += ex * rho[k];
    }
    *rho_hat = sr / se;
    *lse = m + log(se);
}

/*
 * Soft-argmin inverse depth of every pixel over the planes' costs, each plane
 * standing for its hypothesis value at the pixel (or_soft_hypothesis).
 */
void or_soft_forward(const or_params *p, const or_camera *rc, const or_image *ref, int32_t S,
                     const or_camera *scs, const or_image *srcs, const or_pose *poses,
                     int64_t n_pix, const int32_t *pix, double *rho_hat, double *lse)
{
    const int P = n_planes(p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < n_pix; ++e) {
        int i = pix ? pix[2 * e] : (int)(e % ref->width);
        int j = pix ? pix[2 * e + 1] : (int)(e / ref->width);
        double *C = (double *)malloc(sizeof(double) * P);
        double *rho = (double *)malloc(sizeof(double) * P);
        pixel_costs(p, rc, ref, S, scs, srcs, poses, i, j, C, NULL, NULL);
        for (int k = 0; k < P; ++k) rho[k] = or_soft_hypothesis(p, rc, k, i, j);
        or_soft_argmin(C, rho, P, p->temperature, &rho_hat[e], &lse[e]);
        free(rho);
        free(C);
    }
}

/*
 * Gradient of L = sum_p g_p rho_hat_p over the pixels of the rectangle
 * [x0, x0+w) x [y0, y0+h) (g row-major w x h) with respect to
 *   - every source image value (grad_src[s], W_s x H_s, accumulated), and
 *   - the 6-DoF pose of every source as a left perturbation
 *     X_s -> X_s + v + omega x X_s, ordered (v, omega) (grad_pose[6 s + .]).
 * Chain: rho_hat -> C_k (softmax) -> best-K mean -> per-source cost
 * (1 - Z)/2 -> ZNCC of the window -> bilinear samples -> projection -> pose.
 * Windows whose ZNCC is clamped, that are invalid or fall below the variance
 * floor pass no gradient.
 */
void or_soft_backward(const or_params *p, const or_camera *rc, const or_image *ref, int32_t S,
                      const or_camera *scs, const or_image *srcs, const or_pose *poses,
                      int32_t x0, int32_t y0, int32_t w, int32_t h, const double *g,
                      double *const *grad_src, double *grad_pose)
{
    const int P = n_planes(p), win = p->window, hw = win / 2, N = win * win;
    const double T = p->temperature;
    for (int s = 0; s < 6 * S; ++s) grad_pose[s] = 0.0;
    double *C = (double *)malloc(sizeof(double) * P);
    double *Cs = (double *)malloc(sizeof(double) * P * S);
    double *bb = (double *)malloc(sizeof(double) * N);
    for (int jj = 0; jj < h; ++jj)
        for (int ii = 0; ii < w; ++ii) {
            const int i = x0 + ii, j = y0 + jj;
            const double gp = g[(int64_t)jj * w + ii];
            if (gp == 0.0) continue;
            pixel_costs(p, rc, ref, S, scs, srcs, poses, i, j, C, Cs, NULL);
            double m = -INFINITY;
            for (int k = 0; k < P; ++k)
                if (!isnan(C[k]) && -C[k] / T > m) m = -C[k] / T;
            if (isinf(m)) continue;
            double se = 0, sr = 0;
            for (int k = 0; k < P; ++k) {
                if (isnan(C[k])) continue;
                double ex = exp(-C[k] / T - m);
                se += ex; sr += ex * or_soft_hypothesis(p, rc, k, i, j);
            }
            double rh = sr / se;
            for (int k = 0; k < P; ++k) {
                if (isnan(C[k])) continue;
                double pk = exp(-C[k] / T - m) / se;
                double dC = gp * (-1.0 / T) * pk * (or_soft_hypothesis(p, rc, k, i, j) - rh);
                double cs[64];
                int vs[64], chosen[64];
                for (int s = 0; s < S; ++s) { cs[s] = Cs[(int64_t)k * S + s]; vs[s] = !isnan(cs[s]); }
                aggregate(S, p->best_k, cs, vs, chosen);
                int kk = 0;
                for (int s = 0; s < S; ++s) kk += chosen[s];
                for (int s = 0; s < S; ++s) {
                    if (!chosen[s]) continue;
                    win_stats st = pixel_cost(p, rc, ref, &scs[s], &srcs[s], &poses[s], k, i, j, bb);
                    if (!st.valid || fabs(st.zncc) >= 1.0) continue;
                    double dZ = -0.5 * dC / kk;           /* dL/dZ */
                    double D = sqrt(st.s_aa * st.s_bb);
                    for (int dj = -hw; dj <= hw; ++dj)
                        for (int di = -hw; di <= hw; ++di) {
                            double us, vs2, Xs[3], b, wt[4], dbu, dbv;
                            int64_t idx[4];
                            or_warp(p, rc, &scs[s], &poses[s], k, i + di, j + dj, &us, &vs2, Xs);
                            bilinear(&srcs[s], us, vs2, &b, idx, wt, &dbu, &dbv);
                            double a = ref->data[(int64_t)(j + dj) * ref->width + i + di];
                            double dZdb = (a - st.mean_a) / D - st.zncc * (b - st.mean_b) / st.s_bb;
                            double gb = dZ * dZdb;
                            for (int t = 0; t < 4; ++t) grad_src[s][idx[t]] += gb * wt[t];
                            /* projection Jacobian d(u, v)/dXs */
                            const or_camera *c = &scs[s];
                            double mm = sqrt(Xs[0] * Xs[0] + Xs[1] * Xs[1] + Xs[2] * Xs[2]);
                            double den = Xs[2] + c->xi * mm;
                            double dden[3] = {c->xi * Xs[0] / mm, c->xi * Xs[1] / mm, 1.0 + c->xi * Xs[2] / mm};
                            double gX[3];
                            for (int a3 = 0; a3 < 3; ++a3) {
                                double dudX = c->fx * ((a3 == 0 ? 1.0 : 0.0) / den - Xs[0] * dden[a3] / (den * den));
                                double dvdX = c->fy * ((a3 == 1 ? 1.0 : 0.0) / den - Xs[1] * dden[a3] / (den * den));
                                gX[a3] = gb * (dbu * dudX + dbv * dvdX);
                            }
                            double *gpz = grad_pose + 6 * s;
                            gpz[0] += gX[0]; gpz[1] += gX[1]; gpz[2] += gX[2];
                            gpz[3] += Xs[1] * gX[2] - Xs[2] * gX[1];
                            gpz[4] += Xs[2] * gX[0] - Xs[0] * gX[2];
                            gpz[5] += Xs[0] * gX[1] - Xs[1] * gX[0];
                        }
                }
            }
        }
    free(C); free(Cs); free(bb);
}

/* ------------------------------------------------------------------------ */
/* depth-map filtering (Sec. III-A, depth map filtering)                    */
/* ------------------------------------------------------------------------ */

/*
 * Three tests, applied in the order the paper shows them (Fig. 3):
 *   1. best cost: c1 > alpha is an outlier, with alpha_upper for pixels whose
 *      ray points above the ground plane's horizon (n_g . r <= 0, the upper
 *      part of the view) and alpha_lower below it;
 *   2. uniqueness: the ratio c2 / c1 of the second best to the best cost
 *      must reach ratio_min (a larger ratio is a more unique depth);
 *   3. local continuity: among the other pixels of the win x win window that
 *      survived tests 1-2, count those whose range differs from the centre's
 *      by less than gamma; the pixel is rejected when that count over
 *      (win^2 - 1) is below delta_frac.
 * Inputs are the sweep's full-resolution maps; out_depth is the range with
 * rejected pixels set to NaN, code is 0 kept, 1 cost, 2 uniqueness,
 * 3 continuity, 255 invalid before filtering.
 */
void or_filter(const or_camera *cam, const double ground_n[3], int32_t w, int32_t h,
               const double *depth, const double *c1, const double *c2,
               double alpha_upper, double alpha_lower, double ratio_min, double gamma, double delta_frac,
               int32_t win, double *out_depth, uint8_t *code)
{
    const int hw = win / 2;
    double *d1 = (double *)malloc(sizeof(double) * (size_t)w * h);
    for (int j = 0; j < h; ++j)
        for (int i = 0; i < w; ++i) {
            int64_t e = (int64_t)j * w + i;
            d1[e] = NAN;
            if (isnan(depth[e])) { code[e] = 255; continue; }
            double r[3];
            or_unproject(cam, i, j, r);
            double up = ground_n[0] * r[0] + ground_n[1] * r[1] + ground_n[2] * r[2];
            double alpha = up <= 0.0 ? alpha_upper : alpha_lower;
            if (c1[e] > alpha) { code[e] = 1; continue; }
            if (!(c2[e] >= ratio_min * c1[e])) { code[e] = 2; continue; }
            code[e] = 0;
            d1[e] = depth[e];
        }
    for (int j = 0; j < h; ++j)
        for (int i = 0; i < w; ++i) {
            int64_t e = (int64_t)j * w + i;
            out_depth[e] = NAN;
            if (code[e] != 0) continue;
            int cons = 0;
            for (int dj = -hw; dj <= hw; ++dj)
                for (int di = -hw; di <= hw; ++di) {
                    if (di == 0 && dj == 0) continue;
                    int ii = i + di, jj = j + dj;
                    if (ii < 0 || jj < 0 || ii >= w || jj >= h) continue;
                    double q = d1[(int64_t)jj * w + ii];
                    if (!isnan(q) && fabs(q - d1[e]) < gamma) ++cons;
                }
            if ((double)cons < delta_frac * (win * win - 1)) { code[e] = 3; continue; }
            out_depth[e] = d1[e];
        }
    free(d1);
}

/* Threads the parallel loops above use (for reporting the baseline's cores). */
int or_threads(void) { return omp_get_max_threads(); }

/* Set that thread count (n >= 1) for the calling thread's later loops. */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
