/*
 * Seeded synthetic scene renderer: input generator for the fisheye plane-sweep
 * tests and benchmarks.  It renders what a set of fisheye cameras would see of
 * a scene made of a textured ground plane and textured axis-aligned boxes, and
 * the ground-truth range/depth of the centre ray of every pixel.
 *
 * This file holds no part of the plane-sweep method (no warping, no matching
 * cost, no plane hypotheses).  It needs a camera model only to turn a pixel
 * into a viewing ray; that inverse is derived here on its own: a unit vector s
 * on the viewing sphere projects to normalized coordinates (x, y) =
 * (s_x, s_y) / (s_z + xi), so s_z solves the quadratic
 *     (x^2 + y^2 + 1) s_z^2 + 2 xi (x^2 + y^2) s_z + xi^2 (x^2 + y^2) - 1 = 0
 * (larger root) and (s_x, s_y) = (x, y) (s_z + xi).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC render.c -o librender.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    double lo[3], hi[3];
    int32_t tex[6];          /* texture id per face: -x, +x, -y, +y, -z, +z */
} rg_box;

typedef struct {
    int64_t offset;          /* into the texel atlas */
    int32_t nu, nv;          /* texel grid size */
    double u0, v0;           /* world coordinate of texel (0, 0) centre */
    double pitch;            /* metres per texel */
} rg_tex;

typedef struct {
    double xi, fx, fy, cx, cy;
    int32_t width, height;
    double Rcw[9];           /* camera -> world rotation, row-major */
    double centre[3];        /* camera centre in world coordinates */
} rg_cam;

typedef struct {
    int32_t n_boxes;
    const rg_box *boxes;
    double ground_y;         /* ground plane: world y = ground_y (y points down) */
    int32_t ground_tex;
    double ground_max_range; /* ground hits beyond this range are sky */
    double sky_range;        /* any hit beyond this range is sky */
    double sky_value;
    const rg_tex *texs;
    const float *atlas;
} rg_scene;

static double tex_lookup(const rg_scene *sc, int id, double u, double v)
{
    const rg_tex *t = &sc->texs[id];
    double s = (u - t->u0) / t->pitch, r = (v - t->v0) / t->pitch;
    if (s < 0) s = 0;
    if (r < 0) r = 0;
    if (s > t->nu - 1) s = t->nu - 1;
    if (r > t->nv - 1) r = t->nv - 1;
    int i0 = (int)floor(s), j0 = (int)floor(r);
    if (i0 > t->nu - 2) i0 = t->nu - 2;
    if (j0 > t->nv - 2) j0 = t->nv - 2;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    double fs = s - i0, fr = r - j0;
    const float *g = sc->atlas + t->offset;
    double p00 = g[(int64_t)j0 * t->nu + i0], p10 = g[(int64_t)j0 * t->nu + i0 + 1];
    double p01 = g[(int64_t)(j0 + 1) * t->nu + i0], p11 = g[(int64_t)(j0 + 1) * t->nu + i0 + 1];
    return (1 - fr) * ((1 - fs) * p00 + fs * p10) + fr * ((1 - fs) * p01 + fs * p11);
}

/* Nearest hit of the ray o + t d (t > 0).  Returns the distance (inf if none)
 * and the intensity at the hit. */
static double trace(const rg_scene *sc, const double o[3], const double d[3], double *val)
{
    double best = INFINITY;
    double bval = sc->sky_value;
    /* ground */
    if (d[1] > 1e-12) {
        double t = (sc->ground_y - o[1]) / d[1];
        if (t > 1e-9 && t < sc->ground_max_range) {
            best = t;
            double px = o[0] + t * d[0], pz = o[2] + t * d[2];
            bval = tex_lookup(sc, sc->ground_tex, px, pz);
        }
    }
    for (int b = 0; b < sc->n_boxes; ++b) {
        const rg_box *bx = &sc->boxes[b];
        double tn = -INFINITY, tf = INFINITY;
        int axis_n = -1, side_n = 0;
        int miss = 0;
        for (int a = 0; a < 3; ++a) {
            if (fabs(d[a]) < 1e-15) {
                if (o[a] < bx->lo[a] || o[a] > bx->hi[a]) { miss = 1; break; }
                continue;
            }
            double t1 = (bx->lo[a] - o[a]) / d[a], t2 = (bx->hi[a] - o[a]) / d[a];
            int s1 = 0;
            if (t1 > t2) { double tmp = t1; t1 = t2; t2 = tmp; s1 = 1; }
            if (t1 > tn) { tn = t1; axis_n = a; side_n = s1; }
            if (t2 < tf) tf = t2;
        }
        if (miss || tn > tf || tn <= 1e-9 || axis_n < 0) continue;
        if (tn < best) {
            best = tn;
            double p[3] = {o[0] + tn * d[0], o[1] + tn * d[1], o[2] + tn * d[2]};
            int face = 2 * axis_n + side_n;
            int tid = bx->tex[face];
            double u, v;
            if (axis_n == 0) { u = p[2]; v = p[1]; }
            else if (axis_n == 1) { u = p[0]; v = p[2]; }
            else { u = p[0]; v = p[1]; }
            bval = tex_lookup(sc, tid, u, v);
        }
    }
    if (best > sc->sky_range) { best = INFINITY; bval = sc->sky_value; }
    *val = bval;
    return best;
}

/* Viewing ray (unit, camera frame) of normalized coordinates (x, y). */
static int pixel_ray(double xi, double x, double y, double s[3])
{
    double q = x * x + y * y;
    double A = q + 1.0, B = 2.0 * xi * q, C = xi * xi * q - 1.0;
    double disc = B * B - 4.0 * A * C;
    if (disc < 0) return 0;
    double sz = (-B + sqrt(disc)) / (2.0 * A);
    double k = sz + xi;
    s[0] = x * k; s[1] = y * k; s[2] = sz;
    double n = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    s[0] /= n; s[1] /= n; s[2] /= n;
    return 1;
}

/*
 * Render one camera.  img: float [H][W] mean intensity over ss x ss
 * sub-pixel rays.  gt_range / gt_z (may be NULL): distance along the unit
 * centre ray and its camera-frame z, NaN where the centre ray sees sky.
 * Pixel (i, j) has its centre at (u, v) = (i, j).
 */
void rg_render(const rg_scene *sc, const rg_cam *cam, int32_t ss,
               float *img, float *gt_range, float *gt_z)
{
    const int W = cam->width, H = cam->height;
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < H; ++j) {
        for (int i = 0; i < W; ++i) {
            double acc = 0.0;
            for (int sj = 0; sj < ss; ++sj)
                for (int si = 0; si < ss; ++si) {
                    double u = i + ((si + 0.5) / ss - 0.5), v = j + ((sj + 0.5) / ss - 0.5);
                    double x = (u - cam->cx) / cam->fx, y = (v - cam->cy) / cam->fy;
                    double s[3], d[3], val = sc->sky_value;
                    if (pixel_ray(cam->xi, x, y, s)) {
                        for (int a = 0; a < 3; ++a)
                            d[a] = cam->Rcw[3 * a] * s[0] + cam->Rcw[3 * a + 1] * s[1] + cam->Rcw[3 * a + 2] * s[2];
                        trace(sc, cam->centre, d, &val);
                    }
                    acc += val;
                }
            img[(int64_t)j * W + i] = (float)(acc / (ss * ss));
            if (gt_range) {
                double x = (i - cam->cx) / cam->fx, y = (j - cam->cy) / cam->fy;
                double s[3], d[3], val;
                double t = INFINITY;
                if (pixel_ray(cam->xi, x, y, s)) {
                    for (int a = 0; a < 3; ++a)
                        d[a] = cam->Rcw[3 * a] * s[0] + cam->Rcw[3 * a + 1] * s[1] + cam->Rcw[3 * a + 2] * s[2];
                    t = trace(sc, cam->centre, d, &val);
                }
                gt_range[(int64_t)j * W + i] = isinf(t) ? NAN : (float)t;
                if (gt_z) gt_z[(int64_t)j * W + i] = isinf(t) ? NAN : (float)(t * s[2]);
            }
        }
    }
}
