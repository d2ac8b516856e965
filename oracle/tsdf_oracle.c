/*
 * FP64 CPU oracle for fisheye TSDF depth-map fusion (Sec. III-C).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library.
 *
 * The map is a box of nb[0] x nb[1] x nb[2] voxel blocks (8 x 8 x 8 voxels of
 * edge `voxel` metres) whose first block has integer block coordinates b0
 * (world x, y, z); a block covers [b B, (b + 1) B) per axis with B = 8 voxel,
 * and a voxel's sample point is its centre.  Arrays are indexed
 * [z][y][x] (blocks) and [z][y][x] over the box's voxel grid.
 *
 * One depth map is fused in the steps of Sec. III-C:
 *   1. allocation: for every pixel with a valid depth d (range along the
 *      Eq. (1) ray, metres) the segment of the ray from max(d - mu, 0) to
 *      d + mu, taken to world coordinates with the camera pose, marks every
 *      block of the box whose closed cube it meets (exact slab test);
 *   2. visibility: an allocated block is visible when one of its eight
 *      corners projects into the depth image;
 *   3. integration (Eq. (2)): every voxel of a visible block is taken into the
 *      camera frame, X_d = R_d X + t_d, projected with the unified model to
 *      its nearest pixel; with that pixel's depth d_obs and
 *      eta = d_obs - |X_d| >= -mu, D <- (w D + min(1, eta / mu)) / (w + 1)
 *      and w <- min(w + 1, w_max).
 * The block observation counts (frames whose rays met the block) are kept by
 * the caller from the allocation marks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double xi, fx, fy, cx, cy; int32_t width, height; } ot_camera;
typedef struct { double R[9]; double t[3]; } ot_pose;     /* X_cam = R X_world + t */

int or_unproject(const ot_camera *c, double u, double v, double r[3]);
int or_project(const ot_camera *c, const double X[3], double *u, double *v);

static void to_world(const ot_pose *p, const double Xc[3], double Xw[3])
{
    /* X_world = R^T (X_cam - t) */
    double d[3] = {Xc[0] - p->t[0], Xc[1] - p->t[1], Xc[2] - p->t[2]};
    for (int i = 0; i < 3; ++i) Xw[i] = p->R[0 * 3 + i] * d[0] + p->R[1 * 3 + i] * d[1] + p->R[2 * 3 + i] * d[2];
}

static void to_cam(const ot_pose *p, const double Xw[3], double Xc[3])
{
    for (int i = 0; i < 3; ++i)
        Xc[i] = p->R[i * 3 + 0] * Xw[0] + p->R[i * 3 + 1] * Xw[1] + p->R[i * 3 + 2] * Xw[2] + p->t[i];
}

/* Whether segment A + s (B - A), s in [0, 1], meets the closed box [lo, hi]
 * (slab test); if so, how deep it reaches into the box: the largest distance
 * from a point of its piece inside the box to the nearest face (0 for a
 * segment that only touches the box or runs along a face), else -1. */
static double seg_in_box(const double A[3], const double Bp[3], const double lo[3], const double hi[3])
{
    double s0 = 0.0, s1 = 1.0;
    for (int a = 0; a < 3; ++a) {
        double d = Bp[a] - A[a];
        if (d == 0.0) {
            if (A[a] < lo[a] || A[a] > hi[a]) return -1.0;
            continue;
        }
        double ta = (lo[a] - A[a]) / d, tb = (hi[a] - A[a]) / d;
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > s0) s0 = ta;
        if (tb < s1) s1 = tb;
        if (s0 > s1) return -1.0;
    }
    /* the distance to the nearest face is concave along the piece: sample it */
    double best = 0.0;
    for (int k = 0; k <= 64; ++k) {
        double s = s0 + (s1 - s0) * k / 64.0, inner = 1e300;
        for (int a = 0; a < 3; ++a) {
            double p = A[a] + s * (Bp[a] - A[a]);
            double m = p - lo[a] < hi[a] - p ? p - lo[a] : hi[a] - p;
            if (m < inner) inner = m;
        }
        if (inner > best) best = inner;
    }
    return best;
}

/* Step 1.  touched[nb]: 1 for every block met by some pixel's segment;
 * pen[nb]: the deepest any segment reaches into the block (metres, see
 * seg_in_box), for telling blocks that are only grazed. */
void or_tsdf_alloc(const ot_camera *cam, const ot_pose *pose, const double *depth, int64_t pitch, double voxel,
                   double mu, const int32_t b0[3], const int32_t nb[3], int32_t *touched, double *pen)
{
    const double B = 8.0 * voxel;
    const size_t nblk = (size_t)nb[0] * nb[1] * nb[2];
    for (size_t i = 0; i < nblk; ++i) { touched[i] = 0; pen[i] = -1.0; }
    for (int v = 0; v < cam->height; ++v)
        for (int u = 0; u < cam->width; ++u) {
            double d = depth[(int64_t)v * pitch + u];
            if (!(d > 0.0) || !isfinite(d)) continue;
            double r[3];
            if (!or_unproject(cam, u, v, r)) continue;
            double l0 = d - mu > 0.0 ? d - mu : 0.0, l1 = d + mu;
            double P0c[3] = {l0 * r[0], l0 * r[1], l0 * r[2]}, P1c[3] = {l1 * r[0], l1 * r[1], l1 * r[2]};
            double A[3], Bw[3];
            to_world(pose, P0c, A);
            to_world(pose, P1c, Bw);
            int lo_b[3], hi_b[3];
            for (int a = 0; a < 3; ++a) {
                double mn = A[a] < Bw[a] ? A[a] : Bw[a], mx = A[a] < Bw[a] ? Bw[a] : A[a];
                lo_b[a] = (int)floor(mn / B) - 1;
                hi_b[a] = (int)floor(mx / B) + 1;
                if (lo_b[a] < b0[a]) lo_b[a] = b0[a];
                if (hi_b[a] > b0[a] + nb[a] - 1) hi_b[a] = b0[a] + nb[a] - 1;
            }
            for (int bz = lo_b[2]; bz <= hi_b[2]; ++bz)
                for (int by = lo_b[1]; by <= hi_b[1]; ++by)
                    for (int bx = lo_b[0]; bx <= hi_b[0]; ++bx) {
                        double lo[3] = {bx * B, by * B, bz * B}, hi[3] = {(bx + 1) * B, (by + 1) * B, (bz + 1) * B};
                        double len = seg_in_box(A, Bw, lo, hi);
                        if (len < 0.0) continue;
                        size_t i = ((size_t)(bz - b0[2]) * nb[1] + (by - b0[1])) * nb[0] + (bx - b0[0]);
                        touched[i] = 1;
                        if (len > pen[i]) pen[i] = len;
                    }
        }
}

/* FP32 error bounds of the decisions the GPU takes, for the parity tests'
 * exclusion flags (no part of the fusion).  The GPU works on positions
 * relative to the box's first block: with L = |X - origin| + |c - origin|
 * (point and camera centre), the rigid transform's result is within
 * 8 u L of the exact one per coordinate (u = 2^-24: three products and
 * three sums of magnitude <= L, each rounded once); the range |X_d| and eta
 * within 9 u L; a projection u = fx x / den + cx within
 * fx 8 u L (1 + 2 |x / den|) / den + 4 u |u| (den = z + xi |X_d|, the quotient
 * and the final FMA rounded once more).  The flags take four times these. */
#define OT_U 5.9604644775390625e-8   /* 2^-24 */
static double ot_lever(const ot_pose *pose, const double Xw[3], const double origin[3])
{
    /* |X - origin| + |camera centre - origin|, centre = -R^T t */
    double c[3], mt[3] = {-pose->t[0], -pose->t[1], -pose->t[2]};
    for (int i = 0; i < 3; ++i) c[i] = pose->R[0 * 3 + i] * mt[0] + pose->R[1 * 3 + i] * mt[1] + pose->R[2 * 3 + i] * mt[2];
    double a = 0, b = 0;
    for (int i = 0; i < 3; ++i) { a += (Xw[i] - origin[i]) * (Xw[i] - origin[i]); b += (c[i] - origin[i]) * (c[i] - origin[i]); }
    return sqrt(a) + sqrt(b);
}
static double ot_proj_margin(const ot_camera *cam, const double Xc[3], double u, double f, double c, double L)
{
    const double m = sqrt(Xc[0] * Xc[0] + Xc[1] * Xc[1] + Xc[2] * Xc[2]);
    const double den = Xc[2] + cam->xi * m;
    const double r = fabs(u - c) / f;   /* |x / den| */
    return 4.0 * (f * 8.0 * OT_U * L * (1.0 + 2.0 * r) / den + 4.0 * OT_U * (fabs(u) + 1.0));
}

/* Step 2.  vis[nb]: allocated blocks with a corner that projects into
 * [0, W-1] x [0, H-1].  edge[nb]: 1 where a corner projection lies within
 * its FP32 error bound of that border (a decision FP32 arithmetic may take
 * the other way). */
void or_tsdf_visible(const ot_camera *cam, const ot_pose *pose, double voxel, const int32_t b0[3],
                     const int32_t nb[3], const int32_t *alloc, int32_t *vis, int32_t *edge)
{
    const double B = 8.0 * voxel;
    for (int z = 0; z < nb[2]; ++z)
        for (int y = 0; y < nb[1]; ++y)
            for (int x = 0; x < nb[0]; ++x) {
                size_t i = ((size_t)z * nb[1] + y) * nb[0] + x;
                vis[i] = 0;
                edge[i] = 0;
                if (!alloc[i]) continue;
                for (int c = 0; c < 8; ++c) {
                    double Xw[3] = {(b0[0] + x + (c & 1)) * B, (b0[1] + y + ((c >> 1) & 1)) * B,
                                    (b0[2] + z + ((c >> 2) & 1)) * B};
                    double Xc[3], u, v;
                    to_cam(pose, Xw, Xc);
                    if (!or_project(cam, Xc, &u, &v)) continue;
                    double m = fmin(fmin(u, cam->width - 1 - u), fmin(v, cam->height - 1 - v));
                    const double origin[3] = {b0[0] * B, b0[1] * B, b0[2] * B};
                    const double L = ot_lever(pose, Xw, origin);
                    const double tol = fmax(ot_proj_margin(cam, Xc, u, cam->fx, cam->cx, L),
                                            ot_proj_margin(cam, Xc, v, cam->fy, cam->cy, L));
                    if (fabs(m) < tol) edge[i] = 1;
                    if (m >= 0.0) vis[i] = 1;
                }
            }
}

/* Step 3 (Eq. (2)).  D, W over the box's voxel grid.  edge_vox: 1 where the
 * voxel's update is decided within the FP32 error bound of the pixel choice
 * (a projection that close to a pixel boundary) or of the eta >= -mu test. */
void or_tsdf_integrate(const ot_camera *cam, const ot_pose *pose, const double *depth, int64_t pitch, double voxel,
                       double mu, double w_max, const int32_t b0[3], const int32_t nb[3], const int32_t *vis,
                       double *D, double *W, int32_t *edge_vox)
{
    const int nx = nb[0] * 8, ny = nb[1] * 8, nz = nb[2] * 8;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t o = ((size_t)k * ny + j) * nx + i;
                edge_vox[o] = 0;
                size_t bi = ((size_t)(k / 8) * nb[1] + j / 8) * nb[0] + i / 8;
                if (!vis[bi]) continue;
                double Xw[3] = {((double)b0[0] * 8 + i + 0.5) * voxel, ((double)b0[1] * 8 + j + 0.5) * voxel,
                                ((double)b0[2] * 8 + k + 0.5) * voxel};
                double Xc[3], u, v;
                to_cam(pose, Xw, Xc);
                if (!or_project(cam, Xc, &u, &v)) continue;
                double fu = floor(u + 0.5), fv = floor(v + 0.5);
                const double origin[3] = {(double)b0[0] * 8 * voxel, (double)b0[1] * 8 * voxel, (double)b0[2] * 8 * voxel};
                const double L = ot_lever(pose, Xw, origin);
                const double tu = ot_proj_margin(cam, Xc, u, cam->fx, cam->cx, L);
                const double tv = ot_proj_margin(cam, Xc, v, cam->fy, cam->cy, L);
                if (fabs(u + 0.5 - fu) < tu || fabs(u + 0.5 - fu - 1.0) < tu ||
                    fabs(v + 0.5 - fv) < tv || fabs(v + 0.5 - fv - 1.0) < tv)
                    edge_vox[o] = 1;
                if (fu < 0 || fv < 0 || fu > cam->width - 1 || fv > cam->height - 1) continue;
                double d_obs = depth[(int64_t)fv * pitch + (int64_t)fu];
                if (!(d_obs > 0.0) || !isfinite(d_obs)) continue;
                double range = sqrt(Xc[0] * Xc[0] + Xc[1] * Xc[1] + Xc[2] * Xc[2]);
                double eta = d_obs - range;
                if (fabs(eta + mu) < 4.0 * 9.0 * OT_U * L) edge_vox[o] = 1;
                if (eta < -mu) continue;
                double f = eta / mu < 1.0 ? eta / mu : 1.0;
                D[o] = (W[o] * D[o] + f) / (W[o] + 1.0);
                W[o] = W[o] + 1.0 < w_max ? W[o] + 1.0 : w_max;
            }
}
