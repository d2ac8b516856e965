"""Pins of the oracle's TSDF fusion (Sec. III-C, Eq. (1)-(2)): geometry of a
fused wall, the running average and its weight cap, block allocation against
dense sampling of the truncation segments, the moving local map and the
observation threshold."""
import numpy as np
import pytest

import oracle
from scenegen import Camera, Pose

VOX, MU = 0.1, 0.3
CAM = Camera(0.0, 100.0, 100.0, 31.5, 23.5, 64, 48)        # xi = 0: a pinhole, for closed forms
FISH = Camera(0.9, 40.0, 40.0, 31.5, 23.5, 64, 48)
I = Pose(np.eye(3), np.zeros(3))


def _wall_ranges(cam, z0):
    """Range along each pixel's Eq. (1) ray to the plane z = z0 (camera frame)."""
    v, u = np.mgrid[0:cam.height, 0:cam.width]
    out = np.full((cam.height, cam.width), np.nan)
    for j in range(cam.height):
        for i in range(cam.width):
            r = oracle.unproject(cam, i, j)
            if r is not None and r[2] > 1e-9:
                out[j, i] = z0 / r[2]
    return out


def _axis_column(o, D):
    ix = -o.b0[0] * 8          # voxel whose centre is x = +0.05 (just right of the axis)
    iy = -o.b0[1] * 8
    z = (o.b0[2] * 8 + np.arange(D.shape[0]) + 0.5) * VOX
    return z, D[:, iy, ix]


def test_wall_zero_crossing_and_slope():
    z0 = 5.03
    o = oracle.TsdfOracle(VOX, MU, (8, 4, 16), min_obs=1)
    o.integrate(CAM, I, _wall_ranges(CAM, z0), (0.0, 0.0, 5.0))
    z, d = _axis_column(o, o.extract())
    ok = np.isfinite(d)
    z, d = z[ok], d[ok]
    # D = 1 in front of the band, no update further than mu behind the wall
    assert np.all(d[z < z0 - MU - 0.05] == 1.0)
    assert z.max() <= z0 + MU + 1e-9
    # a zero crossing within half a voxel of the wall, slope -1/mu inside the band
    k = np.nonzero((d[:-1] > 0) & (d[1:] <= 0))[0]
    assert len(k) == 1
    zc = z[k[0]] + VOX * d[k[0]] / (d[k[0]] - d[k[0] + 1])
    assert abs(zc - z0) < 0.5 * VOX
    band = (z > z0 - MU + 0.05) & (z < z0 + MU - 0.05)
    slope = np.diff(d[band]) / VOX
    assert np.allclose(slope, -1.0 / MU, rtol=0.02)


def test_running_average_and_weight_cap():
    z0, z1 = 5.03, 5.11
    r0, r1 = _wall_ranges(CAM, z0), _wall_ranges(CAM, z1)
    a = oracle.TsdfOracle(VOX, MU, (8, 4, 16), min_obs=1)
    b = oracle.TsdfOracle(VOX, MU, (8, 4, 16), min_obs=1)
    a.integrate(CAM, I, r0, (0, 0, 5.0))
    D0, W0 = a.D.copy(), a.W.copy()
    a.integrate(CAM, I, r0, (0, 0, 5.0))            # the same map again: same values, twice the weight
    upd = W0 > 0
    assert np.allclose(a.D[upd], D0[upd]) and np.all(a.W[upd] == 2)
    b.integrate(CAM, I, r1, (0, 0, 5.0))
    D1, W1 = b.D.copy(), b.W.copy()
    c = oracle.TsdfOracle(VOX, MU, (8, 4, 16), min_obs=1)
    c.integrate(CAM, I, r0, (0, 0, 5.0))
    c.integrate(CAM, I, r1, (0, 0, 5.0))
    both = (W0 > 0) & (W1 > 0)
    assert both.sum() > 100
    assert np.allclose(c.D[both], 0.5 * (D0[both] + D1[both]))
    cap = oracle.TsdfOracle(VOX, MU, (8, 4, 16), w_max=3, min_obs=1)
    for _ in range(5):
        cap.integrate(CAM, I, r0, (0, 0, 5.0))
    assert cap.W.max() == 3 and np.allclose(cap.D[upd], D0[upd])


def test_allocation_matches_dense_sampling():
    """Every block that holds a point of some pixel's segment [d - mu, d + mu]
    is allocated; every allocated block not merely grazed holds such a point."""
    rng = np.random.default_rng(3)
    depth = rng.uniform(2.0, 9.0, (48, 64))
    depth[rng.random((48, 64)) < 0.2] = np.nan
    th = 0.2
    R = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
    pose = Pose(R, np.array([0.3, -0.1, 0.4]))
    o = oracle.TsdfOracle(VOX, MU, (32, 8, 32), min_obs=1)
    centre = (0.0, 0.0, 4.0)
    info = o.integrate(FISH, pose, depth, centre)
    B = 8 * VOX
    sampled = np.zeros_like(o.alloc)
    s = np.linspace(0.0, 1.0, 2001)
    for j in range(48):
        for i in range(64):
            d = depth[j, i]
            if not np.isfinite(d):
                continue
            r = oracle.unproject(FISH, i, j)
            lam = max(d - MU, 0.0) + s * (d + MU - max(d - MU, 0.0))
            Pc = lam[:, None] * np.asarray(r)[None]
            Pw = (Pc - pose.t) @ R                     # R^T (P - t), row vectors
            b = np.floor(Pw / B).astype(int) - o.b0
            inside = np.all((b >= 0) & (b < o.nb), 1)
            for bx, by, bz in b[inside]:
                sampled[bz, by, bx] = 1
    assert np.all(o.alloc[sampled == 1] == 1)
    extra = (o.alloc == 1) & (sampled == 0)
    # a block holding no sample point is met by a piece shorter than the
    # sample spacing, which cannot reach deeper into it than that spacing
    assert np.all(info["pen"][extra] < (2 * MU) / 2000)
    assert o.alloc.sum() > 200


def test_map_follows_its_centre():
    o = oracle.TsdfOracle(VOX, MU, (8, 4, 16), min_obs=1)
    o.integrate(CAM, I, _wall_ranges(CAM, 5.03), (0.0, 0.0, 5.0))
    A, D = o.alloc.copy(), o.D.copy()
    b0 = o.b0.copy()
    o.set_centre((0.8, 0.0, 5.0))                   # one block to the right
    assert o.b0[0] == b0[0] + 1
    assert np.array_equal(o.alloc[:, :, :-1], A[:, :, 1:]) and np.all(o.alloc[:, :, -1] == 0)
    assert np.array_equal(o.D[:, :, :-8], D[:, :, 8:]) and np.all(o.D[:, :, -8:] == 1.0)
    o.set_centre((100.0, 0.0, 5.0))                 # far away: everything leaves the map
    assert o.alloc.sum() == 0 and np.all(o.W == 0)


def test_blocks_need_three_observations():
    r = _wall_ranges(CAM, 5.03)
    o = oracle.TsdfOracle(VOX, MU, (8, 4, 16), min_obs=3)
    for n in range(1, 4):
        o.integrate(CAM, I, r, (0.0, 0.0, 5.0))
        e = o.extract()
        assert (np.isfinite(e).sum() > 0) == (n >= 3)


def test_nothing_behind_the_camera_is_visible():
    o = oracle.TsdfOracle(VOX, MU, (8, 4, 16), min_obs=1)
    info = o.integrate(CAM, I, _wall_ranges(CAM, 5.03), (0.0, 0.0, 0.0))
    zb = (o.b0[2] + np.arange(o.nb[2]) + 1) * 8 * VOX     # far face of every block row
    assert np.all(info["visible"][zb <= 0] == 0)
    assert np.array_equal(info["visible"], o.alloc)      # a frontal wall: its band is in view
