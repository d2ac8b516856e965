"""Degenerate and extreme inputs of the GPU sweep, through the C ABI:
images no larger than the window, textureless images, sources that see
nothing of the reference view, fewer usable sources than K, and a large
frame checked on sampled pixels."""
import dataclasses

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import Frame, Level, Pose, Settings
from tests.parity import assert_wta_parity, to_np, wta_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sweep(st, fr, **kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    ps = PlaneSweep(st, fr.ref_cam.width, fr.ref_cam.height, len(fr.srcs), **kw)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    torch.cuda.synchronize()
    g = to_np(out["merged"])
    ps.close()
    return g


def _all_invalid(g):
    assert np.all(g["index"] == -1) and np.all(np.isnan(g["depth"])) and np.all(g["cost1"] == np.inf)


@pytest.mark.parametrize("w,h,win", [(12, 10, 15), (9, 9, 9), (15, 40, 15)])
def test_image_not_wider_than_the_window(w, h, win):
    """A window as large as (or larger than) the image leaves at most one
    column of results; the oracle agrees on which."""
    fr = scenegen.random_small_frame(w=w, h=h, n_src=2, seed=41, f=0.62 * max(w, 16))
    lv = Level(n_fronto=6, near=1.0, far=25.0, window=win)
    st = Settings(levels=[lv], best_k=1)
    g = _sweep(st, fr)
    ref = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, volume=True)
    assert np.array_equal(g["index"] >= 0, ref["index"] >= 0)
    if w < win or h < win:
        _all_invalid(g)


def test_textureless_images_give_no_depth():
    fr = scenegen.random_small_frame(w=96, h=72, n_src=2, seed=42, f=60.0)
    flat = Frame(ref=np.full_like(fr.ref, 90), srcs=[np.full_like(s, 90) for s in fr.srcs], ref_cam=fr.ref_cam,
                 src_cams=fr.src_cams, poses=fr.poses, gt_range=fr.gt_range, gt_z=fr.gt_z)
    st = Settings(levels=[Level(n_fronto=8, near=1.0, far=25.0, n_ground=4, h_lo=-0.4, h_hi=0.4, window=7)],
                  best_k=2)
    _all_invalid(_sweep(st, flat))


def test_sources_looking_away_give_no_depth():
    """Every source turned 180 degrees about the vertical axis: no sample of
    any plane lands in a source image (points behind them), so no window is
    usable."""
    fr = scenegen.random_small_frame(w=96, h=72, n_src=2, seed=43, f=60.0)
    R = np.diag([-1.0, 1.0, -1.0])
    away = Frame(ref=fr.ref, srcs=fr.srcs, ref_cam=fr.ref_cam, src_cams=fr.src_cams,
                 poses=[Pose(R, np.array([0.3 * (i + 1), 0.0, 0.0])) for i in range(2)],
                 gt_range=fr.gt_range, gt_z=fr.gt_z)
    # a pinhole-like source (xi = 0) cannot see behind itself
    cams = [scenegen.Camera(0.0, c.fx, c.fy, c.cx, c.cy, c.width, c.height) for c in fr.src_cams]
    away.src_cams[:] = cams
    st = Settings(levels=[Level(n_fronto=8, near=1.0, far=25.0, window=7)], best_k=1)
    g = _sweep(st, away)
    _all_invalid(g)


def test_fewer_usable_sources_than_k():
    """K = 3 with one source that sees nothing: every plane averages the two
    usable sources (K' = min(K, valid)), as the oracle does."""
    fr = scenegen.random_small_frame(w=100, h=70, n_src=3, seed=44, f=62.0)
    R = np.diag([-1.0, 1.0, -1.0])
    cams = list(fr.src_cams)
    cams[2] = scenegen.Camera(0.0, cams[2].fx, cams[2].fy, cams[2].cx, cams[2].cy, cams[2].width, cams[2].height)
    poses = list(fr.poses)
    poses[2] = Pose(R, np.array([0.5, 0.0, 0.0]))
    part = Frame(ref=fr.ref, srcs=fr.srcs, ref_cam=fr.ref_cam, src_cams=cams, poses=poses,
                 gt_range=fr.gt_range, gt_z=fr.gt_z)
    lv = Level(n_fronto=10, near=1.0, far=25.0, window=5)
    st = Settings(levels=[lv], best_k=3)
    g = _sweep(st, part)
    ref = oracle.sweep_level(lv, st, part.ref_cam, part.ref, part.src_cams, part.srcs, part.poses, volume=True)
    s = wta_stats(g, ref, ref["volume"])
    print(s)
    assert s["n_oracle_valid"] > 500
    assert_wta_parity(s)


def test_large_frame_sampled():
    """4096 x 2048 with two sources and 48 + 16 planes (the largest frame the
    tests sweep), on 1000 sampled pixels.  (With a coarse plane set a flat
    cost curve turns FP32 cost rounding into visible subpixel shifts of far
    ranges, so the plane density is kept realistic.)"""
    fr = scenegen._street_frame(4096, 2048, 0.3516 * 4096, 1010, 2010, ss=1)
    fr = Frame(ref=fr.ref, srcs=fr.srcs[:2], ref_cam=fr.ref_cam, src_cams=fr.src_cams[:2], poses=fr.poses[:2],
               gt_range=fr.gt_range, gt_z=fr.gt_z)
    lv = Level(n_fronto=48, near=0.5, far=30.0, n_ground=16, h_lo=-0.5, h_hi=0.5, window=9)
    st = Settings(levels=[lv], best_k=2)
    g = _sweep(st, fr)
    rng = np.random.default_rng(9)
    pix = np.stack([rng.integers(0, 4096, 1000), rng.integers(0, 2048, 1000)], 1).astype(np.int32)
    ref = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, pixels=pix, volume=True)
    s = wta_stats({k: v[pix[:, 1], pix[:, 0]] for k, v in g.items()}, ref, ref["volume"])
    print(s)
    assert_wta_parity(s)


@pytest.mark.parametrize("family,chunks", [("fronto", 1), ("fronto", 4), ("ground", 1), ("ground", 3)])
def test_exact_ties_pick_the_lowest_plane(family, chunks):
    """A source at the reference's centre (pure rotation) sees every plane
    through the same map H = R, so the planes of one family tie exactly: the
    winner must be the family's first plane on every valid pixel, with
    cost2 = cost1 and no subpixel step, also when the planes are cut into
    chunks.  (Across families the costs agree only to rounding: the running
    window sums of a tile carry the rows above a pixel, and the ground family
    has none above the horizon.)"""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device
    fr = scenegen.random_small_frame(w=120, h=80, n_src=1, seed=3, f=70.0)
    th = np.radians(2.0)
    R = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
    src = Frame(ref=fr.ref, srcs=[fr.ref], ref_cam=fr.ref_cam, src_cams=[fr.ref_cam], poses=[Pose(R, np.zeros(3))],
                gt_range=None, gt_z=None)
    nf, ng = (12, 0) if family == "fronto" else (0, 6)
    lv = Level(n_fronto=nf, near=1.0, far=20.0, n_ground=ng, h_lo=-0.3, h_hi=0.3, window=5)
    st = Settings(levels=[lv], best_k=1)
    ps = PlaneSweep(st, 120, 80, 1)
    ps.set_cameras(0, src.ref_cam, src.src_cams, src.poses)
    ps.set_chunks(0, chunks)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(src)], [out])
    torch.cuda.synchronize()
    g = to_np(out["merged"])
    ps.close()
    v = g["index"] >= 0
    assert v.sum() > (2000 if family == "fronto" else 1000)
    assert np.all(g["index"][v] == 0)
    assert np.array_equal(g["cost2"][v], g["cost1"][v])
    assert np.all(g["delta"][v] == 0.0)


def test_maximum_frame_sampled():
    """The largest frame the library takes, 8192 x 8192 (one source, 48 + 16
    planes, 7x7), on 40,000 sampled pixels (about 3,400 oracle-valid): every
    index and offset of the sweep, the plane chunks and their merge at full
    size.  The variance floor is 9 grey levels squared per sample (window
    deviation at least 3 levels).  At this size FP32 source coordinates near
    8,000 px resolve about 1e-3 px, and the scene's texture is smooth at this
    scale: with the default floor of 1, windows of 1 to 1.5 levels of
    deviation pass, where ZNCC turns a 1e-3-level interpolation difference
    into a cost difference of about 1e-3, and the FP32 maps then leave the
    oracle's bar on a few pixels in a thousand."""
    fr = scenegen._street_frame(8192, 8192, 0.3516 * 8192, 1012, 2012, ss=1)
    fr = Frame(ref=fr.ref, srcs=fr.srcs[:1], ref_cam=fr.ref_cam, src_cams=fr.src_cams[:1], poses=fr.poses[:1],
               gt_range=None, gt_z=None)
    lv = Level(n_fronto=48, near=0.5, far=30.0, n_ground=16, h_lo=-0.5, h_hi=0.5, window=7)
    st = Settings(levels=[lv], best_k=1, var_floor=9.0)
    g = _sweep(st, fr)
    rng = np.random.default_rng(12)
    pix = np.stack([rng.integers(0, 8192, 40000), rng.integers(0, 8192, 40000)], 1).astype(np.int32)
    ref = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, pixels=pix, volume=True)
    s = wta_stats({k: v[pix[:, 1], pix[:, 0]] for k, v in g.items()}, ref, ref["volume"])
    print(s)
    assert_wta_parity(s)
    # the last row and column of the map are written (border marks included)
    assert np.all(g["index"][-3:] == -1) and np.all(g["index"][:, -3:] == -1)
    assert (g["index"] >= 0).mean() > 0.05   # about 8.5 % of the frame clears the floor


def test_non_finite_poses_and_cameras_are_rejected():
    """set_cameras refuses a NaN rotation, a non-finite translation and a NaN
    principal point with EINVAL, and leaves the context usable."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06132_amd import psweep as P
    from paper_1809_06132_amd.sweep import PlaneSweep
    fr = scenegen.random_small_frame(w=64, h=48, n_src=1, seed=3, f=40.0)
    st = Settings(levels=[Level(n_fronto=8, near=1.0, far=10.0, window=5)], best_k=1)
    ps = PlaneSweep(st, 64, 48, 1)
    good = fr.poses[0]
    bad_R = dataclasses.replace(good, R=np.where(np.eye(3) > 0, np.nan, 0.0))
    bad_t = dataclasses.replace(good, t=np.array([np.inf, 0.0, 0.0]))
    bad_cam = dataclasses.replace(fr.ref_cam, cx=float("nan"))
    for ref, poses in ((fr.ref_cam, [bad_R]), (fr.ref_cam, [bad_t]), (bad_cam, fr.poses)):
        with pytest.raises(P.PsweepError) as ei:
            ps.set_cameras(0, ref, fr.src_cams, poses)
        assert ei.value.status == -1
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    ps.close()
