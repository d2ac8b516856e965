"""Pins of the oracle's soft-argmin forward and its analytic FP64 gradient
(a differentiable form of the paper's plane sweep; the paper itself has no
learning in this stage).  The gradient is pinned by central finite
differences (eps = 1e-3) of the forward."""
import math

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import Level, Pose, Settings

LEVEL = Level(n_fronto=16, near=1.0, far=15.0, window=5)
SET = Settings(levels=[LEVEL], best_k=2, mode="soft", temperature=0.1)
# the finite-difference checks use a negligible variance floor so that no
# window crosses it under a perturbation (the loss would jump there)
SET_FD = Settings(levels=[LEVEL], best_k=2, mode="soft", temperature=0.1, var_floor=1e-6)
RECT = (14, 22, 12, 8)      # below the horizon: every window is textured


@pytest.fixture(scope="module")
def frame():
    return scenegen.random_small_frame(w=48, h=36, n_src=2, seed=4, f=30.0)


@pytest.fixture(scope="module")
def smooth_frame():
    """Images blurred (sigma = 1 px, kept as floats): the bilinear warp is
    only piecewise smooth, and its kinks at texel lines put an O(eps) error
    on pose finite differences; blurring shrinks the kinks."""
    from scipy.ndimage import gaussian_filter
    fr = scenegen.random_small_frame(w=48, h=36, n_src=2, seed=4, f=30.0)
    return scenegen.Frame(ref=gaussian_filter(fr.ref.astype(np.float64), 1.0),
                          srcs=[gaussian_filter(s.astype(np.float64), 1.0) for s in fr.srcs],
                          ref_cam=fr.ref_cam, src_cams=fr.src_cams, poses=fr.poses,
                          gt_range=fr.gt_range, gt_z=fr.gt_z)


def _loss(fr, srcs, poses, g, st=SET_FD):
    x0, y0, w, h = RECT
    ys, xs = np.mgrid[y0:y0 + h, x0:x0 + w]
    pix = np.stack([xs.ravel(), ys.ravel()], 1)
    rh, _ = oracle.soft_forward(LEVEL, st, fr.ref_cam, fr.ref, fr.src_cams, srcs, poses, pixels=pix)
    rh = np.where(np.isnan(rh), 0.0, rh)
    return float((rh * g.ravel()).sum())


def _rodrigues(w):
    th = np.linalg.norm(w)
    if th == 0:
        return np.eye(3)
    a = w / th
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def _perturbed(ps, xi):
    """Left perturbation exp(xi) * T: X_s -> R' X + t' with R' = exp(w) R,
    t' = exp(w) t + v (first order: X_s + v + w x X_s)."""
    v, w = xi[:3], xi[3:]
    Rw = _rodrigues(w)
    return Pose(Rw @ ps.R, Rw @ ps.t + v)


def test_soft_forward_limits(frame):
    """Low temperature turns the soft-argmin into the winner's inverse depth;
    rho_hat always lies inside the plane range."""
    x0, y0, w, h = RECT
    ys, xs = np.mgrid[y0:y0 + h, x0:x0 + w]
    pix = np.stack([xs.ravel(), ys.ravel()], 1)
    rh, lse = oracle.soft_forward(LEVEL, SET, frame.ref_cam, frame.ref, frame.src_cams, frame.srcs,
                                  frame.poses, pixels=pix)
    ok = np.isfinite(rh)
    assert ok.mean() > 0.9
    assert np.all(rh[ok] >= 1 / 15.0 - 1e-12) and np.all(rh[ok] <= 1.0 + 1e-12)
    cold = Settings(levels=[LEVEL], best_k=2, mode="soft", temperature=1e-4)
    rc, _ = oracle.soft_forward(LEVEL, cold, frame.ref_cam, frame.ref, frame.src_cams, frame.srcs,
                                frame.poses, pixels=pix)
    wta = oracle.sweep_level(LEVEL, SET, frame.ref_cam, frame.ref, frame.src_cams, frame.srcs, frame.poses,
                             pixels=pix, volume=True)
    vol = np.where(np.isnan(wta["volume"]), np.inf, wta["volume"])
    srt = np.sort(vol, 1)
    clear = ok & np.isfinite(srt[:, 1]) & (srt[:, 1] - srt[:, 0] > 0.01)
    rho_w = np.array([oracle.plane_param(LEVEL, SET, int(k))[0] for k in wta["index"][clear]])
    assert np.allclose(rc[clear], rho_w, atol=1e-9)


@pytest.mark.parametrize("eps,tol", [(1e-3, 1e-2), (1e-4, 2e-3)])
def test_pose_gradient_matches_central_differences(smooth_frame, eps, tol):
    """Measured relative l2 error 3.7e-3 at eps = 1e-3 and 8.7e-4 at
    eps = 1e-4: it shrinks with eps, as the texel-kink error does."""
    fr = smooth_frame
    rng = np.random.default_rng(0)
    g = rng.normal(size=(RECT[3], RECT[2]))
    _, gp = oracle.soft_backward(LEVEL, SET_FD, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, RECT, g)
    fd = np.zeros_like(gp)
    for s in range(2):
        for a in range(6):
            xi = np.zeros(6)
            xi[a] = eps
            pp = list(fr.poses)
            pp[s] = _perturbed(fr.poses[s], xi)
            lp = _loss(fr, fr.srcs, pp, g)
            pp[s] = _perturbed(fr.poses[s], -xi)
            lm = _loss(fr, fr.srcs, pp, g)
            fd[s, a] = (lp - lm) / (2 * eps)
    rel = np.linalg.norm(fd - gp) / np.linalg.norm(fd)
    assert rel < tol, (rel, fd, gp)


def test_image_gradient_matches_central_differences(frame):
    """The loss is smooth in the source values (no kinks), so eps = 1e-3
    agrees to 1e-5 relative."""
    rng = np.random.default_rng(1)
    g = rng.normal(size=(RECT[3], RECT[2]))
    gs, _ = oracle.soft_backward(LEVEL, SET_FD, frame.ref_cam, frame.ref, frame.src_cams, frame.srcs,
                                 frame.poses, RECT, g)
    eps = 1e-3
    srcs = [s.astype(np.float64) for s in frame.srcs]
    checked = 0
    for s in range(2):
        nz = np.argwhere(np.abs(gs[s]) > 1e-4 * np.abs(gs[s]).max())
        for j, i in nz[rng.choice(len(nz), size=6, replace=False)]:
            sp = [x.copy() for x in srcs]
            sp[s][j, i] += eps
            lp = _loss(frame, sp, frame.poses, g)
            sp[s][j, i] -= 2 * eps
            lm = _loss(frame, sp, frame.poses, g)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - gs[s][j, i]) <= 1e-5 * max(1e-3, abs(fd)) + 1e-9, (s, j, i, fd, gs[s][j, i])
            checked += 1
    assert checked == 12


GLEVEL = Level(n_fronto=8, near=1.0, far=15.0, n_ground=6, h_lo=-0.4, h_hi=0.4, window=5)
GSET_FD = Settings(levels=[GLEVEL], best_k=2, mode="soft", temperature=0.1, var_floor=1e-6)


def test_ground_hypothesis_is_the_inverse_depth_of_the_cut(frame):
    """A ground plane's value at a pixel is 1 / z of the point where the
    pixel's ray meets it: the oracle's own warp with an identity pose gives
    that point; a fronto plane's value is its parameter."""
    ident = Pose(np.eye(3), np.zeros(3))
    cam = frame.ref_cam
    checked = 0
    for k in range(GLEVEL.n_fronto + GLEVEL.n_ground):
        for (i, j) in ((5, 30), (24, 20), (40, 33), (10, 2)):
            w = oracle.warp(GLEVEL, GSET_FD, cam, cam, ident, k, i, j)
            rho = oracle.soft_hypothesis(GLEVEL, GSET_FD, cam, k, i, j)
            if k < GLEVEL.n_fronto:
                assert rho == pytest.approx(oracle.plane_param(GLEVEL, GSET_FD, k)[0], rel=1e-15)
            if w is None:
                continue
            assert rho == pytest.approx(1.0 / w[2][2], rel=1e-12), (k, i, j)
            checked += 1
    assert checked > 20


@pytest.mark.parametrize("eps,tol", [(1e-4, 2e-3)])
def test_pose_gradient_with_ground_planes_matches_central_differences(smooth_frame, eps, tol):
    """Fronto and ground planes together: each plane stands for its
    per-pixel inverse depth, in the forward and in the gradient alike."""
    fr = smooth_frame
    rng = np.random.default_rng(5)
    g = rng.normal(size=(RECT[3], RECT[2]))
    _, gp = oracle.soft_backward(GLEVEL, GSET_FD, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, RECT, g)
    x0, y0, w, h = RECT
    ys, xs = np.mgrid[y0:y0 + h, x0:x0 + w]
    pix = np.stack([xs.ravel(), ys.ravel()], 1)

    def loss(poses):
        rh, _ = oracle.soft_forward(GLEVEL, GSET_FD, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, poses, pixels=pix)
        return float((np.where(np.isnan(rh), 0.0, rh) * g.ravel()).sum())

    fd = np.zeros_like(gp)
    for s_ in range(2):
        for a in range(6):
            xi = np.zeros(6)
            xi[a] = eps
            pp = list(fr.poses)
            pp[s_] = _perturbed(fr.poses[s_], xi)
            lp = loss(pp)
            pp[s_] = _perturbed(fr.poses[s_], -xi)
            fd[s_, a] = (lp - loss(pp)) / (2 * eps)
    rel = np.linalg.norm(fd - gp) / np.linalg.norm(fd)
    assert np.linalg.norm(fd) > 0
    assert rel < tol, (rel, fd, gp)


def test_soft_argmin_golden():
    """The soft-argmin step against the hand-computed closed-form values of
    tests/golden/soft_argmin_hand.txt: a wrong temperature scale (exp(-C/2T)),
    a dropped max shift or a sign error in lse moves these by far more than
    the tolerance."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "soft_argmin_hand.txt")
    rows = [l for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for row in rows:
        T, C, rho, rh, lse = [f.split() for f in row.split("|")]
        got_rh, got_lse = oracle.soft_argmin([float(c) for c in C], [float(r) for r in rho], float(T[0]))
        want_rh, want_lse = float(rh[0]), float(lse[0])
        if np.isnan(want_rh):
            assert np.isnan(got_rh) and got_lse == -np.inf
        else:
            assert abs(got_rh - want_rh) <= 1e-14 and abs(got_lse - want_lse) <= 1e-14, (row, got_rh, got_lse)
