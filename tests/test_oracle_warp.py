"""Pins of the oracle's plane-induced warp (Sec. III-A: each plane position
defines a mapping of reference pixels into the other images)."""
import math

import numpy as np
import pytest

import oracle
from scenegen import Camera, Level, Pose, Settings


def _rot(axis, deg):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    t = math.radians(deg)
    return np.eye(3) + math.sin(t) * K + (1 - math.cos(t)) * K @ K


LEVEL = Level(n_fronto=8, near=0.5, far=30.0, n_ground=6, h_lo=-0.5, h_hi=0.5, window=7)
SET = Settings(levels=[LEVEL], ground_n=(0.0, 1.0, 0.0), ground_d=1.5)


def test_identity_pose_is_identity_warp():
    cam = Camera(0.9, 180.0, 180.0, 160.0, 128.0, 320, 256)
    ps = Pose(np.eye(3), np.zeros(3))
    rng = np.random.default_rng(0)
    for k in range(LEVEL.n_fronto + LEVEL.n_ground):
        for _ in range(30):
            u, v = rng.uniform(0, 319), rng.uniform(0, 255)
            w = oracle.warp(LEVEL, SET, cam, cam, ps, k, u, v)
            if w is None:     # ray misses the plane (e.g. above the horizon)
                continue
            assert abs(w[0] - u) < 1e-9 and abs(w[1] - v) < 1e-9


def test_pinhole_matches_textbook_homography():
    """With xi = 0 the warp is the plane-induced homography
    K_s (R + t n^T / d) K_r^-1 of the plane n . X = d."""
    rc = Camera(0.0, 200.0, 210.0, 160.0, 120.0, 320, 240)
    sc = Camera(0.0, 190.0, 195.0, 150.0, 125.0, 300, 250)
    R = _rot([0.2, 1.0, 0.1], 4.0)
    t = np.array([0.4, -0.05, 0.1])
    ps = Pose(R, t)
    Kr = np.array([[rc.fx, 0, rc.cx], [0, rc.fy, rc.cy], [0, 0, 1.0]])
    Ks = np.array([[sc.fx, 0, sc.cx], [0, sc.fy, sc.cy], [0, 0, 1.0]])
    rng = np.random.default_rng(1)
    n_checked = 0
    for k in range(LEVEL.n_fronto + LEVEL.n_ground):
        if k < LEVEL.n_fronto:
            rho = 1 / 30.0 + k * (1 / 0.5 - 1 / 30.0) / (LEVEL.n_fronto - 1)
            n, d = np.array([0, 0, 1.0]), 1 / rho
        else:
            h = -0.5 + (k - LEVEL.n_fronto) * 1.0 / (LEVEL.n_ground - 1)
            n, d = np.array([0, 1.0, 0]), 1.5 - h
        Hm = Ks @ (R + np.outer(t, n) / d) @ np.linalg.inv(Kr)
        for _ in range(20):
            u, v = rng.uniform(0, 319), rng.uniform(0, 239)
            w = oracle.warp(LEVEL, SET, rc, sc, ps, k, u, v)
            ray = np.linalg.inv(Kr) @ [u, v, 1.0]
            if n @ ray <= 0:
                assert w is None
                continue
            p = Hm @ [u, v, 1.0]
            if p[2] <= 0:
                continue
            assert w is not None
            assert abs(w[0] - p[0] / p[2]) < 1e-8 and abs(w[1] - p[1] / p[2]) < 1e-8
            n_checked += 1
    assert n_checked > 100


def test_ray_plane_residual():
    """The 3D point behind a warp lies on its plane: n . (R^T (X_s - t)) = d."""
    cam = Camera(0.9, 180.0, 180.0, 160.0, 128.0, 320, 256)
    R = _rot([1.0, 0.3, -0.2], 3.0)
    t = np.array([-0.5, 0.02, 0.1])
    ps = Pose(R, t)
    rng = np.random.default_rng(2)
    for k in range(LEVEL.n_fronto + LEVEL.n_ground):
        if k < LEVEL.n_fronto:
            rho = 1 / 30.0 + k * (1 / 0.5 - 1 / 30.0) / (LEVEL.n_fronto - 1)
            n, d = np.array([0, 0, 1.0]), 1 / rho
        else:
            h = -0.5 + (k - LEVEL.n_fronto) * 1.0 / (LEVEL.n_ground - 1)
            n, d = np.array([0, 1.0, 0]), 1.5 - h
        for _ in range(20):
            w = oracle.warp(LEVEL, SET, cam, cam, ps, k, rng.uniform(0, 319), rng.uniform(0, 255))
            if w is None:
                continue
            X = R.T @ (w[2] - t)
            assert abs(n @ X - d) < 1e-9 * max(1.0, d)


def test_plane_parameters():
    """Fronto planes uniform in inverse depth far -> near, ground planes
    uniform in height low -> high (the plane-spacing reading)."""
    r0, dr = oracle.plane_param(LEVEL, SET, 0)
    r7, _ = oracle.plane_param(LEVEL, SET, 7)
    assert abs(r0 - 1 / 30.0) < 1e-15 and abs(r7 - 2.0) < 1e-12
    assert abs(dr - (2.0 - 1 / 30.0) / 7) < 1e-15
    h0, dh = oracle.plane_param(LEVEL, SET, 8)
    h5, _ = oracle.plane_param(LEVEL, SET, 13)
    assert abs(h0 + 0.5) < 1e-15 and abs(h5 - 0.5) < 1e-12 and abs(dh - 0.2) < 1e-15
