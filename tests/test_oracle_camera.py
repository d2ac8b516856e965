"""Pins of the oracle's camera model (Sec. III-C, Eq. (1)) against closed
forms that do not go through the oracle's own formulas."""
import math

import numpy as np
import pytest

import oracle
from scenegen import Camera


def _cams():
    yield Camera(0.9, 360.0, 360.0, 512.0, 384.0, 1024, 768)
    yield Camera(0.0, 200.0, 210.0, 160.0, 120.0, 320, 240)
    yield Camera(0.5, 180.0, 180.0, 159.5, 127.5, 320, 256)
    yield Camera(1.0, 300.0, 300.0, 300.0, 200.0, 600, 400)


@pytest.mark.parametrize("cam", list(_cams()), ids=lambda c: f"xi{c.xi}")
def test_unit_norm_and_round_trip(cam):
    rng = np.random.default_rng(3)
    for _ in range(400):
        u = rng.uniform(0, cam.width - 1)
        v = rng.uniform(0, cam.height - 1)
        r = oracle.unproject(cam, u, v)
        assert r is not None
        assert abs(np.linalg.norm(r) - 1.0) < 1e-12
        for lam in (0.3, 7.0, 55.0):
            uv = oracle.project(cam, lam * r)
            assert uv is not None
            assert abs(uv[0] - u) < 1e-9 and abs(uv[1] - v) < 1e-9


def test_pinhole_special_case():
    """xi = 0 reduces Eq. (1) to the pinhole ray (x, y, 1) / |(x, y, 1)|."""
    cam = Camera(0.0, 200.0, 210.0, 160.0, 120.0, 320, 240)
    for u, v in [(0, 0), (10.5, 200.25), (319, 239), (160, 120)]:
        x, y = (u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy
        ref = np.array([x, y, 1.0]) / math.sqrt(x * x + y * y + 1)
        assert np.allclose(oracle.unproject(cam, u, v), ref, atol=1e-14)


@pytest.mark.parametrize("xi", [0.0, 0.4, 0.9, 1.0, 1.3])
def test_projection_polar_closed_form(xi):
    """A point at polar angle theta and azimuth phi lands at normalized radius
    sin(theta) / (cos(theta) + xi) (the unified model on the unit sphere)."""
    cam = Camera(xi, 250.0, 240.0, 300.0, 200.0, 600, 400)
    rng = np.random.default_rng(11)
    for _ in range(200):
        th = rng.uniform(0, math.radians(110))
        if math.cos(th) + xi <= 0.05:
            continue
        ph = rng.uniform(-math.pi, math.pi)
        rad = rng.uniform(0.2, 80.0)
        X = rad * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        m = math.sin(th) / (math.cos(th) + xi)
        exp_u = cam.cx + cam.fx * m * math.cos(ph)
        exp_v = cam.cy + cam.fy * m * math.sin(ph)
        u, v = oracle.project(cam, X)
        assert abs(u - exp_u) < 1e-9 and abs(v - exp_v) < 1e-9


def test_unprojection_numeric_inverse():
    """Eq. (1) against a numerical inversion of the polar closed form: solve
    sin(t) / (cos(t) + xi) = m for the polar angle with a bracketing root
    finder."""
    from scipy.optimize import brentq
    cam = Camera(0.9, 360.0, 360.0, 512.0, 384.0, 1024, 768)
    rng = np.random.default_rng(5)
    for _ in range(100):
        u, v = rng.uniform(0, 1023), rng.uniform(0, 767)
        x, y = (u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy
        m = math.hypot(x, y)
        th = brentq(lambda t: math.sin(t) / (math.cos(t) + cam.xi) - m, 0.0, math.acos(-cam.xi) - 1e-9,
                    xtol=1e-15)
        ph = math.atan2(y, x)
        exp = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        assert np.allclose(oracle.unproject(cam, u, v), exp, atol=1e-10)


def test_behind_viewpoint_rejected():
    cam = Camera(0.5, 100.0, 100.0, 50.0, 50.0, 100, 100)
    # polar angle 150 deg: cos + xi = -0.366 < 0
    th = math.radians(150)
    assert oracle.project(cam, [math.sin(th), 0.0, math.cos(th)]) is None
