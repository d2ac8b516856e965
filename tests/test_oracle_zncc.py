"""Pins of the oracle's matching cost: negative ZNCC over a window, with
cost 1 at ZNCC -1 and cost 0 at ZNCC +1 (Sec. III-A)."""
import os

import numpy as np
import pytest

import oracle
from scenegen import Camera, Level, Pose, Settings

GOLD = os.path.join(os.path.dirname(__file__), "golden")

CAM = Camera(0.9, 40.0, 40.0, 16.0, 12.0, 32, 24)
ID = Pose(np.eye(3), np.zeros(3))
LEVEL = Level(n_fronto=4, near=1.0, far=20.0, window=7)
SET = Settings(levels=[LEVEL], best_k=1, var_floor=1.0)


def _cost(ref, src, i=16, j=12, k=0, level=LEVEL):
    return oracle.window_cost(level, SET, CAM, ref, CAM, src, ID, k, i, j)


def _img(seed):
    return np.random.default_rng(seed).uniform(0, 255, size=(24, 32))


def test_matches_numpy_corrcoef():
    """With an identity warp the window samples are the source pixels, so the
    oracle's ZNCC must equal the library correlation coefficient."""
    for seed in range(20):
        ref, src = _img(seed), _img(100 + seed)
        for (i, j) in [(5, 5), (16, 12), (26, 17)]:
            c = _cost(ref, src, i, j)
            a = ref[j - 3:j + 4, i - 3:i + 4].ravel()
            b = src[j - 3:j + 4, i - 3:i + 4].ravel()
            z = np.corrcoef(a, b)[0, 1]
            assert c["valid"]
            assert abs(c["zncc"] - z) < 1e-12
            assert abs(c["cost"] - (1 - z) / 2) < 1e-12


def test_paper_endpoints_golden():
    """Cost endpoints printed in Sec. III-A: ZNCC -1 -> 1, ZNCC +1 -> 0."""
    rows = [l.split() for l in open(os.path.join(GOLD, "cost_endpoints.txt")) if l.strip() and l[0] != "#"]
    ref = _img(1)
    for z_s, c_s in rows:
        z, c = float(z_s), float(c_s)
        src = ref * (2.0 if z > 0 else -2.0) + 300.0   # affine copy: ZNCC is exactly +-1
        got = _cost(ref, src)
        assert got["valid"]
        assert abs(got["zncc"] - z) < 1e-12 and abs(got["cost"] - c) < 1e-12


@pytest.mark.parametrize("a,b", [(0.5, 10.0), (3.0, -40.0), (-1.5, 20.0), (-0.2, 0.0)])
def test_affine_invariance(a, b):
    """ZNCC is unchanged by I -> a I + b for a > 0 and flips sign for a < 0."""
    ref, src = _img(3), _img(4)
    base = _cost(ref, src)["zncc"]
    got = _cost(ref, a * src + b)["zncc"]
    assert abs(got - np.sign(a) * base) < 1e-12
    got_r = _cost(a * ref + b, src)["zncc"]
    assert abs(got_r - np.sign(a) * base) < 1e-12


def test_self_and_range():
    ref = _img(5)
    assert abs(_cost(ref, ref)["zncc"] - 1.0) < 1e-14
    rng = np.random.default_rng(9)
    for s in range(50):
        c = _cost(ref, rng.uniform(0, 255, (24, 32)), 16, 12)
        assert -1.0 <= c["zncc"] <= 1.0 and 0.0 <= c["cost"] <= 1.0


def test_variance_floor_and_borders():
    ref = _img(6)
    flat = np.full((24, 32), 77.0)
    assert not _cost(ref, flat)["valid"]          # source patch flat
    assert not _cost(flat, ref)["valid"]          # reference patch flat
    tiny = 77.0 + 0.5 * np.sign(np.random.default_rng(1).normal(size=(24, 32)))   # variance 0.25 < tau
    assert not _cost(ref, tiny)["valid"]
    assert not _cost(ref, ref, i=2, j=12)["valid"]   # window leaves the image
    assert _cost(ref, ref, i=5, j=5)["valid"]


def test_out_of_view_sample_invalidates_window():
    """A window with a single sample outside the source image is unusable."""
    ref = _img(7)
    ps = Pose(np.eye(3), np.array([0.0, 0.0, 0.0]))
    # shift the source camera's principal point so that column 0 of the
    # reference maps to u = -0.5 in the source
    sc = Camera(CAM.xi, CAM.fx, CAM.fy, CAM.cx - 0.5, CAM.cy, CAM.width, CAM.height)
    c_edge = oracle.window_cost(LEVEL, SET, CAM, ref, sc, ref, ps, 0, 3, 12)
    c_in = oracle.window_cost(LEVEL, SET, CAM, ref, sc, ref, ps, 0, 4, 12)
    assert not c_edge["valid"] and c_in["valid"]
