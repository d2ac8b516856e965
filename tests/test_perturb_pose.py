"""The library's pose update for the soft backward's left perturbation
xi = (v, omega): R' = Exp(omega) R, t' = Exp(omega) t + v (host code, no GPU).
Pinned against scipy's rotation-vector exponential, the first-order form at
small angles, and a rotation by pi about an axis."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from tests.test_abi import _lib_or_skip


def _perturb(R, t, xi):
    from paper_1809_06132_amd import psweep
    Ro, to = psweep.psweep_perturb_pose(np.ravel(R), np.ravel(t), np.ravel(xi))
    return np.asarray(Ro).reshape(3, 3), np.asarray(to)


@pytest.mark.parametrize("angle", [0.0, 1e-12, 1e-6, 9.9e-5, 1.01e-4, 0.01, 0.7, 2.5, math.pi])
def test_matches_rotation_vector_exponential(angle):
    _lib_or_skip()
    rng = np.random.default_rng(int(angle * 1e6) % 1000 + 3)
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    omega, v = axis * angle, rng.normal(size=3)
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t = rng.normal(size=3) * 2.0
    Ro, to = _perturb(R, t, np.concatenate([v, omega]))
    E = Rotation.from_rotvec(omega).as_matrix()
    assert np.allclose(Ro, E @ R, rtol=0, atol=1e-14)
    assert np.allclose(to, E @ t + v, rtol=0, atol=1e-13)
    assert np.allclose(Ro @ Ro.T, np.eye(3), atol=1e-14)


def test_first_order_is_the_left_perturbation():
    """X -> X + v + omega x X to first order in xi."""
    _lib_or_skip()
    rng = np.random.default_rng(9)
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t, X = rng.normal(size=3), rng.normal(size=3) * 5.0
    xi = rng.normal(size=6) * 1e-7
    Ro, to = _perturb(R, t, xi)
    Xs = R @ X + t
    first = Xs + xi[:3] + np.cross(xi[3:], Xs)
    assert np.allclose(Ro @ X + to, first, rtol=0, atol=1e-12)


def test_rejects_bad_arguments():
    _lib_or_skip()
    import ctypes
    from paper_1809_06132_amd import psweep
    L = psweep.lib()
    d9, d3, d6 = (ctypes.c_double * 9)(*np.eye(3).ravel()), (ctypes.c_double * 3)(), (ctypes.c_double * 6)()
    o9, o3 = (ctypes.c_double * 9)(), (ctypes.c_double * 3)()
    assert L.psweep_perturb_pose(None, d3, d6, o9, o3) == psweep.EINVAL
    assert L.psweep_perturb_pose(d9, d3, d6, None, o3) == psweep.EINVAL
    d6[4] = float("nan")
    assert L.psweep_perturb_pose(d9, d3, d6, o9, o3) == psweep.EINVAL
