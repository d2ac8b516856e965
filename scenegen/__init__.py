"""Seeded synthetic inputs for the fisheye plane-sweep tests and benchmarks.

This package is the one input generator shared by the oracle side and the
GPU side.  It holds none of the plane-sweep method's arithmetic: it builds
camera rigs, textured ray-cast scenes and the per-workload sweep settings
(plane counts, ranges, windows), and renders what each camera sees.

Workloads (the synthetic stand-ins for the paper's private 1024x544 NIR
sequences, whose settings are given in Sec. III-A and Sec. IV-A):

* ``C1``  320x256, 1 source, 32 fronto planes, ZNCC 7x7, WTA (tiny parity case)
* ``C2``  1024x768, 3 sources, 128 fronto + 64 ground planes, 9x9, best-2
* ``C3``  C2 rig/scene, two levels: 512x384 downsampled (96 planes, 7x7) plus
          a full-resolution 512x384 centre crop (64 planes over 15-60 m, 9x9)
* ``C4``  640x480, 2 sources, 64 fronto planes, 7x7, soft-argmin (T = 0.1)
* ``C5``  16 frame sets of mixed size (1280x960 / 1024x768 / 640x480),
          4 sources, 192 fronto + 64 ground planes per level, two levels
* ``paper`` 1024x544, 4 sources, 64 fronto + 30 ground planes, 512x272 low
          level (7x7) plus a 572x332 crop (9x9), as in Sec. III-A
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librender.so")


def build(force: bool = True) -> str:
    """Compile the renderer with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "render.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


# ----------------------------------------------------------------------------
# data types
# ----------------------------------------------------------------------------
@dataclass
class Camera:
    """Unified (Mei) fisheye camera: mirror parameter xi plus a pinhole part."""
    xi: float
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


@dataclass
class Pose:
    """Rigid transform from the reference frame to a source frame:
    X_src = R @ X_ref + t (metres)."""
    R: np.ndarray
    t: np.ndarray


@dataclass
class Level:
    n_fronto: int
    near: float
    far: float
    n_ground: int = 0
    h_lo: float = -0.5
    h_hi: float = 0.5
    window: int = 9
    downsample: int = 1
    crop: tuple = (0, 0, 0, 0)   # (x, y, w, h) in full-resolution pixels; w == 0: none


@dataclass
class Settings:
    levels: list
    best_k: int = 2
    var_floor: float = 1.0
    ground_n: tuple = (0.0, 1.0, 0.0)
    ground_d: float = 1.5
    mode: str = "wta"            # "wta" or "soft"
    temperature: float = 0.1


@dataclass
class Frame:
    ref: np.ndarray              # uint8 [H, W]
    srcs: list                   # uint8 [H_s, W_s] per source
    ref_cam: Camera
    src_cams: list
    poses: list                  # Pose per source
    gt_range: np.ndarray         # float32 [H, W], NaN = sky
    gt_z: np.ndarray


@dataclass
class Workload:
    name: str
    frames: list
    settings: Settings
    seeds: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# renderer binding
# ----------------------------------------------------------------------------
class _Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("tex", ctypes.c_int32 * 6)]


class _Tex(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("u0", ctypes.c_double), ("v0", ctypes.c_double), ("pitch", ctypes.c_double)]


class _Cam(ctypes.Structure):
    _fields_ = [("xi", ctypes.c_double), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("Rcw", ctypes.c_double * 9), ("centre", ctypes.c_double * 3)]


class _Scene(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int32), ("boxes", ctypes.POINTER(_Box)),
                ("ground_y", ctypes.c_double), ("ground_tex", ctypes.c_int32),
                ("ground_max_range", ctypes.c_double), ("sky_range", ctypes.c_double),
                ("sky_value", ctypes.c_double),
                ("texs", ctypes.POINTER(_Tex)), ("atlas", ctypes.POINTER(ctypes.c_float))]


@functools.lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.rg_render.argtypes = [ctypes.POINTER(_Scene), ctypes.POINTER(_Cam), ctypes.c_int32,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.rg_render.restype = None
    return lib


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------
class Scene:
    """Ground plane (world y = ground_y, y pointing down) plus textured boxes.

    Every surface carries a world-space texel grid of values drawn from
    U{0..255} (numpy PCG64) and blurred with a Gaussian of sigma = 1 texel
    (truncated at 3 sigma); the renderer interpolates it bilinearly."""

    def __init__(self, rng: np.random.Generator, ground_y: float = 1.5):
        from scipy.ndimage import gaussian_filter
        self._blur = lambda g: gaussian_filter(g, sigma=1.0, truncate=3.0, mode="nearest")
        self.rng = rng
        self.ground_y = ground_y
        self.boxes = []
        self.tex_meta = []
        self.tex_data = []
        self._offset = 0
        self.ground_tex = self._new_tex(-40.0, 40.0, -10.0, 90.0, 0.10)

    def _new_tex(self, u_lo, u_hi, v_lo, v_hi, pitch):
        nu = int(math.ceil((u_hi - u_lo) / pitch)) + 3
        nv = int(math.ceil((v_hi - v_lo) / pitch)) + 3
        g = self.rng.integers(0, 256, size=(nv, nu)).astype(np.float64)
        g = self._blur(g).astype(np.float32)
        self.tex_meta.append((self._offset, nu, nv, u_lo - pitch, v_lo - pitch, pitch))
        self.tex_data.append(g.ravel())
        self._offset += g.size
        return len(self.tex_meta) - 1

    def add_box(self, lo, hi, pitch=0.05):
        lo = [float(v) for v in lo]
        hi = [float(v) for v in hi]
        texs = []
        for axis in range(3):
            if axis == 0:
                ua, va = 2, 1
            elif axis == 1:
                ua, va = 0, 2
            else:
                ua, va = 0, 1
            for _side in range(2):
                texs.append(self._new_tex(lo[ua], hi[ua], lo[va], hi[va], pitch))
        self.boxes.append((lo, hi, texs))

    def _struct(self):
        nb = len(self.boxes)
        boxes = (_Box * max(nb, 1))()
        for i, (lo, hi, texs) in enumerate(self.boxes):
            boxes[i].lo[:] = lo
            boxes[i].hi[:] = hi
            boxes[i].tex[:] = texs
        texs = (_Tex * len(self.tex_meta))()
        for i, (off, nu, nv, u0, v0, p) in enumerate(self.tex_meta):
            texs[i].offset, texs[i].nu, texs[i].nv = off, nu, nv
            texs[i].u0, texs[i].v0, texs[i].pitch = u0, v0, p
        atlas = np.ascontiguousarray(np.concatenate(self.tex_data).astype(np.float32))
        sc = _Scene()
        sc.n_boxes = nb
        sc.boxes = ctypes.cast(boxes, ctypes.POINTER(_Box))
        sc.ground_y = self.ground_y
        sc.ground_tex = self.ground_tex
        sc.ground_max_range = 80.0
        sc.sky_range = 100.0
        sc.sky_value = 128.0
        sc.texs = ctypes.cast(texs, ctypes.POINTER(_Tex))
        sc.atlas = atlas.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        return sc, (boxes, texs, atlas)

    def render(self, cam: Camera, Rcw: np.ndarray, centre, ss: int = 4, with_gt: bool = False):
        """Image (uint8, round-half-even of the sub-pixel mean) and, if asked,
        ground-truth range and z of each pixel's centre ray."""
        sc, keep = self._struct()
        c = _Cam()
        c.xi, c.fx, c.fy, c.cx, c.cy = cam.xi, cam.fx, cam.fy, cam.cx, cam.cy
        c.width, c.height = cam.width, cam.height
        c.Rcw[:] = [float(v) for v in np.asarray(Rcw, dtype=np.float64).ravel()]
        c.centre[:] = [float(v) for v in centre]
        img = np.empty((cam.height, cam.width), np.float32)
        rng_ = np.empty_like(img) if with_gt else None
        z_ = np.empty_like(img) if with_gt else None
        _lib().rg_render(ctypes.byref(sc), ctypes.byref(c), ss, img.ctypes.data,
                         rng_.ctypes.data if with_gt else None, z_.ctypes.data if with_gt else None)
        del keep
        u8 = np.clip(np.rint(img), 0, 255).astype(np.uint8)
        return (u8, rng_, z_) if with_gt else u8


# ----------------------------------------------------------------------------
# rigs
# ----------------------------------------------------------------------------
def _small_rotation(rng: np.random.Generator, max_deg: float = 5.0) -> np.ndarray:
    """Rotation about an axis uniform on the sphere by an angle U[0, max_deg)."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = math.radians(rng.uniform(0.0, max_deg))
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def _pose_from(Rcw: np.ndarray, centre) -> Pose:
    """Pose mapping reference-frame points into a camera with camera->world
    rotation Rcw and centre `centre` (the reference frame is the world)."""
    R = Rcw.T.copy()
    t = -R @ np.asarray(centre, dtype=np.float64)
    return Pose(R=R, t=t)


def _fisheye(w: int, h: int, f: float, xi: float = 0.9) -> Camera:
    return Camera(xi=xi, fx=f, fy=f, cx=w / 2.0, cy=h / 2.0, width=w, height=h)


# ----------------------------------------------------------------------------
# scenes per workload
# ----------------------------------------------------------------------------
def _boxes_scene(rng, n_boxes, z_lo, z_hi, x_lo, x_hi, facades: bool) -> Scene:
    sc = Scene(rng)
    gy = sc.ground_y
    if facades:
        for sign in (-1.0, 1.0):
            x0 = sign * rng.uniform(6.0, 9.0)
            lo = [min(x0, x0 + sign * 0.5), gy - 10.0, -5.0]
            hi = [max(x0, x0 + sign * 0.5), gy, 100.0]
            sc.add_box(lo, hi)
    for _ in range(n_boxes):
        zf = rng.uniform(z_lo, z_hi)
        xc = rng.uniform(x_lo, x_hi)
        sx, sy, sz = rng.uniform(0.5, 2.5, size=3)
        sc.add_box([xc - sx / 2, gy - sy, zf], [xc + sx / 2, gy, zf + sz])
    return sc


def _render_frame(sc: Scene, ref_cam: Camera, src_cams, rots, centres, ss) -> Frame:
    ref, gt_r, gt_z = sc.render(ref_cam, np.eye(3), (0.0, 0.0, 0.0), ss=ss, with_gt=True)
    srcs, poses = [], []
    for cam, Rcw, c in zip(src_cams, rots, centres):
        srcs.append(sc.render(cam, Rcw, c, ss=ss))
        poses.append(_pose_from(Rcw, c))
    return Frame(ref=ref, srcs=srcs, ref_cam=ref_cam, src_cams=list(src_cams), poses=poses,
                 gt_range=gt_r, gt_z=gt_z)


def _street_rig(rng, extra_right: bool = False):
    b = rng.uniform(0.3, 1.2, size=3)
    side = 1.0 if rng.uniform() < 0.5 else -1.0
    centres = [(-b[0], 0.0, 0.0), (b[1], 0.0, 0.0), (side * b[2], 0.0, -0.2)]
    if extra_right:
        centres.append((0.9, 0.0, 0.0))
    rots = [_small_rotation(rng) for _ in centres]
    return centres, rots


def _c1(ss=4) -> Workload:
    srng, rrng = np.random.default_rng(1001), np.random.default_rng(2001)
    cam = Camera(xi=0.9, fx=180.0, fy=180.0, cx=160.0, cy=128.0, width=320, height=256)
    sc = _boxes_scene(srng, 3, 2.0, 25.0, -4.0, 4.0, facades=False)
    _ = rrng  # rig is fixed for C1: one source 0.3 m to the right, no rotation
    fr = _render_frame(sc, cam, [cam], [np.eye(3)], [(0.3, 0.0, 0.0)], ss)
    st = Settings(levels=[Level(n_fronto=32, near=0.5, far=30.0, window=7)], best_k=1)
    return Workload("C1", [fr], st, {"scene": 1001, "rig": 2001})


def _street_frame(w, h, f, scene_seed, rig_seed, ss, extra_right=False) -> Frame:
    srng, rrng = np.random.default_rng(scene_seed), np.random.default_rng(rig_seed)
    cam = _fisheye(w, h, f)
    sc = _boxes_scene(srng, 20, 2.0, 40.0, -5.0, 5.0, facades=True)
    centres, rots = _street_rig(rrng, extra_right)
    return _render_frame(sc, cam, [cam] * len(centres), rots, centres, ss)


def _c2(ss=4) -> Workload:
    fr = _street_frame(1024, 768, 360.0, 1002, 2002, ss)
    st = Settings(levels=[Level(n_fronto=128, near=0.5, far=30.0, n_ground=64, h_lo=-0.5, h_hi=0.5,
                                window=9)], best_k=2)
    return Workload("C2", [fr], st, {"scene": 1002, "rig": 2002})


def c3_settings() -> Settings:
    return Settings(levels=[
        Level(n_fronto=96, near=0.5, far=30.0, window=7, downsample=2),
        Level(n_fronto=64, near=15.0, far=60.0, window=9, downsample=1, crop=(256, 192, 512, 384)),
    ], best_k=2)


def _c3(ss=4) -> Workload:
    fr = _street_frame(1024, 768, 360.0, 1002, 2002, ss)
    return Workload("C3", [fr], c3_settings(), {"scene": 1002, "rig": 2002})


def _c4(ss=4) -> Workload:
    srng, rrng = np.random.default_rng(1004), np.random.default_rng(2004)
    cam = _fisheye(640, 480, 225.0)
    sc = _boxes_scene(srng, 20, 2.0, 40.0, -5.0, 5.0, facades=True)
    centres = [(-0.3, 0.0, 0.0), (0.6, 0.0, 0.0)]
    rots = [_small_rotation(rrng) for _ in centres]
    fr = _render_frame(sc, cam, [cam, cam], rots, centres, ss)
    st = Settings(levels=[Level(n_fronto=64, near=0.5, far=30.0, window=7)], best_k=2,
                  mode="soft", temperature=0.1)
    return Workload("C4", [fr], st, {"scene": 1004, "rig": 2004})


C5_SIZES = [(1280, 960), (1024, 768), (640, 480)]


def c5_settings(w: int, h: int) -> Settings:
    cw, ch = w // 2, h // 2
    return Settings(levels=[
        Level(n_fronto=192, near=0.5, far=30.0, n_ground=64, window=7, downsample=2),
        Level(n_fronto=192, near=15.0, far=60.0, n_ground=64, window=9, downsample=1,
              crop=((w - cw) // 2, (h - ch) // 2, cw, ch)),
    ], best_k=2)


def _c5(ss=2, n_frames=16) -> Workload:
    frames = []
    for f in range(n_frames):
        w, h = C5_SIZES[f % 3]
        frames.append(_street_frame(w, h, 0.3516 * w, 5000 + f, 6000 + f, ss, extra_right=True))
    # every frame carries its own sizes; settings are per frame size
    return Workload("C5", frames, c5_settings(*C5_SIZES[0]), {"frames": "5000+f / 6000+f"})


def paper_settings() -> Settings:
    """Sec. III-A: 64 fronto + 30 ground planes, 7x7 on the 512x272 level,
    9x9 on the full-resolution 572x332 centre crop."""
    return Settings(levels=[
        Level(n_fronto=64, near=0.5, far=30.0, n_ground=30, window=7, downsample=2),
        Level(n_fronto=64, near=0.5, far=30.0, n_ground=30, window=9, downsample=1,
              crop=((1024 - 572) // 2, (544 - 332) // 2, 572, 332)),
    ], best_k=2)


def _paper(ss=4) -> Workload:
    fr = _street_frame(1024, 544, 360.0, 1006, 2006, ss, extra_right=True)
    return Workload("paper", [fr], paper_settings(), {"scene": 1006, "rig": 2006})


@dataclass
class DepthSequence:
    """Depth maps of one scene from a vehicle driving forward: the camera, per
    frame the pose world -> camera (the world is the first camera's frame),
    the vehicle position and the ground-truth range map (float32 metres along
    the Eq. (1) ray; NaN where nothing is hit)."""
    cam: Camera
    poses: list
    centres: list
    depths: list


def depth_sequence(n_frames=6, w=320, h=240, f=None, step_m=0.5, seed=1007, yaw_deg=2.0, ss=1) -> DepthSequence:
    """A street scene (ground, facades, boxes) seen from camera positions
    step_m apart along z, each turned by a small seeded yaw."""
    rng = np.random.default_rng(seed)
    sc = _boxes_scene(rng, 20, 2.0, 40.0, -5.0, 5.0, facades=True)
    cam = _fisheye(w, h, f if f is not None else 0.3516 * w)
    poses, centres, depths = [], [], []
    for k in range(n_frames):
        yaw = math.radians(rng.uniform(-yaw_deg, yaw_deg))
        Rcw = np.array([[math.cos(yaw), 0.0, math.sin(yaw)], [0.0, 1.0, 0.0], [-math.sin(yaw), 0.0, math.cos(yaw)]])
        c = (0.0, 0.0, k * step_m)
        _, rng_map, _ = sc.render(cam, Rcw, c, ss=ss, with_gt=True)
        poses.append(_pose_from(Rcw, c))
        centres.append(c)
        depths.append(rng_map.astype(np.float32))
    return DepthSequence(cam, poses, centres, depths)


_MAKERS = {"C1": _c1, "C2": _c2, "C3": _c3, "C4": _c4, "C5": _c5, "paper": _paper}


@functools.lru_cache(maxsize=8)
def workload(name: str, **kw) -> Workload:
    """Build (and cache per process) one of the named synthetic workloads."""
    return _MAKERS[name](**kw)


def fronto_wall_frame(w=96, h=64, f=120.0, depth=5.0, baseline=0.3, seed=7, ss=2) -> Frame:
    """A textured wall perpendicular to the optical axis at z = depth,
    filling the reference view, seen by one source shifted along x."""
    rng = np.random.default_rng(seed)
    sc = Scene(rng, ground_y=1000.0)
    sc.add_box([-12.0, -12.0, depth], [12.0, 12.0, depth + 0.5], pitch=0.06)
    cam = _fisheye(w, h, f)
    return _render_frame(sc, cam, [cam], [np.eye(3)], [(baseline, 0.0, 0.0)], ss)


def random_small_frame(w=48, h=40, n_src=2, seed=0, f=30.0, xi=0.9, ss=2) -> Frame:
    """A tiny street-like frame for brute-force checks."""
    rng = np.random.default_rng(seed)
    sc = _boxes_scene(rng, 6, 2.0, 12.0, -3.0, 3.0, facades=True)
    cam = _fisheye(w, h, f, xi)
    centres = [(0.25 * (i + 1) * (-1) ** i, 0.02 * i, 0.0) for i in range(n_src)]
    rots = [_small_rotation(rng, 3.0) for _ in centres]
    return _render_frame(sc, cam, [cam] * n_src, rots, centres, ss)
