"""FP64 CPU oracle for fisheye plane-sweep stereo -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it; the two share no code.

The arithmetic lives in ``psweep_oracle.c`` (plain C, double precision,
OpenMP over pixels); this module only marshals arguments.  Every function
cites the part of Cui et al. (Sec. III-A plane sweep and multi-scale strategy,
Sec. III-C Eq. (1) camera model) it follows; the readings of points the paper
leaves open are listed in the C source.

Parity status: every function is pinned by the CPU tests in ``tests/`` except
the level merge (``merge``), which is pinned only by construction checks
(parity unpinned against the paper, which gives no merge rule).
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE double)."""
    if force or not os.path.exists(_LIB_PATH):
        srcs = [os.path.join(_HERE, "psweep_oracle.c"), os.path.join(_HERE, "tsdf_oracle.c")]
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-shared", "-fPIC", *srcs, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrCamera(ctypes.Structure):
    _fields_ = [("xi", _d), ("fx", _d), ("fy", _d), ("cx", _d), ("cy", _d),
                ("width", _i32), ("height", _i32)]


class OrPose(ctypes.Structure):
    _fields_ = [("R", _d * 9), ("t", _d * 3)]


class OrImage(ctypes.Structure):
    _fields_ = [("width", _i32), ("height", _i32), ("data", ctypes.POINTER(_d))]


class OrParams(ctypes.Structure):
    _fields_ = [("n_fronto", _i32), ("near_m", _d), ("far_m", _d),
                ("n_ground", _i32), ("h_lo", _d), ("h_hi", _d),
                ("window", _i32), ("best_k", _i32), ("var_floor", _d),
                ("ground_n", _d * 3), ("ground_d", _d), ("temperature", _d)]


@functools.lru_cache(maxsize=1)
def lib():
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    L = ctypes.CDLL(_LIB_PATH)
    PC, PP, PI, PR = (ctypes.POINTER(OrCamera), ctypes.POINTER(OrPose), ctypes.POINTER(OrImage),
                      ctypes.POINTER(OrParams))
    L.or_unproject.argtypes = [PC, _d, _d, _p]
    L.or_unproject.restype = ctypes.c_int
    L.or_project.argtypes = [PC, _p, _p, _p]
    L.or_project.restype = ctypes.c_int
    L.or_parabola.argtypes = [_d, _d, _d]
    L.or_parabola.restype = _d
    L.or_plane_param.argtypes = [PR, ctypes.c_int, _p]
    L.or_plane_param.restype = _d
    L.or_warp.argtypes = [PR, PC, PC, PP, ctypes.c_int, _d, _d, _p, _p, _p]
    L.or_warp.restype = ctypes.c_int
    L.or_sweep.argtypes = [PR, PC, PI, _i32, PC, PI, PP, _i64, _p] + [_p] * 11
    L.or_sweep.restype = None
    L.or_window_cost.argtypes = [PR, PC, PI, PC, PI, PP, _i32, _i32, _i32, _p]
    L.or_window_cost.restype = None
    L.or_downsample2.argtypes = [_p, _i32, _i32, _p]
    L.or_downsample2.restype = None
    L.or_level_camera.argtypes = [PC, _i32, _i32, _i32, _i32, _i32, PC]
    L.or_level_camera.restype = None
    L.or_merge.argtypes = [PC, PR, PR, _i32, _i32, _i32, _p, _p, _i32, _i32, _i32, _i32, _p, _p,
                           _p, _p, _p, _p]
    L.or_merge.restype = None
    L.or_soft_forward.argtypes = [PR, PC, PI, _i32, PC, PI, PP, _i64, _p, _p, _p]
    L.or_soft_argmin.argtypes = [_p, _p, _i32, _d, _p, _p]
    L.or_soft_argmin.restype = None
    L.or_soft_forward.restype = None
    L.or_soft_backward.argtypes = [PR, PC, PI, _i32, PC, PI, PP, _i32, _i32, _i32, _i32, _p, _p, _p]
    L.or_soft_backward.restype = None
    L.or_soft_hypothesis.argtypes = [PR, PC, _i32, _i32, _i32]
    L.or_soft_hypothesis.restype = _d
    L.or_filter.argtypes = [PC, _p, _i32, _i32, _p, _p, _p, _d, _d, _d, _d, _d, _i32, _p, _p]
    L.or_filter.restype = None
    L.or_threads.argtypes = []
    L.or_threads.restype = _i32
    L.or_set_threads.argtypes = [_i32]
    L.or_set_threads.restype = None
    L.or_tsdf_alloc.argtypes = [PC, PP, _p, _i64, _d, _d, _p, _p, _p, _p]
    L.or_tsdf_alloc.restype = None
    L.or_tsdf_visible.argtypes = [PC, PP, _d, _p, _p, _p, _p, _p]
    L.or_tsdf_visible.restype = None
    L.or_tsdf_integrate.argtypes = [PC, PP, _p, _i64, _d, _d, _d, _p, _p, _p, _p, _p, _p]
    L.or_tsdf_integrate.restype = None
    return L


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------
def camera(c) -> OrCamera:
    return OrCamera(float(c.xi), float(c.fx), float(c.fy), float(c.cx), float(c.cy),
                    int(c.width), int(c.height))


def pose(ps) -> OrPose:
    o = OrPose()
    o.R[:] = [float(v) for v in np.asarray(ps.R, np.float64).ravel()]
    o.t[:] = [float(v) for v in np.asarray(ps.t, np.float64).ravel()]
    return o


class _Img:
    """Keeps the float64 copy alive while the struct points at it."""

    def __init__(self, arr):
        self.arr = np.ascontiguousarray(np.asarray(arr, dtype=np.float64))
        self.s = OrImage(self.arr.shape[1], self.arr.shape[0], self.arr.ctypes.data_as(ctypes.POINTER(_d)))


def params(level, settings) -> OrParams:
    o = OrParams()
    o.n_fronto, o.near_m, o.far_m = int(level.n_fronto), float(level.near), float(level.far)
    o.n_ground, o.h_lo, o.h_hi = int(level.n_ground), float(level.h_lo), float(level.h_hi)
    o.window, o.best_k, o.var_floor = int(level.window), int(settings.best_k), float(settings.var_floor)
    o.ground_n[:] = [float(v) for v in settings.ground_n]
    o.ground_d = float(settings.ground_d)
    o.temperature = float(settings.temperature)
    return o


def _ptr(a):
    return None if a is None else a.ctypes.data


# ----------------------------------------------------------------------------
# camera model (Sec. III-C, Eq. (1))
# ----------------------------------------------------------------------------
def unproject(cam, u: float, v: float):
    """Unit ray of pixel (u, v) by Eq. (1); None where it is undefined."""
    r = np.zeros(3)
    ok = lib().or_unproject(ctypes.byref(camera(cam)), float(u), float(v), r.ctypes.data)
    return r if ok else None


def project(cam, X):
    """Unified-model projection (u, v) of a camera-frame point; None if the
    point is behind the model's viewpoint."""
    X = np.ascontiguousarray(np.asarray(X, np.float64))
    u, v = np.zeros(1), np.zeros(1)
    ok = lib().or_project(ctypes.byref(camera(cam)), X.ctypes.data, u.ctypes.data, v.ctypes.data)
    return (float(u[0]), float(v[0])) if ok else None


def plane_param(level, settings, k: int):
    """(parameter, step) of plane k: inverse depth for fronto planes, height
    above the ground for ground planes (Sec. III-A)."""
    st = np.zeros(1)
    val = lib().or_plane_param(ctypes.byref(params(level, settings)), int(k), st.ctypes.data)
    return float(val), float(st[0])


def parabola(cm: float, c0: float, cp: float) -> float:
    """Subpixel offset (plane steps) of the parabola through the costs of
    the winner's two neighbours and the winner."""
    return float(lib().or_parabola(float(cm), float(c0), float(cp)))


def warp(level, settings, ref_cam, src_cam, ps, k: int, u: float, v: float):
    """Position in the source of reference pixel (u, v) under plane k, and
    the source-frame point; None if the plane is missed or the point does not
    project (Sec. III-A: every plane position maps reference pixels into the
    other images)."""
    us, vs, X = np.zeros(1), np.zeros(1), np.zeros(3)
    ok = lib().or_warp(ctypes.byref(params(level, settings)), ctypes.byref(camera(ref_cam)),
                       ctypes.byref(camera(src_cam)), ctypes.byref(pose(ps)), int(k), float(u), float(v),
                       us.ctypes.data, vs.ctypes.data, X.ctypes.data)
    return (float(us[0]), float(vs[0]), X) if ok else None


def window_cost(level, settings, ref_cam, ref_img, src_cam, src_img, ps, k, i, j):
    """Dict with valid, zncc, cost (= (1 - ZNCC)/2, Sec. III-A) and the
    window statistics of one (pixel, plane, source)."""
    out = np.zeros(8)
    R, S = _Img(ref_img), _Img(src_img)
    lib().or_window_cost(ctypes.byref(params(level, settings)), ctypes.byref(camera(ref_cam)),
                         ctypes.byref(R.s), ctypes.byref(camera(src_cam)), ctypes.byref(S.s),
                         ctypes.byref(pose(ps)), int(k), int(i), int(j), out.ctypes.data)
    keys = ["valid", "zncc", "cost", "mean_a", "mean_b", "s_aa", "s_bb", "s_ab"]
    d = dict(zip(keys, out.tolist()))
    d["valid"] = bool(d["valid"])
    return d


# ----------------------------------------------------------------------------
# one level
# ----------------------------------------------------------------------------
def sweep_level(level, settings, ref_cam, ref_img, src_cams, src_imgs, poses, pixels=None,
                volume: bool = False, srcvol: bool = False, srcsig: bool = False):
    """Winner-take-all plane sweep of one level (Sec. III-A).

    pixels: None (every pixel) or an int array [n, 2] of (x, y).
    Returns a dict of per-pixel arrays (shape [H, W] for all pixels, [n]
    otherwise): depth (range), z, index, delta, cost1, cost2, cost2_nonadj,
    param (refined plane parameter), optionally volume [.., P],
    srcvol [.., P, S] and srcsig [.., P, S] (standard deviation of each
    source window's samples; NaN where a sample is unusable, set also for
    windows below the variance floor)."""
    H, W = ref_img.shape
    if pixels is None:
        n, pix, shape = H * W, None, (H, W)
    else:
        pix = np.ascontiguousarray(np.asarray(pixels, np.int32).reshape(-1, 2))
        n, shape = pix.shape[0], (pix.shape[0],)
    P = level.n_fronto + level.n_ground
    S = len(src_imgs)
    out = {k: np.empty(n, np.float64) for k in ("depth", "z", "delta", "cost1", "cost2", "cost2_nonadj", "param")}
    out["index"] = np.empty(n, np.int32)
    vol = np.empty((n, P), np.float64) if volume else None
    svol = np.empty((n, P, S), np.float64) if srcvol else None
    ssig = np.empty((n, P, S), np.float64) if srcsig else None
    R = _Img(ref_img)
    Ss = [_Img(s) for s in src_imgs]
    sarr = (OrImage * S)(*[s.s for s in Ss])
    carr = (OrCamera * S)(*[camera(c) for c in src_cams])
    parr = (OrPose * S)(*[pose(p) for p in poses])
    lib().or_sweep(ctypes.byref(params(level, settings)), ctypes.byref(camera(ref_cam)), ctypes.byref(R.s), S,
                   carr, sarr, parr, n, _ptr(pix),
                   out["depth"].ctypes.data, out["z"].ctypes.data, out["index"].ctypes.data,
                   out["delta"].ctypes.data, out["cost1"].ctypes.data, out["cost2"].ctypes.data,
                   out["cost2_nonadj"].ctypes.data, out["param"].ctypes.data, _ptr(vol), _ptr(svol), _ptr(ssig))
    res = {k: v.reshape(shape) for k, v in out.items()}
    if volume:
        res["volume"] = vol.reshape(shape + (P,))
    if srcvol:
        res["srcvol"] = svol.reshape(shape + (P, S))
    if srcsig:
        res["srcsig"] = ssig.reshape(shape + (P, S))
    return res


# ----------------------------------------------------------------------------
# resolution levels (Sec. III-A, multi-scale strategy)
# ----------------------------------------------------------------------------
def downsample2(img: np.ndarray) -> np.ndarray:
    """2x2 box filter, (s00 + s01 + s10 + s11 + 2) >> 2."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    out = np.empty((H // 2, W // 2), np.uint8)
    lib().or_downsample2(img.ctypes.data, W, H, out.ctypes.data)
    return out


def level_camera(cam, downsample: int, crop=(0, 0, 0, 0)):
    """Intrinsics of a level (downsampled and/or cropped view of `cam`)."""
    from scenegen import Camera
    o = OrCamera()
    lib().or_level_camera(ctypes.byref(camera(cam)), int(downsample), int(crop[0]), int(crop[1]),
                          int(crop[2]), int(crop[3]), ctypes.byref(o))
    return Camera(o.xi, o.fx, o.fy, o.cx, o.cy, o.width, o.height)


def level_inputs(frame, level):
    """Reference image/camera and source images/cameras of one level: the
    downsampled level shrinks every image; a crop cuts only the reference."""
    ref, srcs = frame.ref, list(frame.srcs)
    if level.downsample == 2:
        ref = downsample2(ref)
        srcs = [downsample2(s) for s in srcs]
    ref_cam = level_camera(frame.ref_cam, level.downsample, level.crop)
    src_cams = [level_camera(c, level.downsample) for c in frame.src_cams]
    if level.crop[2] > 0:
        x, y, w, h = level.crop
        ref = np.ascontiguousarray(ref[y:y + h, x:x + w])
    return ref_cam, ref, src_cams, srcs


def merge(frame, settings, low, crop):
    """Fuse the level results into full-resolution maps (reading of the
    paper's up-sample-and-fuse step; parity unpinned against the paper)."""
    full = frame.ref_cam
    H, W = full.height, full.width
    l0 = settings.levels[0]
    l1 = settings.levels[1] if len(settings.levels) > 1 else None
    depth, z = np.empty(H * W), np.empty(H * W)
    lev = np.empty(H * W, np.uint8)
    src = np.empty(H * W, np.int64)
    lp = np.ascontiguousarray(low["param"].ravel())
    li = np.ascontiguousarray(low["index"].ravel().astype(np.int32))
    p0 = params(l0, settings)
    if l1 is not None:
        cp = np.ascontiguousarray(crop["param"].ravel())
        ci = np.ascontiguousarray(crop["index"].ravel().astype(np.int32))
        p1 = ctypes.byref(params(l1, settings))
        cx, cy, cw, ch = l1.crop
    else:
        cp = ci = None
        p1 = None
        cx = cy = cw = ch = 0
    lh, lw = low["index"].shape
    lib().or_merge(ctypes.byref(camera(full)), ctypes.byref(p0), p1, int(l0.downsample), lw, lh,
                   lp.ctypes.data, li.ctypes.data, cx, cy, cw, ch, _ptr(cp), _ptr(ci),
                   depth.ctypes.data, z.ctypes.data, lev.ctypes.data, src.ctypes.data)
    out = {"depth": depth.reshape(H, W), "z": z.reshape(H, W), "level": lev.reshape(H, W)}
    for key in ("index", "delta", "cost1", "cost2"):
        a = np.empty(H * W, low[key].dtype)
        lv = low[key].ravel()
        cv = crop[key].ravel() if l1 is not None else None
        fill = -1 if key == "index" else (0.0 if key == "delta" else np.inf)
        a[:] = fill
        m0, m1 = lev == 0, lev == 1
        a[m0] = lv[src[m0]]
        if l1 is not None:
            a[m1] = cv[src[m1]]
        out[key] = a.reshape(H, W)
    return out


def run(frame, settings, pixels=None):
    """Whole method on one frame: every level, then (with two levels, or a
    downsampled level) the merge to full resolution.  With pixels given only a
    single full-resolution level is supported (sampled parity checks)."""
    levels = settings.levels
    if pixels is not None:
        assert len(levels) == 1 and levels[0].downsample == 1 and levels[0].crop[2] == 0
    res = []
    for lv in levels:
        rc, ref, scs, srcs = level_inputs(frame, lv)
        res.append(sweep_level(lv, settings, rc, ref, scs, srcs, frame.poses, pixels=pixels))
    if len(levels) == 1 and levels[0].downsample == 1 and levels[0].crop[2] == 0:
        out = dict(res[0])
        if pixels is None:
            out["level"] = np.where(res[0]["index"] >= 0, 0, 255).astype(np.uint8)
        return {"merged": out, "levels": res}
    merged = merge(frame, settings, res[0], res[1] if len(res) > 1 else None)
    return {"merged": merged, "levels": res}


# ----------------------------------------------------------------------------
# soft-argmin forward and analytic gradient
# ----------------------------------------------------------------------------
def _src_arrays(src_cams, src_imgs, poses):
    S = len(src_imgs)
    Ss = [_Img(s) for s in src_imgs]
    return (Ss, (OrImage * S)(*[s.s for s in Ss]), (OrCamera * S)(*[camera(c) for c in src_cams]),
            (OrPose * S)(*[pose(p) for p in poses]))


def soft_argmin(costs, rhos, temperature):
    """Soft-argmin of one pixel: costs C_k (NaN = unusable plane) and plane
    parameters rho_k -> (rho_hat, lse) with p = softmax(-C / T)."""
    C = np.ascontiguousarray(costs, np.float64)
    r = np.ascontiguousarray(rhos, np.float64)
    rh, lse = ctypes.c_double(), ctypes.c_double()
    lib().or_soft_argmin(C.ctypes.data, r.ctypes.data, len(C), float(temperature), ctypes.byref(rh),
                         ctypes.byref(lse))
    return rh.value, lse.value


def soft_hypothesis(level, settings, ref_cam, k: int, i: int, j: int) -> float:
    """The soft-argmin's value of plane k at reference pixel (i, j): the
    inverse z-depth of the point where the pixel's Eq. (1) ray meets the plane
    (the parameter of a fronto plane)."""
    return lib().or_soft_hypothesis(ctypes.byref(params(level, settings)), ctypes.byref(camera(ref_cam)), k, i, j)


def soft_forward(level, settings, ref_cam, ref_img, src_cams, src_imgs, poses, pixels=None):
    """Soft-argmin inverse depth rho_hat and logsumexp per pixel."""
    H, W = ref_img.shape
    if pixels is None:
        n, pix, shape = H * W, None, (H, W)
    else:
        pix = np.ascontiguousarray(np.asarray(pixels, np.int32).reshape(-1, 2))
        n, shape = pix.shape[0], (pix.shape[0],)
    rh, lse = np.empty(n), np.empty(n)
    R = _Img(ref_img)
    keep, sarr, carr, parr = _src_arrays(src_cams, src_imgs, poses)
    lib().or_soft_forward(ctypes.byref(params(level, settings)), ctypes.byref(camera(ref_cam)), ctypes.byref(R.s),
                          len(src_imgs), carr, sarr, parr, n, _ptr(pix), rh.ctypes.data, lse.ctypes.data)
    del keep
    return rh.reshape(shape), lse.reshape(shape)


def soft_backward(level, settings, ref_cam, ref_img, src_cams, src_imgs, poses, rect, grad):
    """Analytic FP64 gradient of sum(grad * rho_hat) over rect = (x0, y0, w, h)
    with respect to the source images and the se(3) left perturbation (v,
    omega) of every source pose.  Returns (list of [H_s, W_s], [S, 6])."""
    x0, y0, w, h = [int(v) for v in rect]
    g = np.ascontiguousarray(np.asarray(grad, np.float64).reshape(h, w))
    R = _Img(ref_img)
    keep, sarr, carr, parr = _src_arrays(src_cams, src_imgs, poses)
    gs = [np.zeros(np.asarray(s).shape, np.float64) for s in src_imgs]
    gptrs = (ctypes.c_void_p * len(gs))(*[a.ctypes.data for a in gs])
    gp = np.zeros(6 * len(src_imgs))
    lib().or_soft_backward(ctypes.byref(params(level, settings)), ctypes.byref(camera(ref_cam)),
                           ctypes.byref(R.s), len(src_imgs), carr, sarr, parr, x0, y0, w, h,
                           g.ctypes.data, gptrs, gp.ctypes.data)
    del keep
    return gs, gp.reshape(-1, 6)


# ----------------------------------------------------------------------------
# depth-map filtering (Sec. III-A)
# ----------------------------------------------------------------------------
def depth_filter(cam, ground_n, depth, cost1, cost2, alpha_upper=0.05, alpha_lower=0.3, ratio_min=1.05,
                 gamma=0.5, delta=0.3, window=5):
    """Best-cost, uniqueness-ratio and local-continuity filters, in that
    order.  Returns (filtered range with NaN for rejected pixels, code: 0
    kept, 1 cost, 2 uniqueness, 3 continuity, 255 invalid)."""
    d = np.ascontiguousarray(np.asarray(depth, np.float64))
    a = np.ascontiguousarray(np.asarray(cost1, np.float64))
    b = np.ascontiguousarray(np.asarray(cost2, np.float64))
    h, w = d.shape
    gn = np.ascontiguousarray(np.asarray(ground_n, np.float64))
    out = np.empty_like(d)
    code = np.empty((h, w), np.uint8)
    lib().or_filter(ctypes.byref(camera(cam)), gn.ctypes.data, w, h, d.ctypes.data, a.ctypes.data, b.ctypes.data,
                    float(alpha_upper), float(alpha_lower), float(ratio_min), float(gamma), float(delta),
                    int(window), out.ctypes.data, code.ctypes.data)
    return out, code


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of the oracle's parallel loops."""
    lib().or_set_threads(int(n))


# ----------------------------------------------------------------------------
# dynamic-object masking (Sec. III overview, Sec. IV-B)
# ----------------------------------------------------------------------------
def mask_boxes(depth, boxes, code=None):
    """Pixels inside any detected box [x0, x1) x [y0, y1) leave the depth map
    (NaN; code 4).  Returns new arrays."""
    d = np.array(depth, dtype=np.float64, copy=True)
    c = None if code is None else np.array(code, copy=True)
    h, w = d.shape
    for x0, y0, x1, y1 in boxes:
        for y in range(max(y0, 0), min(y1, h)):
            for x in range(max(x0, 0), min(x1, w)):
                d[y, x] = np.nan
                if c is not None:
                    c[y, x] = 4
    return d, c


# ----------------------------------------------------------------------------
# TSDF depth-map fusion (Sec. III-C, Eq. (1)-(2))
# ----------------------------------------------------------------------------
def tsdf_region(centre, voxel, nb):
    """First block (integer block coordinates) of the box of nb blocks centred
    on `centre` (world metres): floor(centre / B) - nb // 2 per axis."""
    B = 8.0 * voxel
    return np.array([int(np.floor(c / B)) - n // 2 for c, n in zip(centre, nb)], np.int32)


def tsdf_shift(a, sh, scale, fill):
    """Array `a` over a [z][y][x] box (scale cells per block) after the box
    moved by sh = (x, y, z) blocks: what stays in the box keeps its world
    place, the rest is `fill`."""
    out = np.full_like(a, fill)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    for ax, s in zip((2, 1, 0), sh):   # array axes are z, y, x
        n = a.shape[ax]
        k = int(s) * scale
        if abs(k) >= n:
            src[ax] = slice(0, 0)
            dst[ax] = slice(0, 0)
        elif k >= 0:
            src[ax] = slice(k, n)
            dst[ax] = slice(0, n - k)
        else:
            src[ax] = slice(0, n + k)
            dst[ax] = slice(-k, n)
    out[tuple(dst)] = a[tuple(src)]
    return out


class TsdfOracle:
    """The local map as plain arrays over a box of nb = (nbx, nby, nbz) blocks
    of 8^3 voxels that follows a centre point.  D starts at 1 and w at 0; a
    block's observation count is the number of fused depth maps whose rays met
    it; blocks leave the map (cleared) when the box moves past them."""

    def __init__(self, voxel, mu, nb, w_max=100.0, min_obs=3):
        self.voxel, self.mu, self.w_max, self.min_obs = float(voxel), float(mu), float(w_max), int(min_obs)
        self.nb = np.array(nb, np.int32)
        self.b0 = None
        nbz, nby, nbx = self.nb[2], self.nb[1], self.nb[0]
        self.alloc = np.zeros((nbz, nby, nbx), np.int32)
        self.count = np.zeros((nbz, nby, nbx), np.int32)
        self.D = np.ones((nbz * 8, nby * 8, nbx * 8))
        self.W = np.zeros((nbz * 8, nby * 8, nbx * 8))

    def set_centre(self, centre):
        b0 = tsdf_region(centre, self.voxel, self.nb)
        if self.b0 is not None and not np.array_equal(b0, self.b0):
            sh = b0 - self.b0      # blocks the box moved by (x, y, z)
            for name, scale, fill in (("alloc", 1, 0), ("count", 1, 0), ("D", 8, 1.0), ("W", 8, 0.0)):
                setattr(self, name, tsdf_shift(getattr(self, name), sh, scale, fill))
        self.b0 = b0

    def integrate(self, cam, cam_pose, depth, centre):
        """Fuse one depth map (range along the Eq. (1) ray; NaN = invalid)
        taken with `cam_pose` (X_cam = R X_world + t).  Returns the per-step
        diagnostics: touched blocks, their longest segment piece, visible
        blocks, visibility and voxel edge flags."""
        self.set_centre(centre)
        dep = np.ascontiguousarray(np.asarray(depth, np.float64))
        h, w = dep.shape
        c, p = camera(cam), pose(cam_pose)
        b0 = np.ascontiguousarray(self.b0)
        nb = np.ascontiguousarray(self.nb)
        touched = np.zeros_like(self.alloc)
        pen = np.zeros(self.alloc.shape)
        lib().or_tsdf_alloc(ctypes.byref(c), ctypes.byref(p), dep.ctypes.data, w, self.voxel, self.mu,
                            b0.ctypes.data, nb.ctypes.data, touched.ctypes.data, pen.ctypes.data)
        self.alloc |= touched
        self.count += touched
        vis = np.zeros_like(self.alloc)
        vedge = np.zeros_like(self.alloc)
        lib().or_tsdf_visible(ctypes.byref(c), ctypes.byref(p), self.voxel, b0.ctypes.data, nb.ctypes.data,
                              self.alloc.ctypes.data, vis.ctypes.data, vedge.ctypes.data)
        edge = np.zeros(self.D.shape, np.int32)
        lib().or_tsdf_integrate(ctypes.byref(c), ctypes.byref(p), dep.ctypes.data, w, self.voxel, self.mu,
                                self.w_max, b0.ctypes.data, nb.ctypes.data, vis.ctypes.data,
                                self.D.ctypes.data, self.W.ctypes.data, edge.ctypes.data)
        return {"touched": touched, "pen": pen, "visible": vis, "vis_edge": vedge, "voxel_edge": edge}

    def extract(self):
        """D where the voxel was observed and its block has at least min_obs
        observations; NaN elsewhere (Sec. III-C)."""
        ok_blk = np.repeat(np.repeat(np.repeat(self.count >= self.min_obs, 8, 0), 8, 1), 8, 2)
        return np.where(ok_blk & (self.W > 0), self.D, np.nan)
