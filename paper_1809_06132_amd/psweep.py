"""ctypes binding of the psweep C ABI (include/psweep.h), same names.

Argument marshalling only: every computation happens in libpsweep.so on the
GPU.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import functools
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsweep.so")

MAX_SOURCES = 4
MAX_LEVELS = 2

OK, EINVAL, ESTATE, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STORAGE_F32, STORAGE_F16, STORAGE_BF16 = 0, 1, 2
MODE_WTA, MODE_SOFT = 0, 1
LAUNCH_GRID, LAUNCH_PERSISTENT = 0, 1
IMAGE_U8, IMAGE_F32 = 0, 1

_d, _i32, _i64, _p = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p

# every symbol include/psweep.h declares
EXPORTS = ["psweep_create", "psweep_workspace_size", "psweep_set_workspace", "psweep_set_cameras",
           "psweep_set_crop", "psweep_run", "psweep_run_noalloc", "psweep_soft_depth_backward", "psweep_set_tile",
           "psweep_graph_capture", "psweep_graph_launch", "psweep_set_timing", "psweep_sweep_kernel_ms",
           "psweep_sweep_kernel_times", "psweep_set_chunks", "psweep_filter", "psweep_mask_boxes",
           "psweep_plane_pixels", "psweep_plane_pixels_met", "psweep_perturb_pose", "psweep_destroy",
           "psweep_last_error", "psweep_version",
           "psweep_tsdf_create", "psweep_tsdf_workspace_size", "psweep_tsdf_set_workspace", "psweep_tsdf_reset",
           "psweep_tsdf_integrate", "psweep_tsdf_extract", "psweep_tsdf_region", "psweep_tsdf_stats",
           "psweep_tsdf_last_error", "psweep_tsdf_destroy"]


class PsweepError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"psweep status {status}: {msg}")
        self.status = status


class psweep_camera(ctypes.Structure):
    _fields_ = [("xi", _d), ("fx", _d), ("fy", _d), ("cx", _d), ("cy", _d), ("width", _i32), ("height", _i32)]


class psweep_pose(ctypes.Structure):
    _fields_ = [("R", _d * 9), ("t", _d * 3)]


class psweep_level(ctypes.Structure):
    _fields_ = [("n_fronto", _i32), ("near_m", _d), ("far_m", _d), ("n_ground", _i32), ("h_lo", _d),
                ("h_hi", _d), ("window", _i32), ("downsample", _i32), ("crop_x", _i32), ("crop_y", _i32),
                ("crop_w", _i32), ("crop_h", _i32)]


class psweep_config(ctypes.Structure):
    _fields_ = [("n_levels", _i32), ("level", psweep_level * MAX_LEVELS), ("ground_n", _d * 3), ("ground_d", _d),
                ("best_k", _i32), ("var_floor", _d), ("storage", _i32), ("mode", _i32), ("temperature", _d),
                ("launch", _i32), ("max_width", _i32), ("max_height", _i32), ("max_sources", _i32),
                ("max_frames", _i32), ("max_camera_sets", _i32), ("image_format", _i32)]


class psweep_frame(ctypes.Structure):
    _fields_ = [("ref", _p), ("ref_pitch", _i64), ("src", _p * MAX_SOURCES), ("src_pitch", _i64 * MAX_SOURCES),
                ("camera_set", _i32)]


class psweep_maps(ctypes.Structure):
    _fields_ = [("depth", _p), ("z", _p), ("index", _p), ("delta", _p), ("cost1", _p), ("cost2", _p),
                ("level", _p), ("pitch", _i64)]


class psweep_filter_params(ctypes.Structure):
    _fields_ = [("alpha_upper", _d), ("alpha_lower", _d), ("ratio_min", _d), ("gamma_m", _d), ("delta", _d),
                ("window", _i32)]


class psweep_tsdf_config(ctypes.Structure):
    _fields_ = [("voxel_m", _d), ("mu_m", _d), ("blocks", _i32 * 3), ("w_max", _d), ("min_observations", _i32),
                ("max_width", _i32), ("max_height", _i32)]


class psweep_output(ctypes.Structure):
    _fields_ = [("merged", psweep_maps), ("level", psweep_maps * MAX_LEVELS), ("soft_invdepth", _p),
                ("soft_lse", _p), ("soft_pitch", _i64), ("cost_volume", _p * MAX_LEVELS)]


@functools.lru_cache(maxsize=1)
def lib() -> ctypes.CDLL:
    """The loaded library.  Raises if it is missing: there is no fallback."""
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_1809_06132_amd._build)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.psweep_create.argtypes = [P(psweep_config), P(_p)]
    L.psweep_workspace_size.argtypes = [_p, P(ctypes.c_size_t)]
    L.psweep_set_workspace.argtypes = [_p, _p, ctypes.c_size_t]
    L.psweep_set_cameras.argtypes = [_p, _i32, P(psweep_camera), _i32, P(psweep_camera), P(psweep_pose)]
    L.psweep_set_crop.argtypes = [_p, _i32, _i32, _i32, _i32, _i32]
    L.psweep_run.argtypes = [_p, P(psweep_frame), _i32, P(psweep_output), _p]
    L.psweep_run_noalloc.argtypes = [_p, P(psweep_frame), _i32, P(psweep_output), _p]
    L.psweep_soft_depth_backward.argtypes = [_p, _p, P(_p), _p, _p]
    L.psweep_set_tile.argtypes = [_p, _i32, _i32, _i32]
    L.psweep_set_chunks.argtypes = [_p, _i32, _i32]
    L.psweep_filter.argtypes = [_p, _i32, P(psweep_maps), P(psweep_filter_params), _p, _p, _i64, _p]
    L.psweep_mask_boxes.argtypes = [_p, _i32, _p, _p, _i64, _i32, P(_i32), _p]
    L.psweep_tsdf_create.argtypes = [P(psweep_tsdf_config), P(_p)]
    L.psweep_tsdf_workspace_size.argtypes = [_p, P(ctypes.c_size_t)]
    L.psweep_tsdf_set_workspace.argtypes = [_p, _p, ctypes.c_size_t]
    L.psweep_tsdf_reset.argtypes = [_p, _p]
    L.psweep_tsdf_integrate.argtypes = [_p, P(psweep_camera), P(psweep_pose), P(_d), _p, _i64, _p]
    L.psweep_tsdf_extract.argtypes = [_p, _p, _p, _p, _p]
    L.psweep_tsdf_region.argtypes = [_p, P(_i32)]
    L.psweep_tsdf_stats.argtypes = [_p, _p, _p]
    L.psweep_tsdf_last_error.argtypes = [_p]
    L.psweep_tsdf_last_error.restype = ctypes.c_char_p
    L.psweep_tsdf_destroy.argtypes = [_p]
    L.psweep_tsdf_destroy.restype = None
    L.psweep_graph_capture.argtypes = [_p, P(psweep_frame), _i32, P(psweep_output), _p]
    L.psweep_graph_launch.argtypes = [_p, _p]
    L.psweep_set_timing.argtypes = [_p, _i32]
    L.psweep_sweep_kernel_ms.argtypes = [_p, P(_d), P(_i32)]
    L.psweep_sweep_kernel_times.argtypes = [_p, P(_d), _i32, P(_i32)]
    L.psweep_plane_pixels.argtypes = [_p, P(psweep_frame), _i32, P(_i64)]
    L.psweep_plane_pixels_met.argtypes = [_p, P(psweep_frame), _i32, P(_i64)]
    L.psweep_perturb_pose.argtypes = [P(_d), P(_d), P(_d), P(_d), P(_d)]
    L.psweep_destroy.argtypes = [_p]
    L.psweep_destroy.restype = None
    L.psweep_last_error.argtypes = [_p]
    L.psweep_last_error.restype = ctypes.c_char_p
    L.psweep_version.argtypes = []
    L.psweep_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("psweep_destroy", "psweep_last_error", "psweep_version", "psweep_tsdf_destroy",
                        "psweep_tsdf_last_error"):
            getattr(L, name).restype = _i32
    return L


def _check(st: int, ctx=None):
    if st != OK:
        raise PsweepError(st, psweep_last_error(ctx))


def psweep_version() -> str:
    return lib().psweep_version().decode()


def psweep_last_error(ctx=None) -> str:
    return lib().psweep_last_error(ctx).decode()


def psweep_create(cfg: psweep_config):
    ctx = _p()
    _check(lib().psweep_create(ctypes.byref(cfg), ctypes.byref(ctx)))
    return ctx


def psweep_workspace_size(ctx) -> int:
    n = ctypes.c_size_t()
    _check(lib().psweep_workspace_size(ctx, ctypes.byref(n)), ctx)
    return n.value


def psweep_set_workspace(ctx, dev_ptr: int, nbytes: int):
    _check(lib().psweep_set_workspace(ctx, dev_ptr, nbytes), ctx)


def psweep_set_cameras(ctx, camera_set: int, ref: psweep_camera, srcs, poses):
    n = len(srcs)
    sa = (psweep_camera * n)(*srcs)
    pa = (psweep_pose * n)(*poses)
    _check(lib().psweep_set_cameras(ctx, camera_set, ctypes.byref(ref), n, sa, pa), ctx)


def psweep_set_crop(ctx, camera_set: int, x: int, y: int, w: int, h: int):
    _check(lib().psweep_set_crop(ctx, camera_set, x, y, w, h), ctx)


def psweep_run(ctx, frames, outputs, stream: int = 0):
    n = len(frames)
    fa = (psweep_frame * n)(*frames)
    oa = (psweep_output * n)(*outputs)
    _check(lib().psweep_run(ctx, fa, n, oa, stream), ctx)


def psweep_run_noalloc(ctx, frames, outputs, stream: int = 0):
    n = len(frames)
    fa = (psweep_frame * n)(*frames)
    oa = (psweep_output * n)(*outputs)
    _check(lib().psweep_run_noalloc(ctx, fa, n, oa, stream), ctx)


def psweep_soft_depth_backward(ctx, grad_invdepth: int, grad_src_ptrs, grad_pose: int, stream: int = 0):
    arr = (_p * MAX_SOURCES)(*(list(grad_src_ptrs) + [None] * (MAX_SOURCES - len(grad_src_ptrs))))
    _check(lib().psweep_soft_depth_backward(ctx, grad_invdepth, arr, grad_pose, stream), ctx)


def psweep_set_tile(ctx, level: int, rows_per_wave: int, waves: int):
    _check(lib().psweep_set_tile(ctx, level, rows_per_wave, waves), ctx)


def psweep_set_chunks(ctx, level: int, n_chunks: int):
    _check(lib().psweep_set_chunks(ctx, level, n_chunks), ctx)


def psweep_mask_boxes(ctx, camera_set: int, depth: int, code: int, pitch: int, boxes, stream: int = 0):
    """boxes: sequence of (x0, y0, x1, y1) half-open pixel rectangles."""
    flat = [int(v) for b in boxes for v in b]
    arr = (_i32 * max(1, len(flat)))(*flat)
    _check(lib().psweep_mask_boxes(ctx, camera_set, depth, code, pitch, len(flat) // 4, arr, stream), ctx)


def psweep_filter(ctx, camera_set: int, maps: psweep_maps, params: psweep_filter_params, out_depth: int,
                  out_code: int, out_pitch: int = 0, stream: int = 0):
    _check(lib().psweep_filter(ctx, camera_set, ctypes.byref(maps), ctypes.byref(params), out_depth, out_code,
                               out_pitch, stream), ctx)


def psweep_graph_capture(ctx, frames, outputs, stream: int = 0):
    n = len(frames)
    fa = (psweep_frame * n)(*frames)
    oa = (psweep_output * n)(*outputs)
    _check(lib().psweep_graph_capture(ctx, fa, n, oa, stream), ctx)


def psweep_graph_launch(ctx, stream: int = 0):
    _check(lib().psweep_graph_launch(ctx, stream), ctx)


def psweep_set_timing(ctx, on: bool):
    _check(lib().psweep_set_timing(ctx, 1 if on else 0), ctx)


def psweep_sweep_kernel_ms(ctx):
    ms, n = _d(), _i32()
    _check(lib().psweep_sweep_kernel_ms(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def psweep_sweep_kernel_times(ctx, capacity: int = 64):
    arr = (_d * capacity)()
    n = _i32()
    _check(lib().psweep_sweep_kernel_times(ctx, arr, capacity, ctypes.byref(n)), ctx)
    return list(arr[:min(n.value, capacity)])


def psweep_plane_pixels(ctx, frames) -> int:
    n = len(frames)
    fa = (psweep_frame * n)(*frames)
    c = _i64()
    _check(lib().psweep_plane_pixels(ctx, fa, n, ctypes.byref(c)), ctx)
    return c.value


def psweep_plane_pixels_met(ctx, frames) -> int:
    n = len(frames)
    fa = (psweep_frame * n)(*frames)
    c = _i64()
    _check(lib().psweep_plane_pixels_met(ctx, fa, n, ctypes.byref(c)), ctx)
    return c.value


def psweep_perturb_pose(R, t, xi):
    """(R', t') = (Exp(omega) R, Exp(omega) t + v) for xi = (v, omega), in FP64."""
    Ra, ta, xa = (_d * 9)(*[float(v) for v in R]), (_d * 3)(*[float(v) for v in t]), (_d * 6)(*[float(v) for v in xi])
    Ro, to = (_d * 9)(), (_d * 3)()
    _check(lib().psweep_perturb_pose(Ra, ta, xa, Ro, to))
    return list(Ro), list(to)


def psweep_destroy(ctx):
    lib().psweep_destroy(ctx)


# ---------------------------------------------------------------------------
# TSDF fusion (include/psweep_tsdf.h)
# ---------------------------------------------------------------------------
def _tcheck(st: int, ts=None):
    if st != OK:
        raise PsweepError(st, (lib().psweep_tsdf_last_error(ts) or b"").decode())


def psweep_tsdf_create(cfg: psweep_tsdf_config):
    h = _p()
    _tcheck(lib().psweep_tsdf_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def psweep_tsdf_workspace_size(ts) -> int:
    n = ctypes.c_size_t()
    _tcheck(lib().psweep_tsdf_workspace_size(ts, ctypes.byref(n)), ts)
    return n.value


def psweep_tsdf_set_workspace(ts, ptr: int, nbytes: int):
    _tcheck(lib().psweep_tsdf_set_workspace(ts, ptr, nbytes), ts)


def psweep_tsdf_reset(ts, stream: int = 0):
    _tcheck(lib().psweep_tsdf_reset(ts, stream), ts)


def psweep_tsdf_integrate(ts, cam: psweep_camera, pose: psweep_pose, centre, depth: int, pitch: int,
                          stream: int = 0):
    c = (_d * 3)(*[float(v) for v in centre])
    _tcheck(lib().psweep_tsdf_integrate(ts, ctypes.byref(cam), ctypes.byref(pose), c, depth, pitch, stream), ts)


def psweep_tsdf_extract(ts, d_tsdf: int, d_weight: int, d_count: int, stream: int = 0):
    _tcheck(lib().psweep_tsdf_extract(ts, d_tsdf, d_weight, d_count, stream), ts)


def psweep_tsdf_region(ts):
    b = (_i32 * 3)()
    _tcheck(lib().psweep_tsdf_region(ts, b), ts)
    return [int(v) for v in b]


def psweep_tsdf_stats(ts, d_stats: int, stream: int = 0):
    _tcheck(lib().psweep_tsdf_stats(ts, d_stats, stream), ts)


def psweep_tsdf_last_error(ts) -> str:
    return (lib().psweep_tsdf_last_error(ts) or b"").decode()


def psweep_tsdf_destroy(ts):
    lib().psweep_tsdf_destroy(ts)
