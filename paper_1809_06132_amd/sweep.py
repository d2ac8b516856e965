"""Torch-facing wrapper of the plane-sweep library.

PyTorch supplies device memory (images, outputs, the workspace) and the HIP
stream; every step of the sweep runs in libpsweep.so.  Settings objects are
duck-typed: anything with the attributes of a level (n_fronto, near, far,
n_ground, h_lo, h_hi, window, downsample, crop) and of the settings (levels,
best_k, var_floor, ground_n, ground_d, mode, temperature) works."""
from __future__ import annotations

import math

import numpy as np
import torch

from . import psweep as P

_STORAGE = {"f32": P.STORAGE_F32, "f16": P.STORAGE_F16, "bf16": P.STORAGE_BF16}
_IMAGE = {"u8": (P.IMAGE_U8, torch.uint8), "f32": (P.IMAGE_F32, torch.float32)}
_LAUNCH = {"grid": P.LAUNCH_GRID, "persistent": P.LAUNCH_PERSISTENT}


def make_config(settings, max_width, max_height, max_sources, max_frames=1, max_camera_sets=1,
                storage="f32", launch="grid", image_format="u8") -> P.psweep_config:
    c = P.psweep_config()
    c.n_levels = len(settings.levels)
    for i, lv in enumerate(settings.levels):
        L = c.level[i]
        L.n_fronto, L.near_m, L.far_m = int(lv.n_fronto), float(lv.near), float(lv.far)
        L.n_ground, L.h_lo, L.h_hi = int(lv.n_ground), float(lv.h_lo), float(lv.h_hi)
        L.window, L.downsample = int(lv.window), int(lv.downsample)
        L.crop_x, L.crop_y, L.crop_w, L.crop_h = [int(v) for v in lv.crop]
    c.ground_n[:] = [float(v) for v in settings.ground_n]
    c.ground_d = float(settings.ground_d)
    c.best_k = int(settings.best_k)
    c.var_floor = float(settings.var_floor)
    c.storage = _STORAGE[storage]
    c.mode = P.MODE_SOFT if settings.mode == "soft" else P.MODE_WTA
    c.temperature = float(settings.temperature)
    c.launch = _LAUNCH[launch]
    c.max_width, c.max_height = int(max_width), int(max_height)
    c.max_sources, c.max_frames, c.max_camera_sets = int(max_sources), int(max_frames), int(max_camera_sets)
    c.image_format = _IMAGE[image_format][0]
    return c


def camera(cam) -> P.psweep_camera:
    return P.psweep_camera(float(cam.xi), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy),
                           int(cam.width), int(cam.height))


def pose(ps) -> P.psweep_pose:
    o = P.psweep_pose()
    o.R[:] = [float(v) for v in np.asarray(ps.R, np.float64).ravel()]
    o.t[:] = [float(v) for v in np.asarray(ps.t, np.float64).ravel()]
    return o


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class PlaneSweep:
    """A context, its workspace and output allocation helpers."""

    def __init__(self, settings, max_width, max_height, max_sources, max_frames=1, max_camera_sets=1,
                 storage="f32", launch="grid", device="cuda:0", image_format="u8"):
        if not torch.cuda.is_available():
            raise RuntimeError("PlaneSweep needs a GPU (the sweep has no CPU path)")
        self.settings = settings
        self.device = torch.device(device)
        self.image_dtype = _IMAGE[image_format][1]
        self.cfg = make_config(settings, max_width, max_height, max_sources, max_frames, max_camera_sets,
                               storage, launch, image_format)
        self.ctx = P.psweep_create(self.cfg)
        n = P.psweep_workspace_size(self.ctx)
        self.workspace = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        P.psweep_set_workspace(self.ctx, aligned, n)
        self.cams = {}
        self.crops = {}
        self._keep = []

    def close(self):
        if self.ctx is not None:
            P.psweep_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration ------------------------------------------------------
    def set_cameras(self, camera_set, ref_cam, src_cams, poses):
        P.psweep_set_cameras(self.ctx, camera_set, camera(ref_cam), [camera(c) for c in src_cams],
                             [pose(p) for p in poses])
        self.cams[camera_set] = (ref_cam, list(src_cams))

    def set_crop(self, camera_set, x, y, w, h):
        P.psweep_set_crop(self.ctx, camera_set, x, y, w, h)
        self.crops[camera_set] = (x, y, w, h)

    def set_tile(self, level, rows_per_wave, waves):
        P.psweep_set_tile(self.ctx, level, rows_per_wave, waves)

    def set_chunks(self, level, n_chunks):
        P.psweep_set_chunks(self.ctx, level, n_chunks)

    def set_timing(self, on=True):
        P.psweep_set_timing(self.ctx, on)

    def sweep_kernel_ms(self):
        return P.psweep_sweep_kernel_ms(self.ctx)

    # -- buffers ------------------------------------------------------------
    def alloc_maps(self, h, w, with_level=True):
        d = self.device
        return {"depth": torch.empty((h, w), dtype=torch.float32, device=d),
                "z": torch.empty((h, w), dtype=torch.float32, device=d),
                "index": torch.empty((h, w), dtype=torch.int32, device=d),
                "delta": torch.empty((h, w), dtype=torch.float32, device=d),
                "cost1": torch.empty((h, w), dtype=torch.float32, device=d),
                "cost2": torch.empty((h, w), dtype=torch.float32, device=d),
                **({"level": torch.empty((h, w), dtype=torch.uint8, device=d)} if with_level else {})}

    def level_size(self, camera_set, lv_index):
        ref, _ = self.cams[camera_set]
        lv = self.settings.levels[lv_index]
        w, h = ref.width // lv.downsample, ref.height // lv.downsample
        if lv_index == 1 and camera_set in self.crops:
            w, h = self.crops[camera_set][2:]
        elif lv.crop[2] > 0:
            w, h = lv.crop[2], lv.crop[3]
        return h, w

    def alloc_outputs(self, camera_set=0, level_maps=False):
        ref, _ = self.cams[camera_set]
        out = {"merged": self.alloc_maps(ref.height, ref.width)}
        if self.settings.mode == "soft":
            out["soft_invdepth"] = torch.empty((ref.height, ref.width), dtype=torch.float32, device=self.device)
            out["soft_lse"] = torch.empty((ref.height, ref.width), dtype=torch.float32, device=self.device)
        if level_maps:
            out["levels"] = [self.alloc_maps(*self.level_size(camera_set, l), with_level=False)
                             for l in range(len(self.settings.levels))]
        return out

    def alloc_cost_volumes(self, camera_set=0):
        """Per level, a [P, h, w] float32 tensor filled with +inf, to pass as
        outputs["cost_volume"] (the sweep writes every (pixel, plane) cost it
        computes; the pairs it skips keep +inf)."""
        return [torch.full((lv.n_fronto + lv.n_ground,) + tuple(self.level_size(camera_set, l)), math.inf,
                           dtype=torch.float32, device=self.device) for l, lv in enumerate(self.settings.levels)]

    # -- marshalling --------------------------------------------------------
    @staticmethod
    def _maps(m: dict | None, shape=None) -> P.psweep_maps:
        """Map pointers (pitch = width); `shape` (h, w): the size every map
        must have."""
        pm = P.psweep_maps()
        if m is None:
            return pm
        for key in ("depth", "z", "index", "delta", "cost1", "cost2", "level"):
            t = m.get(key)
            if t is not None:
                if not (t.is_cuda and t.is_contiguous() and t.dim() == 2):
                    raise ValueError(f"map '{key}' must be a contiguous 2-D CUDA tensor")
                if shape is not None and tuple(t.shape) != tuple(shape):
                    raise ValueError(f"map '{key}' has shape {tuple(t.shape)}, expected {tuple(shape)}")
                setattr(pm, key, t.data_ptr())
        pm.pitch = 0
        return pm

    def _frame(self, fr: dict) -> P.psweep_frame:
        """Frame pointers, after checking every image against the size its
        camera set gives it (the library reads width x height pixels)."""
        f = P.psweep_frame()
        f.camera_set = cs = int(fr.get("camera_set", 0))
        if cs not in self.cams:
            raise ValueError(f"camera set {cs} has no cameras")
        ref_cam, src_cams = self.cams[cs]
        dt = self.image_dtype

        def check(img, cam, what):
            if img.dtype != dt or img.device.type != "cuda" or img.dim() != 2 or img.stride(1) != 1:
                raise ValueError(f"{what} must be a 2-D row-major {dt} CUDA tensor")
            if img.shape[0] < cam.height or img.shape[1] < cam.width:
                raise ValueError(f"{what} is {tuple(img.shape)}, smaller than its camera "
                                 f"({cam.height}, {cam.width})")
            return img.data_ptr(), img.stride(0)

        f.ref, f.ref_pitch = check(fr["ref"], ref_cam, "reference")
        if len(fr["srcs"]) != len(src_cams):
            raise ValueError(f"{len(fr['srcs'])} source images for {len(src_cams)} source cameras")
        for s, img in enumerate(fr["srcs"]):
            f.src[s], f.src_pitch[s] = check(img, src_cams[s], f"source {s}")
        return f

    def _output(self, o: dict, camera_set: int) -> P.psweep_output:
        ref, _ = self.cams[camera_set]
        full = (ref.height, ref.width)
        po = P.psweep_output()
        po.merged = self._maps(o.get("merged"), full)
        for l, m in enumerate(o.get("levels", []) or []):
            po.level[l] = self._maps(m, self.level_size(camera_set, l))
        for l, vol in enumerate(o.get("cost_volume", []) or []):
            if vol is None:
                continue
            lv = self.settings.levels[l]
            want = (lv.n_fronto + lv.n_ground,) + tuple(self.level_size(camera_set, l))
            if not (vol.is_cuda and vol.is_contiguous() and vol.dtype == torch.float32 and tuple(vol.shape) == want):
                raise ValueError(f"cost volume of level {l} must be a contiguous float32 CUDA tensor of shape {want}")
            po.cost_volume[l] = vol.data_ptr()
        if "soft_invdepth" in o:
            for key in ("soft_invdepth", "soft_lse"):
                t = o[key]
                if not (t.is_cuda and t.is_contiguous() and tuple(t.shape) == full and t.dtype == torch.float32):
                    raise ValueError(f"'{key}' must be a contiguous float32 CUDA tensor of shape {full}")
            po.soft_invdepth = o["soft_invdepth"].data_ptr()
            po.soft_lse = o["soft_lse"].data_ptr()
        return po

    # -- run ----------------------------------------------------------------
    def run(self, frames, outputs, stream=None):
        """Enqueue one run of the whole sweep for `frames` (list of dicts with
        'ref', 'srcs', 'camera_set') into `outputs` (list of dicts from
        alloc_outputs)."""
        if len(frames) != len(outputs):
            raise ValueError("one output per frame")
        pf = [self._frame(f) for f in frames]
        po = [self._output(o, f.camera_set) for o, f in zip(outputs, pf)]
        P.psweep_run(self.ctx, pf, po, _stream_handle(stream))
        if self.settings.mode == "soft":
            # the backward re-reads the images and the soft outputs (rho, lse)
            # of this run through the pointers it was given: hold the tensors
            # so the caching allocator cannot hand their memory out
            self._soft_frames = list(frames)
            self._soft_outputs = {k: outputs[0][k] for k in ("soft_invdepth", "soft_lse")}
            self._soft_shape = tuple(outputs[0]["soft_invdepth"].shape)
            self.soft_run_id = getattr(self, "soft_run_id", 0) + 1

    def run_noalloc(self, frames, outputs, stream=None):
        """The same run through psweep_run_noalloc: the library's static
        scratch instead of the workspace (winner-take-all mode)."""
        if len(frames) != len(outputs):
            raise ValueError("one output per frame")
        pf = [self._frame(f) for f in frames]
        po = [self._output(o, f.camera_set) for o, f in zip(outputs, pf)]
        P.psweep_run_noalloc(self.ctx, pf, po, _stream_handle(stream))

    def capture_graph(self, frames, outputs, stream=None):
        if len(frames) != len(outputs):
            raise ValueError("one output per frame")
        pf = [self._frame(f) for f in frames]
        po = [self._output(o, f.camera_set) for o, f in zip(outputs, pf)]
        self._keep = [frames, outputs]
        P.psweep_graph_capture(self.ctx, pf, po, _stream_handle(stream))

    def launch_graph(self, stream=None):
        P.psweep_graph_launch(self.ctx, _stream_handle(stream))

    def filter(self, merged: dict, camera_set=0, alpha_upper=0.05, alpha_lower=0.3, ratio_min=1.05, gamma=0.5,
               delta=0.3, window=5, stream=None):
        """Depth-map filtering of a merged output (Sec. III-A); returns the
        filtered range (NaN = rejected) and the per-pixel code."""
        ref, _ = self.cams[camera_set]
        d = torch.empty((ref.height, ref.width), dtype=torch.float32, device=self.device)
        c = torch.empty((ref.height, ref.width), dtype=torch.uint8, device=self.device)
        prm = P.psweep_filter_params(float(alpha_upper), float(alpha_lower), float(ratio_min), float(gamma),
                                     float(delta), int(window))
        P.psweep_filter(self.ctx, camera_set, self._maps(merged, (ref.height, ref.width)), prm, d.data_ptr(),
                        c.data_ptr(), 0, _stream_handle(stream))
        return d, c

    def mask_boxes(self, depth, boxes, code=None, camera_set=0, stream=None):
        """Mask the pixels inside detected boxes (x0, y0, x1, y1; half-open)
        out of a full-resolution depth map in place: depth NaN, code 4."""
        assert depth.is_cuda and depth.dtype == torch.float32 and depth.stride(1) == 1
        if code is not None:
            assert code.is_cuda and code.dtype == torch.uint8 and code.stride(0) == depth.stride(0)
        P.psweep_mask_boxes(self.ctx, camera_set, depth.data_ptr(), code.data_ptr() if code is not None else 0,
                            depth.stride(0), boxes, _stream_handle(stream))

    def plane_pixels(self, frames) -> int:
        return P.psweep_plane_pixels(self.ctx, [self._frame(f) for f in frames])

    def plane_pixels_met(self, frames) -> int:
        """(pixel, plane) pairs with a window inside the image whose ray meets
        the plane (the method's own work; the rest have no cost at all)."""
        return P.psweep_plane_pixels_met(self.ctx, [self._frame(f) for f in frames])

    def soft_backward(self, grad_invdepth, src_shapes, stream=None, image_grads=True, run_id=None):
        """Gradients of sum(grad * soft_invdepth) of the last soft run: list of
        per-source image gradients (None where not requested) and a [S, 6]
        float64 pose gradient (v, omega).  image_grads: True, False, or one
        flag per source.  run_id: the soft_run_id the forward saw; the
        library differentiates only the latest soft run, so an older one is
        an error."""
        if run_id is not None and run_id != getattr(self, "soft_run_id", None):
            raise RuntimeError("backward of a soft run that a later run has replaced: the library "
                               "differentiates only the latest soft run (run the forward again)")
        if tuple(grad_invdepth.shape) != getattr(self, "_soft_shape", None):
            raise ValueError("the gradient must have the shape of the last soft run's output")
        g = grad_invdepth.contiguous().float()
        if stream is not None and g is not grad_invdepth:
            g.record_stream(stream)   # a temporary read on another stream
        want = [image_grads] * len(src_shapes) if isinstance(image_grads, bool) else list(image_grads)
        gs = [torch.empty(s, dtype=torch.float32, device=self.device) if w else None
              for s, w in zip(src_shapes, want)]
        gp = torch.empty((len(src_shapes), 6), dtype=torch.float64, device=self.device)
        P.psweep_soft_depth_backward(self.ctx, g.data_ptr(), [t.data_ptr() if t is not None else None for t in gs],
                                     gp.data_ptr(), _stream_handle(stream))
        return gs, gp


def frame_to_device(frame, device="cuda:0", dtype=None):
    """Upload a scenegen-style frame (numpy images) to the GPU, converted to
    `dtype` when given (torch.uint8 or torch.float32)."""
    def up(a):
        t = torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return t if dtype is None else t.to(dtype)
    return {"ref": up(frame.ref), "srcs": [up(s) for s in frame.srcs], "camera_set": 0}
