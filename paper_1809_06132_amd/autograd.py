"""Soft-argmin inverse depth as a torch.autograd.Function.

forward:  the soft-mode sweep (softmax over -cost / T of the fronto planes,
          expectation of their inverse depths) on the GPU.
backward: the library's hand-written backward kernel, which recomputes the
          warps and returns dL/d(source image) and dL/d(pose) for every
          source.

The pose variable is an se(3) left perturbation xi = (v, omega) per source
(shape [S, 6]) applied to the camera set's poses: T_s <- exp(xi_s) T_s.  The
returned gradient is the library's left-perturbation gradient, exact at
xi = 0 (the usual use: re-linearise after every update).

Sources may be uint8 (no image gradient) or float tensors holding grey
values.  A sweep built with image_format="f32" sweeps float images as they
are and returns their exact gradient; one built for 8-bit images rounds
float sources to 8 bits for the forward and returns the gradient of the
interpolated intensities (straight-through rounding)."""
from __future__ import annotations

import numpy as np
import torch

from . import psweep as P
from .sweep import PlaneSweep


def perturb_pose(R: np.ndarray, t: np.ndarray, xi: np.ndarray):
    """exp(xi) * T with xi = (v, omega): R' = Exp(omega) R, t' = Exp(omega) t + v
    (first order: X_s + v + omega x X_s), computed by the library."""
    Ro, to = P.psweep_perturb_pose(np.asarray(R, np.float64).ravel(), np.asarray(t, np.float64).ravel(),
                                   np.asarray(xi, np.float64).ravel())
    return np.asarray(Ro).reshape(3, 3), np.asarray(to)


class _Pose:
    def __init__(self, R, t):
        self.R, self.t = R, t


class SoftDepth(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sweep: PlaneSweep, ref: torch.Tensor, pose_xi: torch.Tensor, *srcs: torch.Tensor):
        ref_cam, src_cams = sweep.cams[0]
        base = sweep.base_poses
        xi = pose_xi.detach().to("cpu", torch.float64).numpy()
        poses = [_Pose(*perturb_pose(np.asarray(p.R), np.asarray(p.t), xi[s])) for s, p in enumerate(base)]
        sweep.set_cameras(0, ref_cam, src_cams, poses)
        if sweep.image_dtype == torch.float32:
            u8 = [s.detach().float().contiguous() for s in srcs]
            ref = ref.detach().float().contiguous()
        else:
            u8 = [s if s.dtype == torch.uint8 else s.detach().round().clamp(0, 255).to(torch.uint8) for s in srcs]
        out = sweep.alloc_outputs()
        sweep.run([{"ref": ref, "srcs": u8, "camera_set": 0}], [out])
        ctx.sweep = sweep
        ctx.shapes = [tuple(s.shape) for s in srcs]
        ctx.float_src = [s.dtype != torch.uint8 for s in srcs]
        ctx.keep = (ref, u8)           # the backward reads these images again
        ctx.run_id = sweep.soft_run_id
        ctx.xi_dtype, ctx.xi_device = pose_xi.dtype, pose_xi.device
        ctx.mark_non_differentiable(out["soft_lse"])
        # the backward also reads rho and lse of this run: saved, so that the
        # caller dropping them cannot free their memory
        ctx.save_for_backward(out["soft_invdepth"], out["soft_lse"])
        return out["soft_invdepth"], out["soft_lse"]

    @staticmethod
    def backward(ctx, grad_rho, grad_lse):
        g = grad_rho if grad_rho is not None else None
        if g is None:
            return (None, None, None) + tuple(None for _ in ctx.shapes)
        # image gradients only for float sources that ask for them (inputs
        # 0..2 are the sweep, the reference and the pose)
        want = [f and ctx.needs_input_grad[3 + s] for s, f in enumerate(ctx.float_src)]
        _ = ctx.saved_tensors   # rho and lse of this run, alive until the kernel has read them
        gs, gp = ctx.sweep.soft_backward(g, ctx.shapes, image_grads=want, run_id=ctx.run_id)
        g_src = tuple(gs)
        return (None, None, gp.to(device=ctx.xi_device, dtype=ctx.xi_dtype)) + g_src


class SoftDepthSweep(PlaneSweep):
    """A soft-mode PlaneSweep whose poses can be optimised through autograd."""

    def __init__(self, settings, ref_cam, src_cams, poses, **kw):
        assert settings.mode == "soft"
        super().__init__(settings, ref_cam.width, ref_cam.height, len(src_cams), **kw)
        self.base_poses = list(poses)
        self.set_cameras(0, ref_cam, src_cams, poses)

    def __call__(self, ref, srcs, pose_xi=None):
        if pose_xi is None:
            pose_xi = torch.zeros((len(srcs), 6), dtype=torch.float64)
        return SoftDepth.apply(self, ref, pose_xi, *srcs)
