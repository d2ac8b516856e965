"""Torch-facing wrapper of the TSDF fusion in libpsweep.so (Sec. III-C).

PyTorch supplies the device workspace, the depth maps and the output tensors;
allocation, visibility and the running average run in the library's
kernels."""
from __future__ import annotations

import numpy as np
import torch

from . import psweep as P
from .sweep import _stream_handle, camera, pose


class TsdfMap:
    """A local TSDF map: a box of blocks[0] x blocks[1] x blocks[2] voxel
    blocks (8^3 voxels of voxel metres) that follows the centre point given to
    every integration."""

    def __init__(self, voxel=0.1, mu=0.3, blocks=(75, 4, 75), w_max=100.0, min_obs=3, max_width=1280,
                 max_height=960, device="cuda:0", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("TsdfMap needs a GPU (the fusion has no CPU path)")
        self.device = torch.device(device)
        self.blocks = tuple(int(b) for b in blocks)
        cfg = P.psweep_tsdf_config(float(voxel), float(mu), (P._i32 * 3)(*self.blocks), float(w_max), int(min_obs),
                                   int(max_width), int(max_height))
        self.ts = P.psweep_tsdf_create(cfg)
        n = P.psweep_tsdf_workspace_size(self.ts)
        self.workspace = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        P.psweep_tsdf_set_workspace(self.ts, (base + 255) // 256 * 256, n)
        P.psweep_tsdf_reset(self.ts, _stream_handle(stream))
        self._depth = None

    def close(self):
        if self.ts is not None:
            P.psweep_tsdf_destroy(self.ts)
            self.ts = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        P.psweep_tsdf_reset(self.ts, _stream_handle(stream))

    def integrate(self, cam, world_to_cam, centre, depth: torch.Tensor, stream=None):
        """Fuse one depth map (float32 CUDA tensor [H, W], range along the
        Eq. (1) ray in metres, NaN = invalid) taken by `cam` with the pose
        X_cam = R X_world + t."""
        if depth.dtype != torch.float32 or depth.device.type != "cuda" or depth.dim() != 2 or depth.stride(1) != 1:
            raise ValueError("depth must be a 2-D row-major float32 CUDA tensor")
        self._depth = depth       # read by kernels still in flight
        P.psweep_tsdf_integrate(self.ts, camera(cam), pose(world_to_cam), centre, depth.data_ptr(), depth.stride(0),
                                _stream_handle(stream))

    def extract(self, stream=None) -> dict:
        """The box in world order: tsdf and weight [8 nz, 8 ny, 8 nx] float32
        (tsdf NaN where unobserved or in blocks with too few observations),
        block observation counts [nz, ny, nx] int32, and the first block's
        world block coordinates."""
        nx, ny, nz = self.blocks
        d = torch.empty((nz * 8, ny * 8, nx * 8), dtype=torch.float32, device=self.device)
        w = torch.empty_like(d)
        c = torch.empty((nz, ny, nx), dtype=torch.int32, device=self.device)
        P.psweep_tsdf_extract(self.ts, d.data_ptr(), w.data_ptr(), c.data_ptr(), _stream_handle(stream))
        return {"tsdf": d, "weight": w, "count": c, "first_block": np.array(P.psweep_tsdf_region(self.ts))}

    def stats(self, stream=None):
        """(allocated blocks, visible blocks) of the last integration."""
        out = torch.empty(2, dtype=torch.int32, device=self.device)
        P.psweep_tsdf_stats(self.ts, out.data_ptr(), _stream_handle(stream))
        a, v = out.cpu().tolist()
        return a, v
