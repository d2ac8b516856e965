"""MI355X (gfx950) fisheye plane-sweep stereo: the depth-map stage of Cui et
al., "Real-Time Dense Mapping for Self-Driving Vehicles using Fisheye
Cameras" (Sec. III-A), as hand-written HIP kernels behind a C ABI
(include/psweep.h) with a thin Python binding.

* ``psweep``    -- ctypes binding of the C ABI (same function names)
* ``sweep``     -- torch-facing wrapper (device buffers, streams, graphs)
* ``autograd``  -- soft-argmin depth as a torch.autograd.Function
* ``autotune``  -- tile-shape autotuner with a JSON cache
"""
from . import psweep  # noqa: F401

__all__ = ["psweep"]
