"""mrs: multi-resolution Monte Carlo rendering on AMD Instinct MI355X (gfx950).

Python front end of libmrs (include/mrs.h).  The renderer (LBVH build,
wavefront path tracer, Philox sampling) and the fusion network run as HIP
kernels inside libmrs; this package only marshals arguments.  torch supplies
device memory and streams.
"""
from . import _lib  # noqa: F401
from .tracer import (Batch, GpuScene, render, render_ex, counters, set_tuning, get_tuning,  # noqa: F401
                     release_workspaces)
from .net import FusionNet  # noqa: F401

__all__ = ["Batch", "GpuScene", "render", "render_ex", "counters", "set_tuning", "get_tuning", "FusionNet"]
