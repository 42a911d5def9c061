"""Fusion network front end (mrs_net_* and mrs_fuse of include/mrs.h)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class FusionNet:
    """The HRLS + LRHS fusion network; parameters live on the GPU (FP32 masters + BF16)."""

    def __init__(self, seed: int | None = None):
        import torch  # noqa: F401  (initialises the HIP runtime through torch)
        L.use_current_stream()
        h = C.c_void_p()
        L.check(L.lib().mrs_net_create(C.byref(h)))
        self.handle = h
        self.num_params = int(L.lib().mrs_net_num_params())
        if seed is not None:
            self.init(seed)

    def init(self, seed: int):
        L.use_current_stream()
        L.check(L.lib().mrs_net_init(self.handle, C.c_uint64(int(seed))))

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        L.use_current_stream()
        L.check(L.lib().mrs_net_set_params(self.handle, p.ctypes.data_as(C.c_void_p), p.size))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.num_params, np.float32)
        L.use_current_stream()
        L.check(L.lib().mrs_net_get_params(self.handle, p.ctypes.data_as(C.c_void_p), p.size))
        return p

    def fuse(self, hrls_rgb, hrls_aux, lrhs_rgb, out=None):
        """hrls_rgb [B,H,W,3] or [H,W,3], hrls_aux [...,7], lrhs_rgb [..,H/4,W/4,3] (CUDA fp32)."""
        import torch
        batched = hrls_rgb.dim() == 4
        B = hrls_rgb.shape[0] if batched else 1
        H, W = hrls_rgb.shape[-3], hrls_rgb.shape[-2]
        if out is None:
            out = torch.empty(hrls_rgb.shape, dtype=torch.float32, device=hrls_rgb.device)
        L.use_current_stream()
        L.check(L.lib().mrs_fuse_batch(self.handle, B, L.ptr(hrls_rgb), L.ptr(hrls_aux),
                                       L.ptr(lrhs_rgb), W, H, L.ptr(out)))
        return out

    def activation(self, which: int, shape):
        a = np.empty(int(np.prod(shape)), np.float32)
        L.check(L.lib().mrs_debug_net_activation(self.handle, which,
                                                 a.ctypes.data_as(C.c_void_p), a.size))
        return a.reshape(shape)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().mrs_net_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
