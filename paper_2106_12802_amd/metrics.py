"""Evaluation metrics on the GPU (mrs_image_metrics): sRGB PSNR and RelMSE."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def image_metrics(img, ref, lambda1=0.5, lambda2=0.01):
    """{'mse_srgb', 'psnr', 'relmse'} of two CUDA float32 tensors of equal shape."""
    if img.shape != ref.shape:
        raise ValueError("shape mismatch")
    out = np.zeros(3, np.float64)
    L.use_current_stream()
    L.check(L.lib().mrs_image_metrics(L.ptr(img, img.numel(), "f32", "img"),
                                      L.ptr(ref, img.numel(), "f32", "ref"), img.numel(), float(lambda1),
                                      float(lambda2), out.ctypes.data_as(C.c_void_p)))
    return {"mse_srgb": float(out[0]), "psnr": float(out[1]), "relmse": float(out[2])}


def spp_avg(spp_lrhs, spp_hrls, scale=4):
    """Average samples per HR pixel of a hybrid input (paper Sec. 5.1)."""
    return spp_lrhs / scale ** 2 + spp_hrls
