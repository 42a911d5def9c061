"""Fusion network front end (mrs_net_* and mrs_fuse of include/mrs.h)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _lib as L


class FusionNet:
    """The HRLS + LRHS fusion network; parameters live on the GPU (FP32 masters + BF16).

    arch "res16": 16 residual blocks; "rdg": the paper's network of residual
    dense groups, x4 ("rdg_x2", "rdg_x8": the same at x2 and x8; include/mrs.h
    documents them); "res16_layers" / "rdg_layers": the x4 networks whose HRLS
    input also carries the render layers (pass layers=(hr_layers, hr_sumsq, spp)
    to the calls, or bind them once with bind_layers).  .scale is the HR / LR
    size ratio."""

    def __init__(self, seed: int | None = None, arch: str = "res16"):
        import torch  # noqa: F401  (initialises the HIP runtime through torch)
        if arch not in L.NET_ARCHS:
            raise ValueError(f"unknown arch {arch!r}")
        self.arch = arch
        self.scale = L.NET_SCALES[arch]
        L.use_current_stream()
        h = C.c_void_p()
        L.check(L.lib().mrs_net_create_arch(L.NET_ARCHS[arch], C.byref(h)))
        self.handle = h
        self.num_params = int(L.lib().mrs_net_arch_num_params(L.NET_ARCHS[arch]))
        self.ready = False  # parameters loaded (mrs_fuse refuses to run before)
        self.has_layers = arch.endswith("_layers")
        self._bound = None  # keeps the bound layer tensors alive
        if seed is not None:
            self.init(seed)

    def bind_layers(self, hr_layers, hr_sumsq, spp):
        """The HRLS render layers ([..,9]: emission, diffuse, glossy) and sums of
        squares ([..,3]) that later calls of a layered network read (mrs_net_bind_layers)."""
        L.check(L.lib().mrs_net_bind_layers(self.handle, L.ptr(hr_layers, None, "f32", "hr_layers"),
                                            L.ptr(hr_sumsq, None, "f32", "hr_sumsq"), int(spp)))
        self._bound = (hr_layers, hr_sumsq)

    def _layers(self, layers, P):
        if layers is None:
            return
        lay, sq, spp = layers
        if lay.numel() != 9 * P or sq.numel() != 3 * P:
            raise ValueError(f"layers must hold {9 * P} and {3 * P} values")
        self.bind_layers(lay, sq, spp)

    def init(self, seed: int):
        L.use_current_stream()
        L.check(L.lib().mrs_net_init(self.handle, C.c_uint64(int(seed))))
        self.ready = True

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        L.use_current_stream()
        L.check(L.lib().mrs_net_set_params(self.handle, p.ctypes.data_as(C.c_void_p), p.size))
        self.ready = True

    def get_params(self) -> np.ndarray:
        p = np.empty(self.num_params, np.float32)
        L.use_current_stream()
        L.check(L.lib().mrs_net_get_params(self.handle, p.ctypes.data_as(C.c_void_p), p.size))
        return p

    def fuse(self, hrls_rgb, hrls_aux, lrhs_rgb, out=None, layers=None):
        """hrls_rgb [B,H,W,3] or [H,W,3], hrls_aux [...,7], lrhs_rgb [..,H/s,W/s,3] (CUDA fp32);
        layers = (hr_layers, hr_sumsq, spp) for the layered networks."""
        import torch
        batched = hrls_rgb.dim() == 4
        B = hrls_rgb.shape[0] if batched else 1
        H, W = hrls_rgb.shape[-3], hrls_rgb.shape[-2]
        if out is None:
            out = torch.empty(hrls_rgb.shape, dtype=torch.float32, device=hrls_rgb.device)
        P = B * H * W
        self._layers(layers, P)
        L.use_current_stream()
        L.check(L.lib().mrs_fuse_batch(self.handle, B, L.ptr(hrls_rgb, 3 * P, "f32", "hrls_rgb"),
                                       L.ptr(hrls_aux, 7 * P, "f32", "hrls_aux"),
                                       L.ptr(lrhs_rgb, 3 * P // self.scale ** 2, "f32", "lrhs_rgb"), W, H,
                                       L.ptr(out, 3 * P, "f32", "out")))
        return out

    @staticmethod
    def _dims(hrls_rgb):
        batched = hrls_rgb.dim() == 4
        B = hrls_rgb.shape[0] if batched else 1
        return B, hrls_rgb.shape[-3], hrls_rgb.shape[-2]

    def loss_grad(self, hrls_rgb, hrls_aux, lrhs_rgb, target, loss="l1", beta=0.1, layers=None):
        """(grad [num_params] float32, loss (FP64), network output tensor); no update.

        loss "l1" or "robust" (the paper's l_r with robust factor beta)."""
        import torch
        B, H, W = self._dims(hrls_rgb)
        self._layers(layers, B * H * W)
        g = np.empty(self.num_params, np.float32)
        value = C.c_double()
        out = torch.empty(hrls_rgb.shape, dtype=torch.float32, device=hrls_rgb.device)
        L.use_current_stream()
        P = B * H * W
        L.check(L.lib().mrs_net_loss_grad_ex(self.handle, B, L.ptr(hrls_rgb, 3 * P, "f32"),
                                             L.ptr(hrls_aux, 7 * P, "f32"),
                                             L.ptr(lrhs_rgb, 3 * P // self.scale ** 2, "f32"),
                                             L.ptr(target, 3 * P, "f32"), W, H,
                                             L.LOSSES[loss], float(beta),
                                             g.ctypes.data_as(C.c_void_p), C.byref(value),
                                             L.ptr(out)))
        return g, value.value, out

    def backward(self, hrls_rgb, hrls_aux, lrhs_rgb, grad_out, layers=None):
        """Parameter gradient [num_params] float32 for a given dL/dI_SR (CUDA fp32)."""
        B, H, W = self._dims(hrls_rgb)
        self._layers(layers, B * H * W)
        g = np.empty(self.num_params, np.float32)
        L.use_current_stream()
        P = B * H * W
        L.check(L.lib().mrs_net_backward(self.handle, B, L.ptr(hrls_rgb, 3 * P, "f32"),
                                         L.ptr(hrls_aux, 7 * P, "f32"),
                                         L.ptr(lrhs_rgb, 3 * P // self.scale ** 2, "f32"), W, H,
                                         L.ptr(grad_out, 3 * P, "f32"),
                                         g.ctypes.data_as(C.c_void_p)))
        return g

    def train_step(self, hrls_rgb, hrls_aux, lrhs_rgb, target, lr=1e-4, want_loss=False,
                   loss="l1", beta=0.1, optimizer="adam", layers=None):
        """One optimiser step ("adam" or "sgd") on the loss ("l1" or "robust");
        returns the loss of this step (synchronising) if want_loss."""
        B, H, W = self._dims(hrls_rgb)
        self._layers(layers, B * H * W)
        value = C.c_double()
        opts = L.TrainOpts(L.LOSSES[loss], float(beta), L.OPTIMIZERS[optimizer], float(lr))
        L.use_current_stream()
        P = B * H * W
        L.check(L.lib().mrs_train_step_ex(self.handle, B, L.ptr(hrls_rgb, 3 * P, "f32"),
                                          L.ptr(hrls_aux, 7 * P, "f32"),
                                          L.ptr(lrhs_rgb, 3 * P // self.scale ** 2, "f32"),
                                          L.ptr(target, 3 * P, "f32"), W, H, C.byref(opts),
                                          C.byref(value) if want_loss else None))
        return value.value if want_loss else None

    def get_state(self):
        """(params, adam m, adam v, step) as host arrays: a resumable checkpoint."""
        n = self.num_params
        p, m, v = (np.empty(n, np.float32) for _ in range(3))
        step = C.c_int64()
        L.use_current_stream()
        L.check(L.lib().mrs_net_get_state(self.handle, p.ctypes.data_as(C.c_void_p),
                                          m.ctypes.data_as(C.c_void_p),
                                          v.ctypes.data_as(C.c_void_p), n, C.byref(step)))
        return p, m, v, step.value

    def set_state(self, params, m, v, step):
        arrs = [np.ascontiguousarray(a, np.float32) for a in (params, m, v)]
        L.use_current_stream()
        L.check(L.lib().mrs_net_set_state(self.handle, *[a.ctypes.data_as(C.c_void_p) for a in arrs],
                                          self.num_params, int(step)))
        self.ready = True

    def save(self, path, data_counter=0):
        """Resumable checkpoint file (mrs_net_save): versioned header, FP32 masters,
        Adam m and v, step, a data counter and CRC-32 checksums."""
        L.use_current_stream()
        L.check(L.lib().mrs_net_save(self.handle, os.fsencode(str(path)), int(data_counter)))

    def load(self, path):
        """Restores a checkpoint of this architecture (mrs_net_load); returns its
        data counter.  A damaged or foreign file raises and changes nothing."""
        counter = C.c_uint64()
        L.use_current_stream()
        L.check(L.lib().mrs_net_load(self.handle, os.fsencode(str(path)), C.byref(counter)))
        self.ready = True
        return int(counter.value)

    def save_weights(self, path):
        """Weights file: magic, version, count, FP32 parameters, SHA-256 of all before it."""
        import hashlib
        p = self.get_params()
        head = np.array([0x5753524D, 1, self.num_params], np.int64).tobytes()
        with open(path, "wb") as f:
            f.write(head + p.tobytes() + hashlib.sha256(head + p.tobytes()).digest())

    def load_weights(self, path):
        import hashlib
        raw = open(path, "rb").read()
        head, body, digest = raw[:24], raw[24:-32], raw[-32:]
        magic, version, n = np.frombuffer(head, np.int64)
        if magic != 0x5753524D or version != 1 or n != self.num_params:
            raise ValueError("not a weights file of this network")
        if hashlib.sha256(head + body).digest() != digest:
            raise ValueError("weights file checksum mismatch")
        self.set_params(np.frombuffer(body, np.float32))

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
