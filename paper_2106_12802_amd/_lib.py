"""ctypes binding of libmrs (include/mrs.h).

Argument marshalling only: every step of the rendering runs in the library's
HIP kernels.  torch tensors supply device memory and the stream.  Importing this
module does not touch the GPU; loading the library fails loudly if it has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrs.so")

MRS_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARGUMENT", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "NOT_READY",
                5: "UNSUPPORTED"}
NUM_COUNTERS = 16
NUM_KERNEL_IDS = 16
KERNEL_NAMES = ["generate", "extend", "shade", "shadow", "accumulate", "resolve", "cnn_prep",
                "cnn_hr_in", "cnn_lr", "cnn_hr_out", "train_fwd", "train_bwd", "train_adam", "tail"]


class MrsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Material(C.Structure):
    _fields_ = [("kind", C.c_int32), ("color", C.c_float * 3), ("alpha", C.c_float),
                ("emission", C.c_float * 3)]


class QuadLight(C.Structure):
    _fields_ = [("corner", C.c_float * 3), ("edge_u", C.c_float * 3), ("edge_v", C.c_float * 3),
                ("emission", C.c_float * 3), ("tri", C.c_int32 * 2)]


class Camera(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float)]


class SceneDesc(C.Structure):
    _fields_ = [("num_tris", C.c_int32), ("vertices", C.c_void_p), ("normals", C.c_void_p),
                ("tri_material", C.c_void_p), ("tri_flags", C.c_void_p),
                ("num_materials", C.c_int32), ("materials", C.c_void_p),
                ("num_lights", C.c_int32), ("lights", C.c_void_p), ("env", C.c_float * 3),
                ("camera", Camera)]


NET_ARCHS = {"res16": 0, "rdg": 1, "rdg_x2": 2, "rdg_x8": 3, "res16_layers": 4, "rdg_layers": 5}
NET_SCALES = {"res16": 4, "rdg": 4, "rdg_x2": 2, "rdg_x8": 8, "res16_layers": 4, "rdg_layers": 4}
LOSSES = {"l1": 0, "robust": 1}
OPTIMIZERS = {"adam": 0, "sgd": 1}


class TrainOpts(C.Structure):
    _fields_ = [("loss", C.c_int32), ("beta", C.c_float), ("optimizer", C.c_int32),
                ("lr", C.c_float)]


class RenderOpts(C.Structure):
    _fields_ = [("rr_start", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32),
                ("win_w", C.c_int32), ("win_h", C.c_int32), ("accum_fp64", C.c_int32),
                ("mis", C.c_int32), ("lens_radius", C.c_float), ("focus_dist", C.c_float),
                ("cam_motion", C.c_float * 3), ("out_sumsq_dev", C.c_void_p),
                ("out_layers_dev", C.c_void_p)]


class Job(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("W", C.c_int32), ("H", C.c_int32), ("spp", C.c_int32),
                ("max_depth", C.c_int32), ("seed", C.c_uint64), ("opts", RenderOpts),
                ("out_rgb_dev", C.c_void_p), ("out_aux_dev", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("chunk_paths", C.c_int32), ("trace_blocks", C.c_int32), ("schedule", C.c_int32),
                ("bvh_leaf_max", C.c_int32), ("streams", C.c_int32), ("tail_bounce", C.c_int32),
                ("bvh_builder", C.c_int32), ("conv_small_tiles", C.c_int32),
                ("queue_sort", C.c_int32), ("bvh_quantized", C.c_int32),
                ("wave_extend", C.c_int32), ("wave_shadow", C.c_int32),
                ("net_fused_blocks", C.c_int32)]


assert C.sizeof(Material) == 32 and C.sizeof(QuadLight) == 56

_lib = None


def lib():
    """Load libmrs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmrs.so not found at {LIB_PATH}: run __graft_entry__.build() "
                           "(the HIP library is required; there is no fallback)")
    L = C.CDLL(LIB_PATH)
    P, I32, U64 = C.c_void_p, C.c_int32, C.c_uint64
    sigs = {
        "mrs_last_error": ([], C.c_char_p),
        "mrs_set_stream": ([P], I32),
        "mrs_sync": ([], I32),
        "mrs_scene_create": ([C.POINTER(SceneDesc), C.POINTER(P)], I32),
        "mrs_scene_destroy": ([P], I32),
        "mrs_build_bvh": ([P], I32),
        "mrs_render": ([P, I32, I32, I32, I32, U64, P, P], I32),
        "mrs_render_opts_default": ([C.POINTER(RenderOpts)], None),
        "mrs_render_ex": ([P, I32, I32, I32, I32, U64, C.POINTER(RenderOpts), P, P], I32),
        "mrs_get_counters": ([P, I32], I32),
        "mrs_get_tuning": ([C.POINTER(Tuning)], I32),
        "mrs_set_tuning": ([C.POINTER(Tuning)], I32),
        "mrs_debug_philox": ([I32, P, P, P], I32),
        "mrs_debug_closest_hit": ([P, I32, P, P, P, P, P, P], I32),
        "mrs_debug_bvh": ([P, P, P, P, P], I32),
        "mrs_set_count_work": ([I32], I32),
        "mrs_profile_enable": ([I32], I32),
        "mrs_profile_read": ([P, P], I32),
        "mrs_profile_select": ([C.c_uint32], I32),
        "mrs_net_num_params": ([], C.c_int64),
        "mrs_net_create": ([C.POINTER(P)], I32),
        "mrs_net_destroy": ([P], I32),
        "mrs_net_init": ([P, U64], I32),
        "mrs_net_set_params": ([P, P, C.c_int64], I32),
        "mrs_net_get_params": ([P, P, C.c_int64], I32),
        "mrs_fuse": ([P, P, P, P, I32, I32, P], I32),
        "mrs_fuse_batch": ([P, I32, P, P, P, I32, I32, P], I32),
        "mrs_debug_net_activation": ([P, I32, P, C.c_int64], I32),
        "mrs_image_metrics": ([P, P, C.c_int64, C.c_double, C.c_double, P], I32),
        "mrs_net_loss_grad": ([P, I32, P, P, P, P, I32, I32, P, P, P], I32),
        "mrs_train_step": ([P, I32, P, P, P, P, I32, I32, C.c_float, P], I32),
        "mrs_net_get_state": ([P, P, P, P, C.c_int64, P], I32),
        "mrs_net_set_state": ([P, P, P, P, C.c_int64, C.c_int64], I32),
        "mrs_batch_create": ([C.POINTER(Job), I32, C.POINTER(P)], I32),
        "mrs_batch_render": ([P], I32),
        "mrs_batch_render_begin": ([P], I32),
        "mrs_batch_render_fork": ([P], I32),
        "mrs_scene_bvh_builder": ([P, P], I32),
        "mrs_batch_render_end": ([P], I32),
        "mrs_batch_destroy": ([P], I32),
        "mrs_release_workspaces": ([], I32),
        "mrs_batch_set_seeds": ([P, P], I32),
        "mrs_debug_bvh4": ([P, P, P, P, P], I32),
        "mrs_net_arch_num_params": ([I32], C.c_int64),
        "mrs_net_create_arch": ([I32, C.POINTER(P)], I32),
        "mrs_net_loss_grad_ex": ([P, I32, P, P, P, P, I32, I32, I32, C.c_float, P, P, P], I32),
        "mrs_train_step_ex": ([P, I32, P, P, P, P, I32, I32, C.POINTER(TrainOpts), P], I32),
        "mrs_net_backward": ([P, I32, P, P, P, I32, I32, P, P], I32),
        "mrs_debug_conv_launches": ([P, I32], I32),
        "mrs_net_save": ([P, C.c_char_p, U64], I32),
        "mrs_render_ex_noalloc": ([P, I32, I32, I32, I32, U64, C.POINTER(RenderOpts), P, P], I32),
        "mrs_net_bind_layers": ([P, P, P, I32], I32),
        "mrs_net_load": ([P, C.c_char_p, P], I32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(status: int):
    if status != MRS_OK:
        msg = lib().mrs_last_error()
        raise MrsError(status, msg.decode() if msg else "")


def exported_symbols():
    return [
        "mrs_last_error", "mrs_set_stream", "mrs_sync", "mrs_scene_create", "mrs_scene_destroy",
        "mrs_build_bvh", "mrs_render", "mrs_render_opts_default", "mrs_render_ex",
        "mrs_get_counters", "mrs_get_tuning", "mrs_set_tuning", "mrs_debug_philox",
        "mrs_debug_closest_hit", "mrs_debug_bvh", "mrs_set_count_work", "mrs_profile_enable",
        "mrs_profile_read", "mrs_net_num_params", "mrs_net_create", "mrs_net_destroy",
        "mrs_net_init", "mrs_net_set_params", "mrs_net_get_params", "mrs_fuse", "mrs_fuse_batch",
        "mrs_debug_net_activation", "mrs_image_metrics", "mrs_net_loss_grad", "mrs_train_step",
        "mrs_net_get_state", "mrs_net_set_state", "mrs_batch_create", "mrs_batch_render",
        "mrs_batch_destroy", "mrs_release_workspaces", "mrs_batch_set_seeds",
        "mrs_debug_bvh4", "mrs_net_arch_num_params", "mrs_net_create_arch",
        "mrs_net_loss_grad_ex", "mrs_train_step_ex", "mrs_net_backward",
        "mrs_batch_render_begin", "mrs_batch_render_end", "mrs_batch_render_fork", "mrs_scene_bvh_builder",
        "mrs_profile_select", "mrs_debug_conv_launches", "mrs_net_save", "mrs_net_load",
        "mrs_render_ex_noalloc", "mrs_net_bind_layers",
    ]


def ptr(t, numel=None, dtype=None, name="tensor") -> int | None:
    """Device pointer of a contiguous CUDA torch tensor (None passes through).

    With `dtype` / `numel` given, the tensor must have exactly that element type
    and element count: the C ABI takes raw pointers and cannot check them."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if dtype is not None:
        import torch
        want = {"f32": torch.float32, "i32": torch.int32}[dtype]
        if t.dtype != want:
            raise TypeError(f"{name} must be {want}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def use_current_stream():
    """Route library work to torch's current stream on the current device."""
    import torch
    check(lib().mrs_set_stream(C.c_void_p(torch.cuda.current_stream().cuda_stream)))


def scene_desc(scene):
    """Build a SceneDesc from a scene object (numpy arrays); returns (desc, keepalive)."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.c_void_p) if a.size else None

    d = SceneDesc()
    n = int(scene.vertices.shape[0])
    d.num_tris = n
    d.vertices = arr(scene.vertices.reshape(-1), np.float32)
    d.normals = arr(scene.normals.reshape(-1), np.float32) if scene.normals is not None else None
    d.tri_material = arr(scene.tri_material, np.uint32)
    d.tri_flags = arr(scene.tri_flags, np.uint32) if scene.tri_flags is not None else None
    mats = np.ascontiguousarray(scene.materials)
    lights = np.ascontiguousarray(scene.lights)
    keep += [mats, lights]
    d.num_materials = len(mats)
    d.materials = mats.ctypes.data_as(C.c_void_p) if len(mats) else None
    d.num_lights = len(lights)
    d.lights = lights.ctypes.data_as(C.c_void_p) if len(lights) else None
    for i in range(3):
        d.env[i] = float(scene.env[i])
    cam = scene.camera
    for i in range(3):
        d.camera.pos[i] = cam.pos[i]
        d.camera.look_at[i] = cam.look_at[i]
        d.camera.up[i] = cam.up[i]
    d.camera.vfov_deg = cam.vfov_deg
    return d, keep
