"""ctypes front end of the FP64 reference path tracer (oracle/tracer.cpp).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_scene_create.restype = P
        L.orc_scene_create.argtypes = [C.c_int32, P, P, P, P, C.c_int32, P, C.c_int32, P, P, P]
        L.orc_scene_destroy.argtypes = [P]
        L.orc_bvh_nodes.argtypes = [P]
        L.orc_bvh_nodes.restype = C.c_int32
        L.orc_closest_hit.argtypes = [P, C.c_int32, C.c_int32, P, P, P, P, P, P]
        L.orc_camera_ray.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_double, P, P]
        L.orc_onb.argtypes = [P, P, P]
        L.orc_sample_cosine.argtypes = [C.c_double, C.c_double, P]
        L.orc_ggx_D.argtypes = [C.c_double, C.c_double]
        L.orc_ggx_D.restype = C.c_double
        L.orc_ggx_G1.argtypes = [C.c_double, C.c_double]
        L.orc_ggx_G1.restype = C.c_double
        L.orc_sample_ggx_h.argtypes = [C.c_double, C.c_double, C.c_double, P]
        L.orc_ggx_eval.argtypes = [C.c_double, P, P, P, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_render.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_uint64, C.c_int32, P, P, P, P, C.c_int32, C.c_int32,
                                 C.c_int32, P, P, P]
        L.orc_camera_ray_fx.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_double, P, P, P]
        L.orc_render.restype = C.c_int32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniform(seed: int, p: int, s: int, d: int, tag: int = 0) -> float:
    """u(p, s, d): word d%4 of Philox block (p, s, d//4, tag), top 24 bits / 2^24."""
    w = philox4x32_10([p, s, d // 4, tag], [seed & 0xFFFFFFFF, seed >> 32])[d % 4]
    return float(int(w) >> 8) / 16777216.0


class OracleScene:
    def __init__(self, scene):
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dt)
            self._keep.append(a)
            return a

        V = keep(scene.vertices.reshape(-1), np.float32)
        N = keep(scene.normals.reshape(-1), np.float32)
        M = keep(scene.tri_material, np.uint32)
        F = keep(scene.tri_flags, np.uint32)
        mats = keep(scene.materials, scene.materials.dtype)
        lights = keep(scene.lights, scene.lights.dtype)
        env = keep(scene.env, np.float32)
        c = scene.camera
        cam = keep(np.array(list(c.pos) + list(c.look_at) + list(c.up) + [c.vfov_deg]),
                   np.float32)
        self.num_tris = scene.num_tris
        self.h = lib().orc_scene_create(scene.num_tris, _p(V), _p(N), _p(M), _p(F),
                                        len(scene.materials), _p(mats), len(scene.lights),
                                        _p(lights), _p(env), _p(cam))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_scene_destroy(self.h)
            self.h = None

    def closest_hit(self, o, d, skip=None, use_bvh=True):
        o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
        n = len(o)
        sk = None if skip is None else np.ascontiguousarray(skip, np.int32)
        t = np.zeros(n)
        prim = np.zeros(n, np.int32)
        b = np.zeros((n, 2))
        lib().orc_closest_hit(self.h, int(use_bvh), n, _p(o), _p(d), _p(sk), _p(t), _p(prim),
                              _p(b))
        return t, prim, b

    @staticmethod
    def _fx(lens_radius, focus_dist, cam_motion):
        return np.array([lens_radius, focus_dist, *cam_motion], np.float64)

    def camera_ray_fx(self, W, H, x, y, ul0, ul1, tau, lens_radius=0.0, focus_dist=0.0,
                      cam_motion=(0.0, 0.0, 0.0)):
        o = np.zeros(3)
        d = np.zeros(3)
        fx = self._fx(lens_radius, focus_dist, cam_motion)
        lib().orc_camera_ray_fx(self.h, W, H, float(x), float(y), float(ul0), float(ul1),
                                float(tau), _p(fx), _p(o), _p(d))
        return o, d

    def camera_ray(self, W, H, x, y):
        o = np.zeros(3)
        d = np.zeros(3)
        lib().orc_camera_ray(self.h, W, H, float(x), float(y), _p(o), _p(d))
        return o, d

    def render(self, W, H, spp, max_depth, seed, rr_start=3, pixels=None, nthreads=None,
               use_bvh=True, want_aux=True, want_sumsq=False, mis=False, lens_radius=0.0,
               focus_dist=0.0, cam_motion=(0.0, 0.0, 0.0), want_layers=False):
        """FP64 render.  Returns dict(rgb [n,3], aux [n,7], sumsq [n,3], layers [n,9],
        nonfinite, rays).

        `pixels` (flat indices y*W+x) selects a subset; default all pixels, row-major.
        `mis` combines next-event estimation and BSDF sampling of the quad lights
        (power heuristic).  `lens_radius` / `focus_dist`: thin lens; `cam_motion`:
        camera translation over the shutter.  `layers` (Sec. 3.1, Eqs. 1-2 without
        subsurface and transmission): emission seen at the first vertex, then the rest of
        the radiance of samples whose first vertex is diffuse (Lambert) or glossy (GGX).
        """
        if nthreads is None:
            nthreads = os.cpu_count() or 1
        pix = None if pixels is None else np.ascontiguousarray(pixels, np.int32)
        n = W * H if pix is None else len(pix)
        rgb = np.zeros((n, 3))
        aux = np.zeros((n, 7)) if want_aux else None
        sq = np.zeros((n, 3)) if want_sumsq else None
        lay = np.zeros((n, 9)) if want_layers else None
        cnt = np.zeros(2, np.int64)
        rc = lib().orc_render(self.h, W, H, spp, max_depth, rr_start, C.c_uint64(seed), n,
                              _p(pix), _p(rgb), _p(aux), _p(sq), int(nthreads), int(use_bvh),
                              int(bool(mis)), _p(self._fx(lens_radius, focus_dist, cam_motion)),
                              _p(cnt), _p(lay))
        if rc != 0:
            raise ValueError("oracle render: invalid arguments")
        return {"rgb": rgb, "aux": aux, "sumsq": sq, "layers": lay, "nonfinite": int(cnt[0]),
                "rays": int(cnt[1])}


def onb(n):
    n = np.ascontiguousarray(n, np.float64)
    T = np.zeros(3)
    B = np.zeros(3)
    lib().orc_onb(_p(n), _p(T), _p(B))
    return T, B


def sample_cosine(u1, u2):
    out = np.zeros(3)
    lib().orc_sample_cosine(float(u1), float(u2), _p(out))
    return out


def ggx_D(alpha, cos_h):
    return lib().orc_ggx_D(float(alpha), float(cos_h))


def ggx_G1(alpha, cos_v):
    return lib().orc_ggx_G1(float(alpha), float(cos_v))


def sample_ggx_h(alpha, u1, u2):
    out = np.zeros(3)
    lib().orc_sample_ggx_h(float(alpha), float(u1), float(u2), _p(out))
    return out


def ggx_eval(alpha, f0, n, wo, wi):
    args = [np.ascontiguousarray(a, np.float64) for a in (f0, n, wo, wi)]
    out = np.zeros(3)
    lib().orc_ggx_eval(float(alpha), *[_p(a) for a in args], _p(out))
    return out
