"""Rendering front end: device scenes and mrs_render / mrs_render_ex calls."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class GpuScene:
    """A scene copied to the GPU with its LBVH built (mrs_scene_create + mrs_build_bvh)."""

    def __init__(self, scene, build_bvh: bool = True):
        import torch  # noqa: F401  (initialises the HIP runtime through torch)
        L.use_current_stream()
        desc, keep = L.scene_desc(scene)
        h = C.c_void_p()
        L.check(L.lib().mrs_scene_create(C.byref(desc), C.byref(h)))
        del keep
        self.handle = h
        self.num_tris = int(scene.vertices.shape[0])
        self.camera = scene.camera
        if build_bvh:
            self.build_bvh()

    def build_bvh(self):
        L.use_current_stream()
        L.check(L.lib().mrs_build_bvh(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().mrs_scene_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- debug hooks (tests)
    def closest_hit(self, o, d, skip=None):
        import torch
        o = torch.as_tensor(np.ascontiguousarray(o, np.float32), device="cuda").reshape(-1, 3)
        d = torch.as_tensor(np.ascontiguousarray(d, np.float32), device="cuda").reshape(-1, 3)
        n = o.shape[0]
        sk = None if skip is None else torch.as_tensor(np.asarray(skip, np.int32), device="cuda")
        t = torch.empty(n, dtype=torch.float32, device="cuda")
        prim = torch.empty(n, dtype=torch.int32, device="cuda")
        b = torch.empty(n, 2, dtype=torch.float32, device="cuda")
        L.use_current_stream()
        L.check(L.lib().mrs_debug_closest_hit(self.handle, n, L.ptr(o, 3 * n, "f32"),
                                              L.ptr(d, 3 * n, "f32"), L.ptr(sk, n, "i32"),
                                              L.ptr(t, n, "f32"), L.ptr(prim, n, "i32"),
                                              L.ptr(b, 2 * n, "f32")))
        torch.cuda.synchronize()
        return t.cpu().numpy(), prim.cpu().numpy(), b.cpu().numpy()

    def bvh(self):
        n = self.num_tris
        nodes = np.zeros((max(n - 1, 0), 16), np.float32)
        leaf = np.zeros(n, np.int32)
        morton = np.zeros(n, np.uint32)
        root = C.c_int32()
        L.use_current_stream()
        L.check(L.lib().mrs_debug_bvh(self.handle, nodes.ctypes.data_as(C.c_void_p) if n > 1 else None,
                                      leaf.ctypes.data_as(C.c_void_p) if n else None,
                                      morton.ctypes.data_as(C.c_void_p) if n else None,
                                      C.byref(root)))
        return nodes, leaf, morton, root.value & 0xFFFFFFFF

    @property
    def bvh_builder(self):
        """"lbvh" or "ploc": the builder that made this scene's BVH."""
        b = C.c_int32()
        L.check(L.lib().mrs_scene_bvh_builder(self.handle, C.byref(b)))
        return {v: k for k, v in BVH_BUILDERS.items()}[b.value]

    def bvh4(self):
        """(nodes [count, 32] float32, root ref, leaf_max) of the four-wide BVH."""
        count, root, lmax = C.c_int32(), C.c_uint32(), C.c_int32()
        L.use_current_stream()
        L.check(L.lib().mrs_debug_bvh4(self.handle, None, C.byref(count), C.byref(root),
                                       C.byref(lmax)))
        nodes = np.zeros((count.value, 32), np.float32)
        if count.value:
            L.check(L.lib().mrs_debug_bvh4(self.handle, nodes.ctypes.data_as(C.c_void_p),
                                           C.byref(count), C.byref(root), C.byref(lmax)))
        return nodes, root.value, lmax.value


def render_ex(scene: GpuScene, W, H, spp, max_depth, seed, out_rgb, out_aux=None, rr_start=3,
              window=None, accum_fp64=-1, out_sumsq=None, mis=False, lens_radius=0.0,
              focus_dist=0.0, cam_motion=(0.0, 0.0, 0.0), out_layers=None):
    """Enqueue mrs_render_ex on torch's current stream.  Outputs are CUDA float32 tensors.

    mis: combine next-event estimation and BSDF sampling of the quad lights;
    lens_radius / focus_dist: thin lens; cam_motion: camera translation over the shutter;
    out_layers ([.., 9]): emission, diffuse and glossy render layers (Sec. 3.1)."""
    o = L.RenderOpts()
    L.lib().mrs_render_opts_default(C.byref(o))
    o.rr_start = rr_start
    o.mis = int(bool(mis))
    o.lens_radius = float(lens_radius)
    o.focus_dist = float(focus_dist)
    o.cam_motion[:] = [float(v) for v in cam_motion]
    if window is not None:
        o.x0, o.y0, o.win_w, o.win_h = (int(v) for v in window)
    o.accum_fp64 = accum_fp64
    npix = (int(W) * int(H)) if window is None else int(window[2]) * int(window[3])
    o.out_sumsq_dev = L.ptr(out_sumsq, 3 * npix, "f32", "out_sumsq")
    o.out_layers_dev = L.ptr(out_layers, 9 * npix, "f32", "out_layers")
    L.use_current_stream()
    L.check(L.lib().mrs_render_ex(scene.handle, int(W), int(H), int(spp), int(max_depth),
                                  C.c_uint64(int(seed)), C.byref(o),
                                  L.ptr(out_rgb, 3 * npix, "f32", "out_rgb"),
                                  L.ptr(out_aux, 7 * npix, "f32", "out_aux")))


def render(scene: GpuScene, W, H, spp, max_depth, seed, want_aux=True, **kw):
    """Allocate outputs and render; returns (rgb [H,W,3], aux [H,W,7] or None) CUDA tensors."""
    import torch
    win = kw.get("window")
    ww, wh = (W, H) if win is None else (win[2], win[3])
    rgb = torch.empty(wh, ww, 3, dtype=torch.float32, device="cuda")
    aux = torch.empty(wh, ww, 7, dtype=torch.float32, device="cuda") if want_aux else None
    render_ex(scene, W, H, spp, max_depth, seed, rgb, aux, **kw)
    return rgb, aux


def release_workspaces():
    """Free the per-stream render workspaces (mrs_release_workspaces; synchronises)."""
    L.check(L.lib().mrs_release_workspaces())


def counters(reset=False):
    out = np.zeros(L.NUM_COUNTERS, np.int64)
    L.use_current_stream()
    L.check(L.lib().mrs_get_counters(out.ctypes.data_as(C.c_void_p), int(reset)))
    keys = ["nonfinite", "rays", "shadow_rays", "spills", "paths", "overflows",
            "extend_visits", "extend_tests", "shadow_visits", "shadow_tests", "extend_max_steps",
            "shadow_max_steps", "tail_rays", "tail_shadow_rays", "tail_visits", "tail_tests"]
    return dict(zip(keys, (int(x) for x in out)))


def set_count_work(on: bool):
    L.check(L.lib().mrs_set_count_work(int(bool(on))))


def profile_enable(on: bool = True):
    L.check(L.lib().mrs_profile_enable(int(bool(on))))


def profile_select(names=None):
    """Record only these kernels (names of profile_read's keys); None: all."""
    if names is None:
        mask = 0xFFFFFFFF
    else:
        mask = 0
        for n in names:
            mask |= 1 << L.KERNEL_NAMES.index(n)
    L.check(L.lib().mrs_profile_select(mask))


def profile_read():
    """{kernel name: (total ms, launches)} for the launches recorded since profile_enable."""
    ms = np.zeros(L.NUM_KERNEL_IDS, np.float64)
    n = np.zeros(L.NUM_KERNEL_IDS, np.int64)
    L.check(L.lib().mrs_profile_read(ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)))
    names = L.KERNEL_NAMES + [f"k{i}" for i in range(len(L.KERNEL_NAMES), L.NUM_KERNEL_IDS)]
    return {names[i]: (float(ms[i]), int(n[i])) for i in range(L.NUM_KERNEL_IDS) if n[i]}


TUNING_KEYS = ("chunk_paths", "trace_blocks", "schedule", "bvh_leaf_max", "streams", "tail_bounce",
               "bvh_builder", "conv_small_tiles", "queue_sort", "bvh_quantized", "wave_extend",
               "wave_shadow", "net_fused_blocks")
BVH_BUILDERS = {"lbvh": 0, "ploc": 1}


def get_tuning():
    t = L.Tuning()
    L.check(L.lib().mrs_get_tuning(C.byref(t)))
    return {k: int(getattr(t, k)) for k in TUNING_KEYS}


def set_tuning(chunk_paths=None, trace_blocks=None, schedule=None, bvh_leaf_max=None,
               streams=None, tail_bounce=None, bvh_builder=None, conv_small_tiles=None,
               queue_sort=None, bvh_quantized=None, wave_extend=None, wave_shadow=None,
               net_fused_blocks=None):
    """bvh_builder: 0 / "lbvh" (Karras) or 1 / "ploc" (clustering, the default);
    conv_small_tiles: the network's 3x3 convs with fewer 16x16 output tiles than
    this run on the small-tile plan (0: never); wave_extend / wave_shadow: the
    bounces below these trace their closest-hit / shadow rays a wave at a time;
    net_fused_blocks: the network trunk's residual blocks run as one kernel each."""
    cur = get_tuning()
    if isinstance(bvh_builder, str):
        bvh_builder = BVH_BUILDERS[bvh_builder]
    new = dict(chunk_paths=chunk_paths, trace_blocks=trace_blocks, schedule=schedule,
               bvh_leaf_max=bvh_leaf_max, streams=streams, tail_bounce=tail_bounce,
               bvh_builder=bvh_builder, conv_small_tiles=conv_small_tiles,
               queue_sort=queue_sort, bvh_quantized=bvh_quantized, wave_extend=wave_extend,
               wave_shadow=wave_shadow, net_fused_blocks=net_fused_blocks)
    t = L.Tuning()
    for k in TUNING_KEYS:
        setattr(t, k, int(new[k] if new[k] is not None else cur[k]))
    L.check(L.lib().mrs_set_tuning(C.byref(t)))


CONV_KINDS = ("lds64_small", "lds64_large", "lds16", "lds8", "lds80_narrow", "lds64_narrow",
              "direct64", "direct16", "dgrad_lds_small", "dgrad_lds_large", "res_block")


def conv_launches(reset=False):
    """{conv kernel instance: launches} counted since the last reset (host side)."""
    out = np.zeros(len(CONV_KINDS), np.int64)
    L.check(L.lib().mrs_debug_conv_launches(out.ctypes.data_as(C.c_void_p), int(reset)))
    return dict(zip(CONV_KINDS, out.tolist()))


def philox(ctr, key):
    """Device Philox4x32-10 on n counters [n,4] and keys [n,2] (uint32); returns [n,4]."""
    import torch
    c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, np.uint32).reshape(-1, 2)
    n = c.shape[0]
    ct = torch.from_numpy(c.view(np.int32)).cuda()
    kt = torch.from_numpy(k.view(np.int32)).cuda()
    out = torch.empty(n, 4, dtype=torch.int32, device="cuda")
    L.use_current_stream()
    L.check(L.lib().mrs_debug_philox(n, L.ptr(ct), L.ptr(kt), L.ptr(out)))
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


class Batch:
    """Several renders (uneven scenes, sizes, spp, depths) enqueued as one wavefront.

    jobs: dicts with keys scene (GpuScene), W, H, spp, max_depth, seed, and optional
    out_rgb / out_aux / out_sumsq / out_layers (CUDA float32 tensors; rgb and aux are
    allocated if missing, aux only when want_aux is true), rr_start, window, accum_fp64,
    mis, lens_radius, focus_dist, cam_motion.  Outputs are in .outputs."""

    def __init__(self, jobs):
        import torch
        n = len(jobs)
        self.njobs = n
        arr = (L.Job * n)()
        self.outputs = []
        self._keep = []
        for i, j in enumerate(jobs):
            W, H = int(j["W"]), int(j["H"])
            win = j.get("window")
            ww, wh = (W, H) if win is None else (int(win[2]), int(win[3]))
            rgb = j.get("out_rgb")
            if rgb is None:
                rgb = torch.empty(wh, ww, 3, dtype=torch.float32, device="cuda")
            aux = j.get("out_aux")
            if aux is None and j.get("want_aux", True):
                aux = torch.empty(wh, ww, 7, dtype=torch.float32, device="cuda")
            sq = j.get("out_sumsq")
            lay = j.get("out_layers")
            o = L.RenderOpts()
            L.lib().mrs_render_opts_default(C.byref(o))
            o.rr_start = int(j.get("rr_start", 3))
            if win is not None:
                o.x0, o.y0, o.win_w, o.win_h = (int(v) for v in win)
            o.accum_fp64 = int(j.get("accum_fp64", -1))
            o.mis = int(bool(j.get("mis", False)))
            o.lens_radius = float(j.get("lens_radius", 0.0))
            o.focus_dist = float(j.get("focus_dist", 0.0))
            o.cam_motion[:] = [float(v) for v in j.get("cam_motion", (0.0, 0.0, 0.0))]
            o.out_sumsq_dev = L.ptr(sq, 3 * ww * wh, "f32", "out_sumsq")
            o.out_layers_dev = L.ptr(lay, 9 * ww * wh, "f32", "out_layers")
            arr[i].scene = j["scene"].handle.value
            arr[i].W, arr[i].H = W, H
            arr[i].spp, arr[i].max_depth = int(j["spp"]), int(j["max_depth"])
            arr[i].seed = int(j["seed"])
            arr[i].opts = o
            arr[i].out_rgb_dev = L.ptr(rgb, 3 * ww * wh, "f32", "out_rgb")
            arr[i].out_aux_dev = L.ptr(aux, 7 * ww * wh, "f32", "out_aux")
            self.outputs.append((rgb, aux))
            self._keep += [rgb, aux, sq, lay, j["scene"]]
        L.use_current_stream()
        h = C.c_void_p()
        L.check(L.lib().mrs_batch_create(arr, n, C.byref(h)))
        self.handle = h
        self.paths = sum(int(j["spp"]) * (int(j["W"]) * int(j["H"]) if j.get("window") is None
                                           else int(j["window"][2]) * int(j["window"][3]))
                         for j in jobs)

    def render(self):
        L.use_current_stream()
        L.check(L.lib().mrs_batch_render(self.handle))

    def render_begin(self):
        """First half of render(): the wavefront is enqueued; the outputs still
        hold the previous render's values until render_end() (same stream)."""
        L.use_current_stream()
        L.check(L.lib().mrs_batch_render_begin(self.handle))

    def render_fork(self):
        """Marks the start of the next render on the current stream ahead of its
        launches (mrs_batch_render_fork): work enqueued before the following
        render_begin runs beside that render.  Set seeds before forking."""
        L.use_current_stream()
        L.check(L.lib().mrs_batch_render_fork(self.handle))

    def render_end(self):
        L.use_current_stream()
        L.check(L.lib().mrs_batch_render_end(self.handle))

    def set_seeds(self, seeds):
        """New seed per job (stream-ordered device update; no allocation)."""
        arr = np.asarray([int(x) for x in seeds], dtype=np.uint64)
        if arr.size != self.njobs:
            raise ValueError(f"set_seeds: need {self.njobs} seeds, got {arr.size}")
        L.use_current_stream()
        L.check(L.lib().mrs_batch_set_seeds(self.handle, arr.ctypes.data_as(C.c_void_p)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().mrs_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
