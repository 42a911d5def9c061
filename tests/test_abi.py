"""CPU-side checks of the C ABI: the library loads, exports every declared symbol,
and rejects invalid arguments before touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    syms = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            syms |= set(re.findall(r"\b(mrs_\w+)\s*\(", text))
    return sorted(syms)


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("mrs_build_bvh", "mrs_render", "mrs_scene_create", "mrs_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2106_12802_amd import _lib
    L = _lib.lib()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_validation_without_gpu():
    from paper_2106_12802_amd import _lib
    L = _lib.lib()
    h = C.c_void_p()
    assert L.mrs_scene_create(None, C.byref(h)) == 1
    assert b"NULL" in L.mrs_last_error()
    assert L.mrs_render(None, 4, 4, 1, 1, 0, None, None) == 1
    # a descriptor with an out-of-range material index is rejected before any upload
    from mrs_inputs import scenes as S
    sc = S.cornell(1)
    sc.tri_material = sc.tri_material.copy()
    sc.tri_material[3] = 999
    desc, keep = _lib.scene_desc(sc)
    assert L.mrs_scene_create(C.byref(desc), C.byref(h)) == 1
    assert b"material index" in L.mrs_last_error()
    assert not h.value
    sc2 = S.cornell(1)
    sc2.lights = sc2.lights.copy()
    sc2.lights["tri"][0, 0] = 10_000
    desc, keep = _lib.scene_desc(sc2)
    assert L.mrs_scene_create(C.byref(desc), C.byref(h)) == 1
    sc3 = S.cornell(1)
    sc3.camera = S.Camera((0, 0, 0), (0, 1, 0), (0, 1, 0), 40.0)  # up parallel to view
    desc, keep = _lib.scene_desc(sc3)
    assert L.mrs_scene_create(C.byref(desc), C.byref(h)) == 1
    assert L.mrs_scene_destroy(None) == 0
    assert L.mrs_get_counters(None, 0) == 1


def test_tuning_validation():
    from paper_2106_12802_amd import _lib
    L = _lib.lib()
    t = _lib.Tuning()
    assert L.mrs_get_tuning(C.byref(t)) == 0
    assert (t.chunk_paths, t.trace_blocks, t.schedule, t.bvh_leaf_max, t.streams,
            t.tail_bounce, t.bvh_builder) == (1 << 23, 8192, 0, 3, 3, 3, 1)
    for bad in (_lib.Tuning(1, 10, 0, 4, 1, 3), _lib.Tuning(1 << 22, 0, 0, 4, 1, 3),
                _lib.Tuning(1 << 22, 2048, 2, 4, 1, 3), _lib.Tuning(1 << 22, 2048, -1, 4, 1, 3),
                _lib.Tuning(1 << 22, 2048, 0, 0, 1, 3),
                _lib.Tuning(1 << 22, 2048, 0, 5, 1, 3), _lib.Tuning(1 << 22, 2048, 0, 4, 0, 3),
                _lib.Tuning(1 << 22, 2048, 0, 4, 5, 3), _lib.Tuning(1 << 22, 2048, 0, 4, 1, 0),
                _lib.Tuning(1 << 22, 2048, 0, 4, 1, 66), _lib.Tuning(1 << 22, 2048, 0, 4, 1, 3, 2),
                _lib.Tuning(1 << 22, 2048, 0, 4, 1, 3, -1),
                _lib.Tuning(1 << 22, 2048, 0, 4, 1, 3, 1, 0, 0, 0, 66),
                _lib.Tuning(1 << 22, 2048, 0, 4, 1, 3, 1, 0, 0, 0, 0, -1),
                _lib.Tuning(1 << 22, 2048, 0, 4, 1, 3, 1, 0, 0, 0, 0, 0, 2)):
        assert L.mrs_set_tuning(C.byref(bad)) == 1
    assert L.mrs_set_tuning(C.byref(t)) == 0


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2106_12802_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libmrs.so")
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.lib()


def test_net_arch_and_training_option_validation():
    from oracle import cnn, cnn_rdg
    from paper_2106_12802_amd import _lib
    L = _lib.lib()
    assert L.mrs_net_arch_num_params(_lib.NET_ARCHS["res16"]) == cnn.num_params()
    assert L.mrs_net_arch_num_params(_lib.NET_ARCHS["rdg"]) == cnn_rdg.num_params()
    assert L.mrs_net_arch_num_params(_lib.NET_ARCHS["rdg_x2"]) == cnn_rdg.num_params(2)
    assert L.mrs_net_arch_num_params(_lib.NET_ARCHS["rdg_x8"]) == cnn_rdg.num_params(8)
    assert L.mrs_net_arch_num_params(7) == -1
    h = C.c_void_p()
    assert L.mrs_net_create_arch(7, C.byref(h)) == 1 and not h.value
    assert b"arch" in L.mrs_last_error()
    assert C.sizeof(_lib.TrainOpts) == 16
    opts = _lib.TrainOpts(_lib.LOSSES["robust"], 0.1, _lib.OPTIMIZERS["sgd"], 1e-4)
    assert L.mrs_train_step_ex(None, 1, None, None, None, None, 4, 4, C.byref(opts), None) == 1
    assert L.mrs_net_loss_grad_ex(None, 1, None, None, None, None, 4, 4, 1, 0.1, None, None,
                                  None) == 1


def test_render_opts_layout_matches_the_header():
    """mrs_render_opts_default writes each documented default into its own field
    (a layout mismatch between the header and the binding would misplace them)."""
    from paper_2106_12802_amd import _lib
    o = _lib.RenderOpts(7, 7, 7, 7, 7, 7, 7, 7.0, 7.0, (C.c_float * 3)(7, 7, 7), 12345, 678)
    _lib.lib().mrs_render_opts_default(C.byref(o))
    assert (o.rr_start, o.x0, o.y0, o.win_w, o.win_h, o.accum_fp64, o.mis) == (3, 0, 0, 0, 0, -1, 0)
    assert (o.lens_radius, o.focus_dist, list(o.cam_motion)) == (0.0, 0.0, [0.0, 0.0, 0.0])
    assert not o.out_sumsq_dev and not o.out_layers_dev
    assert C.sizeof(_lib.Job) == 112
    # a lens needs a positive focus distance; motion must be finite (rejected on the host)
    from mrs_inputs import scenes as S
    L = _lib.lib()
    for kw in (dict(lens_radius=0.1), dict(lens_radius=-1.0),
               dict(cam_motion=(float("nan"), 0.0, 0.0))):
        bad = _lib.RenderOpts()
        L.mrs_render_opts_default(C.byref(bad))
        for k, v in kw.items():
            if k == "cam_motion":
                bad.cam_motion[:] = list(v)
            else:
                setattr(bad, k, v)
        assert L.mrs_render_ex(None, 4, 4, 1, 1, 0, C.byref(bad), None, None) == 1
        assert b"lens_radius" in L.mrs_last_error() or b"cam_motion" in L.mrs_last_error()


def test_tuning_bvh_builder_by_name():
    """set_tuning takes the builder by name or number; the library keeps it."""
    from paper_2106_12802_amd import tracer as R
    old = R.get_tuning()
    try:
        R.set_tuning(bvh_builder="lbvh")
        assert R.get_tuning()["bvh_builder"] == 0
        R.set_tuning(bvh_builder=1)
        assert R.get_tuning()["bvh_builder"] == 1
        with pytest.raises(KeyError):
            R.set_tuning(bvh_builder="sah")
        with pytest.raises(_lib_error()):
            R.set_tuning(bvh_builder=7)
    finally:
        R.set_tuning(**old)
    assert R.get_tuning() == old


def _lib_error():
    from paper_2106_12802_amd._lib import MrsError
    return MrsError
