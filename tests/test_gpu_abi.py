"""Error and failure paths of the C ABI on a live device (status codes, no writes),
forced from the host: every kernel that runs here exits normally."""
import ctypes as C
import sys

import numpy as np
import pytest

from mrs_inputs import scenes as S

pytestmark = pytest.mark.gpu

FLT_MAX = float(np.finfo(np.float32).max)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mrs(torch_cuda):
    import paper_2106_12802_amd as m
    return m


def _sentinel(torch, H, W, C_, value=7.25):
    return torch.full((H, W, C_), value, dtype=torch.float32, device="cuda")


def test_render_before_build_is_not_ready(mrs, torch_cuda):
    from paper_2106_12802_amd import _lib
    torch = torch_cuda
    gs = mrs.GpuScene(S.cornell(1), build_bvh=False)
    rgb, aux = _sentinel(torch, 8, 8, 3), _sentinel(torch, 8, 8, 7)
    L = _lib.lib()
    _lib.use_current_stream()
    rc = L.mrs_render(gs.handle, 8, 8, 1, 1, C.c_uint64(1), rgb.data_ptr(), aux.data_ptr())
    assert rc == 4 and b"mrs_build_bvh" in L.mrs_last_error()
    torch.cuda.synchronize()
    assert torch.all(rgb == 7.25) and torch.all(aux == 7.25)
    b = C.c_int32()
    assert L.mrs_scene_bvh_builder(gs.handle, C.byref(b)) == 4
    gs.build_bvh()
    out, _ = mrs.render(gs, 8, 8, 1, 1, 1)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()


@pytest.mark.parametrize("W,H,spp,depth,what", [
    (0, 8, 1, 1, "W and H"), (8, 0, 1, 1, "W and H"), (16385, 8, 1, 1, "W and H"),
    (8, 16385, 1, 1, "W and H"), (8, 8, 0, 1, "spp"), (8, 8, (1 << 20) + 1, 1, "spp"),
    (8, 8, 1, -1, "max_depth"), (8, 8, 1, 65, "max_depth")])
def test_limits_on_a_live_scene(mrs, torch_cuda, W, H, spp, depth, what):
    """Out-of-range sizes on a built scene: INVALID_ARGUMENT naming the argument,
    and the outputs stay untouched."""
    from paper_2106_12802_amd import _lib
    torch = torch_cuda
    gs = mrs.GpuScene(S.cornell(2))
    rgb, aux = _sentinel(torch, 8, 8, 3), _sentinel(torch, 8, 8, 7)
    L = _lib.lib()
    _lib.use_current_stream()
    rc = L.mrs_render(gs.handle, W, H, spp, depth, C.c_uint64(3), rgb.data_ptr(), aux.data_ptr())
    assert rc == 1 and what.encode() in L.mrs_last_error()
    # NULL and misaligned outputs on the same live scene
    assert L.mrs_render(gs.handle, 8, 8, 1, 1, C.c_uint64(3), None, None) == 1
    assert L.mrs_render(gs.handle, 8, 8, 1, 1, C.c_uint64(3), rgb.data_ptr() + 2, None) == 1
    torch.cuda.synchronize()
    assert torch.all(rgb == 7.25) and torch.all(aux == 7.25)


def test_absurd_batch_is_out_of_memory(mrs, torch_cuda):
    """32 jobs of 16384 x 16384 pixels at 1024 spp with render layers need 32 x 47 GB
    of FP64 pixel sums, far beyond the device: mrs_batch_create reports
    OUT_OF_MEMORY (before any launch) and the library keeps working."""
    from paper_2106_12802_amd import _lib
    torch = torch_cuda
    gs = mrs.GpuScene(S.cornell(3))
    dummy = _sentinel(torch, 4, 4, 9)  # never written: creation fails before any launch
    jobs = (_lib.Job * 32)()
    for j in jobs:
        j.scene = gs.handle.value
        j.W = j.H = 16384
        j.spp = 1024
        j.max_depth = 4
        j.seed = 5
        _lib.lib().mrs_render_opts_default(C.byref(j.opts))
        j.opts.out_layers_dev = dummy.data_ptr()
        j.out_rgb_dev = dummy.data_ptr()
        j.out_aux_dev = None
    h = C.c_void_p()
    _lib.use_current_stream()
    rc = _lib.lib().mrs_batch_create(jobs, 32, C.byref(h))
    _log(f"absurd batch: status {rc}, {_lib.lib().mrs_last_error().decode()}")
    assert rc == 2 and not h.value
    torch.cuda.synchronize()
    assert torch.all(dummy == 7.25)
    out, _ = mrs.render(gs, 16, 16, 2, 2, 9)  # the device is still usable
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()


def _with_degenerate(scene):
    """The scene plus zero-area triangles appended after its own (prim ids of the
    originals unchanged): points, and collinear corners along each axis."""
    pts = [[[0.3, 0.4, 0.5]] * 3, [[0.7, 0.2, 0.6]] * 3]
    lines = [[[0.25, 0.5, 0.5], [0.5, 0.5, 0.5], [0.75, 0.5, 0.5]],
             [[0.5, 0.25, 0.5], [0.5, 0.5, 0.5], [0.5, 0.75, 0.5]],
             [[0.5, 0.5, 0.25], [0.5, 0.5, 0.5], [0.5, 0.5, 0.75]]]
    extra = np.array(pts + lines, np.float32)
    n = len(extra)
    return S.Scene(np.concatenate([scene.vertices, extra]),
                   np.concatenate([scene.normals, np.zeros_like(extra)]),
                   np.concatenate([scene.tri_material, np.zeros(n, np.uint32)]),
                   np.concatenate([scene.tri_flags, np.zeros(n, np.uint32)]),
                   scene.materials, scene.lights, scene.env, scene.camera, scene.name + "+deg")


def test_zero_area_triangles_are_never_hit(mrs, oracle_tracer, torch_cuda):
    """Zero-area triangles (their geometric normal is 0/0) have a zero determinant
    for every ray, so both sides count them as misses (E4): the image is bitwise the
    one without them, matches the oracle, and no sample turns non-finite."""
    torch = torch_cuda
    base = S.cornell(1)
    deg = _with_degenerate(base)
    mrs.counters(reset=True)
    g0, _ = mrs.render(mrs.GpuScene(base), 48, 48, 8, 4, 21)
    g1, a1 = mrs.render(mrs.GpuScene(deg), 48, 48, 8, 4, 21)
    torch.cuda.synchronize()
    c = mrs.counters(reset=True)
    assert c["nonfinite"] == 0 and c["overflows"] == 0
    assert torch.equal(g0, g1)
    o = oracle_tracer.OracleScene(deg).render(48, 48, 8, 4, 21)
    g = g1.cpu().numpy().reshape(-1, 3).astype(np.float64)
    floor = 1e-3 * np.abs(o["rgb"]).mean()
    ok = np.all(np.abs(g - o["rgb"]) <= 1e-4 * np.maximum(np.abs(o["rgb"]), floor), -1)
    assert ok.mean() >= 0.999 and o["nonfinite"] == 0


def _overflow_scene():
    """A Lambert floor (rho 0.9) under a 1 x 1 quad light of emission 3.4e38 centred
    0.2 above the point the camera sees (tiny field of view)."""
    b = S._Builder()
    b.add_quad((-50.0, 0.0, -50.0), (0.0, 0.0, 100.0), (100.0, 0.0, 0.0),
               b.material(S.LAMBERT, color=(0.9, 0.9, 0.9)))
    b.add_light((-0.5, 0.2, -0.5), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), (3.4e38,) * 3)
    cam = S.Camera((0.0, 0.1, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0.01)
    return b.build((0.0, 0.0, 0.0), cam, "overflow")


def test_nonfinite_samples_counted_and_dropped(mrs, oracle_tracer, torch_cuda):
    """One sample per pixel, next-event estimation only (depth 1), emission near
    FLT_MAX: a sample whose FP32 contribution exceeds FLT_MAX becomes +inf on the
    GPU, is counted and replaced by 0 (E12); the FP64 oracle computes the same
    samples without overflow.  Each pixel is one sample, so the GPU pixel is 0
    exactly where the oracle's value exceeds FLT_MAX, and the oracle's value
    elsewhere."""
    torch = torch_cuda
    scene = _overflow_scene()
    W = H = 64
    mrs.counters(reset=True)
    rgb, _ = mrs.render(mrs.GpuScene(scene), W, H, 1, 1, 77)
    torch.cuda.synchronize()
    c = mrs.counters(reset=True)
    g = rgb.cpu().numpy().reshape(-1, 3).astype(np.float64)
    o = oracle_tracer.OracleScene(scene).render(W, H, 1, 1, 77)["rgb"]
    assert np.all(np.isfinite(g))
    over = o.max(1) > FLT_MAX * (1 + 1e-5)
    under = o.max(1) < FLT_MAX * (1 - 1e-5)
    _log(f"nonfinite: counter {c['nonfinite']}, oracle samples over FLT_MAX {over.sum()}, "
         f"under {under.sum()} of {W * H}")
    assert over.sum() > 100 and under.sum() > 100  # both cases occur
    assert np.all(g[over] == 0.0)
    assert np.all(np.abs(g[under] - o[under]) <= 1e-4 * np.abs(o[under]) + 1e-30)
    assert over.sum() <= c["nonfinite"] <= W * H - under.sum()
