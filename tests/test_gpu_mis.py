"""GPU parity of the multiple-importance-sampling estimator (next-event estimation
and BSDF sampling of the quad lights, power heuristic) against the FP64 oracle,
through the C ABI, and its invariances."""
import sys

import numpy as np
import pytest

from mrs_inputs import scenes as S

pytestmark = pytest.mark.gpu

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_tracer import _parity, gpu_render  # noqa: E402


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


@pytest.mark.parametrize("scene_seed", [1, 3])
def test_cornell_mis_parity(mrs, oracle_tracer, scene_seed):
    scene = S.cornell(scene_seed)
    W = H = 64
    spp, D, seed = 16, 4, 2000 + scene_seed
    _log(f"mis cornell {scene_seed}")
    g_rgb, g_aux, _ = gpu_render(mrs, scene, W, H, spp, D, seed, mis=True)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, D, seed, mis=True)
    frac, mean_rel, aux_frac = _parity(g_rgb, g_aux, o, f"mis cornell {scene_seed}")
    assert frac >= 0.999 and mean_rel <= 1e-5 and aux_frac >= 0.999


def test_procedural_mis_parity_ragged(mrs, oracle_tracer):
    """The 101k-triangle scene (Lambert and GGX, 3 quad lights), 97 x 55 at 4 spp."""
    scene = S.procedural(7)
    W, H, spp, D, seed = 97, 55, 4, 8, 31
    _log("mis procedural 97x55x4")
    g_rgb, g_aux, _ = gpu_render(mrs, scene, W, H, spp, D, seed, mis=True)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, D, seed, mis=True)
    frac, mean_rel, aux_frac = _parity(g_rgb, g_aux, o, "mis procedural 97x55x4")
    assert frac >= 0.999 and mean_rel <= 1e-4 and aux_frac >= 0.999


def test_procedural_mis_parity_lrhs_full_size(mrs, oracle_tracer, torch_cuda):
    """The LRHS image at full size, 320 x 180 at 64 spp, against the oracle."""
    scene = S.procedural(7)
    _log("mis procedural 320x180x64")
    g_rgb, g_aux, _ = gpu_render(mrs, scene, 320, 180, 64, 8, 33, mis=True)
    o = oracle_tracer.OracleScene(scene).render(320, 180, 64, 8, 33, mis=True)
    frac, mean_rel, aux_frac = _parity(g_rgb.reshape(-1, 3), g_aux.reshape(-1, 7), o,
                                       "mis procedural 320x180x64")
    assert frac >= 0.999 and mean_rel <= 1e-5 and aux_frac >= 0.999


def test_mis_changes_only_light_paths_and_is_tuning_invariant(mrs, torch_cuda):
    """Without quad lights MIS changes nothing (bitwise); with them the image
    differs but not its features, and it is bitwise the same whichever kernel
    traces the late bounces (the path tail carries the BSDF density)."""
    torch = torch_cuda
    _log("mis invariances")
    a, aa, _ = gpu_render(mrs, S.lambert_plane(), 32, 16, 8, 3, 5)
    m, ma, _ = gpu_render(mrs, S.lambert_plane(), 32, 16, 8, 3, 5, mis=True)
    assert np.array_equal(a, m) and np.array_equal(aa, ma)
    gs = mrs.GpuScene(S.procedural(7))
    old = mrs.get_tuning()
    try:
        ref, raux = mrs.render(gs, 640, 360, 4, 8, 41, mis=True)
        plain, paux = mrs.render(gs, 640, 360, 4, 8, 41)
        torch.cuda.synchronize()
        assert not torch.equal(ref, plain) and torch.equal(raux, paux)
        for tune in (dict(tail_bounce=1), dict(tail_bounce=65), dict(streams=1)):
            mrs.set_tuning(**dict(old, **tune))
            img, _ = mrs.render(gs, 640, 360, 4, 8, 41, mis=True)
            torch.cuda.synchronize()
            assert torch.equal(img, ref), tune
    finally:
        mrs.set_tuning(**old)


def test_mis_batch_job_equals_single_render(mrs, torch_cuda):
    torch = torch_cuda
    _log("mis batch")
    gs = mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))
    b = mrs.Batch([dict(scene=gs, W=96, H=64, spp=8, max_depth=5, seed=3, mis=True),
                   dict(scene=gs, W=64, H=64, spp=4, max_depth=5, seed=4)])
    b.render()
    r1, _ = mrs.render(gs, 96, 64, 8, 5, 3, mis=True)
    r2, _ = mrs.render(gs, 64, 64, 4, 5, 4)
    torch.cuda.synchronize()
    assert torch.equal(b.outputs[0][0], r1) and torch.equal(b.outputs[1][0], r2)
