"""What the trained fusion network gains over the method without it.

Held-out procedural scene (seed 200: not among the training scenes 100..198), 1280x720,
PSNR (Eq. 3 sRGB, peak 1) against a 1024-spp render with an independent seed.  Each
trained network (the 16-block trunk and the paper's network) must beat every input it
fuses and the same network untrained."""
import os
import sys

import pytest

from mrs_inputs import scenes as S

pytestmark = pytest.mark.gpu

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                           "paper_2106_12802_amd", "weights")


@pytest.mark.parametrize("arch,weights", [("res16", "fusion_l1_textured.bin"),
                                          ("rdg", "fusion_rdg_l1.bin")])
def test_trained_network_beats_its_inputs_and_untrained(arch, weights):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as HY
    from paper_2106_12802_amd.metrics import image_metrics
    seed, tris = S.training_scene_specs(200, 1)[0]
    gs = mrs.GpuScene(S.procedural_sized(seed, tris))
    W, H = 1280, 720
    ref = HY.reference(gs, W, H, 1024, HY.REF_SEED + 3)
    trained = mrs.FusionNet(arch=arch)
    trained.load_weights(os.path.join(WEIGHTS_DIR, weights))
    untrained = mrs.FusionNet(seed=1, arch=arch)
    psnr = {}
    for name, net in (("trained", trained), ("untrained", untrained), ("plain_same_paths", None)):
        out, _ = HY.hybrid_frame(gs, net, W, H, 3)
        psnr[name] = image_metrics(out, ref)["psnr"]
    hr, aux, lr = HY.render_inputs(gs, W, H, 3)
    up = torch.nn.functional.interpolate(lr.permute(2, 0, 1)[None], scale_factor=4,
                                         mode="bilinear", align_corners=False)[0]
    psnr["hrls_4spp"] = image_metrics(hr, ref)["psnr"]
    psnr["lrhs_bilinear"] = image_metrics(up.permute(1, 2, 0).contiguous(), ref)["psnr"]
    print(arch, "PSNR dB:", {k: round(v, 2) for k, v in psnr.items()}, file=sys.stderr, flush=True)
    others = [v for k, v in psnr.items() if k != "trained"]
    assert psnr["trained"] >= max(others) + 0.5
