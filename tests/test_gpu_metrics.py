"""GPU metrics (sRGB PSNR, RelMSE; FP64 reductions) vs the metric oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_metrics_match_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import metrics as M
    from paper_2106_12802_amd.metrics import image_metrics
    rng = np.random.default_rng(0)
    for shape in [(7, 5, 3), (720, 1280, 3), (33, 3)]:
        ref = rng.gamma(1.0, 0.5, shape).astype(np.float32)
        img = (ref + rng.normal(0, 0.05, shape)).astype(np.float32)
        img.flat[::97] = -0.5
        img.flat[::89] = 1e-4
        img.flat[::101] = 7.0
        r = image_metrics(torch.from_numpy(img).cuda(), torch.from_numpy(ref).cuda())
        mse = np.mean((M.srgb(img) - M.srgb(ref)) ** 2)
        assert r["mse_srgb"] == pytest.approx(mse, rel=1e-12)
        assert r["psnr"] == pytest.approx(M.psnr(img, ref), abs=1e-9)
        assert r["relmse"] == pytest.approx(M.relmse(img, ref), rel=1e-12)
        r2 = image_metrics(torch.from_numpy(img).cuda(), torch.from_numpy(ref).cuda(), 1.0, 1e-4)
        assert r2["relmse"] == pytest.approx(M.relmse(img, ref, 1.0, 1e-4), rel=1e-12)
    same = torch.ones(10, 3, device="cuda")
    assert image_metrics(same, same)["psnr"] == float("inf")
