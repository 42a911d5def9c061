"""GPU parity of the fusion networks whose HRLS input carries the render layers
(MRS_NET_RES16_LAYERS, MRS_NET_RDG_LAYERS; paper Sec. 4, first paragraph) against
the FP64 oracle (oracle/cnn.py preprocess_layers), through the C ABI: forward on
synthetic and on rendered layers, gradients, training, binding rules."""
import math
import sys

import numpy as np
import pytest

from mrs_inputs import scenes as S

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel_l2(g, o):
    return float(np.linalg.norm(g - o) / np.linalg.norm(o))


def _inputs(seed, B, H, W, spp=4):
    """rgb, aux, layers, sums of squares of explicit samples, LRHS rgb (float32)."""
    rng = np.random.default_rng(seed)
    em = rng.gamma(0.3, 0.5, (B, H, W, spp, 3)) * (rng.random((B, H, W, spp, 1)) < 0.1)
    di = rng.gamma(1.0, 0.4, (B, H, W, spp, 3))
    gl = rng.gamma(0.7, 0.6, (B, H, W, spp, 3))
    gl[rng.random((B, H, W, spp)) < 0.01] *= 300.0
    L = (em + di + gl).astype(np.float32)
    rgb = L.mean(3)
    lay = np.concatenate([em.mean(3), di.mean(3), gl.mean(3)], -1)
    sq = (L.astype(np.float64) ** 2).sum(3)
    aux = np.concatenate([rng.uniform(0, 1, (B, H, W, 3)), rng.normal(0, 1, (B, H, W, 3)),
                          rng.uniform(0, 20, (B, H, W, 1))], -1)
    lr = rng.gamma(1.0, 0.5, (B, H // 4, W // 4, 3))
    return [a.astype(np.float32) for a in (rgb, aux, lay, sq, lr)], spp


def _bf16_weights(params, specs):
    p = params.astype(np.float32).copy()
    off = 0
    for _, co, ci, k in specs:
        nw = co * ci * k * k
        u = p[off:off + nw].view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        p[off:off + nw] = u.astype(np.uint32).view(np.float32)
        off += nw + co
    return p.astype(np.float64)


def test_binding_rules(torch_cuda):
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd._lib import MrsError
    torch = torch_cuda
    f = dict(dtype=torch.float32, device="cuda")
    hr, aux, lr = torch.zeros(8, 8, 3, **f), torch.zeros(8, 8, 7, **f), torch.zeros(2, 2, 3, **f)
    lay, sq = torch.zeros(8, 8, 9, **f), torch.zeros(8, 8, 3, **f)
    net = mrs.FusionNet(seed=1, arch="res16_layers")
    assert net.num_params == 1_412_339
    with pytest.raises(MrsError, match="NOT_READY"):
        net.fuse(hr, aux, lr)  # no layers bound
    with pytest.raises(MrsError, match="spp"):
        net.bind_layers(lay, sq, 0)
    out = net.fuse(hr, aux, lr, layers=(lay, sq, 4))
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
    with pytest.raises(MrsError, match="no render layers"):
        mrs.FusionNet(seed=1).bind_layers(lay, sq, 4)
    assert mrs.FusionNet(seed=1, arch="rdg_layers").num_params == 5_911_363


@pytest.mark.parametrize("arch,B,H,W", [("res16_layers", 2, 16, 24), ("res16_layers", 1, 96, 128),
                                        ("res16_layers", 8, 256, 256), ("rdg_layers", 2, 16, 24),
                                        ("rdg_layers", 1, 96, 136)])
def test_forward_parity(torch_cuda, arch, B, H, W):
    """Synthetic layers from explicit samples; bars as for the networks without
    layers (16-block: 5e-3 against the FP32 masters; the paper's network: 5e-3
    against its BF16-weight oracle, 8e-3 against the FP32 masters)."""
    import paper_2106_12802_amd as mrs
    from oracle import cnn, cnn_rdg
    torch = torch_cuda
    _log(f"{arch} forward parity {B}x{H}x{W}")
    (rgb, aux, lay, sq, lr), spp = _inputs(B * H + W, B, H, W)
    net = mrs.FusionNet(seed=55, arch=arch)
    params = net.get_params().astype(np.float64)
    t = [torch.from_numpy(a).cuda() for a in (rgb, aux, lay, sq, lr)]
    out = net.fuse(t[0], t[1], t[4], layers=(t[2], t[3], spp))
    torch.cuda.synchronize()
    g = out.cpu().numpy().astype(np.float64)
    layers = (lay, sq, spp)
    if arch == "res16_layers":
        o = cnn.forward(params, rgb, aux, lr, layers=layers)
        e = _rel_l2(g, o)
        _log(f"  rel L2 out {e:.2e}")
        assert e <= 5e-3
    else:
        o = cnn_rdg.forward(_bf16_weights(params, cnn_rdg.layer_specs(4, 16)), rgb, aux, lr,
                            layers=layers)
        e, e32 = _rel_l2(g, o), _rel_l2(g, cnn_rdg.forward(params, rgb, aux, lr, layers=layers))
        _log(f"  rel L2 vs BF16-weight oracle {e:.2e}, vs FP32 masters {e32:.2e}")
        assert e <= 5e-3 and e32 <= 8e-3


def test_forward_parity_on_rendered_layers(torch_cuda, oracle_tracer):
    """The inputs as the tracer renders them (a 128 x 96 window of the bench scene at
    4 spp: image, features, render layers, sums of squares; LRHS at 64 spp)."""
    import paper_2106_12802_amd as mrs
    from oracle import cnn
    torch = torch_cuda
    gs = mrs.GpuScene(S.procedural(7))
    W, H, win = 1280, 720, (576, 320, 128, 96)
    f = dict(dtype=torch.float32, device="cuda")
    rgb, aux = torch.empty(96, 128, 3, **f), torch.empty(96, 128, 7, **f)
    lay, sq = torch.empty(96, 128, 9, **f), torch.zeros(96, 128, 3, **f)
    lr = torch.empty(24, 32, 3, **f)
    mrs.render_ex(gs, W, H, 4, 8, 41, rgb, aux, window=win, out_layers=lay, out_sumsq=sq)
    mrs.render_ex(gs, W // 4, H // 4, 64, 8, 42, lr, None, window=(144, 80, 32, 24))
    net = mrs.FusionNet(seed=9, arch="res16_layers")
    out = net.fuse(rgb, aux, lr, layers=(lay, sq, 4))
    torch.cuda.synchronize()
    h = [a.cpu().numpy()[None] for a in (rgb, aux, lay, sq, lr)]
    o = cnn.forward(net.get_params().astype(np.float64), h[0], h[1], h[4],
                    layers=(h[2], h[3], 4))
    e = _rel_l2(out.cpu().numpy()[None].astype(np.float64), o)
    v = cnn.layer_variance(h[0], h[3], 4)
    _log(f"rendered layers: rel L2 {e:.2e}; variance channel median {np.median(v):.3e}, "
         f"max {v.max():.3e}")
    assert e <= 5e-3


def test_gradient_parity(torch_cuda):
    """GPU backward of the layered 16-block network against the FP64 hand backward
    from the same output gradient (bars of the network without layers: 4e-2 per
    layer, 1e-2 whole)."""
    import paper_2106_12802_amd as mrs
    from oracle import cnn
    torch = torch_cuda
    B, H, W = 2, 32, 48
    (rgb, aux, lay, sq, lr), spp = _inputs(7, B, H, W)
    net = mrs.FusionNet(seed=77, arch="res16_layers")
    params = net.get_params().astype(np.float64)
    tgt = np.random.default_rng(3).gamma(1.0, 0.5, (B, H, W, 3))
    o, acts = cnn.forward(params, rgb, aux, lr, keep=True, layers=(lay, sq, spp))
    gout = cnn.l1_grad(o, tgt)
    g_ref = cnn.backward(params, acts, gout)
    t = [torch.from_numpy(a).cuda() for a in (rgb, aux, lay, sq, lr)]
    g_gpu = net.backward(t[0], t[1], t[4], torch.from_numpy(gout.astype(np.float32)).cuda(),
                         layers=(t[2], t[3], spp)).astype(np.float64)
    off, errs = 0, {}
    for name, co, ci, k in cnn.layer_specs(16):
        n = co * ci * k * k + co
        errs[name] = _rel_l2(g_gpu[off:off + n], g_ref[off:off + n])
        off += n
    e_all = _rel_l2(g_gpu, g_ref)
    worst = max(errs, key=errs.get)
    _log(f"layered grad: all {e_all:.2e}; worst {worst} {errs[worst]:.2e}; hrls {errs['hrls']:.2e}")
    assert all(v <= 4e-2 for v in errs.values()), errs
    assert e_all <= 1e-2


def test_training_steps_reduce_the_loss(torch_cuda):
    import paper_2106_12802_amd as mrs
    torch = torch_cuda
    (rgb, aux, lay, sq, lr), spp = _inputs(11, 4, 32, 32)
    tgt = (rgb * 0.8 + 0.05).astype(np.float32)
    t = [torch.from_numpy(a).cuda() for a in (rgb, aux, lay, sq, lr, tgt)]
    net = mrs.FusionNet(seed=5, arch="res16_layers")
    losses = [net.train_step(t[0], t[1], t[4], t[5], lr=1e-3, want_loss=True,
                             layers=(t[2], t[3], spp)) for _ in range(60)]
    _log(f"layered training: {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert math.isfinite(losses[-1]) and losses[-1] < 0.5 * losses[0]
