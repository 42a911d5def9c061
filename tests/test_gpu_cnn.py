"""GPU parity of the BF16 MFMA fusion network against the FP64 oracle (via the C ABI)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def net(torch_cuda):
    import paper_2106_12802_amd as mrs
    return mrs.FusionNet(seed=1234)


def _inputs(seed, B, H, W):
    rng = np.random.default_rng(seed)
    hr = rng.gamma(1.0, 0.5, (B, H, W, 3))
    hr[rng.random((B, H, W)) < 0.01] *= 300.0
    aux = np.concatenate([rng.uniform(0, 1, (B, H, W, 3)),
                          rng.normal(0, 1, (B, H, W, 3)),
                          rng.uniform(0, 20, (B, H, W, 1))], -1)
    lr = rng.gamma(1.0, 0.5, (B, H // 4, W // 4, 3))
    return [a.astype(np.float32) for a in (hr, aux, lr)]


def _rel_l2(g, o):
    return float(np.linalg.norm(g - o) / np.linalg.norm(o))


def test_init_statistics(net):
    from oracle import cnn
    p = net.get_params().astype(np.float64)
    assert p.size == cnn.num_params() == 1_408_883
    off = 0
    for name, co, ci, k in cnn.layer_specs():
        nw = co * ci * k * k
        w, b = p[off:off + nw], p[off + nw:off + nw + co]
        bound = math.sqrt(6.0 / (ci * k * k))
        assert np.all(np.abs(w) <= bound) and np.all(b == 0), name
        if nw > 10_000:
            assert abs(w.mean()) < 0.02 * bound and abs(w.var() / (bound ** 2 / 3) - 1) < 0.03
        off += nw + co
    import paper_2106_12802_amd as mrs
    assert np.array_equal(mrs.FusionNet(seed=1234).get_params(), net.get_params())
    assert not np.array_equal(mrs.FusionNet(seed=1235).get_params(), net.get_params())


@pytest.mark.parametrize("B,H,W", [(2, 16, 24), (1, 20, 36), (1, 96, 128)])
def test_forward_parity(net, torch_cuda, B, H, W):
    from oracle import cnn
    torch = torch_cuda
    hr, aux, lr = _inputs(B * H + W, B, H, W)
    params = net.get_params().astype(np.float64)
    t = [torch.from_numpy(a).cuda() for a in (hr, aux, lr)]
    out = net.fuse(*t)
    torch.cuda.synchronize()
    g = out.cpu().numpy().astype(np.float64)
    o, acts = cnn.forward(params, hr, aux, lr, keep=True)
    f0 = net.activation(0, acts["f0"].shape)
    fdf = net.activation(1, acts["fdf"].shape)
    e_out, e_f0, e_fdf = _rel_l2(g, o), _rel_l2(f0, acts["f0"]), _rel_l2(fdf, acts["fdf"])
    _log(f"cnn {B}x{H}x{W}: rel L2 out {e_out:.2e}, F0 {e_f0:.2e}, FDF {e_fdf:.2e}")
    assert e_f0 <= 5e-3 and e_fdf <= 5e-3
    assert e_out <= 5e-3


def test_fuse_not_ready_and_validation(torch_cuda):
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd._lib import MrsError
    torch = torch_cuda
    n = mrs.FusionNet()
    hr = torch.zeros(8, 8, 3, device="cuda")
    aux = torch.zeros(8, 8, 7, device="cuda")
    lr = torch.zeros(2, 2, 3, device="cuda")
    with pytest.raises(MrsError, match="NOT_READY"):
        n.fuse(hr, aux, lr)
    n.init(1)
    with pytest.raises(MrsError, match="multiples of 4"):
        n.fuse(torch.zeros(6, 8, 3, device="cuda"), torch.zeros(6, 8, 7, device="cuda"), lr)
