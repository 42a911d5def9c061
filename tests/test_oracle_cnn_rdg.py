"""Pins for the FP64 oracle of the paper's own fusion network (oracle/cnn_rdg.py).

The network's forward is checked against closed forms of its structure (the
stacked deshuffle's index map, the residual skeleton with every dense branch
switched off) and against an independent float64 torch implementation of the
architecture; the hand-written backward against torch autograd and central
differences; the robust loss against its limits and its derivative.
"""
import math

import numpy as np
import pytest
import torch

from oracle import cnn, cnn_rdg as rdg


def _rand_params(seed, scale=1.0, branch_scale=0.1, sr=4):
    rng = np.random.default_rng(seed)
    out = []
    for name, co, ci, k in rdg.layer_specs(sr):
        bound = math.sqrt(6.0 / (ci * k * k)) * scale
        if name.endswith(f"c{rdg.N_CONVS - 1}"):
            bound *= branch_scale  # keep the 15-block residual chain at its input's scale
        out.append(rng.uniform(-bound, bound, co * ci * k * k))
        out.append(rng.uniform(-0.1, 0.1, co))
    return np.concatenate(out)


def _inputs(seed, B, H, W, sr=4):
    rng = np.random.default_rng(seed)
    hr = rng.gamma(1.0, 0.5, (B, H, W, 3))
    hr[rng.random((B, H, W)) < 0.01] *= 300.0
    aux = np.concatenate([rng.uniform(0, 1, (B, H, W, 3)),
                          rng.normal(0, 1, (B, H, W, 3)),
                          rng.uniform(0, 20, (B, H, W, 1))], -1)
    lr = rng.gamma(1.0, 0.5, (B, H // sr, W // sr, 3))
    return hr, aux, lr


def test_param_count():
    # encoders 5,824 + 1,792; fuse 64*1088 + 64 = 69,696;
    # one RDB: 9*64*(64 + 128 + 192 + 256) + 4*64 = 368,896, times 15 = 5,533,440;
    # two upscale convs 2*(256*64*9 + 256) = 295,424; reconstruction 3*64*9 + 3 = 1,731
    assert rdg.num_params() == 5_907_907
    names = [s[0] for s in rdg.layer_specs()]
    assert len(names) == 3 + 60 + 3 and len(set(names)) == len(names)
    # x2: fuse 64*(64 + 256) + 64 = 20,544, one upscale conv 147,712
    assert rdg.num_params(2) == 5_824 + 1_792 + 20_544 + 5_533_440 + 147_712 + 1_731
    # x8: fuse 64*(64 + 4096) + 64 = 266,304, three upscale convs 443,136
    assert rdg.num_params(8) == 5_824 + 1_792 + 266_304 + 5_533_440 + 443_136 + 1_731
    with pytest.raises(ValueError):
        rdg.layer_specs(3)


def test_deshuffle_stack_index_map():
    rng = np.random.default_rng(1)
    C = 3
    x = rng.normal(size=(2, 8, 12, C))
    u = rdg.deshuffle_stack(x)
    assert u.shape == (2, 2, 3, 16 * C)
    # HR pixel (4Y+I, 4X+J), channel c lands in LR channel
    # ((I//2)*2 + J//2) * 4C + ((I%2)*2 + J%2) * C + c:
    # the first stride-2 deshuffle consumes the low bit of I and J.
    for b in range(2):
        for Y in range(2):
            for X in range(3):
                for I in range(4):
                    for J in range(4):
                        for c in range(C):
                            ch = ((I // 2) * 2 + J // 2) * 4 * C + ((I % 2) * 2 + J % 2) * C + c
                            assert u[b, Y, X, ch] == x[b, 4 * Y + I, 4 * X + J, c]
    # a permutation: shuffling twice restores the input
    assert np.array_equal(cnn.shuffle(cnn.shuffle(u, 2), 2), x)


def test_branches_off_leave_the_residual_skeleton():
    """With every RDB's fusing conv zeroed, each block is the identity, each
    group doubles its input (F_g = F_{g-1} + F_{g-1}) and F_DF = 8 F_0 + F_0."""
    params = _rand_params(2)
    off = 0
    for name, co, ci, k in rdg.layer_specs():
        n = co * ci * k * k + co
        if name.endswith(f"c{rdg.N_CONVS - 1}"):
            params[off:off + n] = 0.0
        off += n
    hr, aux, lr = _inputs(3, 1, 16, 16)
    out, acts = rdg.forward(params, hr, aux, lr, keep=True)
    assert np.allclose(acts["fdf"], 9.0 * acts["f0"], rtol=1e-13, atol=1e-13)
    # and the block outputs are exactly their inputs
    for g in range(rdg.N_GROUPS):
        for b in range(rdg.N_BLOCKS - 1):
            nxt = acts["dense"][g, b + 1][0]
            assert np.array_equal(nxt, acts["dense"][g, b][0])


def _torch_forward(flat, hr, aux, lr, sr=4):
    """Independent float64 torch implementation of the same architecture, NCHW,
    with torch's pixel (un)shuffle and the channel permutations between its
    convention and the oracle's."""
    D = {2: 1, 4: 2, 8: 3}[sr]
    offs = {}
    off = 0
    for name, co, ci, k in rdg.layer_specs(sr):
        offs[name] = (off, co, ci, k)
        off += co * ci * k * k + co

    def conv(x, n):
        o, co, ci, k = offs[n]
        w = flat[o:o + co * ci * k * k].reshape(co, ci, k, k)
        b = flat[o + co * ci * k * k:o + co * ci * k * k + co]
        return torch.nn.functional.conv2d(x, w, b, padding=k // 2)

    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).permute(0, 3, 1, 2)
    xh = torch.cat([torch.log1p(T(hr).clamp(0, 100)), T(aux[..., :6]),
                    torch.log1p(T(aux[..., 6:]).clamp(min=0))], 1)
    xl = torch.log1p(T(lr).clamp(0, 100))
    h0 = torch.relu(conv(xh, "hrls"))
    fl = torch.relu(conv(xl, "lrhs"))
    fh = h0
    for _ in range(D):  # torch: channel c*4 + q; oracle: q*C + c
        C = fh.shape[1]
        fh = torch.nn.functional.pixel_unshuffle(fh, 2)
        fh = fh[:, torch.tensor([c * 4 + q for q in range(4) for c in range(C)])]
    f0 = torch.relu(conv(torch.cat([fl, fh], 1), "fuse"))
    F = f0
    for g in range(3):
        s = F
        for b in range(5):
            xs = [s]
            for c in range(3):
                xs.append(torch.relu(conv(torch.cat(xs, 1), f"g{g}b{b}c{c}")))
            s = s + conv(torch.cat(xs, 1), f"g{g}b{b}c3")
        F = s + F
    u = F + f0
    for i in range(D):
        a = torch.relu(conv(u, f"up{i}"))
        C = a.shape[1] // 4
        a = a[:, torch.tensor([q * C + c for c in range(C) for q in range(4)])]
        u = torch.nn.functional.pixel_shuffle(a, 2)
    return conv(u, "rec").permute(0, 2, 3, 1)


def test_forward_cross_check_torch():
    params = _rand_params(4)
    hr, aux, lr = _inputs(5, 2, 16, 24)
    out = rdg.forward(params, hr, aux, lr)
    ref = _torch_forward(torch.from_numpy(params), hr, aux, lr).numpy()
    assert out.shape == (2, 16, 24, 3)
    scale = np.abs(ref).max()
    assert scale > 1e-3
    assert np.allclose(out, ref, rtol=1e-10, atol=1e-12 * scale)


@pytest.mark.parametrize("sr", [2, 8])
def test_other_scales_cross_check_torch(sr):
    """x2 (one deshuffle, one upscaling step) and x8 (three of each): forward
    against the torch implementation, backward against torch autograd."""
    params = _rand_params(20 + sr, sr=sr)
    hr, aux, lr = _inputs(21 + sr, 1, 16, 24, sr=sr)
    target = np.random.default_rng(22).gamma(1.0, 0.5, (1, 16, 24, 3))
    out, acts = rdg.forward(params, hr, aux, lr, keep=True, scale=sr)
    p = torch.from_numpy(params.copy()).requires_grad_(True)
    y = _torch_forward(p, hr, aux, lr, sr=sr)
    assert out.shape == (1, 16, 24, 3)
    assert np.allclose(out, y.detach().numpy(), rtol=1e-10, atol=1e-12 * np.abs(out).max())
    g = rdg.backward(params, acts, rdg.robust_grad(out, target, 0.1), scale=sr)
    d = (y - torch.from_numpy(target).clamp(0, 100)).abs()
    (d / (0.1 + d)).mean().backward()
    ref = p.grad.numpy()
    assert np.allclose(g, ref, rtol=1e-8, atol=1e-12 * np.abs(ref).max())


def test_backward_cross_check_autograd_robust_loss():
    params = _rand_params(6)
    hr, aux, lr = _inputs(7, 2, 8, 12)
    target = np.random.default_rng(8).gamma(1.0, 0.5, (2, 8, 12, 3))
    target[0, 0, 0, 0] = 500.0  # above the clip
    out, acts = rdg.forward(params, hr, aux, lr, keep=True)
    g = rdg.backward(params, acts, rdg.robust_grad(out, target, 0.1))
    p = torch.from_numpy(params.copy()).requires_grad_(True)
    y = _torch_forward(p, hr, aux, lr)
    d = (y - torch.from_numpy(target).clamp(0, 100)).abs()
    loss = (d / (0.1 + d)).mean()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(rdg.robust_loss(out, target, 0.1), rel=1e-12)
    ref = p.grad.numpy()
    assert np.allclose(g, ref, rtol=1e-8, atol=1e-12 * np.abs(ref).max())


def test_backward_central_differences():
    params = _rand_params(9)
    hr, aux, lr = _inputs(10, 1, 8, 8)
    target = np.random.default_rng(11).gamma(1.0, 0.5, (1, 8, 8, 3))

    def loss(pv):
        return 0.5 * np.sum((rdg.forward(pv, hr, aux, lr) - target) ** 2)

    out, acts = rdg.forward(params, hr, aux, lr, keep=True)
    g = rdg.backward(params, acts, out - target)
    rng = np.random.default_rng(12)
    specs = rdg.layer_specs()
    offs = np.cumsum([0] + [co * ci * k * k + co for _, co, ci, k in specs])
    # one parameter in each of a spread of layers, including every conv of one RDB
    layers = [0, 1, 2, 3, 4, 5, 6, 30, 62, 63, 64, 65]
    h = 1e-6
    roundoff = 64 * np.finfo(float).eps * abs(loss(params)) / h
    for li in layers:
        i = int(rng.integers(offs[li], offs[li + 1]))
        e = np.zeros_like(params)
        e[i] = h
        fd = (loss(params + e) - loss(params - e)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=roundoff), (specs[li][0], i)


def test_robust_loss_limits_and_derivative():
    rng = np.random.default_rng(13)
    t = rng.uniform(0, 5, 1000)
    assert rdg.robust_loss(t, t) == 0.0
    # small errors: l_r ~ mean|d| / beta, with the next term -mean d^2 / beta^2
    d = rng.normal(0, 1e-6, 1000)
    l1 = np.abs(d).mean()
    assert rdg.robust_loss(t + d, t, 0.1) == pytest.approx(l1 / 0.1, rel=1e-4)
    # huge errors: l_r -> 1 from below (targets clip at 100, outputs do not)
    big = rdg.robust_loss(t + 1e9, t, 0.1)
    assert 1.0 - 1e-9 < big < 1.0
    # always below both 1 and l1 / beta
    o = t + rng.normal(0, 3, 1000)
    lr_ = rdg.robust_loss(o, t, 0.1)
    assert lr_ < 1.0 and lr_ < np.abs(o - t).mean() / 0.1
    # beta -> infinity: beta * l_r -> l1
    assert 1e8 * rdg.robust_loss(o, t, 1e8) == pytest.approx(np.abs(o - t).mean(), rel=1e-7)
    # derivative: central differences, one element at a time (N = 1), then 1/N
    g = rdg.robust_grad(o, t, 0.1)
    for i in rng.choice(1000, 10, replace=False):
        oi, ti = o[i:i + 1], t[i:i + 1]
        fd = (rdg.robust_loss(oi + 1e-7, ti, 0.1) - rdg.robust_loss(oi - 1e-7, ti, 0.1)) / 2e-7
        assert fd / 1000 == pytest.approx(g[i], rel=1e-6)
    assert rdg.robust_grad(t, t).tolist() == [0.0] * 1000  # sign(0) = 0


def test_sgd_matches_torch():
    rng = np.random.default_rng(14)
    p = rng.normal(size=40)
    tp = torch.from_numpy(p.copy()).requires_grad_(True)
    opt = torch.optim.SGD([tp], lr=1e-4)
    for _ in range(3):
        g = rng.normal(size=40)
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        p = rdg.sgd_step(p, g, 1e-4)
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-15, atol=0)
