"""Pins for the FP64 fusion-network oracle (oracle/cnn.py).

The convolution is checked against its definition summed term by term; torch
(CPU, float64) serves only as an independent cross-check of the oracle, as do
central finite differences for the hand-written backward pass.
"""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import cnn


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for _, co, ci, k in cnn.layer_specs():
        bound = math.sqrt(6.0 / (ci * k * k)) * scale
        out.append(rng.uniform(-bound, bound, co * ci * k * k))
        out.append(rng.uniform(-0.1, 0.1, co))
    return np.concatenate(out)


def _inputs(seed, B, H, W):
    rng = np.random.default_rng(seed)
    hr = rng.gamma(1.0, 0.5, (B, H, W, 3))
    hr[rng.random((B, H, W)) < 0.01] *= 300.0  # fireflies above the clip
    aux = np.concatenate([rng.uniform(0, 1, (B, H, W, 3)),
                          rng.normal(0, 1, (B, H, W, 3)),
                          rng.uniform(0, 20, (B, H, W, 1))], -1)
    lr = rng.gamma(1.0, 0.5, (B, H // 4, W // 4, 3))
    return hr, aux, lr


def test_param_count():
    assert cnn.num_params() == 1_408_883


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 3))
    w = rng.normal(size=(2, 3, 3, 3))
    b = rng.normal(size=2)
    y = cnn.conv(x, w, b)
    B, H, W, C = x.shape
    for bb, yy, xx, o in itertools.product(range(B), range(H), range(W), range(2)):
        s = b[o]
        for c, ky, kx in itertools.product(range(C), range(3), range(3)):
            sy, sx = yy + ky - 1, xx + kx - 1
            if 0 <= sy < H and 0 <= sx < W:
                s += w[o, c, ky, kx] * x[bb, sy, sx, c]
        assert y[bb, yy, xx, o] == pytest.approx(s, abs=1e-12)


def test_conv_cross_check_torch():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 9, 7, 5))
    for k in (1, 3):
        w = rng.normal(size=(4, 5, k, k))
        b = rng.normal(size=4)
        ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w),
                                         torch.from_numpy(b), padding=k // 2).permute(0, 2, 3, 1)
        assert np.allclose(cnn.conv(x, w, b), ref.numpy(), atol=1e-12)


def test_unshuffle_convention_and_inverse():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 8, 12, 5))
    u = cnn.unshuffle(x)
    assert u.shape == (2, 2, 3, 80)
    # channel (i*4 + j)*C + c of pixel (Y, X) holds x[4Y+i, 4X+j, c]
    for Y, X, i, j, c in [(0, 0, 0, 0, 0), (1, 2, 3, 1, 4), (1, 0, 2, 3, 2)]:
        assert u[1, Y, X, (i * 4 + j) * 5 + c] == x[1, 4 * Y + i, 4 * X + j, c]
    # same values as torch.pixel_unshuffle up to a fixed channel permutation
    t = torch.nn.functional.pixel_unshuffle(torch.from_numpy(x).permute(0, 3, 1, 2), 4)
    t = t.permute(0, 2, 3, 1).numpy()  # torch channel c*16 + i*4 + j
    perm = np.array([c * 16 + q for q in range(16) for c in range(5)])
    assert np.array_equal(u, t[..., perm])
    assert np.array_equal(cnn.shuffle(u), x)


def test_preprocess_closed_forms():
    hr = np.array([[[[-1.0, 0.0, 1e6]]]])
    aux = np.array([[[[0.5, 0.5, 0.5, 0, 1, 0, math.e - 1]]]])
    lr = np.zeros((1, 0, 0, 3))
    xh, _ = cnn.preprocess(hr, aux, lr)
    assert np.allclose(xh[0, 0, 0], [0, 0, math.log(101), 0.5, 0.5, 0.5, 0, 1, 0, 1.0])


def _torch_forward(params, hr, aux, lr):
    """Independent float64 torch implementation of the same network (cross-check)."""
    L = cnn.unpack(params)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).permute(0, 3, 1, 2)
    conv = lambda x, n: torch.nn.functional.conv2d(x, torch.from_numpy(L[n][0]),
                                                   torch.from_numpy(L[n][1]),
                                                   padding=L[n][0].shape[2] // 2)
    xh = torch.cat([torch.log1p(T(hr).clamp(0, 100)), T(aux[..., :6]),
                    torch.log1p(T(aux[..., 6:]).clamp(min=0))], 1)
    xl = torch.log1p(T(lr).clamp(0, 100))
    h0 = torch.relu(conv(xh, "hrls"))
    fl = torch.relu(conv(xl, "lrhs"))
    un = torch.nn.functional.pixel_unshuffle(h0, 4)  # channel c*16 + q
    perm = torch.tensor([c * 16 + q for q in range(16) for c in range(64)])
    f0 = torch.relu(conv(torch.cat([fl, un[:, perm]], 1), "fuse"))
    r = f0
    for i in range(cnn.N_RES):
        r = r + 0.1 * conv(torch.relu(conv(r, f"res{i}a")), f"res{i}b")
    fdf = r + f0
    u_lr = torch.relu(conv(fdf, "up"))  # channel q*16 + c  ->  torch wants c*16 + q
    inv = torch.tensor([q * 16 + c for c in range(16) for q in range(16)])
    u = torch.nn.functional.pixel_shuffle(u_lr[:, inv], 4)
    out = conv(torch.cat([u, h0], 1), "rec")
    return out.permute(0, 2, 3, 1)


def test_forward_cross_check_torch():
    params = _rand_params(3)
    hr, aux, lr = _inputs(4, 2, 16, 24)
    out = cnn.forward(params, hr, aux, lr)
    ref = _torch_forward(params, hr, aux, lr).numpy()
    assert out.shape == (2, 16, 24, 3)
    assert np.allclose(out, ref, rtol=1e-10, atol=1e-10)


def test_backward_cross_check_autograd():
    params = _rand_params(5)
    hr, aux, lr = _inputs(6, 2, 8, 12)
    target = np.random.default_rng(7).gamma(1.0, 0.5, (2, 8, 12, 3))
    out, acts = cnn.forward(params, hr, aux, lr, keep=True)
    g = cnn.backward(params, acts, cnn.l1_grad(out, target))
    # autograd through the independent torch implementation
    p = torch.from_numpy(params.copy()).requires_grad_(True)
    L = {}
    off = 0
    for name, co, ci, k in cnn.layer_specs():
        nw = co * ci * k * k
        L[name] = off
        off += nw + co

    def fwd(pv):
        flat = pv
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).permute(0, 3, 1, 2)

        def conv(x, n):
            _, co, ci, k = [s for s in cnn.layer_specs() if s[0] == n][0]
            o = L[n]
            w = flat[o:o + co * ci * k * k].reshape(co, ci, k, k)
            b = flat[o + co * ci * k * k:o + co * ci * k * k + co]
            return torch.nn.functional.conv2d(x, w, b, padding=k // 2)

        xh = torch.cat([torch.log1p(T(hr).clamp(0, 100)), T(aux[..., :6]),
                        torch.log1p(T(aux[..., 6:]).clamp(min=0))], 1)
        xl = torch.log1p(T(lr).clamp(0, 100))
        h0 = torch.relu(conv(xh, "hrls"))
        fl = torch.relu(conv(xl, "lrhs"))
        un = torch.nn.functional.pixel_unshuffle(h0, 4)
        perm = torch.tensor([c * 16 + q for q in range(16) for c in range(64)])
        f0 = torch.relu(conv(torch.cat([fl, un[:, perm]], 1), "fuse"))
        r = f0
        for i in range(cnn.N_RES):
            r = r + 0.1 * conv(torch.relu(conv(r, f"res{i}a")), f"res{i}b")
        u_lr = torch.relu(conv(r + f0, "up"))
        inv = torch.tensor([q * 16 + c for c in range(16) for q in range(16)])
        u = torch.nn.functional.pixel_shuffle(u_lr[:, inv], 4)
        return conv(torch.cat([u, h0], 1), "rec").permute(0, 2, 3, 1)

    loss = (fwd(p) - torch.from_numpy(target)).abs().mean()
    loss.backward()
    assert np.allclose(g, p.grad.numpy(), rtol=1e-8, atol=1e-12)


def test_backward_central_differences():
    params = _rand_params(8)
    hr, aux, lr = _inputs(9, 1, 8, 8)
    target = np.random.default_rng(10).gamma(1.0, 0.5, (1, 8, 8, 3))

    # a smooth loss (squared error) avoids the kink of |.| at 0
    def loss(pv):
        return 0.5 * np.sum((cnn.forward(pv, hr, aux, lr) - target) ** 2)

    out, acts = cnn.forward(params, hr, aux, lr, keep=True)
    g = cnn.backward(params, acts, out - target)
    rng = np.random.default_rng(11)
    offs = np.cumsum([0] + [co * ci * k * k + co for _, co, ci, k in cnn.layer_specs()])
    idx = [int(rng.integers(offs[i], offs[i + 1])) for i in range(len(offs) - 1)][::3]
    h = 1e-6
    # rounding of the two loss values bounds the difference quotient's error
    roundoff = 64 * np.finfo(float).eps * abs(loss(params)) / h
    for i in idx:
        e = np.zeros_like(params)
        e[i] = h
        fd = (loss(params + e) - loss(params - e)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=roundoff), i


def test_adam_first_step_and_torch():
    rng = np.random.default_rng(12)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = cnn.adam_step(p, g, np.zeros(50), np.zeros(50), 1)
    # first step: mhat = g, vhat = g^2, so the update is lr * g / (|g| + eps)
    assert np.allclose(p - p1, 1e-4 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    tp = torch.from_numpy(p.copy()).requires_grad_(True)
    opt = torch.optim.Adam([tp], lr=1e-4, betas=(0.9, 0.999), eps=1e-8)
    pp, mm, vv = p.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        gs = rng.normal(size=50)
        tp.grad = torch.from_numpy(gs.copy())
        opt.step()
        pp, mm, vv = cnn.adam_step(pp, gs, mm, vv, step)
    assert np.allclose(pp, tp.detach().numpy(), rtol=1e-12, atol=1e-14)
