"""Pins for the oracle's network input with the HRLS render layers (paper Sec. 4,
first paragraph: RGB plus albedo, normal, diffuse, specular and variance layers):
oracle/cnn.py preprocess_layers / layer_variance and the 16-channel variants of
both networks.  The variance is pinned against numpy's own variance of explicit
samples, the channel layout by values whose logarithms are exact, and the whole
forward and backward by an independent float64 torch implementation."""
import math

import numpy as np
import torch

from oracle import cnn, cnn_rdg


def _layer_inputs(seed, B, H, W, spp=6):
    """Explicit per-sample radiance split into emission, diffuse and glossy parts,
    reduced the way a render reduces them (means and sums of squares)."""
    rng = np.random.default_rng(seed)
    em = rng.gamma(0.3, 0.5, (B, H, W, spp, 3)) * (rng.random((B, H, W, spp, 1)) < 0.1)
    di = rng.gamma(1.0, 0.4, (B, H, W, spp, 3))
    gl = rng.gamma(0.7, 0.6, (B, H, W, spp, 3))
    gl[rng.random((B, H, W, spp)) < 0.01] *= 400.0  # fireflies
    L = em + di + gl
    rgb = L.mean(3)
    lay = np.concatenate([em.mean(3), di.mean(3), gl.mean(3)], -1)
    sumsq = (L * L).sum(3)
    aux = np.concatenate([rng.uniform(0, 1, (B, H, W, 3)), rng.normal(0, 1, (B, H, W, 3)),
                          rng.uniform(0, 20, (B, H, W, 1))], -1)
    lr = rng.gamma(1.0, 0.5, (B, H // 4, W // 4, 3))
    return rgb, aux, lay, sumsq, spp, lr, L


def test_variance_equals_numpy_var_of_the_samples():
    rgb, _, _, sumsq, spp, _, L = _layer_inputs(1, 2, 5, 7)
    want = np.clip(np.var(L, axis=3).mean(-1), 0.0, cnn.VAR_MAX)  # population variance
    got = cnn.layer_variance(rgb, sumsq, spp)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-12)
    # identical samples have no variance; the clamp bounds fireflies
    const = np.full((1, 1, 1, 3), 2.5)
    assert cnn.layer_variance(const, 4 * const * const, 4)[0, 0, 0] == 0.0
    huge = cnn.layer_variance(np.zeros((1, 3)), np.full((1, 3), 1e9), 2)
    assert huge[0] == cnn.VAR_MAX
    # two samples per channel: (0, 1), (2, 2), (1, 1): variances 1/4, 0, 0 -> mean 1/12
    v = cnn.layer_variance(np.array([[0.5, 2.0, 1.0]]), np.array([[1.0, 8.0, 2.0]]), 2)
    assert v[0] == 1.0 / 12.0


def test_layered_input_channels():
    """Channels 0-8 are the base input's rgb, albedo and normal; 9-11 and 12-14 the
    diffuse and glossy layers (log1p of their clipped values: e - 1 -> 1, e^2 - 1 ->
    2, above 100 -> log 101); 15 the variance.  Emission and depth do not enter."""
    rgb = np.array([[[[0.5, 2.0, 1e6]]]])
    aux = np.array([[[[0.2, 0.3, 0.4, 0.0, 1.0, 0.0, 5.0]]]])
    lay = np.array([[[[7.0, 7.0, 7.0, math.e - 1, math.e - 1, 300.0,
                       math.e ** 2 - 1, 0.0, -1.0]]]])
    sumsq = np.array([[[[2 * 0.25 + 2 * (math.e - 1), 8.0, 4e12]]]])  # spp 2
    lr = np.zeros((1, 0, 0, 3))
    xh, _ = cnn.preprocess_layers(rgb, aux, lay, sumsq, 2, lr)
    base, _ = cnn.preprocess(rgb, aux, lr)
    assert xh.shape == (1, 1, 1, 16)
    assert np.array_equal(xh[..., :9], base[..., :9])
    assert np.allclose(xh[0, 0, 0, 9:15], [1.0, 1.0, math.log(101.0), 2.0, 0.0, 0.0])
    # variance: channel 0 (0.25 + e - 1) - 0.25 = e - 1, channel 1 4 - 4 = 0, channel 2
    # beyond the clamp in sum -> mean over channels clamped to 1e4
    assert xh[0, 0, 0, 15] == np.log1p(cnn.VAR_MAX)
    lay2, aux2 = lay.copy(), aux.copy()
    lay2[..., 0:3] = 123.0   # emission
    aux2[..., 6] = 99.0      # depth
    xh2, _ = cnn.preprocess_layers(rgb, aux2, lay2, sumsq, 2, lr)
    assert np.array_equal(xh, xh2)


def test_param_counts_of_the_layered_variants():
    assert cnn.num_params(16) == cnn.num_params() + 64 * 6 * 9 == 1_412_339
    assert cnn_rdg.num_params(4, 16) == cnn_rdg.num_params(4) + 64 * 6 * 9
    assert cnn.hr_in_of(cnn.num_params(16)) == 16 and cnn.hr_in_of(cnn.num_params()) == 10


def _rand_params(specs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _, co, ci, k in specs:
        bound = math.sqrt(6.0 / (ci * k * k))
        out.append(rng.uniform(-bound, bound, co * ci * k * k))
        out.append(rng.uniform(-0.1, 0.1, co))
    return np.concatenate(out)


def _torch_res16(params, xh, xl):
    """Independent float64 torch forward of the 16-block network from its inputs."""
    L = cnn.unpack(params)
    conv = lambda x, n: torch.nn.functional.conv2d(x, torch.from_numpy(L[n][0]),
                                                   torch.from_numpy(L[n][1]),
                                                   padding=L[n][0].shape[2] // 2)
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


def _torch_inputs(rgb, aux, lay, sumsq, spp, lr):
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).permute(0, 3, 1, 2)
    m = torch.from_numpy(rgb)
    var = (torch.from_numpy(sumsq) / spp - m * m).mean(-1, keepdim=True).clamp(0, 1e4)
    xh = torch.cat([torch.log1p(T(rgb).clamp(0, 100)), T(aux[..., :6]),
                    torch.log1p(T(lay[..., 3:9]).clamp(0, 100)),
                    torch.log1p(var.permute(0, 3, 1, 2))], 1)
    return xh, torch.log1p(T(lr).clamp(0, 100))


def test_layered_res16_forward_and_backward_against_torch():
    rgb, aux, lay, sumsq, spp, lr, _ = _layer_inputs(3, 2, 8, 12)
    params = _rand_params(cnn.layer_specs(16), 4)
    out, acts = cnn.forward(params, rgb, aux, lr, keep=True, layers=(lay, sumsq, spp))
    xh, xl = _torch_inputs(rgb, aux, lay, sumsq, spp, lr)
    ref = _torch_res16(params, xh, xl)
    assert np.allclose(out, ref.numpy(), rtol=1e-10, atol=1e-10)
    tgt = np.random.default_rng(5).gamma(1.0, 0.5, out.shape)
    g = cnn.backward(params, acts, cnn.l1_grad(out, tgt))
    p = torch.from_numpy(params.copy()).requires_grad_(True)
    # autograd of the same loss through the torch forward (params as one leaf)
    offs = np.cumsum([0] + [co * ci * k * k + co for _, co, ci, k in cnn.layer_specs(16)])
    names = [n for n, *_ in cnn.layer_specs(16)]

    def unpack_t(pv):
        d = {}
        for i, (n, co, ci, k) in enumerate(cnn.layer_specs(16)):
            a = int(offs[i])
            d[n] = (pv[a:a + co * ci * k * k].reshape(co, ci, k, k),
                    pv[a + co * ci * k * k:int(offs[i + 1])])
        return d
    Lt = unpack_t(p)
    conv = lambda x, n: torch.nn.functional.conv2d(x, Lt[n][0], Lt[n][1],
                                                   padding=Lt[n][0].shape[2] // 2)
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
    o = conv(torch.cat([u, h0], 1), "rec").permute(0, 2, 3, 1)
    loss = (o - torch.from_numpy(cnn.clip_target(tgt))).abs().mean()
    loss.backward()
    assert names[0] == "hrls"
    assert np.allclose(g, p.grad.numpy(), rtol=1e-8, atol=1e-12)


def test_layered_rdg_forward_against_the_base_input_path():
    """The paper's network with the layered input equals the same network run on the
    base input path whose first conv sees the 16 layered channels: built here by
    feeding preprocess_layers' channels through the 10-channel entry with the input
    conv's weights split (the first conv is linear in its input channels)."""
    rgb, aux, lay, sumsq, spp, lr, _ = _layer_inputs(7, 1, 16, 16)
    specs16 = cnn_rdg.layer_specs(4, 16)
    params = _rand_params(specs16, 8)
    out = cnn_rdg.forward(params, rgb, aux, lr, layers=(lay, sumsq, spp))
    # the same network in torch from the layered inputs
    xh, xl = _torch_inputs(rgb, aux, lay, sumsq, spp, lr)
    L = cnn_rdg.unpack(params)
    assert L["hrls"][0].shape == (64, 16, 3, 3)
    conv = lambda x, n: torch.nn.functional.conv2d(x, torch.from_numpy(L[n][0]),
                                                   torch.from_numpy(L[n][1]),
                                                   padding=L[n][0].shape[2] // 2)
    h0 = torch.relu(conv(xh, "hrls"))
    want_h0 = cnn.relu(cnn.conv(cnn.preprocess_layers(rgb, aux, lay, sumsq, spp, lr)[0],
                                *L["hrls"]))
    assert np.allclose(h0.permute(0, 2, 3, 1).numpy(), want_h0, rtol=1e-12, atol=1e-12)
    assert out.shape == (1, 16, 16, 3) and np.all(np.isfinite(out))
