"""FP64 reference of the HRLS+LRHS fusion network -- TEST INFRASTRUCTURE ONLY.

Plain numpy, float64, written from the architecture description (paper Sec. 4
and the network row of the build's configuration): two shallow encoders
(Eqs. for F_LRHS and F^0_HRLS), a deshuffle (pixel unshuffle, Fig. 4) of the
HRLS features down to the LRHS size, concatenation and a 1x1 fusion conv
giving F_0, a residual trunk with a global residual (F_DF = trunk(F_0) + F_0),
and a pixel-shuffle upscaler followed by the reconstruction conv H_Rec, which
also sees the HRLS features.  Every conv is 3x3 except the 1x1 fusion conv;
every conv except the last is followed by ReLU (Sec. 4, implementation
details); 64 feature channels.  The trunk is 16 residual blocks
r <- r + 0.1 * conv(ReLU(conv(r))) (the configuration's "16 residual blocks").

Conventions fixed here (the GPU library documents the same ones):
  * tensors are NHWC;
  * unshuffle by r maps x[b, r*Y+i, r*X+j, c] to channel (i*r + j)*C + c of
    pixel (Y, X); shuffle is its inverse (a fixed permutation of the channel
    order of torch.pixel_unshuffle / pixel_shuffle);
  * inputs: RGB clipped to [0, 100] (Sec. 3.2) then log1p; albedo and normal
    as rendered; depth log1p(max(d, 0)).  HRLS = 3 RGB + 7 features (10
    channels), LRHS = 3 RGB.  The output is linear RGB.
  * parameters: one flat float32 vector, layer by layer, each as the weight
    [C_out, C_in, k, k] followed by the bias [C_out].

With the HRLS render layers (paper Sec. 4, first paragraph: I_HRLS is RGB plus
albedo, normal, diffuse, specular and variance layers; the layers of Sec. 3.1),
the HRLS input has 16 channels instead of 10: log1p of the clipped RGB, albedo,
normal, log1p of the clipped diffuse and glossy (specular) layers, and log1p of
the per-sample variance averaged over the three colour channels (clamped to
[0, 1e4]), computed from the per-pixel sums of squares and the sample count.
Depth is not part of it (the paper's list has none); the emission layer enters
implicitly as RGB minus the two lobes.  Only the input conv changes (16 -> 64).

Only tests/, the smoke check and the bench's CPU-baseline leg use this module.
"""
from __future__ import annotations

import numpy as np

SCALE = 4
FEAT = 64
N_RES = 16
RES_SCALE = 0.1
UP_CH = 16  # channels per HR pixel after the x4 shuffle of 256 channels
HR_IN = 10          # HRLS input: rgb, albedo, normal, depth
HR_IN_LAYERS = 16   # with the render layers: rgb, albedo, normal, diffuse, glossy, variance
VAR_MAX = 1.0e4     # the variance channel's clamp


def layer_specs(hr_in=HR_IN):
    """[(name, c_out, c_in, k)] in parameter order."""
    specs = [("hrls", FEAT, hr_in, 3), ("lrhs", FEAT, 3, 3),
             ("fuse", FEAT, FEAT + SCALE * SCALE * FEAT, 1)]
    for i in range(N_RES):
        specs += [(f"res{i}a", FEAT, FEAT, 3), (f"res{i}b", FEAT, FEAT, 3)]
    specs += [("up", UP_CH * SCALE * SCALE, FEAT, 3), ("rec", 3, UP_CH + FEAT, 3)]
    return specs


def num_params(hr_in=HR_IN):
    return sum(co * ci * k * k + co for _, co, ci, k in layer_specs(hr_in))


def hr_in_of(n_params, count=num_params):
    """The HRLS input width of a parameter vector of n_params values (count(hr_in)
    gives the size of each variant)."""
    for hr_in in (HR_IN, HR_IN_LAYERS):
        if count(hr_in) == n_params:
            return hr_in
    raise ValueError(f"{n_params} parameters fit no variant of the network")


def unpack(params):
    params = np.asarray(params, np.float64)
    out = {}
    off = 0
    for name, co, ci, k in layer_specs(hr_in_of(params.size)):
        nw = co * ci * k * k
        out[name] = (params[off:off + nw].reshape(co, ci, k, k), params[off + nw:off + nw + co])
        off += nw + co
    assert off == params.size, (off, params.size)
    return out


def pack(layers):
    hr_in = layers["hrls"][0].shape[1]
    return np.concatenate([np.concatenate([layers[n][0].ravel(), layers[n][1].ravel()])
                           for n, *_ in layer_specs(hr_in)])


# ----------------------------------------------------------------- primitives


def conv(x, w, b):
    """'same' zero-padded stride-1 convolution; x [B,H,W,Cin], w [Cout,Cin,k,k]."""
    B, H, W, _ = x.shape
    k = w.shape[2]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    out = np.zeros((B, H, W, w.shape[0]))
    for ky in range(k):
        for kx in range(k):
            # a contiguous copy of the tap's weights lets numpy hand the product to BLAS
            out += xp[:, ky:ky + H, kx:kx + W, :] @ np.ascontiguousarray(w[:, :, ky, kx].T)
    return out + b


def conv_backward(x, w, gy):
    """Gradients of conv(x, w, b) given dL/dy: returns (dx, dw, db)."""
    B, H, W, _ = x.shape
    k = w.shape[2]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(k):
        for kx in range(k):
            win = xp[:, ky:ky + H, kx:kx + W, :]
            dw[:, :, ky, kx] = np.einsum("bhwo,bhwi->oi", gy, win)
            dxp[:, ky:ky + H, kx:kx + W, :] += gy @ np.ascontiguousarray(w[:, :, ky, kx])
    return dxp[:, p:p + H, p:p + W, :], dw, gy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def unshuffle(x, r=SCALE):
    B, H, W, C = x.shape
    y = x.reshape(B, H // r, r, W // r, r, C)  # b, Y, i, X, j, c
    return y.transpose(0, 1, 3, 2, 4, 5).reshape(B, H // r, W // r, r * r * C)


def shuffle(x, r=SCALE):
    B, h, w, CC = x.shape
    C = CC // (r * r)
    y = x.reshape(B, h, w, r, r, C)  # b, Y, X, i, j, c
    return y.transpose(0, 1, 3, 2, 4, 5).reshape(B, h * r, w * r, C)


def preprocess(hrls_rgb, hrls_aux, lrhs_rgb):
    """Network inputs: HRLS [B,H,W,10], LRHS [B,H/4,W/4,3] (float64)."""
    hr = np.log1p(np.clip(np.asarray(hrls_rgb, np.float64), 0.0, 100.0))
    aux = np.asarray(hrls_aux, np.float64).copy()
    aux[..., 6] = np.log1p(np.maximum(aux[..., 6], 0.0))
    lr = np.log1p(np.clip(np.asarray(lrhs_rgb, np.float64), 0.0, 100.0))
    return np.concatenate([hr, aux], axis=-1), lr


def layer_variance(hrls_rgb, hrls_sumsq, spp):
    """Per-sample variance of each pixel's samples, averaged over the three colour
    channels: mean_c (sumsq_c / spp - mean_c^2), clamped to [0, VAR_MAX]."""
    m = np.asarray(hrls_rgb, np.float64)
    v = np.asarray(hrls_sumsq, np.float64) / spp - m * m
    return np.clip(v.mean(-1), 0.0, VAR_MAX)


def preprocess_layers(hrls_rgb, hrls_aux, hrls_layers, hrls_sumsq, spp, lrhs_rgb):
    """Network inputs with the render layers: HRLS [B,H,W,16] (rgb, albedo, normal,
    diffuse, glossy, variance), LRHS [B,H/4,W/4,3] (float64).  hrls_layers [...,9]:
    emission, diffuse, glossy; hrls_sumsq [...,3]: per-pixel sums of squared samples."""
    hr = np.log1p(np.clip(np.asarray(hrls_rgb, np.float64), 0.0, 100.0))
    aux = np.asarray(hrls_aux, np.float64)
    lay = np.log1p(np.clip(np.asarray(hrls_layers, np.float64)[..., 3:9], 0.0, 100.0))
    var = np.log1p(layer_variance(hrls_rgb, hrls_sumsq, spp))[..., None]
    lr = np.log1p(np.clip(np.asarray(lrhs_rgb, np.float64), 0.0, 100.0))
    return np.concatenate([hr, aux[..., 0:6], lay, var], axis=-1), lr


# ----------------------------------------------------------------- network


def forward(params, hrls_rgb, hrls_aux, lrhs_rgb, keep=False, layers=None):
    """I_SR [B,H,W,3] from HRLS rgb [B,H,W,3], aux [B,H,W,7], LRHS rgb [B,H/4,W/4,3];
    layers = (hrls_layers [B,H,W,9], hrls_sumsq [B,H,W,3], spp) for the variant
    whose HRLS input carries the render layers."""
    L = unpack(params)
    if layers is None:
        xh, xl = preprocess(hrls_rgb, hrls_aux, lrhs_rgb)
    else:
        xh, xl = preprocess_layers(hrls_rgb, hrls_aux, *layers, lrhs_rgb)
    if xh.shape[-1] != L["hrls"][0].shape[1]:
        raise ValueError("the parameters and the inputs belong to different variants")
    acts = {"xh": xh, "xl": xl}
    h0 = relu(conv(xh, *L["hrls"]))                   # F^0_HRLS
    fl = relu(conv(xl, *L["lrhs"]))                   # F_LRHS
    cat = np.concatenate([fl, unshuffle(h0)], -1)     # [F_LRHS, DSF^D(F^0_HRLS)]
    f0 = relu(conv(cat, *L["fuse"]))                  # F_0
    r = f0
    acts.update(h0=h0, fl=fl, cat=cat, f0=f0, r=[r], t=[])
    for i in range(N_RES):
        t = relu(conv(r, *L[f"res{i}a"]))
        r = r + RES_SCALE * conv(t, *L[f"res{i}b"])
        acts["t"].append(t)
        acts["r"].append(r)
    fdf = r + f0                                      # F_DF
    u_lr = relu(conv(fdf, *L["up"]))
    u = shuffle(u_lr)                                 # UP(F_DF)
    cat2 = np.concatenate([u, h0], -1)
    out = conv(cat2, *L["rec"])                       # H_Rec, no ReLU
    acts.update(fdf=fdf, u_lr=u_lr, u=u, cat2=cat2, out=out)
    return (out, acts) if keep else out


def clip_target(target):
    """Training targets are clipped to [0, 100] (Sec. 3.2: firefly outliers)."""
    return np.clip(np.asarray(target, np.float64), 0.0, 100.0)


def l1_loss(out, target):
    return np.abs(out - clip_target(target)).mean()


def backward(params, acts, gout):
    """dL/dparams (flat, float64) given dL/dI_SR, by hand through forward()."""
    L = unpack(params)
    g = {}
    dcat2, g["rec_w"], g["rec_b"] = conv_backward(acts["cat2"], L["rec"][0], gout)
    du = dcat2[..., :UP_CH]
    dh0 = dcat2[..., UP_CH:].copy()
    du_lr = unshuffle(du) * (acts["u_lr"] > 0)
    dfdf, g["up_w"], g["up_b"] = conv_backward(acts["fdf"], L["up"][0], du_lr)
    dr = dfdf.copy()
    df0 = dfdf.copy()
    for i in reversed(range(N_RES)):
        r_in, t = acts["r"][i], acts["t"][i]
        dy = RES_SCALE * dr
        dt, g[f"res{i}b_w"], g[f"res{i}b_b"] = conv_backward(t, L[f"res{i}b"][0], dy)
        dt = dt * (t > 0)
        dri, g[f"res{i}a_w"], g[f"res{i}a_b"] = conv_backward(r_in, L[f"res{i}a"][0], dt)
        dr = dr + dri
    df0 = df0 + dr
    df0 = df0 * (acts["f0"] > 0)
    dcat, g["fuse_w"], g["fuse_b"] = conv_backward(acts["cat"], L["fuse"][0], df0)
    dfl = dcat[..., :FEAT] * (acts["fl"] > 0)
    dh0 = (dh0 + shuffle(dcat[..., FEAT:])) * (acts["h0"] > 0)
    _, g["lrhs_w"], g["lrhs_b"] = conv_backward(acts["xl"], L["lrhs"][0], dfl)
    _, g["hrls_w"], g["hrls_b"] = conv_backward(acts["xh"], L["hrls"][0], dh0)
    return np.concatenate([np.concatenate([g[f"{n}_w"].ravel(), g[f"{n}_b"].ravel()])
                           for n, *_ in layer_specs(L["hrls"][0].shape[1])])


def l1_grad(out, target):
    """d mean|out - clip(target)| / d out with sign(0) = 0."""
    return np.sign(out - clip_target(target)) / out.size


def adam_step(params, grads, m, v, step, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, ICLR 2015, Algorithm 1); step counts from 1."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
