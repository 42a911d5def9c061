"""FP64 reference of the paper's own fusion network -- TEST INFRASTRUCTURE ONLY.

Plain numpy, float64, written from the network description of paper Sec. 4
(Fig. 4 and the equations for F_LRHS, F^0_HRLS, F_HRLS, F_g, F_DF and I_SR):

  F_LRHS   = ReLU(H_lrhs(I_LRHS))                 3x3, 3 -> 64         @LR
  F^0_HRLS = ReLU(H_hrls(I_HRLS))                 3x3, 10 -> 64        @HR
  F_HRLS   = DSF^D(F^0_HRLS)                      D stacked stride-2 deshuffles (alpha = 2;
                                                  scale 2^D: x2, x4 (the default), x8)
  F_0      = ReLU(fuse([F_LRHS, F_HRLS]))         1x1, 64 + 64 4^D -> 64 @LR
  RDB:  x_0 = input; x_c = ReLU(conv3x3([x_0 .. x_{c-1}])) for c = 1..3 (64 each);
        output = x_0 + conv3x3([x_0 .. x_3]) (256 -> 64)
  F_g      = RDB_5(...RDB_1(F_{g-1})...) + F_{g-1},   g = 1..3
  F_DF     = F_3 + F_0
  UP       = D times: ReLU(conv3x3 64 -> 256) then shuffle by 2 (sub-pixel conv)
  I_SR     = H_rec(UP(F_DF))                      3x3, 64 -> 3, no ReLU  @HR

Readings where the paper is silent (each one is listed with its reason in the
design notes of the repository):
  * an RDB's four 3x3 convs are dense: conv c sees the block input and every
    earlier conv's output; the fourth conv fuses the 256 channels back to 64
    and feeds the block's local residual, so it has no ReLU (as in the
    residual dense blocks the paper follows); growth rate 64;
  * the equation for F_DF adds F_0 (the text names F_LRHS);
  * UP mirrors the deshuffle: D stride-2 sub-pixel steps, each conv
    followed by ReLU (every conv but the last has one);
  * the stride-2 deshuffle uses the channel convention of oracle/cnn.py
    (HR pixel (2Y+i, 2X+j), channel c -> channel (2i+j) C + c), applied D times;
  * inputs, preprocessing and parameter layout are those of oracle/cnn.py.

The robust loss is the paper's l_r with robust factor beta (Sec. 4, loss
function), as a mean over all output elements against targets clipped to
[0, 100]; SGD is the plain update w <- w - lr g.

Only tests/, the smoke check and the bench's CPU-baseline leg use this module.
"""
from __future__ import annotations

import numpy as np

from .cnn import (FEAT, HR_IN, clip_target, conv, conv_backward, hr_in_of, preprocess,
                  preprocess_layers, relu, shuffle, unshuffle)

N_GROUPS = 3      # G
N_BLOCKS = 5      # B, RDBs per group
N_CONVS = 4       # convs per RDB
GROWTH = 64
ALPHA = 2         # deshuffle / shuffle stride
SCALES = (2, 4, 8)


def n_dsf(scale):
    """D, the stacked stride-2 deshuffles (and upscaling steps) of a scale."""
    if scale not in SCALES:
        raise ValueError(f"scale {scale} not in {SCALES}")
    return {2: 1, 4: 2, 8: 3}[scale]


def rdb_name(g, b, c):
    return f"g{g}b{b}c{c}"


def layer_specs(scale=4, hr_in=HR_IN):
    """[(name, c_out, c_in, k)] in parameter order; hr_in 16 for the variant whose
    HRLS input carries the render layers (oracle/cnn.py, preprocess_layers)."""
    specs = [("hrls", FEAT, hr_in, 3), ("lrhs", FEAT, 3, 3),
             ("fuse", FEAT, FEAT + scale * scale * FEAT, 1)]
    for g in range(N_GROUPS):
        for b in range(N_BLOCKS):
            for c in range(N_CONVS):
                cout = GROWTH if c < N_CONVS - 1 else FEAT
                specs.append((rdb_name(g, b, c), cout, FEAT + c * GROWTH, 3))
    for i in range(n_dsf(scale)):
        specs.append((f"up{i}", ALPHA * ALPHA * FEAT, FEAT, 3))
    specs.append(("rec", 3, FEAT, 3))
    return specs


def num_params(scale=4, hr_in=HR_IN):
    return sum(co * ci * k * k + co for _, co, ci, k in layer_specs(scale, hr_in))


def unpack(params, scale=4):
    params = np.asarray(params, np.float64)
    out = {}
    off = 0
    hr_in = hr_in_of(params.size, lambda h: num_params(scale, h))
    for name, co, ci, k in layer_specs(scale, hr_in):
        nw = co * ci * k * k
        out[name] = (params[off:off + nw].reshape(co, ci, k, k), params[off + nw:off + nw + co])
        off += nw + co
    assert off == params.size, (off, params.size)
    return out


def deshuffle_stack(x, scale=4):
    """F_HRLS = DSF^D(...DSF^1(x)...): D stride-ALPHA deshuffles."""
    for _ in range(n_dsf(scale)):
        x = unshuffle(x, ALPHA)
    return x


def rdb(x0, L, g, b):
    """One residual dense block; returns (output, [x_0, x_1, x_2, x_3])."""
    xs = [x0]
    for c in range(N_CONVS - 1):
        xs.append(relu(conv(np.concatenate(xs, -1), *L[rdb_name(g, b, c)])))
    return x0 + conv(np.concatenate(xs, -1), *L[rdb_name(g, b, N_CONVS - 1)]), xs


def forward(params, hrls_rgb, hrls_aux, lrhs_rgb, keep=False, scale=4, layers=None):
    """I_SR [B,H,W,3] from HRLS rgb [B,H,W,3], aux [B,H,W,7], LRHS rgb [B,H/s,W/s,3];
    layers = (hrls_layers, hrls_sumsq, spp) for the variant with the render layers."""
    L = unpack(params, scale)
    if layers is None:
        xh, xl = preprocess(hrls_rgb, hrls_aux, lrhs_rgb)
    else:
        xh, xl = preprocess_layers(hrls_rgb, hrls_aux, *layers, lrhs_rgb)
    if xh.shape[-1] != L["hrls"][0].shape[1]:
        raise ValueError("the parameters and the inputs belong to different variants")
    h0 = relu(conv(xh, *L["hrls"]))                   # F^0_HRLS
    fl = relu(conv(xl, *L["lrhs"]))                   # F_LRHS
    cat = np.concatenate([fl, deshuffle_stack(h0, scale)], -1)
    f0 = relu(conv(cat, *L["fuse"]))                  # F_0
    acts = {"xh": xh, "xl": xl, "h0": h0, "fl": fl, "cat": cat, "f0": f0, "dense": {}}
    F = f0
    for g in range(N_GROUPS):
        s = F
        for b in range(N_BLOCKS):
            s, xs = rdb(s, L, g, b)
            acts["dense"][g, b] = xs
        F = s + F                                     # F_g
    fdf = F + f0                                      # F_DF
    acts["fdf"] = fdf
    u = fdf
    acts["up_in"], acts["up_act"] = [], []
    for i in range(n_dsf(scale)):
        a = relu(conv(u, *L[f"up{i}"]))
        acts["up_in"].append(u)
        acts["up_act"].append(a)
        u = shuffle(a, ALPHA)
    acts["u"] = u
    out = conv(u, *L["rec"])                          # H_Rec, no ReLU
    acts["out"] = out
    return (out, acts) if keep else out


def backward(params, acts, gout, scale=4):
    """dL/dparams (flat, float64) given dL/dI_SR, by hand through forward()."""
    L = unpack(params, scale)
    g = {}
    du, g["rec_w"], g["rec_b"] = conv_backward(acts["u"], L["rec"][0], gout)
    for i in reversed(range(n_dsf(scale))):
        da = unshuffle(du, ALPHA) * (acts["up_act"][i] > 0)
        du, g[f"up{i}_w"], g[f"up{i}_b"] = conv_backward(acts["up_in"][i], L[f"up{i}"][0], da)
    dfdf = du
    dF = dfdf.copy()                                  # dL/dF_G
    for gi in reversed(range(N_GROUPS)):
        ds = dF.copy()                                # gradient of the chain's end
        for b in reversed(range(N_BLOCKS)):
            xs = acts["dense"][gi, b]
            last = rdb_name(gi, b, N_CONVS - 1)
            dcat, g[last + "_w"], g[last + "_b"] = conv_backward(
                np.concatenate(xs, -1), L[last][0], ds)
            dx = [dcat[..., FEAT + (k - 1) * GROWTH:FEAT + k * GROWTH] if k else dcat[..., :FEAT]
                  for k in range(N_CONVS)]
            dx[0] = dx[0] + ds                        # local residual
            for c in reversed(range(N_CONVS - 1)):   # conv c produced x_{c+1}
                name = rdb_name(gi, b, c)
                dy = dx[c + 1] * (xs[c + 1] > 0)
                dcat, g[name + "_w"], g[name + "_b"] = conv_backward(
                    np.concatenate(xs[:c + 1], -1), L[name][0], dy)
                dx[0] = dx[0] + dcat[..., :FEAT]
                for k in range(1, c + 1):
                    dx[k] = dx[k] + dcat[..., FEAT + (k - 1) * GROWTH:FEAT + k * GROWTH]
            ds = dx[0]
        dF = ds + dF                                  # through the chain + the group skip
    df0 = (dF + dfdf) * (acts["f0"] > 0)              # + the global skip of F_DF
    dcat, g["fuse_w"], g["fuse_b"] = conv_backward(acts["cat"], L["fuse"][0], df0)
    dfl = dcat[..., :FEAT] * (acts["fl"] > 0)
    dfh = dcat[..., FEAT:]
    for _ in range(n_dsf(scale)):                     # adjoint of the stacked deshuffle
        dfh = shuffle(dfh, ALPHA)
    dh0 = dfh * (acts["h0"] > 0)
    _, g["lrhs_w"], g["lrhs_b"] = conv_backward(acts["xl"], L["lrhs"][0], dfl)
    _, g["hrls_w"], g["hrls_b"] = conv_backward(acts["xh"], L["hrls"][0], dh0)
    return np.concatenate([np.concatenate([g[f"{n}_w"].ravel(), g[f"{n}_b"].ravel()])
                           for n, *_ in layer_specs(scale, L["hrls"][0].shape[1])])


def robust_loss(out, target, beta=0.1):
    """l_r = mean over elements of |d| / (beta + |d|), d = target - out (Sec. 4)."""
    d = np.abs(np.asarray(out, np.float64) - clip_target(target))
    return (d / (beta + d)).mean()


def robust_grad(out, target, beta=0.1):
    """d l_r / d out = sign(out - target) beta / (beta + |d|)^2 / N, sign(0) = 0."""
    e = np.asarray(out, np.float64) - clip_target(target)
    return np.sign(e) * beta / (beta + np.abs(e)) ** 2 / e.size


def sgd_step(params, grads, lr=1e-4):
    """Plain SGD (the paper's optimiser, Sec. 4 implementation details)."""
    return params - lr * grads
