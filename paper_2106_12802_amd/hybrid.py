"""The hybrid multi-resolution frame and the learned part around it.

* hybrid_frame / HybridFrame: HRLS (W x H, 4 spp, features) + LRHS (W/4 x H/4,
  64 spp) + fusion network -> I_SR (paper Sec. 4), each step a libmrs call
  (HybridFrame renders both as one batch).
* build_dataset / train: training pairs rendered by the tracer itself
  (HRLS/LRHS windows against 1024-spp FP64-accumulated targets) and Adam on the
  L1 loss (libmrs mrs_train_step).
* equal_psnr: the plain-render spp whose PSNR (against an independent-seed
  reference) equals the hybrid frame's, and the time that render takes.

Seeds: HRLS 2s, LRHS 2s+1 for frame seed s; references and targets use seeds
at or above 2^40 so that no path is shared with the inputs.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import tracer as T
from .metrics import image_metrics
from .net import FusionNet

SCALE = 4
DEPTH = 8
REF_SEED = 1 << 40


def _empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.float32, device="cuda")


def render_inputs(gs, W, H, seed, spp_h=4, spp_l=64, depth=DEPTH, window=None):
    """HRLS rgb + features and LRHS rgb of one frame (or of a window whose origin and
    size are multiples of 4; the LRHS window is the corresponding quarter-size one)."""
    if window is None:
        x0, y0, w, h = 0, 0, W, H
    else:
        x0, y0, w, h = window
    hr_rgb, hr_aux = _empty((h, w, 3)), _empty((h, w, 7))
    lr_rgb = _empty((h // SCALE, w // SCALE, 3))
    T.render_ex(gs, W, H, spp_h, depth, 2 * seed, hr_rgb, hr_aux,
                window=None if window is None else (x0, y0, w, h))
    T.render_ex(gs, W // SCALE, H // SCALE, spp_l, depth, 2 * seed + 1, lr_rgb, None,
                window=None if window is None else
                (x0 // SCALE, y0 // SCALE, w // SCALE, h // SCALE))
    return hr_rgb, hr_aux, lr_rgb


def fallback_spp(spp_h=4, spp_l=64):
    """spp of the plain render that traces as many paths as the hybrid frame."""
    return max(1, spp_h + spp_l // (SCALE * SCALE))


def pipeline_frames(batches, seeds_of, fuses, seeds, on_frame=None):
    """Renders and fuses the frames of `seeds` on the current stream with
    n = len(batches) frames in flight: frame k renders with batches[k % n] (a
    batch owns its path workspace and outputs) and fuses with fuses[k % n]().

    n = 1: per frame k, render_end (frame k's per-pixel sums and outputs), the
    seeds and render_fork of frame k+1 (the point its sub-chunk streams start
    from), fuse() on frame k's outputs, then render_begin of frame k+1: the
    fusion's launches queue ahead of the next wavefront's and run beside it.

    n = 2: frame k+1 is begun (on the other batch) before frame k is ended.  Its
    sub-chunks queue on the library's sub-chunk streams behind frame k's and start
    as each of frame k's sub-chunks finishes, so frame k's last path tails share
    the GPU with frame k+1's first bounces instead of running alone; frame k's
    sums, outputs and fusion follow on the stream.  A batch is begun again only
    after its previous frame was ended and fused (stream order), so frame k+2's
    outputs are written after frame k's fusion has read them.  (Forking frame k+2
    right after frame k's sums, ahead of frame k's fusion, measured slower: with
    two frames queued on the sub-chunk streams the stream's sums and fusions fall
    behind.)

    Every frame is bitwise what render + fuse of its seeds gives.  on_frame(k)
    runs right after frame k's fusion is enqueued (work it enqueues on the stream
    sees that frame)."""
    seeds = list(seeds)
    n = len(batches)
    if not seeds:
        return
    if n not in (1, 2):
        raise ValueError("pipeline_frames: 1 or 2 frames in flight")
    batches[0].set_seeds(seeds_of(seeds[0]))
    batches[0].render_begin()
    for k in range(len(seeds)):
        cur = batches[k % n]
        more = k + 1 < len(seeds)
        if n == 1:
            cur.render_end()
            if more:
                cur.set_seeds(seeds_of(seeds[k + 1]))
                cur.render_fork()
            fuses[0]()
            if on_frame is not None:
                on_frame(k)
            if more:
                cur.render_begin()
        else:
            if more:
                nxt = batches[(k + 1) % n]
                nxt.set_seeds(seeds_of(seeds[k + 1]))
                nxt.render_begin()
            cur.render_end()
            fuses[k % n]()
            if on_frame is not None:
                on_frame(k)


class _Slot:
    """One frame in flight: its two-job batch and the images it writes."""

    def __init__(self, gs, W, H, spp_h, spp_l, depth, layers):
        self.hr_rgb, self.hr_aux = _empty((H, W, 3)), _empty((H, W, 7))
        self.lr_rgb = _empty((H // SCALE, W // SCALE, 3))
        self.hr_layers = self.hr_sumsq = None
        extra = {}
        if layers:
            self.hr_layers, self.hr_sumsq = _empty((H, W, 9)), _empty((H, W, 3))
            extra = dict(out_layers=self.hr_layers, out_sumsq=self.hr_sumsq)
        self.batch = T.Batch([
            dict(scene=gs, W=W, H=H, spp=spp_h, max_depth=depth, seed=0, out_rgb=self.hr_rgb,
                 out_aux=self.hr_aux, **extra),
            dict(scene=gs, W=W // SCALE, H=H // SCALE, spp=spp_l, max_depth=depth, seed=1,
                 out_rgb=self.lr_rgb, want_aux=False)])


class HybridFrame:
    """HRLS + LRHS rendered as one two-job batch (one wavefront launch sequence over
    both renders), then fused.  Buffers and the batch are made once; render(seed)
    takes seeds 2 seed and 2 seed + 1 as hybrid_frame does.  Without a ready network
    (None, or no parameters) the frame falls back to a plain render with the same
    number of paths (fallback_spp), seed 2 seed.  layers=True also keeps the HRLS
    render layers of Sec. 3.1 (hr_layers [H, W, 9]: emission, diffuse, glossy) and
    its per-pixel sums of squares (hr_sumsq, the variance layer).  hr_rgb, hr_aux,
    lr_rgb, hr_layers and hr_sumsq are the images of the last render()."""

    def __init__(self, gs, net: FusionNet | None, W, H, spp_h=4, spp_l=64, depth=DEPTH,
                 layers=False):
        self.net = net
        self.out = _empty((H, W, 3))
        self.fallback = net is None or not net.ready
        self.spp_h = spp_h
        self._args = (gs, W, H, spp_h, spp_l, depth)
        if not self.fallback and net.has_layers:
            layers = True  # the network reads them
        self.layers = layers
        if self.fallback:
            self.batch = T.Batch([dict(scene=gs, W=W, H=H, spp=fallback_spp(spp_h, spp_l),
                                       max_depth=depth, seed=0, out_rgb=self.out,
                                       want_aux=False)])
            return
        self.slots = [_Slot(*self._args, layers)]
        self._use(self.slots[0])

    def _use(self, sl):
        self.batch = sl.batch
        self.hr_rgb, self.hr_aux, self.lr_rgb = sl.hr_rgb, sl.hr_aux, sl.lr_rgb
        if self.layers:
            self.hr_layers, self.hr_sumsq = sl.hr_layers, sl.hr_sumsq

    def render(self, seed):
        if self.fallback:
            self.batch.set_seeds([2 * seed])
            self.batch.render()
            return self.out
        sl = self.slots[0]
        self._use(sl)
        sl.batch.set_seeds([2 * seed, 2 * seed + 1])
        sl.batch.render()
        return self._fuse(sl)

    def _fuse(self, sl):
        lay = (sl.hr_layers, sl.hr_sumsq, self.spp_h) if self.net.has_layers else None
        return self.net.fuse(sl.hr_rgb, sl.hr_aux, sl.lr_rgb, out=self.out, layers=lay)

    def _seeds(self, seed):
        return [2 * seed] if self.fallback else [2 * seed, 2 * seed + 1]

    def render_stream(self, seeds, on_frame=None, in_flight=2):
        """The frames of `seeds` in order, pipelined on the current stream
        (pipeline_frames): with in_flight=2 (a second batch, made on first use)
        frame k+1 renders while frame k's last paths finish and while frame k is
        fused; with 1, frame k's fusion runs while frame k+1 renders.  Each frame
        equals render(seed) bitwise.  on_frame(k, out) is called once frame k's
        output is enqueued (work it enqueues on the stream sees that frame)."""
        seeds = list(seeds)
        if self.fallback:  # no fusion: plain renders one after the other
            for k, sd in enumerate(seeds):
                self.render(sd)
                if on_frame is not None:
                    on_frame(k, self.out)
            return self.out
        while len(self.slots) < in_flight:
            self.slots.append(_Slot(*self._args, self.layers))
        slots = self.slots[:in_flight]
        pipeline_frames([sl.batch for sl in slots], self._seeds,
                        [lambda sl=sl: self._fuse(sl) for sl in slots], seeds,
                        on_frame=None if on_frame is None else
                        (lambda k: on_frame(k, self.out)))
        if seeds:
            self._use(slots[(len(seeds) - 1) % len(slots)])
        return self.out

    def close(self):
        if self.fallback:
            self.batch.close()
            return
        for sl in self.slots:
            sl.batch.close()


def hybrid_frame(gs, net: FusionNet | None, W, H, seed, spp_h=4, spp_l=64, depth=DEPTH,
                 out=None):
    """One hybrid frame by separate calls; a plain render (fallback_spp, seed 2 seed)
    when the network is missing or has no parameters."""
    if net is None or not net.ready:
        out = _empty((H, W, 3)) if out is None else out
        T.render_ex(gs, W, H, fallback_spp(spp_h, spp_l), depth, 2 * seed, out, None)
        return out, None
    if net.has_layers:  # the HRLS render also keeps its layers and sums of squares
        frame = HybridFrame(gs, net, W, H, spp_h, spp_l, depth)
        if out is not None:
            frame.out = out
        img = frame.render(seed)
        res = (frame.hr_rgb, frame.hr_aux, frame.lr_rgb)
        frame.close()
        return img, res
    hr_rgb, hr_aux, lr_rgb = render_inputs(gs, W, H, seed, spp_h, spp_l, depth)
    out = net.fuse(hr_rgb, hr_aux, lr_rgb, out=out)
    return out, (hr_rgb, hr_aux, lr_rgb)


def reference(gs, W, H, spp=1024, seed=REF_SEED, depth=DEPTH, window=None):
    """High-spp reference render (FP64 per-pixel sums from 1024 spp)."""
    if window is None:
        out = _empty((H, W, 3))
    else:
        out = _empty((window[3], window[2], 3))
    T.render_ex(gs, W, H, spp, depth, seed, out, None, window=window)
    return out


# ---------------------------------------------------------------- training data


class PairSet:
    """Training pairs resident on the GPU: HRLS rgb/features, LRHS rgb, target, and
    (for the networks with layer inputs) the HRLS render layers and sums of squares."""

    def __init__(self, hr_rgb, hr_aux, lr_rgb, target, hr_layers=None, hr_sumsq=None, spp_h=4):
        self.hr_rgb, self.hr_aux, self.lr_rgb, self.target = hr_rgb, hr_aux, lr_rgb, target
        self.hr_layers, self.hr_sumsq, self.spp_h = hr_layers, hr_sumsq, spp_h

    def __len__(self):
        return self.hr_rgb.shape[0]

    def batch(self, idx):
        import torch
        i = torch.as_tensor(idx, device="cuda", dtype=torch.long)
        return [t.index_select(0, i).contiguous() for t in
                (self.hr_rgb, self.hr_aux, self.lr_rgb, self.target)]

    def layers(self, idx):
        """(hr_layers, hr_sumsq, spp) of a batch, for mrs_net_bind_layers."""
        import torch
        if self.hr_layers is None:
            raise ValueError("this pair set was built without render layers")
        i = torch.as_tensor(idx, device="cuda", dtype=torch.long)
        return (self.hr_layers.index_select(0, i).contiguous(),
                self.hr_sumsq.index_select(0, i).contiguous(), self.spp_h)


def build_dataset(first_seed=100, n_scenes=64, windows=16, size=128, W=1280, H=720,
                  spp=(4, 64, 1024), tri_range=(10_000, 200_000), depth=DEPTH, log=print,
                  layers=False):
    """Render `n_scenes` x `windows` training pairs of size x size HR pixels
    (layers: also the HRLS render layers and per-pixel sums of squares)."""
    import torch
    from mrs_inputs import scenes as S
    N = n_scenes * windows
    hr_rgb = _empty((N, size, size, 3))
    hr_aux = _empty((N, size, size, 7))
    lr_rgb = _empty((N, size // SCALE, size // SCALE, 3))
    target = _empty((N, size, size, 3))
    hr_lay = _empty((N, size, size, 9)) if layers else None
    hr_sq = torch.zeros((N, size, size, 3), dtype=torch.float32, device="cuda") if layers else None
    t0 = time.perf_counter()
    k = 0
    for si, (seed, tris) in enumerate(S.training_scene_specs(first_seed, n_scenes, *tri_range)):
        scene = S.procedural_sized(seed, tris)
        gs = T.GpuScene(scene)
        for (x0, y0) in S.training_windows(seed, windows, W, H, size):
            fseed = seed * 1000 + k % windows
            win = (x0, y0, size, size)
            extra = dict(out_layers=hr_lay[k], out_sumsq=hr_sq[k]) if layers else {}
            T.render_ex(gs, W, H, spp[0], depth, 2 * fseed, hr_rgb[k], hr_aux[k], window=win,
                        **extra)
            T.render_ex(gs, W // SCALE, H // SCALE, spp[1], depth, 2 * fseed + 1, lr_rgb[k], None,
                        window=(x0 // SCALE, y0 // SCALE, size // SCALE, size // SCALE))
            T.render_ex(gs, W, H, spp[2], depth, REF_SEED + fseed, target[k], None, window=win)
            k += 1
        torch.cuda.synchronize()
        gs.close()
        if log and (si % 8 == 7 or si == n_scenes - 1):
            log(f"[data] {si + 1}/{n_scenes} scenes, {k} pairs, {time.perf_counter() - t0:.1f} s")
    return PairSet(hr_rgb, hr_aux, lr_rgb, target, hr_lay, hr_sq, spp[0])


def train(net: FusionNet, data: PairSet, steps: int, batch=16, lr=1e-4, seed=0,
          log_every=200, log=print, time_limit=None, start_step=0, loss="l1",
          optimizer="adam", beta=0.1):
    """Optimiser steps (Adam on L1 by default; the paper's setting is
    loss="robust", optimizer="sgd") over random batches; the batch order is a pure
    function of (seed, step), so a run resumed from a checkpoint at step s
    continues identically."""
    losses = []
    t0 = time.perf_counter()
    done = start_step
    for step in range(start_step, steps):
        idx = np.random.default_rng([seed, step]).choice(len(data), batch, replace=False)
        want = (step + 1) % log_every == 0 or step == steps - 1
        value = net.train_step(*data.batch(idx), lr=lr, want_loss=want, loss=loss,
                               optimizer=optimizer, beta=beta,
                               layers=data.layers(idx) if net.has_layers else None)
        done = step + 1
        if want:
            losses.append((done, value))
            if log:
                log(f"[train] step {done} loss {value:.5f} ({time.perf_counter() - t0:.1f} s)")
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
    return losses, done


# ------------------------------------------------- random spp pairs (Sec. 4)

# The spp sets the paper draws from at every training iteration (Sec. 4,
# implementation details); the HRLS spp is kept below the LRHS spp.
SPP_HRLS = (1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 32)
SPP_LRHS = (2, 3, 4, 5, 6, 7, 8, 12, 16, 32, 64, 128, 250, 1000, 4000)


def sample_spp_pair(rng):
    """(spp_hrls, spp_lrhs): HRLS uniform over SPP_HRLS, then LRHS uniform over the
    values of SPP_LRHS above it."""
    h = int(rng.choice(SPP_HRLS))
    lo = [v for v in SPP_LRHS if v > h]
    return h, int(rng.choice(lo))


class OnlinePairs:
    """Training windows whose inputs are re-rendered at every iteration, at that
    iteration's spp pair and with fresh seeds; the 1024-spp targets (FP64 sums,
    seeds >= 2^40) are rendered once.  Window origins and sizes are multiples of
    the network's scale."""

    def __init__(self, specs, windows=16, size=128, W=1280, H=720, scale=SCALE,
                 target_spp=1024, depth=DEPTH, log=print):
        import torch
        from mrs_inputs import scenes as S
        self.scale, self.size, self.W, self.H, self.depth = scale, size, W, H, depth
        self.scenes = []
        self.wins = []
        for seed, tris in specs:
            gs = T.GpuScene(S.procedural_sized(seed, tris))
            self.scenes.append(gs)
            for (x0, y0) in S.training_windows(seed, windows, W, H, size):
                x0 -= x0 % scale
                y0 -= y0 % scale
                self.wins.append((len(self.scenes) - 1, x0, y0, seed))
        self.target = _empty((len(self.wins), size, size, 3))
        for k, (si, x0, y0, seed) in enumerate(self.wins):
            T.render_ex(self.scenes[si], W, H, target_spp, depth, REF_SEED + seed * 1000 + k,
                        self.target[k], None, window=(x0, y0, size, size))
        torch.cuda.synchronize()
        if log:
            log(f"[data] {len(self.wins)} windows of {len(self.scenes)} scenes, targets rendered")

    def __len__(self):
        return len(self.wins)

    def batch(self, idx, spp_h, spp_l, seed):
        """HRLS rgb/features, LRHS rgb and targets of windows idx, inputs rendered
        now at (spp_h, spp_l) with frame seeds derived from `seed`."""
        import torch
        n, z, s = len(idx), self.size, self.scale
        hr_rgb, hr_aux = _empty((n, z, z, 3)), _empty((n, z, z, 7))
        lr_rgb = _empty((n, z // s, z // s, 3))
        for b, k in enumerate(idx):
            si, x0, y0, _ = self.wins[k]
            fseed = (seed << 20) + int(k)
            gs = self.scenes[si]
            T.render_ex(gs, self.W, self.H, spp_h, self.depth, 2 * fseed, hr_rgb[b], hr_aux[b],
                        window=(x0, y0, z, z))
            T.render_ex(gs, self.W // s, self.H // s, spp_l, self.depth, 2 * fseed + 1, lr_rgb[b],
                        None, window=(x0 // s, y0 // s, z // s, z // s))
        i = torch.as_tensor(list(idx), device="cuda", dtype=torch.long)
        return hr_rgb, hr_aux, lr_rgb, self.target.index_select(0, i).contiguous()

    def close(self):
        for gs in self.scenes:
            gs.close()
        self.scenes = []


def train_random_spp(net: FusionNet, data: OnlinePairs, steps: int, batch=16, lr=1e-4,
                     seed=0, loss="robust", optimizer="sgd", log_every=100, log=print,
                     time_limit=None):
    """The paper's training loop: every iteration draws an spp pair
    (sample_spp_pair) and a batch of windows, renders the inputs at that pair and
    takes one optimiser step.  Returns [(step, spp_h, spp_l, loss or None)]."""
    out = []
    t0 = time.perf_counter()
    for step in range(steps):
        rng = np.random.default_rng([seed, step])
        h, l = sample_spp_pair(rng)
        idx = rng.choice(len(data), batch, replace=False)
        want = (step + 1) % log_every == 0 or step == steps - 1
        value = net.train_step(*data.batch(idx, h, l, seed * 1000003 + step), lr=lr,
                               want_loss=want, loss=loss, optimizer=optimizer)
        out.append((step + 1, h, l, value))
        if want and log:
            log(f"[train] step {step + 1} spp {h}/{l} loss {value:.5f} "
                f"({time.perf_counter() - t0:.1f} s)")
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
    return out


def loss_ablation(data: PairSet, settings, eval_scenes, seconds, W=1280, H=720, batch=16,
                  lr=1e-4, seed=1, arch="res16", log=print, optimizer="adam", weights_out=None):
    """One network per loss setting, each trained from the same init on the same
    pairs for the same time, then the hybrid frame's PSNR on each evaluation
    scene: {setting: {"steps": n, scene name: dB}}.  settings: ("l1", None) or
    ("robust", beta).  weights_out {setting key: path} saves the trained weights."""
    refs = {name: reference(gs, W, H, 1024, REF_SEED + k)
            for k, (name, gs) in enumerate(eval_scenes)}
    out = {}
    for loss, beta in settings:
        net = FusionNet(seed=seed, arch=arch)
        losses, done = train(net, data, 10 ** 9, batch, lr, seed=seed, log_every=2000, log=log,
                             time_limit=seconds, loss=loss, beta=0.1 if beta is None else beta,
                             optimizer=optimizer)
        key = loss if beta is None else f"{loss}_beta{beta:g}"
        out[key] = {"steps": done, "optimizer": optimizer, "lr": lr,
                    "last_losses": [round(v, 6) for _, v in losses[-3:]]}
        for k, (name, gs) in enumerate(eval_scenes):
            img, _ = hybrid_frame(gs, net, W, H, k)
            out[key][name] = image_metrics(img, refs[name])["psnr"]
        if weights_out and key in weights_out:
            net.save_weights(weights_out[key])
        if log:
            log(f"[ablation] {key}: {out[key]}")
        net.close()
    return out


def layers_ablation(data: PairSet, eval_scenes, seconds, W=1280, H=720, batch=16, lr=1e-4,
                    seed=1, archs=("res16", "res16_layers"), log=print, weights_out=None):
    """The input-layer ablation (Sec. 5, Fig. 9 on synthetic scenes): the network
    with and without the HRLS render layers as inputs, each trained from the same
    seed on the same pairs (built with layers=True) with L1 and Adam for the same
    time, then the hybrid frame's PSNR on each evaluation scene:
    {arch: {"steps": n, scene name: dB}}.  weights_out {arch: path} saves them."""
    refs = {name: reference(gs, W, H, 1024, REF_SEED + k)
            for k, (name, gs) in enumerate(eval_scenes)}
    out = {}
    for arch in archs:
        net = FusionNet(seed=seed, arch=arch)
        _, done = train(net, data, 10 ** 9, batch, lr, seed=seed, log_every=4000, log=log,
                        time_limit=seconds)
        out[arch] = {"steps": done}
        for k, (name, gs) in enumerate(eval_scenes):
            img, _ = hybrid_frame(gs, net, W, H, k)
            out[arch][name] = image_metrics(img, refs[name])["psnr"]
        if weights_out and arch in weights_out:
            net.save_weights(weights_out[arch])
        if log:
            log(f"[layers ablation] {arch}: {out[arch]}")
        net.close()
    return out


def spp_grid(gs, net, W, H, spp_h=(1, 2, 4, 8), spp_l=(16, 64, 256), seed=0, ref=None):
    """PSNR of the hybrid frame at each (HRLS spp, LRHS spp) pair with HRLS < LRHS
    (the paper's spp-pair table, Table 6): {(h, l): dB} against a 1024-spp
    reference with an independent seed."""
    if ref is None:
        ref = reference(gs, W, H, 1024, REF_SEED + seed)
    table = {}
    for h in spp_h:
        for l in spp_l:
            if l > h:
                out, _ = hybrid_frame(gs, net, W, H, seed, spp_h=h, spp_l=l)
                table[(h, l)] = image_metrics(out, ref)["psnr"]
    return table


def grid_monotone(table, tol=0.1):
    """True when PSNR does not fall (by more than tol dB) as either spp grows."""
    for (h, l), p in table.items():
        for (h2, l2), p2 in table.items():
            if ((h2 == h and l2 > l) or (l2 == l and h2 > h)) and p2 < p - tol:
                return False
    return True


# ---------------------------------------------------------------- equal PSNR


def equal_psnr(psnr_target, plain):
    """plain: [(spp, psnr, ms)] increasing in spp.  Returns (spp*, ms*) where the PSNR
    interpolated linearly in log2(spp) reaches psnr_target (ms interpolated linearly in
    spp), or None if the target lies outside the measured range."""
    for (n0, p0, t0), (n1, p1, t1) in zip(plain, plain[1:]):
        if (p0 - psnr_target) * (p1 - psnr_target) <= 0 and p1 != p0:
            a = (psnr_target - p0) / (p1 - p0)
            n = 2 ** (math.log2(n0) + a * (math.log2(n1) - math.log2(n0)))
            t = t0 + (n - n0) / (n1 - n0) * (t1 - t0)
            return n, t
    return None


def time_ms(fn, reps=3):
    import torch
    torch.cuda.synchronize()
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / reps


def evaluate_scene(gs, net, W=1280, H=720, seed=0, plain_spp=(4, 8, 16, 32, 64, 128, 256),
                   ref_spp=1024, reps=3, extra_nets=None):
    """PSNR/time of the hybrid frame, its baselines and plain renders for one scene;
    extra_nets {name: net}: the same frame with other networks, against the same
    reference and plain renders (res["extra"][name])."""
    import torch
    ref = reference(gs, W, H, ref_spp, REF_SEED + seed)
    res = {}
    frame = HybridFrame(gs, net, W, H)
    t_h = time_ms(lambda: frame.render(seed), reps)
    out = frame.render(seed)
    res["hybrid"] = {"psnr": image_metrics(out, ref)["psnr"], "ms": t_h}
    hr_rgb, hr_aux, lr_rgb = frame.hr_rgb, frame.hr_aux, frame.lr_rgb
    up = torch.nn.functional.interpolate(lr_rgb.permute(2, 0, 1)[None], scale_factor=SCALE,
                                         mode="bilinear", align_corners=False)[0].permute(1, 2, 0)
    res["hrls_4spp"] = {"psnr": image_metrics(hr_rgb, ref)["psnr"]}
    res["lrhs_bilinear"] = {"psnr": image_metrics(up.contiguous(), ref)["psnr"]}
    plain = []
    img = _empty((H, W, 3))
    for n in plain_spp:
        ms = time_ms(lambda: T.render_ex(gs, W, H, n, DEPTH, 2 * seed + 7919, img, None), reps)
        T.render_ex(gs, W, H, n, DEPTH, 2 * seed + 7919, img, None)
        plain.append((n, image_metrics(img, ref)["psnr"], ms))
    res["plain"] = plain
    eq = equal_psnr(res["hybrid"]["psnr"], plain)
    res["equal_psnr"] = None if eq is None else {"spp": eq[0], "ms": eq[1],
                                                 "ratio": t_h / eq[1]}
    frame.close()
    res["extra"] = {}
    for name, other in (extra_nets or {}).items():
        fr = HybridFrame(gs, other, W, H)
        t_o = time_ms(lambda: fr.render(seed), reps)
        p_o = image_metrics(fr.render(seed), ref)["psnr"]
        eq_o = equal_psnr(p_o, plain)
        res["extra"][name] = {"psnr": p_o, "ms": t_o, "equal_psnr": None if eq_o is None else
                              {"spp": eq_o[0], "ms": eq_o[1], "ratio": t_o / eq_o[1]}}
        fr.close()
    return res


def main(argv=None):
    """Render the training set, train the network, save a checkpoint, evaluate."""
    import argparse
    import json
    import sys

    import torch
    from mrs_inputs import scenes as S

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--scenes", type=int, default=64)
    ap.add_argument("--windows", type=int, default=16)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--time-limit", type=float, default=None, help="seconds of training at most")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default="fusion_checkpoint.bin", help="resumable checkpoint")
    ap.add_argument("--weights-out", default=None, help="weights-only file for inference")
    ap.add_argument("--arch", default="res16",
                    choices=("res16", "rdg", "res16_layers", "rdg_layers"),
                    help="network: the configured 16-block trunk or the paper's (x4); "
                         "*_layers: with the HRLS render layers as inputs")
    ap.add_argument("--loss", default="l1", choices=("l1", "robust"))
    ap.add_argument("--optimizer", default="adam", choices=("adam", "sgd"))
    ap.add_argument("--random-spp", action="store_true",
                    help="the paper's training: inputs re-rendered at a random spp pair per "
                         "iteration (default: fixed 4 / 64 spp pairs rendered once)")
    ap.add_argument("--ablate-loss", type=float, default=None, metavar="SECONDS",
                    help="instead of one run: train one network per loss (L1, and the paper's "
                         "robust loss at beta 0.1 and 1) for SECONDS each from the same init and "
                         "report the hybrid frame's PSNR on the bench and held-out scenes")
    ap.add_argument("--ablate-layers", type=float, default=None, metavar="SECONDS",
                    help="instead of one run: the 16-block network without and with the HRLS "
                         "render layers as inputs, SECONDS of training each from the same seed "
                         "on the same pairs; the hybrid frame's PSNR on the bench and held-out "
                         "scenes")
    ap.add_argument("--loss-settings", default="l1,robust:0.1,robust:1",
                    help="losses of --ablate-loss: comma-separated l1 or robust:<beta>")
    ap.add_argument("--ablation-weights", default=None, metavar="PREFIX",
                    help="save each ablation network's weights to PREFIX<name>.bin")
    ap.add_argument("--init-weights", default=None,
                    help="start from these weights (fine-tuning) instead of a fresh init")
    ap.add_argument("--eval-scenes", type=int, default=4)
    ap.add_argument("--eval-size", default="1280x720")
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    if args.ablate_loss or args.ablate_layers:
        data = build_dataset(n_scenes=args.scenes, windows=args.windows, log=log,
                             layers=bool(args.ablate_layers))
        evals = [("bench", T.GpuScene(S.procedural(7)))]
        evals += [(f"heldout_{sd}", T.GpuScene(S.procedural_sized(sd, tr)))
                  for sd, tr in S.training_scene_specs(200, args.eval_scenes)]
        pre = args.ablation_weights
        if args.ablate_layers:
            archs = ("res16", "res16_layers")
            res = layers_ablation(data, evals, args.ablate_layers, batch=args.batch, lr=args.lr,
                                  seed=args.seed, archs=archs, log=log,
                                  weights_out={a: f"{pre}{a}.bin" for a in archs} if pre else None)
        else:
            settings = []
            for item in args.loss_settings.split(","):
                name, _, beta = item.partition(":")
                settings.append((name, float(beta) if beta else None))
            keys = [n if b is None else f"{n}_beta{b:g}" for n, b in settings]
            res = loss_ablation(data, settings, evals, args.ablate_loss, batch=args.batch,
                                lr=args.lr, seed=args.seed, arch=args.arch, log=log,
                                optimizer=args.optimizer,
                                weights_out={k: f"{pre}{k}.bin" for k in keys} if pre else None)
        print(json.dumps(res))
        return
    net = FusionNet(seed=args.seed, arch=args.arch)
    if args.init_weights:
        net.load_weights(args.init_weights)
    if args.random_spp:
        data = OnlinePairs(S.training_scene_specs(100, args.scenes), windows=args.windows,
                           scale=net.scale, log=log)
        hist = train_random_spp(net, data, args.steps, args.batch, args.lr, seed=args.seed,
                                loss=args.loss, optimizer=args.optimizer, log_every=200,
                                log=log, time_limit=args.time_limit)
        losses = [(s, v) for s, _, _, v in hist if v is not None]
        done = hist[-1][0] if hist else 0
    else:
        data = build_dataset(n_scenes=args.scenes, windows=args.windows, log=log)
        losses, done = train(net, data, args.steps, args.batch, args.lr, seed=args.seed,
                             log=log, time_limit=args.time_limit, loss=args.loss,
                             optimizer=args.optimizer)
    net.save(args.out)
    if args.weights_out:
        net.save_weights(args.weights_out)
    log(f"[train] saved {args.out} after {done} steps")
    if hasattr(data, "close"):
        data.close()
    del data
    W, H = (int(v) for v in args.eval_size.split("x"))
    results = []
    for seed, tris in S.training_scene_specs(200, args.eval_scenes):
        gs = T.GpuScene(S.procedural_sized(seed, tris))
        r = evaluate_scene(gs, net, W, H, seed, plain_spp=(4, 8, 16, 32, 64), reps=1)
        results.append(r)
        log(f"[eval] scene {seed}: hybrid {r['hybrid']['psnr']:.2f} dB, "
            f"hrls {r['hrls_4spp']['psnr']:.2f}, lrhs-bilinear {r['lrhs_bilinear']['psnr']:.2f}, "
            f"plain " + " ".join(f"{n}:{p:.2f}" for n, p, _ in r["plain"]))
    print(json.dumps({"steps": done, "losses": losses[-5:], "eval": results}))


if __name__ == "__main__":
    main()
