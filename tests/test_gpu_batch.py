"""Batched renders, HIP-graph replay of the hybrid frame, autotuned launch shapes."""
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


def _jobs(mrs):
    scenes = [mrs.GpuScene(S.cornell(1)), mrs.GpuScene(S.procedural_sized(301, 20000)),
              mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))]
    return [
        dict(scene=scenes[0], W=64, H=48, spp=5, max_depth=4, seed=11),
        dict(scene=scenes[1], W=160, H=96, spp=2, max_depth=8, seed=12, window=(8, 4, 100, 60)),
        dict(scene=scenes[2], W=40, H=40, spp=7, max_depth=3, seed=13, rr_start=1),
        dict(scene=scenes[0], W=8, H=8, spp=1030, max_depth=2, seed=14),  # FP64 sums
        dict(scene=scenes[1], W=16, H=12, spp=3, max_depth=6, seed=15, want_aux=False),
    ]


def _single(mrs, j):
    kw = {k: j[k] for k in ("window", "rr_start") if k in j}
    return mrs.render(j["scene"], j["W"], j["H"], j["spp"], j["max_depth"], j["seed"],
                      want_aux=j.get("want_aux", True), **kw)


@pytest.mark.parametrize("chunk,schedule", [(None, 0), (None, 1), (3000, 1), (257, 0)])
def test_batch_matches_single_renders_bitwise(torch_cuda, chunk, schedule):
    import paper_2106_12802_amd as mrs
    old = mrs.get_tuning()
    try:
        mrs.set_tuning(schedule=schedule)
        if chunk:
            mrs.set_tuning(chunk_paths=chunk, trace_blocks=16)
        jobs = _jobs(mrs)
        b = mrs.Batch(jobs)
        b.render()
        torch_cuda.cuda.synchronize()
        for j, (rgb, aux) in zip(jobs, b.outputs):
            r1, a1 = _single(mrs, j)
            torch_cuda.cuda.synchronize()
            assert torch_cuda.equal(rgb, r1)
            if aux is not None:
                assert torch_cuda.equal(aux, a1)
        b.render()  # a batch can be rendered again (same results)
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(b.outputs[0][0], _single(mrs, jobs[0])[0])
    finally:
        mrs.set_tuning(**old)



@pytest.mark.parametrize("schedule", [0, 1])
def test_wave_traversal_batch_matches_lane_traversal(torch_cuda, schedule):
    """Every bounce's closest-hit and shadow rays traced a wave at a time: the
    batch's outputs equal single renders traced lane by lane, bitwise.  The jobs'
    path counts put waves across two scenes (lanes of a wave walk different trees),
    and the later bounces hold incoherent rays (waves whose lanes enter few common
    nodes)."""
    import paper_2106_12802_amd as mrs
    old = mrs.get_tuning()
    try:
        jobs = _jobs(mrs)
        mrs.set_tuning(wave_extend=0, wave_shadow=0, schedule=schedule)
        singles = [_single(mrs, j) for j in jobs]
        mrs.counters(reset=True)
        mrs.set_tuning(wave_extend=65, wave_shadow=65, tail_bounce=65)
        b = mrs.Batch(jobs)
        b.render()
        torch_cuda.cuda.synchronize()
        for j, (rgb, aux), (r1, a1) in zip(jobs, b.outputs, singles):
            assert torch_cuda.equal(rgb, r1), j
            if aux is not None:
                assert torch_cuda.equal(aux, a1), j
        c = mrs.counters(reset=True)
        assert c["overflows"] == 0 and c["nonfinite"] == 0
    finally:
        mrs.set_tuning(**old)

def test_batch_set_seeds_matches_single_renders(torch_cuda):
    import paper_2106_12802_amd as mrs
    jobs = _jobs(mrs)[:3]
    b = mrs.Batch(jobs)
    with pytest.raises(ValueError):
        b.set_seeds([1, 2])
    for seeds in ([101, 102, 103], [7, (1 << 40) + 5, 9]):
        b.set_seeds(seeds)
        b.render()
        torch_cuda.cuda.synchronize()
        for j, seed, (rgb, aux) in zip(jobs, seeds, b.outputs):
            r1, a1 = _single(mrs, dict(j, seed=seed))
            torch_cuda.cuda.synchronize()
            assert torch_cuda.equal(rgb, r1) and torch_cuda.equal(aux, a1), seed
    b.close()


def test_graph_replay_of_hybrid_frame(torch_cuda):
    """Capture HRLS + LRHS + fusion in a HIP graph; every replay equals the eager frame."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as HY
    torch = torch_cuda
    gs = mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))
    net = mrs.FusionNet(seed=3)
    W, H = 256, 128
    out = torch.empty(H, W, 3, device="cuda")
    eager, _ = HY.hybrid_frame(gs, net, W, H, 5, out=torch.empty(H, W, 3, device="cuda"))
    eager = eager.clone()
    # warm up on the capturing stream (its workspace grows outside the capture)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        HY.hybrid_frame(gs, net, W, H, 5, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        HY.hybrid_frame(gs, net, W, H, 5, out=out)
    for k in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
        # eager work between replays
        other, _ = HY.hybrid_frame(gs, net, W, H, 6 + k, out=torch.empty(H, W, 3, device="cuda"))
        torch.cuda.synchronize()


def test_autotune_applies_choice_and_keeps_results(torch_cuda, tmp_path):
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import autotune
    old = mrs.get_tuning()
    try:
        gs = mrs.GpuScene(S.cornell(2))
        ref, _ = mrs.render(gs, 96, 64, 8, 4, 3)
        torch_cuda.cuda.synchronize()
        wl = lambda: mrs.render(gs, 96, 64, 8, 4, 3)
        cache = str(tmp_path / "tune.json")
        cands = [(1 << 20, 512, 0), (4096, 64, 1), (1 << 22, 2048, 1)]
        r = autotune.tune(wl, "cornell96", cache, reps=2, candidates=cands, log=_log)
        assert (r["chunk_paths"], r["trace_blocks"], r["schedule"]) in cands and not r["cached"]
        now = mrs.get_tuning()
        assert all(now[k] == r[k] for k in ("chunk_paths", "trace_blocks", "schedule"))
        again, _ = mrs.render(gs, 96, 64, 8, 4, 3)
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(again, ref)
        mrs.set_tuning(**old)
        r2 = autotune.tune(wl, "cornell96", cache, candidates=cands)
        assert r2["cached"] and r2["chunk_paths"] == r["chunk_paths"]
    finally:
        mrs.set_tuning(**old)


def test_concurrent_streams_and_batch_tuning_snapshot(torch_cuda):
    """Renders on two streams at once equal sequential ones (one workspace per stream);
    a batch keeps the tuning it was created with."""
    import paper_2106_12802_amd as mrs
    torch = torch_cuda
    gs1 = mrs.GpuScene(S.procedural_sized(302, 30000))
    gs2 = mrs.GpuScene(S.cornell(4))
    r1, _ = mrs.render(gs1, 200, 120, 4, 6, 21)
    r2, _ = mrs.render(gs2, 96, 96, 16, 5, 22)
    torch.cuda.synchronize()
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for k in range(3):
        with torch.cuda.stream(a):
            x1, _ = mrs.render(gs1, 200, 120, 4, 6, 21)
        with torch.cuda.stream(b):
            x2, _ = mrs.render(gs2, 96, 96, 16, 5, 22)
        outs.append((x1, x2))
    torch.cuda.synchronize()
    for x1, x2 in outs:
        assert torch.equal(x1, r1) and torch.equal(x2, r2)
    old = mrs.get_tuning()
    try:
        bt = mrs.Batch([dict(scene=gs2, W=96, H=96, spp=16, max_depth=5, seed=22)])
        mrs.set_tuning(chunk_paths=256, trace_blocks=1, schedule=1)
        bt.render()
        torch.cuda.synchronize()
        assert torch.equal(bt.outputs[0][0], r2)
        bt.close()
    finally:
        mrs.set_tuning(**old)


def test_full_size_render_invariant_to_tuning(torch_cuda):
    """A 1280x720x4 render of the 101k-triangle scene is bitwise the same for every
    sub-chunk count, chunk size, grid size, schedule, path-tail bounce and wave
    traversal (the result must not depend on which rays share a wave, nor on which
    kernel traces a bounce)."""
    import paper_2106_12802_amd as mrs
    torch = torch_cuda
    gs = mrs.GpuScene(S.procedural(7))
    old = mrs.get_tuning()
    try:
        mrs.set_tuning(streams=1)
        ref, raux = mrs.render(gs, 1280, 720, 4, 8, 99)
        torch.cuda.synchronize()
        for tune in (dict(streams=3), dict(streams=2, chunk_paths=1 << 20),
                     dict(streams=3, trace_blocks=1000, schedule=1),
                     dict(streams=1, chunk_paths=777777, trace_blocks=3000),
                     dict(tail_bounce=1), dict(tail_bounce=2), dict(tail_bounce=65),
                     dict(wave_extend=1, wave_shadow=1),
                     dict(wave_extend=3, wave_shadow=3, schedule=1, trace_blocks=700)):
            mrs.set_tuning(**dict(old, **tune))
            img, aux = mrs.render(gs, 1280, 720, 4, 8, 99)
            torch.cuda.synchronize()
            assert torch.equal(img, ref) and torch.equal(aux, raux), tune
    finally:
        mrs.set_tuning(**old)


def test_hybrid_frame_batch_equals_separate_calls(torch_cuda):
    """HybridFrame (HRLS + LRHS as one batch, reseeded per frame) gives bitwise the
    frame of hybrid_frame (two render calls), for several seeds, also in a graph."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as HY
    torch = torch_cuda
    gs = mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))
    net = mrs.FusionNet(seed=4)
    W, H = 320, 192
    fr = HY.HybridFrame(gs, net, W, H)
    for seed in (3, 11):
        a = fr.render(seed).clone()
        b, _ = HY.hybrid_frame(gs, net, W, H, seed, out=torch.empty(H, W, 3, device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(a, b), seed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fr.render(7)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fr.render(7)
    ref, _ = HY.hybrid_frame(gs, net, W, H, 7, out=torch.empty(H, W, 3, device="cuda"))
    for _ in range(3):
        fr.out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(fr.out, ref)
        fr.render(12)  # eager work between replays (its own seeds)
        torch.cuda.synchronize()
    fr.close()


def test_hybrid_frame_with_layers(torch_cuda):
    """A hybrid frame that keeps the HRLS layers fuses bitwise the same frame; its layers
    and sums of squares equal those of a single HRLS render with the frame's seed."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as HY
    torch = torch_cuda
    gs = mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))
    net = mrs.FusionNet(seed=4)
    W, H = 160, 96
    _log("hybrid frame with layers")
    plain = HY.HybridFrame(gs, net, W, H)
    fr = HY.HybridFrame(gs, net, W, H, layers=True)
    a = plain.render(5).clone()
    b = fr.render(5).clone()
    lay = torch.empty(H, W, 9, device="cuda")
    sq = torch.empty(H, W, 3, device="cuda")
    rgb, _ = mrs.render(gs, W, H, 4, HY.DEPTH, 10, want_aux=False, out_layers=lay,
                        out_sumsq=sq)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(fr.hr_rgb, rgb)
    assert torch.equal(fr.hr_layers, lay) and torch.equal(fr.hr_sumsq, sq)
    plain.close()
    fr.close()


def test_fallback_without_network_is_plain_render(torch_cuda):
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as HY
    torch = torch_cuda
    gs = mrs.GpuScene(S.cornell(2))
    empty = mrs.FusionNet()  # no parameters
    plain, _ = mrs.render(gs, 64, 48, HY.fallback_spp(), HY.DEPTH, 2 * 9, want_aux=False)
    for net in (None, empty):
        a, _ = HY.hybrid_frame(gs, net, 64, 48, 9)
        fr = HY.HybridFrame(gs, net, 64, 48)
        b = fr.render(9)
        torch.cuda.synchronize()
        assert torch.equal(a, plain) and torch.equal(b, plain)
        fr.close()


@pytest.mark.parametrize("chunk", [None, 3000])
def test_split_render_matches_render(torch_cuda, chunk):
    """render_begin + render_end is render, bitwise, also over several super-chunks;
    the outputs keep the previous render's values until render_end; misuse is an
    error with no effect."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd._lib import MrsError
    torch = torch_cuda
    old = mrs.get_tuning()
    try:
        if chunk:
            mrs.set_tuning(chunk_paths=chunk, trace_blocks=16)
        jobs = _jobs(mrs)[:3]
        b = mrs.Batch(jobs)
    finally:
        mrs.set_tuning(**old)
    b.render()
    torch.cuda.synchronize()
    prev = [o[0].clone() for o in b.outputs]
    with pytest.raises(MrsError, match="no render of the batch begun"):
        b.render_end()
    seeds = [21, (1 << 33) + 22, 23]
    b.set_seeds(seeds)
    b.render_begin()
    with pytest.raises(MrsError, match="not ended"):
        b.render_begin()
    with pytest.raises(MrsError, match="not ended"):
        b.render()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with pytest.raises(MrsError, match="stream"):
            b.render_end()
    between = [o[0].clone() for o in b.outputs]  # enqueued between begin and end
    b.render_end()
    torch.cuda.synchronize()
    for p, q in zip(prev, between):
        assert torch.equal(p, q)
    for j, seed, (rgb, aux) in zip(jobs, seeds, b.outputs):
        r1, a1 = _single(mrs, dict(j, seed=seed))
        torch.cuda.synchronize()
        assert torch.equal(rgb, r1), seed
        assert torch.equal(aux, a1), seed
    b.close()



@pytest.mark.parametrize("chunk", [None, 3000])
def test_render_fork_keeps_results(torch_cuda, chunk):
    """render_fork marks the next render's start ahead of its launches: fork, other
    work on the stream, begin, end equals render bitwise (one super-chunk or
    several); seeds set after a fork undo it; a fork while a render is begun is an
    error with no effect."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd._lib import MrsError
    torch = torch_cuda
    old = mrs.get_tuning()
    try:
        if chunk:
            mrs.set_tuning(chunk_paths=chunk, trace_blocks=16)
        jobs = _jobs(mrs)[:3]
        b = mrs.Batch(jobs)
    finally:
        mrs.set_tuning(**old)
    seeds_a, seeds_b = [31, 32, 33], [41, (1 << 35) + 42, 43]
    b.set_seeds(seeds_a)
    b.render()
    torch.cuda.synchronize()
    ref_a = [o[0].clone() for o in b.outputs]
    b.set_seeds(seeds_b)
    b.render()
    torch.cuda.synchronize()
    ref_b = [o[0].clone() for o in b.outputs]
    # fork, unrelated work on the stream, begin, end
    b.set_seeds(seeds_a)
    b.render_fork()
    scratch = torch.randn(1 << 20, device="cuda")
    scratch.mul_(2.0)
    b.render_begin()
    with pytest.raises(MrsError, match="not ended"):
        b.render_fork()
    b.render_end()
    torch.cuda.synchronize()
    for got, r in zip(b.outputs, ref_a):
        assert torch.equal(got[0], r)
    # seeds after the fork: the render uses them
    b.render_fork()
    b.set_seeds(seeds_b)
    b.render()
    torch.cuda.synchronize()
    for got, r in zip(b.outputs, ref_b):
        assert torch.equal(got[0], r)
    b.close()

@pytest.mark.parametrize("in_flight", [1, 2])
def test_pipelined_frames_equal_single_frames(torch_cuda, in_flight):
    """HybridFrame.render_stream (frame k+1 rendering while frame k finishes and is
    fused; one or two frames in flight) gives every frame bitwise as render(seed);
    also for the network that reads the render layers and for the no-network
    fallback.  Afterwards the frame's images are the last frame's."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import hybrid as HY
    torch = torch_cuda
    gs = mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))
    seeds = [3, 11, 5, 8, 2]
    for net in (mrs.FusionNet(seed=4), mrs.FusionNet(seed=6, arch="res16_layers"), None):
        fr = HY.HybridFrame(gs, net, 320, 192)
        refs = [fr.render(sd).clone() for sd in seeds]
        last_hr = None if net is None else fr.hr_rgb.clone()
        got = []
        fr.render_stream(seeds, on_frame=lambda k, out: got.append(out.clone()),
                         in_flight=in_flight)
        torch.cuda.synchronize()
        assert len(got) == len(seeds)
        for k, (a, r) in enumerate(zip(got, refs)):
            assert torch.equal(a, r), (net is None, k)
        if net is not None:
            assert torch.equal(fr.hr_rgb, last_hr)
        fr.render_stream([], in_flight=in_flight)
        fr.close()


def test_profile_records_selected_kernels(torch_cuda):
    """HIP-event kernel timing: every launch by default, only the selected kernels
    after profile_select; the counts follow the launch structure of a render.  With
    bounce 0 on the wave traversal (the default) camera rays are generated inside
    the bounce-0 kernels, so no generate launch is recorded; with the lane-by-lane
    traversal at bounce 0 the generate kernel runs."""
    import paper_2106_12802_amd as mrs
    from paper_2106_12802_amd import tracer as R
    torch = torch_cuda
    gs = mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))
    old = mrs.get_tuning()
    try:
        R.profile_select(None)
        R.profile_enable(True)
        mrs.render(gs, 128, 96, 4, 8, 3)
        everything = R.profile_read()
        R.profile_select(["extend"])
        R.profile_enable(True)
        mrs.render(gs, 128, 96, 4, 8, 3)
        only = R.profile_read()
        mrs.set_tuning(wave_extend=0)
        R.profile_select(None)
        R.profile_enable(True)
        mrs.render(gs, 128, 96, 4, 8, 3)
        lane0 = R.profile_read()
    finally:
        R.profile_enable(False)
        R.profile_select(None)
        mrs.set_tuning(**old)
    torch.cuda.synchronize()
    assert set(only) == {"extend"}
    assert only["extend"][1] == everything["extend"][1] > 0
    assert old["wave_extend"] > 0 and "generate" not in everything
    assert {"extend", "shade", "shadow", "accumulate", "resolve"} <= set(everything)
    assert {"generate", "extend", "shade", "shadow", "accumulate", "resolve"} <= set(lane0)
    with pytest.raises(ValueError):
        R.profile_select(["no_such_kernel"])
