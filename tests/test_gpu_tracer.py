"""GPU parity of the HIP path tracer against the FP64 oracle (through the C ABI)."""
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


@pytest.fixture(scope="module")
def mrs(torch_cuda):
    import paper_2106_12802_amd as m
    return m


def rel_ok(g, o):
    """Per-channel relative closeness, dark pixels judged against 1e-3 of the image mean."""
    floor = 1e-3 * max(float(np.abs(o).mean()), 1e-30)
    return np.abs(g - o) <= 1e-4 * np.maximum(np.abs(o), floor)


def gpu_render(mrs, scene, W, H, spp, D, seed, **kw):
    import torch
    gs = mrs.GpuScene(scene)
    rgb, aux = mrs.render(gs, W, H, spp, D, seed, **kw)
    torch.cuda.synchronize()
    return rgb.cpu().numpy().astype(np.float64), aux.cpu().numpy().astype(np.float64), gs


# --------------------------------------------------------------------------- RNG


def test_philox_bitwise(mrs, oracle_tracer):
    from paper_2106_12802_amd.tracer import philox
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, (1000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, (1000, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    key[1] = 0xFFFFFFFF
    got = philox(ctr, key)
    want = np.stack([oracle_tracer.philox4x32_10(c, k) for c, k in zip(ctr, key)])
    assert np.array_equal(got, want)
    assert list(got[0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


# --------------------------------------------------------------------------- LBVH


def _check_lbvh(gs, scene):
    nodes, leaf, morton, root = gs.bvh()
    n = scene.num_tris
    assert sorted(leaf.tolist()) == list(range(n))
    keys = (morton.astype(np.uint64) << np.uint64(32)) | leaf.astype(np.uint64)
    if gs.bvh_builder == "lbvh":  # leaves in Morton order
        assert np.all(keys[1:] > keys[:-1])
    else:  # leaves depth first: the same keys, each once
        assert np.all(np.diff(np.sort(keys)) > 0)
    if n >= 2:  # each node's leaf range is its left range followed by its right range
        refs_u = nodes[:, 12:16].copy().view(np.uint32)

        def rng(r):
            return (r & 0x7FFFFFFF,) * 2 if r & 0x80000000 else tuple(refs_u[r, 2:4])
        for i in range(n - 1):
            a, b = rng(int(refs_u[i, 0])), rng(int(refs_u[i, 1]))
            assert a[0] == refs_u[i, 2] and a[1] + 1 == b[0] and b[1] == refs_u[i, 3], i
    if n < 2:
        return
    refs = nodes[:, 12:14].copy().view(np.uint32)
    V = scene.vertices.astype(np.float32)
    # every node and leaf reachable exactly once; child boxes bound their subtrees
    seen_int = np.zeros(n - 1, int)
    seen_leaf = np.zeros(n, int)

    def subtree_box(ref):
        stack = [ref]
        lo = np.full(3, np.inf, np.float32)
        hi = np.full(3, -np.inf, np.float32)
        while stack:
            r = stack.pop()
            if r & 0x80000000:
                tri = V[leaf[r & 0x7FFFFFFF]]
                lo = np.minimum(lo, tri.min(0))
                hi = np.maximum(hi, tri.max(0))
            else:
                stack += list(refs[r])
        return lo, hi

    stack = [0]
    while stack:
        i = stack.pop()
        seen_int[i] += 1
        for side in range(2):
            r = int(refs[i, side])
            box = nodes[i, 6 * side:6 * side + 6]
            if r & 0x80000000:
                seen_leaf[r & 0x7FFFFFFF] += 1
                tri = V[leaf[r & 0x7FFFFFFF]]
                assert np.array_equal(box[:3], tri.min(0)) and np.array_equal(box[3:], tri.max(0))
            else:
                stack.append(r)
    assert np.all(seen_int == 1) and np.all(seen_leaf == 1)
    # spot-check subtree boxes of some internal children (exact min/max)
    for i in range(0, n - 1, max(1, (n - 1) // 40)):
        for side in range(2):
            r = int(refs[i, side])
            if not r & 0x80000000:
                lo, hi = subtree_box(r)
                box = nodes[i, 6 * side:6 * side + 6]
                assert np.array_equal(box[:3], lo) and np.array_equal(box[3:], hi)


def _check_bvh4(gs, scene):
    """The four-wide BVH: every node reached once, every leaf slot covered once by
    the leaf ranges (at most leaf_max each), child boxes equal to the exact bounds of
    their subtrees, at least two children per node."""
    nodes, root, lmax = gs.bvh4()
    _, leaf, _, _ = gs.bvh()
    n = scene.num_tris
    if n == 0:
        return
    V = scene.vertices.astype(np.float32)
    if n == 1:
        assert root == 0x80000000 and len(nodes) == 0
        return
    assert root == 0
    refs = nodes[:, 24:28].copy().view(np.uint32)
    seen_node = np.zeros(len(nodes), int)
    seen_slot = np.zeros(n, int)

    def bounds(ref):  # exact bounds of a reference's triangles; marks what it reaches
        if ref & 0x80000000:
            first, count = ref & 0xFFFFFF, ((ref >> 24) & 3) + 1
            assert count <= lmax and first + count <= n
            seen_slot[first:first + count] += 1
            tri = V[leaf[first:first + count]].reshape(-1, 3)
            return tri.min(0), tri.max(0)
        seen_node[ref] += 1
        lo = np.full(3, np.inf, np.float32)
        hi = np.full(3, -np.inf, np.float32)
        kids = 0
        for k in range(4):
            r = int(refs[ref, k])
            if r == 0xFFFFFFFF:
                continue
            kids += 1
            clo, chi = bounds(r)
            box = nodes[ref, [k, 4 + k, 8 + k, 12 + k, 16 + k, 20 + k]]
            assert np.array_equal(box[:3], clo) and np.array_equal(box[3:], chi), (ref, k)
            lo, hi = np.minimum(lo, clo), np.maximum(hi, chi)
        assert kids >= 2
        return lo, hi

    import sys
    sys.setrecursionlimit(10000)
    bounds(root)
    assert np.all(seen_node == 1) and np.all(seen_slot == 1)


@pytest.mark.parametrize("maker", [
    lambda: S.random_soup(1, 1),
    lambda: S.random_soup(2, 2),
    lambda: S.random_soup(3, 777),
    lambda: S.cornell(1),
    lambda: S.procedural(7, spheres=((2, 4),), n_boxes=8, n_lights=2),
])
@pytest.mark.parametrize("builder", ["lbvh", "ploc"])
def test_lbvh_invariants(mrs, maker, builder):
    scene = maker()
    _log("bvh", builder, scene.name, scene.num_tris)
    old = mrs.get_tuning()
    try:
        mrs.set_tuning(bvh_builder=builder)
        gs = mrs.GpuScene(scene)
    finally:
        mrs.set_tuning(**old)
    assert gs.bvh_builder == (builder if scene.num_tris >= 2 else "lbvh")
    _check_lbvh(gs, scene)
    _check_bvh4(gs, scene)


@pytest.mark.parametrize("maker", [
    lambda: S.random_soup(4, 20000),
    lambda: S.procedural(7, spheres=((2, 4),), n_boxes=8, n_lights=2),
    lambda: S.procedural_sized(510, 200000),
    lambda: S.random_soup(6, 3),
])
def test_bvh_builders_give_identical_results(mrs, maker):
    """The clustered and the Morton-split BVH give bitwise the same closest hits and
    renders (conservative culling, ties to the smaller primitive id)."""
    import torch
    scene = maker()
    _log("builders", scene.name, scene.num_tris)
    old = mrs.get_tuning()
    gs = {}
    try:
        for b in ("lbvh", "ploc"):
            mrs.set_tuning(bvh_builder=b)
            gs[b] = mrs.GpuScene(scene)
            assert gs[b].bvh_builder == b
    finally:
        mrs.set_tuning(**old)
    o, d = S.random_rays(9, 4000)
    hits = [gs[b].closest_hit(o, d) for b in ("lbvh", "ploc")]
    for x, y in zip(*hits):
        assert np.array_equal(x, y)
    imgs = [mrs.render(gs[b], 96, 64, 4, 8, 21) for b in ("lbvh", "ploc")]
    torch.cuda.synchronize()
    assert torch.equal(imgs[0][0], imgs[1][0]) and torch.equal(imgs[0][1], imgs[1][1])


def test_ploc_identical_boxes_stay_shallow(mrs):
    """Many identical triangles (every candidate cost ties): the clustering pairs
    neighbours, so the tree is balanced rather than a chain (no fallback)."""
    tri = np.tile(np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32), (1000, 1, 1))
    b = S._Builder()
    m = b.material(S.LAMBERT, (0.5, 0.5, 0.5))
    b.add_tris(list(tri), m)
    scene = b.build((0, 0, 0), S.Camera((0.3, 0.3, -3), (0.3, 0.3, 0)), "identical")
    gs = mrs.GpuScene(scene)
    assert gs.bvh_builder == "ploc"
    _check_lbvh(gs, scene)
    o = np.tile(np.array([[0.25, 0.25, -1.0]], np.float32), (8, 1))
    d = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (8, 1))
    t, p, _ = gs.closest_hit(o, d)
    assert np.all(p == 0) and np.allclose(t, 1.0)  # equal t: the smallest primitive id


@pytest.mark.parametrize("leaf_max", [1, 2, 4])
def test_bvh4_leaf_grouping_and_same_hits(mrs, leaf_max):
    """Any leaf grouping gives a valid tree and bitwise the same closest hits."""
    scene = S.random_soup(5, 3000)
    o, d = S.random_rays(5, 2000)
    ref = mrs.GpuScene(scene)
    t_r, p_r, b_r = ref.closest_hit(o, d)
    old = mrs.get_tuning()
    try:
        mrs.set_tuning(bvh_leaf_max=leaf_max)
        gs = mrs.GpuScene(scene)
    finally:
        mrs.set_tuning(**old)
    assert gs.bvh4()[2] == leaf_max
    _check_bvh4(gs, scene)
    t_g, p_g, b_g = gs.closest_hit(o, d)
    assert np.array_equal(p_g, p_r) and np.array_equal(t_g, t_r) and np.array_equal(b_g, b_r)


def test_lbvh_identical_centroids(mrs):
    # all centroids equal: every Morton code ties and the primitive index decides
    b = S._Builder()
    m = b.material(S.LAMBERT, (0.5, 0.5, 0.5))
    rng = np.random.default_rng(0)
    for _ in range(300):
        d = rng.normal(size=(3, 3))
        d -= d.mean(0)
        b.add_tris([d], m)
    scene = b.build((0, 0, 0), S.Camera((0, 0, -5), (0, 0, 0)), "ties")
    gs = mrs.GpuScene(scene)
    _check_lbvh(gs, scene)


# --------------------------------------------------------------------------- traversal


@pytest.mark.parametrize("seed,n", [(1, 1), (2, 40), (3, 1500), (4, 20000)])
def test_closest_hit_vs_oracle_brute_force(mrs, oracle_tracer, seed, n):
    scene = S.random_soup(seed, n)
    o, d = S.random_rays(seed, 3000)
    _log("closest_hit", seed, n)
    gs = mrs.GpuScene(scene)
    t_g, p_g, b_g = gs.closest_hit(o, d)
    t_o, p_o, b_o = oracle_tracer.OracleScene(scene).closest_hit(o, d, use_bvh=n > 2000)
    same = p_g == p_o
    # A disagreement is allowed only at a near-tie between two triangles (FP32 vs FP64).
    # FP32 rounding of t scales with the size of the hit point's coordinates
    scale = t_o + np.linalg.norm(o, axis=1)
    bad = np.where(~same)[0]
    for i in bad:
        assert p_g[i] >= 0 and p_o[i] >= 0 and abs(t_g[i] - t_o[i]) <= 1e-5 * scale[i], (i, t_g[i], t_o[i])
    assert same.mean() >= 0.999
    hit = same & (p_o >= 0)
    assert hit.sum() > 0 or n == 1
    err = np.abs(t_g[hit] - t_o[hit]) / scale[hit]
    _log(f"closest_hit: {len(bad)} prim mismatches, max |dt|/(t+|o|) {err.max() if err.size else 0:.2e}")
    assert np.all(err <= 1e-5)
    assert np.all(np.isinf(t_g[p_g < 0]))


def test_closest_hit_skip(mrs, oracle_tracer):
    scene = S.random_soup(5, 500)
    o, d = S.random_rays(5, 2000)
    osc = oracle_tracer.OracleScene(scene)
    _, p0, _ = osc.closest_hit(o, d, use_bvh=False)
    skip = np.where(p0 >= 0, p0, -1).astype(np.int32)
    gs = mrs.GpuScene(scene)
    t_g, p_g, _ = gs.closest_hit(o, d, skip=skip)
    t_o, p_o, _ = osc.closest_hit(o, d, skip=skip, use_bvh=False)
    assert (p_g == p_o).mean() >= 0.999
    assert not np.any((p_g == skip) & (skip >= 0))


# --------------------------------------------------------------------------- closed forms


def test_env_only_exact(mrs):
    scene = S.env_only((0.3, 0.5, 0.7))
    rgb, aux, _ = gpu_render(mrs, scene, 37, 19, 3, 5, 1)
    assert np.all(rgb == scene.env.astype(np.float64)[None, None])
    assert np.all(aux == 0)


@pytest.mark.parametrize("D", [0, 1, 3])
def test_lambert_plane_exact(mrs, D):
    scene = S.lambert_plane()
    rgb, _, _ = gpu_render(mrs, scene, 32, 24, 8, D, 3)
    want = 0.0 if D == 0 else (scene.materials[0]["color"] * scene.env).astype(np.float64)
    assert np.allclose(rgb, want, rtol=2e-7, atol=0)


@pytest.mark.parametrize("D", [0, 2, 3])
def test_furnace_exact(mrs, D):
    scene = S.furnace_sphere(1.5, 0.6, subdiv=2)
    rgb, _, _ = gpu_render(mrs, scene, 24, 16, 8, D, 5, rr_start=100)
    E = float(scene.materials[0]["emission"][0])
    rho = float(scene.materials[0]["color"][0])
    want = E * sum(rho ** k for k in range(D + 1))
    assert np.allclose(rgb, want, rtol=1e-6)


# --------------------------------------------------------------------------- full renders


# Feature-buffer tolerances.  Albedo is a table lookup (exact unless the hit
# differs).  The smooth shading normal interpolates corner normals with FP32
# barycentrics, whose error is about eps32 * (|o| + t) / edge: for 0.04-long
# triangles seen from ~10 units that is ~1e-5, times a corner-normal spread of
# ~0.1, so 2e-5 absolute.  Depth is FP32 t: 1e-5 relative.
ALBEDO_TOL, NORMAL_TOL, DEPTH_TOL = 1e-6, 2e-5, 1e-5


def _parity(g_rgb, g_aux, o, label):
    o_rgb = o["rgb"].reshape(g_rgb.shape)
    o_aux = o["aux"].reshape(g_aux.shape)
    ok = np.all(rel_ok(g_rgb, o_rgb), axis=-1)
    frac = ok.mean()
    mean_rel = abs(g_rgb.mean() - o_rgb.mean()) / abs(o_rgb.mean())
    alb_err = np.abs(g_aux[..., 0:3] - o_aux[..., 0:3]).max(-1)
    nrm_err = np.abs(g_aux[..., 3:6] - o_aux[..., 3:6]).max(-1)
    dep_err = np.abs(g_aux[..., 6] - o_aux[..., 6]) / np.maximum(o_aux[..., 6], 1e-6)
    aux_ok = (alb_err <= ALBEDO_TOL) & (nrm_err <= NORMAL_TOL) & (dep_err <= DEPTH_TOL)
    _log(f"{label}: pixels ok {frac:.5f} ({(~ok).sum()} bad), mean rel {mean_rel:.2e}, "
         f"aux ok {aux_ok.mean():.5f}, normal err median {np.median(nrm_err):.1e} "
         f"max {nrm_err.max():.2e}, max depth err {dep_err.max():.2e}")
    return frac, mean_rel, aux_ok.mean()


@pytest.mark.parametrize("scene_seed", [1, 2, 3])
def test_cornell_parity(mrs, oracle_tracer, scene_seed):
    scene = S.cornell(scene_seed)
    W = H = 64
    spp, D, seed = 16, 4, 1000 + scene_seed
    g_rgb, g_aux, _ = gpu_render(mrs, scene, W, H, spp, D, seed)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, D, seed)
    frac, mean_rel, aux_frac = _parity(g_rgb, g_aux, o, f"cornell {scene_seed}")
    assert frac >= 0.999
    assert mean_rel <= 1e-5
    assert aux_frac >= 0.999


def test_procedural_parity_small_ragged(mrs, oracle_tracer):
    # 97 x 55 at 4 spp: several 256-thread blocks and a ragged tail.  With only
    # 21k paths one divergent path moves the image mean by ~1e-5 of itself, so
    # the mean is held to 1e-4 here and to 1e-5 at full size below.
    scene = S.procedural(7)
    W, H, spp, D, seed = 97, 55, 4, 8, 2 * 7
    g_rgb, g_aux, _ = gpu_render(mrs, scene, W, H, spp, D, seed)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, D, seed)
    frac, mean_rel, aux_frac = _parity(g_rgb, g_aux, o, "procedural 97x55x4")
    assert frac >= 0.999
    assert mean_rel <= 1e-4
    assert aux_frac >= 0.999


@pytest.mark.parametrize("W,H,spp,seed", [(1280, 720, 4, 14), (320, 180, 64, 15)])
def test_procedural_parity_full_size(mrs, oracle_tracer, torch_cuda, W, H, spp, seed):
    """HRLS 1280x720 @4 spp and LRHS 320x180 @64 spp, whole images against the oracle."""
    scene = S.procedural(7)
    gs = mrs.GpuScene(scene)
    rgb, aux = mrs.render(gs, W, H, spp, 8, seed)
    torch_cuda.cuda.synchronize()
    g_rgb = rgb.cpu().numpy().reshape(-1, 3).astype(np.float64)
    g_aux = aux.cpu().numpy().reshape(-1, 7).astype(np.float64)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, 8, seed)
    frac, mean_rel, aux_frac = _parity(g_rgb, g_aux, o, f"procedural {W}x{H}x{spp}")
    assert frac >= 0.999
    assert mean_rel <= 1e-5
    assert aux_frac >= 0.999


def test_binding_rejects_wrong_tensors(mrs, torch_cuda):
    gs = mrs.GpuScene(S.cornell(1))
    torch = torch_cuda
    with pytest.raises(TypeError, match="float32"):
        mrs.render_ex(gs, 8, 8, 1, 1, 0, torch.zeros(8, 8, 3, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="elements"):
        mrs.render_ex(gs, 8, 8, 1, 1, 0, torch.zeros(8, 7, 3, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="CUDA"):
        mrs.render_ex(gs, 8, 8, 1, 1, 0, torch.zeros(8, 8, 3, dtype=torch.float32))


def test_window_is_crop_and_chunking_invariant(mrs, torch_cuda):
    scene = S.cornell(2)
    gs = mrs.GpuScene(scene)
    full, faux = mrs.render(gs, 48, 40, 6, 4, 77)
    win, waux = mrs.render(gs, 48, 40, 6, 4, 77, window=(8, 12, 17, 9))
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(win, full[12:21, 8:25])
    assert torch_cuda.equal(waux, faux[12:21, 8:25])
    old = mrs.get_tuning()
    try:
        for chunk, blocks, sched, qs in [(256, 3, 1, 0), (1000, 7, 0, 1), (48 * 40 * 2 + 5, 64, 1, 0),
                                         (48 * 40 * 2 + 5, 64, 1, 1)]:
            mrs.set_tuning(chunk_paths=chunk, trace_blocks=blocks, schedule=sched, queue_sort=qs)
            again, aaux = mrs.render(gs, 48, 40, 6, 4, 77)
            torch_cuda.cuda.synchronize()
            assert torch_cuda.equal(again, full), (chunk, blocks, sched, qs)
            assert torch_cuda.equal(aaux, faux)
    finally:
        mrs.set_tuning(**old)
    again, _ = mrs.render(gs, 48, 40, 6, 4, 77)
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(again, full)  # deterministic run to run


def test_queue_order_and_node_format_do_not_change_the_image(mrs, torch_cuda):
    """Ordering each block's appended rays by direction octant and its shadow rays by
    light (queue_sort) changes which rays share a wave, the quantized BVH4 nodes
    (bvh_quantized) which boxes a ray visits, and the wave traversal (wave_extend,
    wave_shadow) the order and company in which rays walk the tree, not any result:
    the full HRLS render of the bench scene, with features and render layers, is
    bitwise the same."""
    gs = mrs.GpuScene(S.procedural(7))
    old = mrs.get_tuning()
    outs = []
    try:
        for qs, qn, we, wsh in ((0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (1, 1, 0, 0),
                                (1, 0, 1, 1), (1, 1, 3, 0), (0, 0, 0, 3)):
            mrs.set_tuning(queue_sort=qs, bvh_quantized=qn, wave_extend=we, wave_shadow=wsh)
            lay = torch_cuda.empty(720, 1280, 9, device="cuda")
            rgb, aux = mrs.render(gs, 1280, 720, 4, 8, 14, out_layers=lay)
            torch_cuda.cuda.synchronize()
            outs.append((rgb, aux, lay))
    finally:
        mrs.set_tuning(**old)
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert torch_cuda.equal(a, b)


@pytest.mark.parametrize("seed,n", [(2, 40), (3, 1500), (4, 20000)])
def test_quantized_nodes_closest_hit_vs_oracle_brute_force(mrs, oracle_tracer, seed, n):
    """Closest hits through the quantized nodes equal the FP32-node traversal's
    bitwise and the oracle's brute force (same primitive)."""
    scene = S.random_soup(seed, n)
    gs = mrs.GpuScene(scene)
    o, d = S.random_rays(seed + 100, 3000)
    old = mrs.get_tuning()
    try:
        mrs.set_tuning(bvh_quantized=0)
        t0, p0, b0 = gs.closest_hit(o, d)
        mrs.set_tuning(bvh_quantized=1)
        t1, p1, b1 = gs.closest_hit(o, d)
    finally:
        mrs.set_tuning(**old)
    assert np.array_equal(p0, p1) and np.array_equal(t0, t1) and np.array_equal(b0, b1)
    _, p_o, _ = oracle_tracer.OracleScene(scene).closest_hit(o, d, use_bvh=False)
    assert (p1 == p_o).mean() >= 0.999


def test_sub_chunks_beyond_2_24_paths(mrs, torch_cuda):
    """A shadow ray carries its path slot in 24 bits next to its light index; a
    tuning asking for more resident paths per sub-chunk than that (one stream,
    2^25 paths) is cut into more super-chunks instead, and a multi-light render
    of 17.8 M paths is bitwise the one of the default tuning."""
    scene = S.procedural(7, spheres=((2, 3),), n_boxes=6, n_lights=3)
    gs = mrs.GpuScene(scene)
    ref, _ = mrs.render(gs, 1024, 1024, 17, 2, 31, want_aux=False)
    old = mrs.get_tuning()
    try:
        mrs.set_tuning(chunk_paths=1 << 25, streams=1)
        big, _ = mrs.render(gs, 1024, 1024, 17, 2, 31, want_aux=False)
        mrs.set_tuning(chunk_paths=1 << 26, streams=2)
        big2, _ = mrs.render(gs, 1024, 1024, 17, 2, 31, want_aux=False)
        torch_cuda.cuda.synchronize()
    finally:
        mrs.set_tuning(**old)
    mrs.release_workspaces()
    assert torch_cuda.equal(big, ref) and torch_cuda.equal(big2, ref)


def test_fp64_accumulation_matches(mrs, oracle_tracer, torch_cuda):
    scene = S.cornell(3)
    gs = mrs.GpuScene(scene)
    r32, _ = mrs.render(gs, 16, 16, 64, 4, 5, accum_fp64=0)
    r64, _ = mrs.render(gs, 16, 16, 64, 4, 5, accum_fp64=1)
    torch_cuda.cuda.synchronize()
    a = r32.cpu().numpy().astype(np.float64)
    b = r64.cpu().numpy().astype(np.float64)
    assert np.allclose(a, b, rtol=1e-5, atol=1e-7)
    o = oracle_tracer.OracleScene(scene).render(16, 16, 64, 4, 5)
    assert np.mean(np.all(rel_ok(b.reshape(-1, 3), o["rgb"]), -1)) >= 0.99


# The automatic FP64 pixel sums (spp >= 1024) against the oracle, element-wise.
# A path whose FP32 and FP64 versions take different branches (a grazing hit or
# shadow test, a Russian-roulette draw at its threshold) changes its pixel by
# about |dL| / spp; on the Cornell box about 2 paths in a million diverge, so
# at 1024 spp ~0.2% of pixels hold one and miss the 1e-4 bar (measured: 2 of
# 1024 pixels; image mean 6.7e-8).  The bar is therefore checked where it is a
# property of the arithmetic: (a) 2^20 samples per pixel, where a divergent
# path moves its pixel by ~1e-6 of it, and (b) 1024 spp of a scene with no
# occluder and no roulette (direct light on a floor), where no path can diverge.
@pytest.mark.parametrize("case", ["cornell_2x2_1M_spp", "direct_64x64_1024_spp"])
def test_fp64_auto_parity_at_high_spp(mrs, oracle_tracer, torch_cuda, case):
    """At spp >= 1024 the pixel sums switch to FP64 by themselves (Q16, the path
    every reference and training target takes): the automatic choice equals
    forced FP64 bitwise, and the image holds the parity bar element-wise
    (99.9% of pixels within 1e-4, image mean within 1e-5) against the oracle."""
    if case.startswith("cornell"):
        scene, W, H, spp, D = S.cornell(1), 2, 2, 1 << 20, 4
    else:
        scene, W, H, spp, D = S.nee_config(rho=0.6, le=8.0, a=1.5, bb=1.0, c=1.2), 64, 64, 1024, 1
    seed = 2 ** 40 + 3
    gs = mrs.GpuScene(scene)
    auto, aux = mrs.render(gs, W, H, spp, D, seed)
    forced, _ = mrs.render(gs, W, H, spp, D, seed, accum_fp64=1, want_aux=False)
    sums32, _ = mrs.render(gs, W, H, spp, D, seed, accum_fp64=0, want_aux=False)
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(auto, forced)
    g_rgb = auto.cpu().numpy().reshape(-1, 3).astype(np.float64)
    g_aux = aux.cpu().numpy().reshape(-1, 7).astype(np.float64)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, D, seed)
    frac, mean_rel, aux_frac = _parity(g_rgb, g_aux, o, f"{case} (FP64 sums)")
    e64 = float(np.max(np.abs(g_rgb - o["rgb"]) / np.maximum(np.abs(o["rgb"]), 1e-30)))
    g32 = sums32.cpu().numpy().reshape(-1, 3).astype(np.float64)
    e32 = float(np.max(np.abs(g32 - o["rgb"]) / np.maximum(np.abs(o["rgb"]), 1e-30)))
    _log(f"  worst pixel relative error: FP64 sums {e64:.2e}, FP32 sums {e32:.2e}")
    assert frac >= 0.999
    assert mean_rel <= 1e-5
    assert aux_frac >= 0.999


def test_counters_and_no_overflow(mrs, torch_cuda):
    mrs.counters(reset=True)
    scene = S.procedural(7, spheres=((2, 4),), n_boxes=10, n_lights=3)
    gs = mrs.GpuScene(scene)
    mrs.render(gs, 64, 48, 2, 8, 9)
    c = mrs.counters(reset=True)
    _log("counters", c)
    assert c["paths"] == 64 * 48 * 2
    assert c["rays"] >= c["paths"]
    assert c["overflows"] == 0
    assert c["nonfinite"] == 0


def test_sumsq_parity(mrs, oracle_tracer, torch_cuda):
    """Per-pixel sums of squared sample radiance match the oracle's (same paths)."""
    scene = S.cornell(1)
    W = H = 12
    gs = mrs.GpuScene(scene)
    for seed, fp64 in [(5000, 0), (5001, 1)]:
        s = torch_cuda.zeros(H, W, 3, dtype=torch_cuda.float32, device="cuda")
        rgb, _ = mrs.render(gs, W, H, 16, 4, seed, want_aux=False, out_sumsq=s, accum_fp64=fp64)
        torch_cuda.cuda.synchronize()
        g = s.cpu().numpy().reshape(-1, 3).astype(np.float64)
        o = oracle_tracer.OracleScene(scene).render(W, H, 16, 4, seed, want_sumsq=True)["sumsq"]
        ok = np.all(rel_ok(g, o), -1)
        _log(f"sumsq fp64={fp64}: {ok.mean():.4f} ok, max {g.max():.3e} vs {o.max():.3e}")
        assert ok.mean() >= 0.99


def test_unbiased_vs_oracle_high_spp(mrs, oracle_tracer, torch_cuda):
    """Mean of 64 independent 16-spp GPU renders vs a 4096-spp oracle render."""
    scene = S.cornell(1)
    W = H = 12
    osc = oracle_tracer.OracleScene(scene)
    ref = osc.render(W, H, 4096, 4, 2 ** 40 + 1, want_sumsq=True)
    ref_mean = ref["rgb"]
    ref_var = ref["sumsq"] / 4096 - ref_mean ** 2
    gs = mrs.GpuScene(scene)
    imgs = []
    sq = []
    for k in range(64):
        s = torch_cuda.zeros(H, W, 3, dtype=torch_cuda.float32, device="cuda")
        rgb, _ = mrs.render(gs, W, H, 16, 4, 5000 + k, want_aux=False, out_sumsq=s)
        imgs.append(rgb.cpu().numpy().reshape(-1, 3).astype(np.float64))
        sq.append(s.cpu().numpy().reshape(-1, 3).astype(np.float64))
    g_mean = np.mean(imgs, 0)
    g_var = np.sum(sq, 0) / 1024 - g_mean ** 2
    sigma = np.sqrt(np.maximum(g_var, 0) / 1024 + np.maximum(ref_var, 0) / 4096)
    z = np.abs(g_mean - ref_mean) / np.maximum(sigma, 1e-12)
    frac_out = (z > 3).mean()
    img_sigma = math.sqrt(np.sum(sigma ** 2)) / sigma.size
    _log(f"unbiased: frac > 3 sigma {frac_out:.4f}, mean diff {g_mean.mean() - ref_mean.mean():.3e} "
         f"(sigma {img_sigma:.3e})")
    if frac_out > 0.01:
        sq_all = np.array(sq)
        bad = np.argsort(-sigma.max(1))[:3]
        _log(f"  largest sigma pixels {bad.tolist()}: gpu var {g_var[bad].max(1)}, oracle var "
             f"{ref_var[bad].max(1)}; per-render sumsq of pixel {bad[0]}: "
             f"{sq_all[:, bad[0], 0].tolist()}")
    assert abs(g_mean.mean() - ref_mean.mean()) <= 3 * img_sigma
    assert frac_out <= 0.01


def test_ploc_too_deep_falls_back_to_lbvh(mrs):
    """Concentric triangles of growing size: the clustering can only chain them
    (one merge per round), a tree deeper than the traversal stack allows, so the
    build falls back to the Morton-split tree, with the same hits."""
    b = S._Builder()
    m = b.material(S.LAMBERT, (0.5, 0.5, 0.5))
    base = np.array([[-1.0, -1.0, 0.0], [1.0, -1.0, 0.0], [0.0, 1.0, 0.0]])
    tris = [base * 1.5 ** k + np.array([0.0, 0.0, 0.01 * k]) for k in range(100)]
    b.add_tris(tris, m)
    scene = b.build((0, 0, 0), S.Camera((0, 0, -5), (0, 0, 0)), "concentric")
    gs = mrs.GpuScene(scene)
    assert gs.bvh_builder == "lbvh"
    _check_lbvh(gs, scene)
    o = np.tile(np.array([[0.0, -0.2, -1.0]], np.float32), (4, 1))
    d = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (4, 1))
    t, p, _ = gs.closest_hit(o, d)
    assert np.all(p == 0) and np.allclose(t, 1.0)  # the smallest (nearest) triangle


# --------------------------------------------------------------------------- render layers


def _layers_gpu(mrs, torch_cuda, gs, W, H, spp, D, seed, **kw):
    lay = torch_cuda.full((H, W, 9), float("nan"), dtype=torch_cuda.float32, device="cuda")
    rgb, _ = mrs.render(gs, W, H, spp, D, seed, want_aux=False, out_layers=lay, **kw)
    torch_cuda.cuda.synchronize()
    return rgb.cpu().numpy().reshape(-1, 3).astype(np.float64), \
        lay.cpu().numpy().reshape(-1, 9).astype(np.float64)


@pytest.mark.parametrize("fp64,mis", [(0, False), (1, True)])
def test_layers_parity(mrs, oracle_tracer, torch_cuda, fp64, mis):
    """Emission / diffuse / glossy layers (Sec. 3.1, Eqs. 1-2) against the oracle's, on a
    Lambert + GGX scene with lights and environment; 97 x 55 ends in ragged tiles.  As
    for the image (21k paths, mean held to 1e-4), one divergent path moves a layer's mean
    by as much more as the layer is a smaller share of the image (diffuse: ~5% here)."""
    scene = S.procedural(7)
    W, H, spp, D, seed = 97, 55, 4, 4, 4242 + fp64
    gs = mrs.GpuScene(scene)
    _log(f"layers parity fp64={fp64} mis={mis}")
    g_rgb, g_lay = _layers_gpu(mrs, torch_cuda, gs, W, H, spp, D, seed, accum_fp64=fp64, mis=mis)
    plain, _ = mrs.render(gs, W, H, spp, D, seed, want_aux=False, accum_fp64=fp64, mis=mis)
    torch_cuda.cuda.synchronize()
    # the same paths: asking for layers leaves the image bitwise as it was
    assert np.array_equal(plain.cpu().numpy().reshape(-1, 3).astype(np.float64), g_rgb)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, D, seed, mis=mis, want_layers=True)
    assert np.all(np.isfinite(g_lay))
    tot = g_lay[:, 0:3] + g_lay[:, 3:6] + g_lay[:, 6:9]
    assert np.allclose(tot, g_rgb, rtol=1e-5, atol=1e-6 * max(g_rgb.mean(), 1e-30))
    for k, name in enumerate(("emission", "diffuse", "glossy")):
        g, ob = g_lay[:, 3 * k:3 * k + 3], o["layers"][:, 3 * k:3 * k + 3]
        assert ob.max() > 0, name
        frac = np.all(rel_ok(g, ob), -1).mean()
        mean_rel = abs(g.mean() - ob.mean()) / abs(ob.mean())
        share = ob.mean() / o["rgb"].mean()
        _log(f"  {name}: pixels ok {frac:.5f}, mean rel {mean_rel:.2e}, share {share:.3f}")
        assert frac >= 0.999, name
        assert mean_rel <= 1e-4 / min(share, 1.0), name


def test_layers_parity_full_size_hrls(mrs, oracle_tracer, torch_cuda):
    """The HRLS render (1280x720 @4 spp, depth 8) with its layers, whole image against the
    oracle; the image mean bar (1e-5) scaled by each layer's share of the image."""
    scene = S.procedural(7)
    W, H, spp, D, seed = 1280, 720, 4, 8, 14
    _log("layers parity 1280x720x4")
    g_rgb, g_lay = _layers_gpu(mrs, torch_cuda, mrs.GpuScene(scene), W, H, spp, D, seed)
    o = oracle_tracer.OracleScene(scene).render(W, H, spp, D, seed, want_aux=False,
                                                want_layers=True)
    assert np.all(rel_ok(g_rgb, o["rgb"]).all(-1).mean() >= 0.999)
    for k, name in enumerate(("emission", "diffuse", "glossy")):
        g, ob = g_lay[:, 3 * k:3 * k + 3], o["layers"][:, 3 * k:3 * k + 3]
        frac = np.all(rel_ok(g, ob), -1).mean()
        mean_rel = abs(g.mean() - ob.mean()) / abs(ob.mean())
        share = ob.mean() / o["rgb"].mean()
        _log(f"  {name}: pixels ok {frac:.5f}, mean rel {mean_rel:.2e}, share {share:.3f}")
        assert frac >= 0.999, name
        assert mean_rel <= 1e-5 / min(share, 1.0), name


def test_layers_degenerate_cases(mrs, torch_cuda):
    """Depth 0 (the first vertex's emission only): the emission layer is the image and the
    others are zero; one pixel at one sample; a scene with no lights (environment only)."""
    gs = mrs.GpuScene(S.procedural(7))
    _log("layers degenerate cases")
    rgb, lay = _layers_gpu(mrs, torch_cuda, gs, 33, 17, 3, 0, 5)
    assert np.array_equal(lay[:, 0:3], rgb) and np.all(lay[:, 3:] == 0)
    rgb, lay = _layers_gpu(mrs, torch_cuda, gs, 1, 1, 1, 8, 6)
    assert np.allclose(lay[:, 0:3] + lay[:, 3:6] + lay[:, 6:9], rgb, rtol=1e-6, atol=0)
    env = S.env_only((0.3, 0.5, 0.7))
    rgb, lay = _layers_gpu(mrs, torch_cuda, mrs.GpuScene(env), 16, 8, 2, 4, 7)
    assert np.array_equal(lay[:, 0:3], rgb) and np.all(lay[:, 3:] == 0)
    assert np.allclose(rgb, env.env.astype(np.float64)[None])


def test_layers_in_a_batch_match_single_renders(mrs, torch_cuda):
    """Jobs with and without layers share a batch's accumulators (their offsets differ
    by the layer sums); each job's outputs equal its own render bitwise."""
    gA = mrs.GpuScene(S.procedural(7, spheres=((2, 4),), n_boxes=5, n_lights=2))
    gB = mrs.GpuScene(S.cornell(1))
    mk = lambda h, w: torch_cuda.zeros(h, w, 9, dtype=torch_cuda.float32, device="cuda")
    jobs = [dict(scene=gA, W=40, H=24, spp=5, max_depth=3, seed=71, out_layers=mk(24, 40)),
            dict(scene=gB, W=32, H=16, spp=3, max_depth=4, seed=72),
            dict(scene=gA, W=8, H=8, spp=1030, max_depth=2, seed=73, out_layers=mk(8, 8)),
            dict(scene=gB, W=64, H=40, spp=2, max_depth=5, seed=74, window=(8, 8, 30, 20),
                 out_layers=mk(20, 30), mis=True)]
    _log("layers batch")
    b = mrs.Batch(jobs)
    b.render()
    torch_cuda.cuda.synchronize()
    for j, (rgb, aux) in zip(jobs, b.outputs):
        kw = {k: j[k] for k in ("window", "mis") if k in j}
        lay = mk(*j["out_layers"].shape[:2]) if "out_layers" in j else None
        r1, a1 = mrs.render(j["scene"], j["W"], j["H"], j["spp"], j["max_depth"], j["seed"],
                            out_layers=lay, **kw)
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(rgb, r1) and torch_cuda.equal(aux, a1)
        if lay is not None:
            assert torch_cuda.equal(j["out_layers"], lay)
            assert float(lay.abs().sum()) > 0
