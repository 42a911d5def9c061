"""Pins for the FP64 reference path tracer (oracle/tracer.cpp).

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, quadrature of the defining integrals, or a
brute-force / independent-algorithm computation.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from mrs_inputs import scenes as S

# --------------------------------------------------------------------------- E1 Philox


def test_philox_known_answers(oracle_tracer):
    # Known-answer vectors of Philox4x32-10 published with Random123 (Salmon et al., SC'11).
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        got = oracle_tracer.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want


def test_uniform_mapping_range(oracle_tracer):
    us = [oracle_tracer.uniform(1234, p, 3, d) for p in range(64) for d in range(8)]
    for u in us:
        assert 0.0 <= u <= 1.0 - 2.0 ** -24
        assert u * 2 ** 24 == int(u * 2 ** 24)  # 24-bit grid: exact in FP32 and FP64
    # different dimensions of one (p, s) are different words
    assert len(set(us)) > 500


# --------------------------------------------------------------------------- E3 camera


def test_camera_corner_angles(oracle_tracer):
    sc = oracle_tracer.OracleScene(S.cornell(1))
    W, H = 64, 48
    vfov = 40.0
    _, top = sc.camera_ray(W, H, W / 2, 0)
    _, bot = sc.camera_ray(W, H, W / 2, H)
    _, left = sc.camera_ray(W, H, 0, H / 2)
    _, right = sc.camera_ray(W, H, W, H / 2)
    ang = lambda a, b: math.degrees(math.acos(np.clip(np.dot(a, b), -1, 1)))
    assert ang(top, bot) == pytest.approx(vfov, abs=1e-9)
    hfov = 2 * math.degrees(math.atan(math.tan(math.radians(vfov / 2)) * W / H))
    assert ang(left, right) == pytest.approx(hfov, abs=1e-9)
    # row 0 is the top of the image: its ray points up relative to the centre ray
    _, ctr = sc.camera_ray(W, H, W / 2, H / 2)
    assert top[1] > ctr[1] > bot[1]
    # image right is f x up; looking along +z with up +y that is -x
    assert left[0] > ctr[0] > right[0]
    f = np.array([0.0, 0.0, 1.7]) / 1.7
    assert np.allclose(ctr, f, atol=1e-12)


def test_thin_lens_rays_meet_on_the_focal_plane(oracle_tracer):
    """Every lens sample of a pixel point leaves from the lens disk (radius R,
    across the view axis) and passes through the point where the pinhole ray
    meets the focal plane (distance `focus` along the view axis)."""
    sc = oracle_tracer.OracleScene(S.cornell(1))
    W, H, R, focus = 64, 48, 0.05, 1.3
    pos = np.array([0.5, 0.5, -1.2], np.float32).astype(np.float64)  # the camera is FP32
    f = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(5)
    for x, y in [(W / 2, H / 2), (3.25, 40.5), (60.0, 1.0)]:
        o0, d0 = sc.camera_ray(W, H, x, y)
        F = o0 + d0 * (focus / (d0 @ f))
        for u0, u1 in rng.random((8, 2)):
            o, d = sc.camera_ray_fx(W, H, x, y, u0, u1, 0.0, lens_radius=R, focus_dist=focus)
            off = o - pos
            assert abs(off @ f) < 1e-15 and np.linalg.norm(off) <= R * (1 + 1e-12)
            assert np.linalg.norm(off) == pytest.approx(R * math.sqrt(u0), rel=1e-12)
            t = (F - o) @ f / (d @ f)
            assert np.allclose(o + t * d, F, atol=1e-12)
        # radius 0 is the pinhole exactly
        o, d = sc.camera_ray_fx(W, H, x, y, 0.3, 0.7, 0.0, focus_dist=focus)
        assert np.array_equal(o, o0) and np.array_equal(d, d0)


def test_circle_of_confusion(oracle_tracer):
    """On a plane at distance z across the axis, the centre pixel's lens samples
    land on a disk of radius R |z - focus| / focus around the pinhole hit."""
    sc = oracle_tracer.OracleScene(S.cornell(1))
    W, H, R, focus = 64, 48, 0.05, 1.3
    pos = np.array([0.5, 0.5, -1.2], np.float32).astype(np.float64)  # the camera is FP32
    for z in (0.6, 2.5):
        pts = []
        for k in range(64):
            u0, u1 = (k + 0.5) / 64, (k * 0.618034) % 1.0
            o, d = sc.camera_ray_fx(W, H, W / 2, H / 2, 1.0 if k % 2 else u0, u1, 0.0,
                                    lens_radius=R, focus_dist=focus)
            pts.append(o + d * ((pos[2] + z - o[2]) / d[2]))
        rad = np.linalg.norm(np.array(pts)[:, :2] - pos[:2], axis=1)
        assert rad.max() == pytest.approx(R * abs(z - focus) / focus, rel=1e-12)


def test_camera_motion_translates_the_ray(oracle_tracer):
    sc = oracle_tracer.OracleScene(S.cornell(1))
    m = (0.2, -0.1, 0.05)
    o0, d0 = sc.camera_ray(32, 32, 10.5, 20.25)
    for tau in (0.0, 0.37, 0.999):
        o, d = sc.camera_ray_fx(32, 32, 10.5, 20.25, 0.5, 0.5, tau, cam_motion=m)
        assert np.allclose(o, o0 + tau * np.array(m), atol=1e-15) and np.array_equal(d, d0)


@pytest.mark.parametrize("max_depth", [1, 3])
def test_lens_and_motion_keep_lambert_plane_exact(oracle_tracer, max_depth):
    """A Lambert plane under a constant environment is rho * env from any point of
    view: it stays exact with a lens and a moving camera (which do draw their
    random numbers)."""
    scene = S.lambert_plane()
    r = oracle_tracer.OracleScene(scene).render(8, 8, 16, max_depth, 3, lens_radius=0.2,
                                                focus_dist=3.0, cam_motion=(0.5, 0.0, 0.2))
    want = scene.materials[0]["color"].astype(np.float64) * scene.env.astype(np.float64)
    assert np.allclose(r["rgb"], want[None], rtol=1e-14, atol=0)


def test_in_focus_plane_matches_pinhole(oracle_tracer):
    """A textured Lambert plane on the focal plane, lit by the environment: every
    lens sample of a pixel point hits the point the pinhole ray hits, so the image
    is the pinhole image (to rounding of the hit points)."""
    b = S._Builder()
    mats = [b.material(S.LAMBERT, color=(0.8, 0.2, 0.1)), b.material(S.LAMBERT, color=(0.1, 0.3, 0.9))]
    for i in range(8):
        for j in range(8):
            b.add_quad((-2.0 + 0.5 * i, -2.0 + 0.5 * j, 3.0), (0.5, 0.0, 0.0), (0.0, 0.5, 0.0),
                       mats[(i + j) % 2])
    cam = S.Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 50.0)
    scene = b.build((1.0, 1.0, 1.0), cam, "focal_checker")
    sc = oracle_tracer.OracleScene(scene)
    pin = sc.render(24, 24, 8, 1, 9)
    dof = sc.render(24, 24, 8, 1, 9, lens_radius=0.1, focus_dist=3.0)
    assert np.allclose(dof["rgb"], pin["rgb"], rtol=1e-9, atol=1e-12)
    blur = sc.render(24, 24, 8, 1, 9, lens_radius=0.1, focus_dist=1.5)
    assert not np.allclose(blur["rgb"], pin["rgb"], atol=1e-3)  # out of focus: checker edges blur


# --------------------------------------------------------------------------- E4 intersection


def _solve_hits(V, o, d, skip=None):
    """Closest hit by solving o + t d = v0 + b1 e1 + b2 e2 with a dense linear solve."""
    n = len(o)
    t_best = np.full(n, np.inf)
    p_best = np.full(n, -1)
    e1 = V[:, 1] - V[:, 0]
    e2 = V[:, 2] - V[:, 0]
    for i in range(n):
        A = np.stack([e1, e2, -np.broadcast_to(d[i], e1.shape)], axis=2)  # [T,3,3]
        rhs = o[i][None, :] - V[:, 0]
        det = np.linalg.det(A)
        ok = np.abs(det) > 1e-300
        sol = np.full((len(V), 3), np.nan)
        sol[ok] = np.linalg.solve(A[ok], rhs[ok][..., None])[..., 0]
        b1, b2, t = sol[:, 0], sol[:, 1], sol[:, 2]
        good = ok & (b1 >= 0) & (b2 >= 0) & (b1 + b2 <= 1) & (t > 0)
        if skip is not None:
            good[skip[i]] = False
        if good.any():
            idx = np.where(good)[0]
            j = idx[np.argmin(t[idx])]
            t_best[i] = t[j]
            p_best[i] = j
    return t_best, p_best


def test_hand_triangle_rational_t(oracle_tracer):
    b = S._Builder()
    m = b.material(S.LAMBERT, (0.5, 0.5, 0.5))
    b.add_tris([[[0, 0, 2], [1, 0, 2], [0, 1, 2]]], m)  # plane z = 2
    b.add_tris([[[0, 0, 5], [4, 0, 5], [0, 4, 5]]], m)  # plane z = 5 behind it
    sc = oracle_tracer.OracleScene(b.build((0, 0, 0), S.Camera((0, 0, 0), (0, 0, 1)), "hand"))
    o = np.array([[0.25, 0.5, 0.0], [0.75, 0.75, 0.0], [0.25, 0.25, 3.0], [0.0, 0.0, 0.0]])
    d = np.array([[0, 0, 1.0], [0, 0, 1.0], [0, 0, 1.0], [0, 0, 1.0]])
    t, prim, bb = sc.closest_hit(o, d, use_bvh=False)
    assert t[0] == 2.0 and prim[0] == 0 and tuple(bb[0]) == (0.25, 0.5)
    assert t[1] == 5.0 and prim[1] == 1  # outside the first triangle (u + v > 1)
    assert t[2] == 2.0 and prim[2] == 1  # origin past the first plane
    assert t[3] == 2.0 and prim[3] == 0  # vertex: edges are inclusive
    # excluding the origin primitive
    t, prim, _ = sc.closest_hit(o[:1], d[:1], skip=[0], use_bvh=False)
    assert prim[0] == 1 and t[0] == 5.0
    # parallel ray is a miss
    t, prim, _ = sc.closest_hit([[0.1, 0.1, 2.0]], [[1.0, 0, 0]], use_bvh=False)
    assert prim[0] == -1 and np.isinf(t[0])


def test_tie_goes_to_smaller_prim(oracle_tracer):
    b = S._Builder()
    m = b.material(S.LAMBERT, (0.5, 0.5, 0.5))
    tri = [[-1, -1, 3], [3, -1, 3], [-1, 3, 3]]
    for _ in range(3):
        b.add_tris([tri], m)
    sc = oracle_tracer.OracleScene(b.build((0, 0, 0), S.Camera((0, 0, 0), (0, 0, 1)), "tie"))
    for bvh in (False, True):
        t, prim, _ = sc.closest_hit([[0.1, 0.2, 0.0]], [[0, 0, 1.0]], use_bvh=bvh)
        assert prim[0] == 0 and t[0] == 3.0
        t, prim, _ = sc.closest_hit([[0.1, 0.2, 0.0]], [[0, 0, 1.0]], skip=[0], use_bvh=bvh)
        assert prim[0] == 1


@pytest.mark.parametrize("seed,n", [(1, 40), (2, 300), (3, 1500)])
def test_brute_force_matches_linear_solve_and_bvh(oracle_tracer, seed, n):
    scene = S.random_soup(seed, n)
    sc = oracle_tracer.OracleScene(scene)
    o, d = S.random_rays(seed, 400)
    o = o.astype(np.float64)
    d = d.astype(np.float64)
    t_bf, p_bf, _ = sc.closest_hit(o, d, use_bvh=False)
    t_bvh, p_bvh, _ = sc.closest_hit(o, d, use_bvh=True)
    assert np.array_equal(p_bf, p_bvh)
    assert np.array_equal(t_bf, t_bvh)
    V = scene.vertices.astype(np.float64)
    k = 120
    t_ls, p_ls = _solve_hits(V, o[:k], d[:k])
    assert np.array_equal(p_ls, p_bf[:k])
    fin = np.isfinite(t_ls)
    assert np.allclose(t_ls[fin], t_bf[:k][fin], rtol=1e-10)
    assert (p_bf >= 0).sum() > 50  # the test exercises hits, not only misses


def test_bvh_on_procedural_scene(oracle_tracer):
    scene = S.procedural(7, spheres=((2, 3),), n_boxes=5, n_lights=1)
    sc = oracle_tracer.OracleScene(scene)
    rng = np.random.default_rng(0)
    o = np.zeros((500, 3)) + np.array([0.0, 3.0, 10.0])
    d = rng.normal(size=(500, 3)) + np.array([0, -0.3, -1.0]) * 2
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t1, p1, _ = sc.closest_hit(o, d, use_bvh=False)
    t2, p2, _ = sc.closest_hit(o, d, use_bvh=True)
    assert np.array_equal(p1, p2) and np.array_equal(t1, t2)
    assert (p1 >= 0).mean() > 0.5


# --------------------------------------------------------------------------- E5 frame


def test_onb_orthonormal(oracle_tracer):
    rng = np.random.default_rng(5)
    ns = list(rng.normal(size=(200, 3))) + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                           np.array([1.0, 0, 0])]
    for n in ns:
        n = n / np.linalg.norm(n)
        T, B = oracle_tracer.onb(n)
        M = np.stack([T, B, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.linalg.det(M) == pytest.approx(1.0, abs=1e-12)  # right-handed


# --------------------------------------------------------------------------- E9 Lambert


def test_cosine_sampling_moments(oracle_tracer):
    # Exact midpoint quadrature of the sampling map over [0,1]^2 reproduces the
    # moments of the cosine-weighted hemisphere: E[z] = 2/3, E[z^2] = 1/2, E[x^2] = 1/4.
    n = 400
    g = (np.arange(n) + 0.5) / n
    pts = np.array([oracle_tracer.sample_cosine(u1, u2) for u1 in g for u2 in g[::8]])
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.0, atol=1e-12)
    assert pts[:, 2].min() > 0
    assert pts[:, 2].mean() == pytest.approx(2 / 3, abs=2e-4)
    assert (pts[:, 2] ** 2).mean() == pytest.approx(1 / 2, abs=2e-4)
    assert (pts[:, 0] ** 2).mean() == pytest.approx(1 / 4, abs=2e-3)
    assert abs(pts[:, 0].mean()) < 1e-3 and abs(pts[:, 1].mean()) < 1e-3


# --------------------------------------------------------------------------- E10 GGX


@pytest.mark.parametrize("alpha", [0.05, 0.3, 0.8])
def test_ggx_D_normalised(oracle_tracer, alpha):
    # int D(h) (n.h) dw_h = 1 over the hemisphere (projected microfacet area).
    f = lambda mu: oracle_tracer.ggx_D(alpha, mu) * mu * 2 * math.pi
    val, _ = integrate.quad(f, 0.0, 1.0, points=[1 - alpha ** 2, 1 - alpha ** 2 / 10], limit=400)
    assert val == pytest.approx(1.0, abs=1e-8)


@pytest.mark.parametrize("alpha", [0.3, 0.8])
@pytest.mark.parametrize("theta_o", [0.1, 0.7, 1.3])
def test_ggx_weak_white_furnace(oracle_tracer, alpha, theta_o):
    # Heitz (JCGT 2014): int G1(wo) max(0, wo.h) D(h) / (n.wo) dw_h = 1 for Smith G1.
    wo = np.array([math.sin(theta_o), 0.0, math.cos(theta_o)])
    g1 = oracle_tracer.ggx_G1(alpha, wo[2])

    def f(phi, th):
        h = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
        return g1 * max(0.0, wo @ h) * oracle_tracer.ggx_D(alpha, h[2]) / wo[2] * math.sin(th)

    val, _ = integrate.dblquad(f, 0, math.pi / 2, 0, 2 * math.pi, epsabs=1e-7)
    assert val == pytest.approx(1.0, abs=2e-5)


@pytest.mark.parametrize("alpha", [0.1, 0.5])
def test_ggx_sampling_density(oracle_tracer, alpha):
    # The sampled half vectors have density D(h)(n.h): compare E[cos^k] with quadrature.
    n = 2000
    g = (np.arange(n) + 0.5) / n
    hs = np.array([oracle_tracer.sample_ggx_h(alpha, u, 0.3) for u in g])
    assert np.allclose(np.linalg.norm(hs, axis=1), 1.0, atol=1e-12)
    for k in (1, 2, 4):
        want, _ = integrate.quad(
            lambda mu: mu ** k * oracle_tracer.ggx_D(alpha, mu) * mu * 2 * math.pi, 0, 1,
            points=[1 - alpha ** 2], limit=200)
        assert (hs[:, 2] ** k).mean() == pytest.approx(want, rel=2e-4)


# --------------------------------------------------------------------------- full paths


def _sigma(r, spp):
    mean = r["rgb"]
    var = np.maximum(r["sumsq"] / spp - mean ** 2, 0) * spp / (spp - 1)
    return np.sqrt(var / spp)


def test_env_only_exact(oracle_tracer):
    scene = S.env_only((0.3, 0.5, 0.7))
    r = oracle_tracer.OracleScene(scene).render(16, 8, 4, 8, 42)
    assert np.array_equal(r["rgb"], np.tile(scene.env.astype(np.float64), (128, 1)))
    assert np.all(r["aux"] == 0)


@pytest.mark.parametrize("max_depth", [1, 2, 7])
def test_lambert_plane_under_env_exact(oracle_tracer, max_depth):
    scene = S.lambert_plane()
    r = oracle_tracer.OracleScene(scene).render(8, 8, 16, max_depth, 3, want_sumsq=True)
    want = scene.materials[0]["color"].astype(np.float64) * scene.env.astype(np.float64)
    assert np.allclose(r["rgb"], want[None], rtol=1e-14, atol=0)
    assert np.allclose(r["sumsq"] / 16, want[None] ** 2, rtol=1e-13)
    r0 = oracle_tracer.OracleScene(scene).render(8, 8, 4, 0, 3)
    assert np.all(r0["rgb"] == 0)  # depth 0: the plane itself does not emit


@pytest.mark.parametrize("max_depth", [0, 1, 2, 3])
def test_furnace_exact_without_rr(oracle_tracer, max_depth):
    E, rho = 1.5, 0.6
    scene = S.furnace_sphere(E, rho, subdiv=2)
    r = oracle_tracer.OracleScene(scene).render(8, 8, 8, max_depth, 5, rr_start=100,
                                                want_sumsq=True)
    # the scene stores FP32 values; the oracle promotes them exactly
    E32 = float(scene.materials[0]["emission"][0])
    rho32 = float(scene.materials[0]["color"][0])
    want = E32 * sum(rho32 ** k for k in range(max_depth + 1))
    assert np.allclose(r["rgb"], want, rtol=1e-12)
    assert np.allclose(r["sumsq"] / 8, want ** 2, rtol=1e-12)  # zero variance


def test_furnace_with_rr_unbiased(oracle_tracer):
    E, rho = 1.0, 0.5
    scene = S.furnace_sphere(E, rho, subdiv=2)
    spp = 2048
    r = oracle_tracer.OracleScene(scene).render(4, 4, spp, 64, 9, rr_start=3, want_sumsq=True)
    rho32 = float(scene.materials[0]["color"][0])
    want = E * (1 - rho32 ** 65) / (1 - rho32)
    mean = r["rgb"].mean()
    sig = _sigma(r, spp).mean() / math.sqrt(r["rgb"].size)  # pixels are independent
    assert abs(mean - want) < 3 * sig + 1e-12
    assert sig < 0.01


def _config_factor(X, Y):
    a = X / math.sqrt(1 + X * X) * math.atan(Y / math.sqrt(1 + X * X))
    b = Y / math.sqrt(1 + Y * Y) * math.atan(X / math.sqrt(1 + Y * Y))
    return (a + b) / (2 * math.pi)


@pytest.mark.parametrize("mis", [False, True])
def test_nee_configuration_factor(oracle_tracer, mis):
    # With mis the light is reached by both strategies (NEE at the floor, the
    # BSDF ray hitting it at depth 1) and the power-heuristic weights must sum
    # to one for every direction: a wrong density on either side biases this.
    rho, le, a, bb, c = 0.5, 10.0, 1.0, 2.0, 1.5
    scene = S.nee_config(rho, le, a, bb, c)
    spp = 200_000
    r = oracle_tracer.OracleScene(scene).render(1, 1, spp, 1, 77, want_sumsq=True, mis=mis)
    want = rho * le * _config_factor(a / c, bb / c)
    sig = _sigma(r, spp)[0]
    assert np.all(np.abs(r["rgb"][0] - want) < 3 * sig), (r["rgb"][0], want, sig)
    # first-hit features: albedo, normal, depth
    assert np.allclose(r["aux"][0, :3], rho)
    assert np.allclose(r["aux"][0, 3:6], [0, 1, 0], atol=1e-6)
    assert r["aux"][0, 6] == pytest.approx(c / 2, rel=1e-6)


def test_light_back_face_does_not_emit(oracle_tracer):
    # Camera above the light, looking down at its back: the emitter is one-sided,
    # and a pure emitter ends the path, so the pixel is black.
    b = S._Builder()
    b.add_light((-1.0, 1.0, -1.0), (2.0, 0, 0), (0, 0, 2.0), (5.0, 5.0, 5.0))
    cam = S.Camera((0.0, 3.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 10.0)
    scene = b.build((0.0, 0.0, 0.0), cam, "backface")
    r = oracle_tracer.OracleScene(scene).render(4, 4, 4, 3, 1)
    assert np.all(r["rgb"] == 0)
    # seen from below, the front face emits its radiance exactly
    cam2 = S.Camera((0.0, -2.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 10.0)
    scene2 = b.build((0.0, 0.0, 0.0), cam2, "frontface")
    r2 = oracle_tracer.OracleScene(scene2).render(4, 4, 4, 3, 1)
    assert np.all(r2["rgb"] == 5.0)


def _ggx_plane_scene(alpha, f0, theta_o, env):
    b = S._Builder()
    b.add_quad((-100.0, 0.0, -100.0), (0.0, 0.0, 200.0), (200.0, 0.0, 0.0),
               b.material(S.GGX, color=f0, alpha=alpha))
    pos = (0.0, 2.0 * math.cos(theta_o), -2.0 * math.sin(theta_o))
    cam = S.Camera(pos, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.01)
    return b.build(env, cam, "ggx_plane")


def test_ggx_plane_under_env_matches_quadrature(oracle_tracer):
    # Camera sees a GGX plane under a constant environment (max depth 1): the pixel
    # mean is env * int f(wo, wi) cos(wi) dw_i, computed here by quadrature over wi
    # with the separately pinned BRDF evaluation.
    alpha, f0, theta_o = 0.4, (0.9, 0.6, 0.3), 0.6
    env = (1.0, 1.0, 1.0)
    scene = _ggx_plane_scene(alpha, f0, theta_o, env)
    spp = 200_000
    r = oracle_tracer.OracleScene(scene).render(1, 1, spp, 1, 11, want_sumsq=True)
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([0.0, math.sin(theta_o), math.cos(theta_o)])  # local frame: z = normal

    def f(phi, th, c):
        wi = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
        return oracle_tracer.ggx_eval(alpha, f0, n, wo, wi)[c] * wi[2] * math.sin(th)

    sig = _sigma(r, spp)[0]
    for c in range(3):
        want, _ = integrate.dblquad(lambda p, t: f(p, t, c), 0, math.pi / 2, 0, 2 * math.pi,
                                    epsabs=1e-6)
        assert abs(r["rgb"][0, c] - want) < 3 * sig[c] + 1e-5, (c, r["rgb"][0, c], want, sig[c])


@pytest.mark.parametrize("alpha,mis", [(0.5, False), (0.5, True), (0.15, True)])
def test_ggx_nee_matches_quadrature(oracle_tracer, alpha, mis):
    # GGX floor lit by one quad light, max depth 1: E[pixel] = int_light f Le cos cos / r^2 dA,
    # by NEE alone or (mis) NEE and BSDF sampling combined.
    f0 = (0.8, 0.7, 0.6)
    le, a, bb, c = 10.0, 1.0, 2.0, 1.5
    b = S._Builder()
    b.add_quad((-50.0, 0.0, -50.0), (0.0, 0.0, 100.0), (100.0, 0.0, 0.0),
               b.material(S.GGX, color=f0, alpha=alpha))
    b.add_light((0.0, c, 0.0), (a, 0.0, 0.0), (0.0, 0.0, bb), (le, le, le))
    cam_pos = (-0.8, 0.9, -0.6)
    cam = S.Camera(cam_pos, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.01)
    scene = b.build((0.0, 0.0, 0.0), cam, "ggx_nee")
    spp = 200_000
    r = oracle_tracer.OracleScene(scene).render(1, 1, spp, 1, 12, want_sumsq=True, mis=mis)
    n = np.array([0.0, 1.0, 0.0])
    wo = np.array(cam_pos) / np.linalg.norm(cam_pos)

    def f(z, x, ch):
        y = np.array([x, c, z])
        dv = y
        r2 = dv @ dv
        wi = dv / math.sqrt(r2)
        return (oracle_tracer.ggx_eval(alpha, f0, n, wo, wi)[ch] * le * wi[1] * wi[1] / r2)

    sig = _sigma(r, spp)[0]
    for ch in range(3):
        want, _ = integrate.dblquad(lambda z, x: f(z, x, ch), 0, a, 0, bb, epsabs=1e-7)
        assert abs(r["rgb"][0, ch] - want) < 3 * sig[ch] + 1e-6, (ch, r["rgb"][0, ch], want)


def _glossy_light_scene(alpha):
    # A glossy GGX floor whose sharp lobe sees a part of a larger light.
    b = S._Builder()
    b.add_quad((-50.0, 0.0, -50.0), (0.0, 0.0, 100.0), (100.0, 0.0, 0.0),
               b.material(S.GGX, color=(0.9, 0.9, 0.9), alpha=alpha))
    b.add_light((0.5, 1.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), (10.0, 10.0, 10.0))
    cam = S.Camera((-1.0, 1.0, -0.5), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.01)
    return b.build((0.0, 0.0, 0.0), cam, "glossy_light")


def test_mis_same_mean_lower_variance_on_glossy(oracle_tracer):
    # Both estimators are unbiased for the same integral; when a sharp lobe sees
    # only a part of a light, light sampling alone wastes most samples and the
    # combined estimator does not (Veach & Guibas 1995): measured 5x lower sigma.
    sc = oracle_tracer.OracleScene(_glossy_light_scene(0.05))
    spp = 100_000
    a = sc.render(1, 1, spp, 1, 31, want_sumsq=True)
    m = sc.render(1, 1, spp, 1, 32, want_sumsq=True, mis=True)
    sa, sm = _sigma(a, spp)[0], _sigma(m, spp)[0]
    assert np.all(np.abs(a["rgb"][0] - m["rgb"][0]) < 3 * np.hypot(sa, sm))
    assert a["rgb"][0, 0] > 1.0  # the reflection is in the pixel
    assert np.all(sm < 0.5 * sa), (sm, sa)


def test_mis_without_lights_changes_nothing(oracle_tracer):
    sc = oracle_tracer.OracleScene(S.lambert_plane())
    a = sc.render(4, 4, 8, 3, 5)
    m = sc.render(4, 4, 8, 3, 5, mis=True)
    assert np.array_equal(a["rgb"], m["rgb"]) and np.array_equal(a["aux"], m["aux"])


def test_mis_cornell_same_mean(oracle_tracer):
    sc = oracle_tracer.OracleScene(S.cornell(1))
    spp = 256
    a = sc.render(16, 16, spp, 4, 41, want_sumsq=True)
    m = sc.render(16, 16, spp, 4, 42, want_sumsq=True, mis=True)
    # image means of independent pixels: sigma = sqrt(sum of pixel variances) / npix
    # (pixels that see the light edge dominate it)
    sa = np.sqrt((_sigma(a, spp) ** 2).sum(axis=0)) / 256
    sm = np.sqrt((_sigma(m, spp) ** 2).sum(axis=0)) / 256
    da = a["rgb"].mean(axis=0) - m["rgb"].mean(axis=0)
    assert np.all(np.abs(da) < 3 * np.hypot(sa, sm)), (da, sa, sm)
    assert np.array_equal(a["aux"], sc.render(16, 16, spp, 4, 41, mis=True)["aux"])


def test_render_threads_and_subset_consistent(oracle_tracer):
    sc = oracle_tracer.OracleScene(S.cornell(2))
    full = sc.render(16, 16, 4, 4, 1002, nthreads=4)
    one = sc.render(16, 16, 4, 4, 1002, nthreads=1)
    assert np.array_equal(full["rgb"], one["rgb"])
    pix = np.array([0, 17, 100, 255])
    sub = sc.render(16, 16, 4, 4, 1002, pixels=pix)
    assert np.array_equal(sub["rgb"], full["rgb"][pix])
    assert np.array_equal(sub["aux"], full["aux"][pix])
    bf = sc.render(16, 16, 4, 4, 1002, use_bvh=False)
    assert np.array_equal(bf["rgb"], full["rgb"])


# --------------------------------------------------------------------------- render layers
# Sec. 3.1, Eqs. 1-2: the image is the sum of its layers.  Here: the emission
# seen at the first vertex (emitters, or the environment for a camera ray that
# misses), then the rest of each sample's radiance filed under the lobe of its
# first vertex, diffuse (Lambert) or glossy (GGX).


def test_layers_env_only_is_all_emission(oracle_tracer):
    scene = S.env_only((0.3, 0.5, 0.7))
    r = oracle_tracer.OracleScene(scene).render(8, 4, 4, 8, 42, want_layers=True)
    lay = r["layers"]
    assert np.array_equal(lay[:, 0:3], np.tile(scene.env.astype(np.float64), (32, 1)))
    assert np.all(lay[:, 3:] == 0)


@pytest.mark.parametrize("max_depth", [1, 3])
def test_layers_lambert_plane_all_diffuse(oracle_tracer, max_depth):
    scene = S.lambert_plane()
    r = oracle_tracer.OracleScene(scene).render(8, 8, 8, max_depth, 3, want_layers=True)
    want = scene.materials[0]["color"].astype(np.float64) * scene.env.astype(np.float64)
    lay = r["layers"]
    assert np.all(lay[:, 0:3] == 0) and np.all(lay[:, 6:9] == 0)
    assert np.allclose(lay[:, 3:6], want[None], rtol=1e-14, atol=0)


@pytest.mark.parametrize("max_depth", [0, 1, 3])
def test_layers_furnace_splits_emission_from_bounces(oracle_tracer, max_depth):
    # emitting Lambert sphere seen from inside: E directly, E sum_{k=1..D} rho^k after
    E, rho = 1.5, 0.6
    scene = S.furnace_sphere(E, rho, subdiv=2)
    r = oracle_tracer.OracleScene(scene).render(4, 4, 8, max_depth, 5, rr_start=100,
                                                want_layers=True)
    E32 = float(scene.materials[0]["emission"][0])
    rho32 = float(scene.materials[0]["color"][0])
    lay = r["layers"]
    assert np.all(lay[:, 0:3] == E32)
    assert np.allclose(lay[:, 3:6], E32 * sum(rho32 ** k for k in range(1, max_depth + 1)),
                       rtol=1e-12, atol=0)
    assert np.all(lay[:, 6:9] == 0)


def test_layers_ggx_plane_all_glossy(oracle_tracer):
    scene = _ggx_plane_scene(0.4, (0.9, 0.6, 0.3), 0.6, (1.0, 1.0, 1.0))
    r = oracle_tracer.OracleScene(scene).render(2, 2, 64, 2, 11, want_layers=True)
    lay = r["layers"]
    assert np.all(lay[:, 0:6] == 0)
    assert np.allclose(lay[:, 6:9], r["rgb"], rtol=1e-12, atol=0)
    assert np.all(lay[:, 6:9] > 0)


def test_layers_front_light_is_emission(oracle_tracer):
    b = S._Builder()
    b.add_light((-1.0, 1.0, -1.0), (2.0, 0, 0), (0, 0, 2.0), (5.0, 5.0, 5.0))
    cam = S.Camera((0.0, -2.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 10.0)
    r = oracle_tracer.OracleScene(b.build((0.0, 0.0, 0.0), cam, "front")).render(
        4, 4, 4, 3, 1, want_layers=True)
    assert np.all(r["layers"][:, 0:3] == 5.0) and np.all(r["layers"][:, 3:] == 0)


@pytest.mark.parametrize("mis", [False, True])
def test_layers_sum_to_image_on_mixed_scene(oracle_tracer, mis):
    # Lambert and GGX objects, quad lights, the environment seen past them
    sc = oracle_tracer.OracleScene(S.procedural(7))
    r = sc.render(24, 16, 4, 4, 77, want_layers=True, mis=mis)
    lay = r["layers"]
    total = lay[:, 0:3] + lay[:, 3:6] + lay[:, 6:9]
    assert np.allclose(total, r["rgb"], rtol=1e-12, atol=1e-14)
    assert np.all(lay >= 0)
    for k in range(3):
        assert lay[:, 3 * k:3 * k + 3].max() > 0, k  # every layer holds something
    # same paths as without layers
    assert np.array_equal(sc.render(24, 16, 4, 4, 77, mis=mis)["rgb"], r["rgb"])
