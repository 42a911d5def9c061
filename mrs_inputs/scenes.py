"""Seeded synthetic scene generators.

These produce the inputs shared by the GPU renderer and the FP64 reference
renderer: triangle soups with per-corner shading normals, a material table,
quad area lights, a constant environment and a pinhole camera.  Nothing here
computes light transport; the module only builds geometry and draws scene
parameters from numpy's seeded PCG64 generator.

The paper renders Blender community scenes with Cycles (Sec. 3.1, 3.2); those
assets are not available, so procedural scenes with the same kind of content
(closed rooms, curved displaced objects, boxes, area lights, an environment)
stand in for them.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

# Material kinds (mirrors the C ABI enum mrs_material_kind).
LAMBERT = 0
GGX = 1
EMITTER = 2  # pure emitter: no BSDF, the path ends on it

# Per-triangle flags.
FLAG_SMOOTH = 1  # use the interpolated per-corner normals for shading

MATERIAL_DTYPE = np.dtype(
    [("kind", "<i4"), ("color", "<f4", (3,)), ("alpha", "<f4"), ("emission", "<f4", (3,))],
    align=True,
)
LIGHT_DTYPE = np.dtype(
    [
        ("corner", "<f4", (3,)),
        ("edge_u", "<f4", (3,)),
        ("edge_v", "<f4", (3,)),
        ("emission", "<f4", (3,)),
        ("tri", "<i4", (2,)),
    ],
    align=True,
)
assert MATERIAL_DTYPE.itemsize == 32
assert LIGHT_DTYPE.itemsize == 56


@dataclass
class Camera:
    pos: tuple
    look_at: tuple
    up: tuple = (0.0, 1.0, 0.0)
    vfov_deg: float = 40.0


@dataclass
class Scene:
    vertices: np.ndarray  # float32 [N, 3, 3]  (triangle, corner, xyz)
    normals: np.ndarray  # float32 [N, 3, 3]  per-corner shading normals
    tri_material: np.ndarray  # uint32 [N]
    tri_flags: np.ndarray  # uint32 [N]
    materials: np.ndarray  # MATERIAL_DTYPE [M]
    lights: np.ndarray  # LIGHT_DTYPE [L]
    env: np.ndarray  # float32 [3]
    camera: Camera
    name: str = "scene"
    meta: dict = field(default_factory=dict)

    @property
    def num_tris(self) -> int:
        return int(self.vertices.shape[0])

    def content_hash(self) -> str:
        h = hashlib.sha256()
        for a in (self.vertices, self.normals, self.tri_material, self.tri_flags,
                  self.materials, self.lights, self.env):
            h.update(np.ascontiguousarray(a).tobytes())
        c = self.camera
        h.update(np.asarray(list(c.pos) + list(c.look_at) + list(c.up) + [c.vfov_deg],
                            dtype=np.float32).tobytes())
        return h.hexdigest()


class _Builder:
    """Accumulates triangles, materials and lights."""

    def __init__(self):
        self.v, self.n, self.m, self.f = [], [], [], []
        self.mats = []
        self.lights = []

    def material(self, kind, color=(0, 0, 0), alpha=0.0, emission=(0, 0, 0)) -> int:
        self.mats.append((kind, tuple(float(x) for x in color), float(alpha),
                          tuple(float(x) for x in emission)))
        return len(self.mats) - 1

    @property
    def ntris(self):
        return sum(len(x) for x in self.v)

    def add_tris(self, verts, mat, normals=None):
        """Append triangles; `mat` is one material index or one per triangle."""
        verts = np.asarray(verts, dtype=np.float32).reshape(-1, 3, 3)
        first = self.ntris
        self.v.append(verts)
        if normals is None:
            self.n.append(np.zeros_like(verts))
            self.f.append(np.zeros(len(verts), np.uint32))
        else:
            self.n.append(np.asarray(normals, np.float32).reshape(-1, 3, 3))
            self.f.append(np.full(len(verts), FLAG_SMOOTH, np.uint32))
        self.m.append(np.broadcast_to(np.asarray(mat, np.uint32), (len(verts),)).copy())
        return first

    def add_grid(self, corner, eu, ev, nu, nv, mats):
        """nu x nv quads tiling the parallelogram, materials in a checkerboard."""
        c = np.asarray(corner, np.float64)
        eu = np.asarray(eu, np.float64) / nu
        ev = np.asarray(ev, np.float64) / nv
        tris, ms = [], []
        for i in range(nu):
            for j in range(nv):
                q = c + i * eu + j * ev
                tris += [[q, q + eu, q + eu + ev], [q, q + eu + ev, q + ev]]
                ms += [mats[(i + j) % len(mats)]] * 2
        return self.add_tris(np.array(tris), np.array(ms))

    def add_box_grid(self, center, size, yaw, mats, n=2):
        """Box rotated by `yaw` about +y, each face an n x n checkerboard, outward winding."""
        sx, sy, sz = (0.5 * float(v) for v in size)
        faces = [((sx, -sy, -sz), (0, 2 * sy, 0), (0, 0, 2 * sz)),
                 ((-sx, -sy, -sz), (0, 0, 2 * sz), (0, 2 * sy, 0)),
                 ((-sx, sy, -sz), (0, 0, 2 * sz), (2 * sx, 0, 0)),
                 ((-sx, -sy, -sz), (2 * sx, 0, 0), (0, 0, 2 * sz)),
                 ((-sx, -sy, sz), (2 * sx, 0, 0), (0, 2 * sy, 0)),
                 ((-sx, -sy, -sz), (0, 2 * sy, 0), (2 * sx, 0, 0))]
        cy, sn = np.cos(yaw), np.sin(yaw)
        rot = np.array([[cy, 0, sn], [0, 1, 0], [-sn, 0, cy]])
        ctr = np.asarray(center, np.float64)
        first = self.ntris
        for corner, eu, ev in faces:
            self.add_grid(rot @ np.asarray(corner, np.float64) + ctr, rot @ np.asarray(eu, np.float64),
                          rot @ np.asarray(ev, np.float64), n, n, mats)
        return first

    def add_quad(self, corner, eu, ev, mat):
        """Two triangles (c, c+eu, c+eu+ev), (c, c+eu+ev, c+ev); front face along eu x ev."""
        c = np.asarray(corner, np.float64)
        eu = np.asarray(eu, np.float64)
        ev = np.asarray(ev, np.float64)
        t = np.array([[c, c + eu, c + eu + ev], [c, c + eu + ev, c + ev]])
        return self.add_tris(t, mat)

    def add_light(self, corner, eu, ev, emission):
        mat = self.material(EMITTER, emission=emission)
        # Store the light exactly as the float32 values of its geometry.
        c32 = np.asarray(corner, np.float32)
        eu32 = np.asarray(eu, np.float32)
        ev32 = np.asarray(ev, np.float32)
        t0 = self.add_quad(c32, eu32, ev32, mat)
        self.lights.append((c32, eu32, ev32, np.asarray(emission, np.float32), (t0, t0 + 1)))
        return mat

    def add_box(self, center, size, yaw, mat, outward=True):
        """Axis box of `size` rotated by `yaw` radians about +y, 12 triangles."""
        sx, sy, sz = (0.5 * float(s) for s in size)
        corners = np.array([[x, y, z] for x in (-sx, sx) for y in (-sy, sy) for z in (-sz, sz)])
        cy, sn = np.cos(yaw), np.sin(yaw)
        rot = np.array([[cy, 0, sn], [0, 1, 0], [-sn, 0, cy]])
        P = corners @ rot.T + np.asarray(center, np.float64)
        # index = 4*ix + 2*iy + iz
        faces = [
            (0, 1, 3, 2),  # -x
            (4, 6, 7, 5),  # +x
            (0, 4, 5, 1),  # -y
            (2, 3, 7, 6),  # +y
            (0, 2, 6, 4),  # -z
            (1, 5, 7, 3),  # +z
        ]
        tris = []
        for a, b, c, d in faces:
            quad = [(a, b, c), (a, c, d)]
            for tri in quad:
                t = P[list(tri)]
                if not outward:
                    t = t[[0, 2, 1]]
                tris.append(t)
        tris = np.array(tris)
        # make the winding outward (or inward) by checking against the centre
        ctr = np.asarray(center, np.float64)
        for i in range(len(tris)):
            ng = np.cross(tris[i, 1] - tris[i, 0], tris[i, 2] - tris[i, 0])
            out = np.dot(ng, tris[i].mean(0) - ctr) > 0
            if out != outward:
                tris[i] = tris[i][[0, 2, 1]]
        return self.add_tris(tris, mat)

    def build(self, env, camera, name, meta=None) -> Scene:
        if self.v:
            V = np.concatenate(self.v).astype(np.float32)
            N = np.concatenate(self.n).astype(np.float32)
            M = np.concatenate(self.m).astype(np.uint32)
            F = np.concatenate(self.f).astype(np.uint32)
        else:
            V = np.zeros((0, 3, 3), np.float32)
            N = np.zeros((0, 3, 3), np.float32)
            M = np.zeros((0,), np.uint32)
            F = np.zeros((0,), np.uint32)
        mats = np.zeros(max(len(self.mats), 0), MATERIAL_DTYPE)
        for i, (k, col, a, e) in enumerate(self.mats):
            mats[i]["kind"] = k
            mats[i]["color"] = col
            mats[i]["alpha"] = a
            mats[i]["emission"] = e
        lights = np.zeros(len(self.lights), LIGHT_DTYPE)
        for i, (c, eu, ev, le, tri) in enumerate(self.lights):
            lights[i]["corner"] = c
            lights[i]["edge_u"] = eu
            lights[i]["edge_v"] = ev
            lights[i]["emission"] = le
            lights[i]["tri"] = tri
        return Scene(V, N, M, F, mats, lights, np.asarray(env, np.float32), camera, name,
                     meta or {})


# --------------------------------------------------------------------------- icospheres

def icosphere(subdiv: int):
    """Unit icosphere: (vertices [V,3] float64, faces [F,3] int64), outward winding."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    for _ in range(subdiv):
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        edges = np.stack([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)], 1)
        es = np.sort(edges.reshape(-1, 2), axis=1)
        uniq, inv = np.unique(es, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = V[uniq[:, 0]] + V[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(V)
        V = np.concatenate([V, mid])
        m = (inv + base).reshape(-1, 3)
        mab, mbc, mca = m[:, 0], m[:, 1], m[:, 2]
        F = np.concatenate([
            np.stack([a, mab, mca], 1),
            np.stack([b, mbc, mab], 1),
            np.stack([c, mca, mbc], 1),
            np.stack([mab, mbc, mca], 1),
        ])
    # ensure outward winding
    ng = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("ij,ij->i", ng, V[F].mean(1)) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def vertex_normals(V, F):
    """Area-weighted vertex normals of an indexed mesh (float64, unit length)."""
    ng = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    acc = np.zeros_like(V)
    for k in range(3):
        np.add.at(acc, F[:, k], ng)
    return acc / np.linalg.norm(acc, axis=1, keepdims=True)


def _displaced_sphere(rng, subdiv, radius, center_xz):
    V, F = icosphere(subdiv)
    k = rng.uniform(2.0, 4.0, 3)
    ph = rng.uniform(0.0, 2.0 * np.pi, 3)
    disp = 0.15 * radius * np.prod(np.sin(k[None, :] * V + ph[None, :]), axis=1)
    P = V * radius + V * disp[:, None]
    P[:, 1] -= P[:, 1].min()  # rest on the ground y = 0
    P[:, 0] += center_xz[0]
    P[:, 2] += center_xz[1]
    N = vertex_normals(P, F)
    return P[F], N[F]


def _random_material(rng, b: _Builder):
    if rng.uniform() < 0.5:
        return b.material(LAMBERT, color=rng.uniform(0.2, 0.8, 3))
    return b.material(GGX, color=rng.uniform(0.5, 0.95, 3), alpha=rng.uniform(0.05, 0.8))


def _material_pair(rng, b: _Builder):
    """Two materials of one kind with different colours: the two 'texture' tones of an
    object (Lambert albedo U[0.2, 0.8]^3, or GGX F0 U[0.5, 0.95]^3 and roughness
    U[0.05, 0.8] shared by both tones)."""
    if rng.uniform() < 0.5:
        return [b.material(LAMBERT, color=rng.uniform(0.2, 0.8, 3)) for _ in range(2)]
    alpha = rng.uniform(0.05, 0.8)
    return [b.material(GGX, color=rng.uniform(0.5, 0.95, 3), alpha=alpha) for _ in range(2)]


def _sphere_pattern(rng, P, F):
    """Per-triangle tone (0/1) of a displaced sphere: a product-of-sines pattern of
    the centroid direction, giving blotches a few triangles to a few dozen wide."""
    u = P[F].mean(1)
    u = u - u.mean(0)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    k = rng.uniform(4.0, 9.0, 3)
    ph = rng.uniform(0.0, 2 * np.pi, 3)
    return (np.prod(np.sin(k[None] * u + ph[None]), axis=1) > 0.1).astype(np.int64)


# --------------------------------------------------------------------------- named scenes

def cornell(seed: int = 1) -> Scene:
    """Cornell-style box: 5 walls (10 tris), two boxes (24 tris), one quad light (2 tris).

    Lambertian albedo is drawn per object and channel from U[0.2, 0.8]; the light
    has emission 15.  36 triangles in total.
    """
    rng = np.random.default_rng(seed)
    b = _Builder()
    walls = [
        # floor y=0 (normal +y), ceiling y=1 (-y), back z=1 (-z), left x=0 (+x), right x=1 (-x)
        ((0, 0, 0), (0, 0, 1), (1, 0, 0)),
        ((0, 1, 0), (1, 0, 0), (0, 0, 1)),
        ((0, 0, 1), (0, 1, 0), (1, 0, 0)),
        ((0, 0, 0), (0, 1, 0), (0, 0, 1)),
        ((1, 0, 0), (0, 0, 1), (0, 1, 0)),
    ]
    for c, eu, ev in walls:
        b.add_quad(c, eu, ev, b.material(LAMBERT, color=rng.uniform(0.2, 0.8, 3)))
    b.add_box((0.68, 0.15, 0.32), (0.3, 0.3, 0.3), np.deg2rad(-18.0),
              b.material(LAMBERT, color=rng.uniform(0.2, 0.8, 3)))
    b.add_box((0.32, 0.30, 0.62), (0.3, 0.6, 0.3), np.deg2rad(18.0),
              b.material(LAMBERT, color=rng.uniform(0.2, 0.8, 3)))
    b.add_light((0.375, 0.999, 0.375), (0.25, 0.0, 0.0), (0.0, 0.0, 0.25), (15.0, 15.0, 15.0))
    cam = Camera((0.5, 0.5, -1.2), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 40.0)
    return b.build((0.0, 0.0, 0.0), cam, f"cornell_{seed}", {"seed": seed})


def procedural(seed: int = 7, spheres=((4, 5), (3, 4)), n_boxes: int = 20,
               n_lights: int = 3, env: float = 0.2, random_camera: bool = False) -> Scene:
    """Ground plane, displaced icospheres, boxes and quad lights.

    `spheres` lists (count, subdivision level) groups.  The defaults give
    3,200 + 4*20,480 + 3*5,120 + 20*48 + 3*2 = 101,446 triangles.  Each non-light
    object is Lambertian (albedo U[0.2, 0.8]^3) or GGX (F0 U[0.5, 0.95]^3,
    roughness U[0.05, 0.8]) with probability 1/2, in two tones laid out as a
    texture: a checkerboard on the ground and on box faces (2 x 2 per face), a
    blotch pattern on the spheres.
    """
    rng = np.random.default_rng(seed)
    b = _Builder()
    # ground: 40 x 40 checkerboard tiles of 1 x 1 (3,200 triangles)
    b.add_grid((-20.0, 0.0, -20.0), (0.0, 0.0, 40.0), (40.0, 0.0, 0.0), 40, 40,
               _material_pair(rng, b))
    for count, subdiv in spheres:
        for _ in range(count):
            r = rng.uniform(0.5, 1.5)
            cxz = rng.uniform(-4.0, 4.0, 2)
            P, N = _displaced_sphere(rng, subdiv, r, cxz)
            mats = np.asarray(_material_pair(rng, b))
            V, F = icosphere(subdiv)
            b.add_tris(P, mats[_sphere_pattern(rng, V, F)], normals=N)
    for _ in range(n_boxes):
        size = rng.uniform(0.2, 1.0, 3)
        cxz = rng.uniform(-4.0, 4.0, 2)
        b.add_box_grid((cxz[0], size[1] / 2, cxz[1]), size, rng.uniform(0, 2 * np.pi),
                       _material_pair(rng, b))
    for _ in range(n_lights):
        a, w = rng.uniform(0.5, 1.5, 2)
        h = rng.uniform(4.0, 6.0)
        cxz = rng.uniform(-3.0, 3.0, 2)
        inten = rng.uniform(10.0, 30.0)
        col = rng.uniform(0.8, 1.0, 3)
        b.add_light((cxz[0] - a / 2, h, cxz[1] - w / 2), (a, 0, 0), (0, 0, w), inten * col)
    cam = Camera((0.0, 3.0, 10.0), (0.0, 0.8, 0.0), (0.0, 1.0, 0.0), 40.0)
    if random_camera:  # orbit the scene: azimuth, elevation and distance from the seed
        az = rng.uniform(0, 2 * np.pi)
        el = rng.uniform(0.15, 0.6)
        dist = rng.uniform(7.0, 11.0)
        pos = (dist * np.cos(el) * np.sin(az), dist * np.sin(el) + 0.5, dist * np.cos(el) * np.cos(az))
        cam = Camera(tuple(float(v) for v in pos), (0.0, 0.8, 0.0), (0.0, 1.0, 0.0),
                     float(rng.uniform(35.0, 50.0)))
    return b.build((env, env, env), cam, f"procedural_{seed}", {"seed": seed})


def sphere_plan(target_tris: int):
    """(count, level) groups whose icosphere triangles approximate `target_tris`."""
    budget = max(int(target_tris) - 3200 - 20 * 48 - 3 * 2, 320)
    plan = []
    for level in (7, 6, 5, 4, 3, 2):
        nt = 20 * 4 ** level
        c = 0
        while budget >= nt and c < 6:
            c += 1
            budget -= nt
        if c:
            plan.append((c, level))
    return tuple(plan) or ((1, 2),)


def procedural_sized(seed: int, target_tris: int, random_camera: bool = True) -> Scene:
    """Procedural scene whose triangle count approximates `target_tris`."""
    sc = procedural(seed, spheres=sphere_plan(target_tris), random_camera=random_camera)
    sc.name = f"procedural_sized_{seed}_{target_tris}"
    sc.meta = {"seed": seed, "target_tris": int(target_tris)}
    return sc


def furnace_sphere(emission: float = 1.0, rho: float = 0.5, subdiv: int = 2) -> Scene:
    """Closed, inward-facing flat-shaded sphere of emissive Lambertian triangles.

    The emitters are not in the light list, so they are found only by BSDF rays.
    The camera sits at the centre.
    """
    V, F = icosphere(subdiv)
    tris = V[F][:, [0, 2, 1]] * 2.0  # flip the winding: front faces look inward
    b = _Builder()
    m = b.material(LAMBERT, color=(rho, rho, rho), emission=(emission, emission, emission))
    b.add_tris(tris, m)
    cam = Camera((0.1, -0.05, 0.07), (0.3, 0.2, 1.0), (0.0, 1.0, 0.0), 60.0)
    return b.build((0.0, 0.0, 0.0), cam, "furnace", {"E": emission, "rho": rho})


def env_only(env=(0.3, 0.5, 0.7)) -> Scene:
    """No geometry at all: every camera ray misses."""
    b = _Builder()
    cam = Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 50.0)
    return b.build(env, cam, "env_only")


def lambert_plane(rho=(0.25, 0.5, 0.75), env=(1.0, 0.5, 0.25)) -> Scene:
    """A large Lambertian plane under a constant environment, seen from above."""
    b = _Builder()
    b.add_quad((-1000.0, 0.0, -1000.0), (0.0, 0.0, 2000.0), (2000.0, 0.0, 0.0),
               b.material(LAMBERT, color=rho))
    cam = Camera((0.0, 1.0, 0.0), (0.0, 0.0, 0.5), (0.0, 1.0, 0.0), 60.0)
    return b.build(env, cam, "lambert_plane")


def nee_config(rho=0.5, le=10.0, a=1.0, bb=2.0, c=1.5) -> Scene:
    """Floor plus a parallel a x bb rectangular light at height c, one corner above the origin.

    The camera looks straight down at the origin with a tiny field of view.
    """
    b = _Builder()
    b.add_quad((-50.0, 0.0, -50.0), (0.0, 0.0, 100.0), (100.0, 0.0, 0.0),
               b.material(LAMBERT, color=(rho, rho, rho)))
    b.add_light((0.0, c, 0.0), (a, 0.0, 0.0), (0.0, 0.0, bb), (le, le, le))
    cam = Camera((0.0, c * 0.5, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0.01)
    return b.build((0.0, 0.0, 0.0), cam, "nee_config",
                   {"rho": rho, "le": le, "a": a, "b": bb, "c": c})


def glossy_lights(alpha: float = 0.05) -> Scene:
    """A glossy GGX floor (roughness alpha) under three quad lights of different
    sizes, seen at a grazing angle: the floor mirrors the lights, the case where
    light sampling alone is noisy (the MIS comparison scene)."""
    b = _Builder()
    b.add_quad((-20.0, 0.0, -20.0), (0.0, 0.0, 40.0), (40.0, 0.0, 0.0),
               b.material(GGX, color=(0.9, 0.85, 0.8), alpha=alpha))
    for x, size, le in ((-2.0, 0.4, 40.0), (0.0, 1.0, 8.0), (2.5, 2.0, 2.0)):
        b.add_light((x - size / 2, 2.0, 4.0 - size / 2), (size, 0.0, 0.0), (0.0, 0.0, size),
                    (le, le, le))
    cam = Camera((0.0, 1.0, -4.0), (0.0, 0.3, 2.0), (0.0, 1.0, 0.0), 50.0)
    return b.build((0.05, 0.05, 0.05), cam, f"glossy_lights_{alpha}")


def random_soup(seed: int, n: int, spread: float = 1.0) -> Scene:
    """Random triangles in a cube (intersection / BVH tests)."""
    rng = np.random.default_rng(seed)
    b = _Builder()
    centers = rng.uniform(-spread, spread, (n, 1, 3))
    tris = centers + rng.normal(0, 0.2 * spread, (n, 3, 3))
    m = b.material(LAMBERT, color=(0.5, 0.5, 0.5))
    b.add_tris(tris, m)
    cam = Camera((0.0, 0.0, -4.0 * spread), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 45.0)
    return b.build((0.1, 0.1, 0.1), cam, f"soup_{seed}_{n}")


def random_rays(seed: int, n: int, spread: float = 1.0):
    """Random float32 rays: origins in a cube of side 4*spread, aimed at points of the
    central cube of side 2*spread (where random_soup puts its triangles)."""
    rng = np.random.default_rng(seed + 12345)
    o = rng.uniform(-2 * spread, 2 * spread, (n, 3))
    tgt = rng.uniform(-spread, spread, (n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def training_scene_specs(first_seed: int, count: int, tri_lo: int = 10_000, tri_hi: int = 200_000):
    """(seed, triangle budget) pairs, budgets log-uniform in [tri_lo, tri_hi]."""
    rng = np.random.default_rng(first_seed * 7919 + count)
    logs = rng.uniform(np.log(tri_lo), np.log(tri_hi), count)
    return [(first_seed + i, int(np.exp(v))) for i, v in enumerate(logs)]


def training_windows(seed: int, count: int, W: int = 1280, H: int = 720, size: int = 128):
    """`count` window origins (x0, y0), multiples of 4, of size x size windows in W x H."""
    rng = np.random.default_rng(seed + 99_991)
    xs = rng.integers(0, (W - size) // 4 + 1, count) * 4
    ys = rng.integers(0, (H - size) // 4 + 1, count) * 4
    return list(zip(xs.tolist(), ys.tolist()))


def batch_specs(first_seed: int = 500, count: int = 32):
    """Uneven render+fuse jobs: (scene seed, triangle budget, W, H, HRLS spp, LRHS spp).

    W x H between 256 x 256 and 1920 x 1080 (multiples of 8), triangle budgets
    log-uniform in [10k, 1M], HRLS 1..8 spp, LRHS 16..128 spp at W/4 x H/4."""
    rng = np.random.default_rng(first_seed * 104_729 + count)
    out = []
    for i in range(count):
        tris = int(np.exp(rng.uniform(np.log(1e4), np.log(1e6))))
        W = int(rng.integers(256 // 8, 1920 // 8 + 1)) * 8
        H = int(rng.integers(256 // 8, 1080 // 8 + 1)) * 8
        out.append((first_seed + i, tris, W, H, int(rng.integers(1, 9)), int(rng.integers(16, 129))))
    return out
