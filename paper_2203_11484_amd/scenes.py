"""Seeded synthetic inputs: scenes, cameras, lights and generation parameters.

This module builds the geometry that both the GPU path and the CPU oracle
consume.  It holds none of the method's arithmetic (no normals, areas, patch
refinement, visibility or shading): it only places triangles, draws albedos
and fixes the camera, light and parameter values of each workload.

The paper's own scenes (a desk, stone carvings with a tea set, a showcase;
all lit by point lights, Section "Results") are not available, so seeded
stand-ins with the same character are built here: a Cornell-style box with an
area light, and procedural rooms full of subdivided boxes and spheres with a
point light, many facets and mutual reflection.

Every array is float32 (vertices, albedo, camera, light) so that the GPU path
and the oracle read identical bytes.  A scene is a plain dict:

    tri     float32 [T, 3, 3]   vertices A, B, C; counter-clockwise seen from
                                the front side (one-sided faces)
    albedo  float32 [T, 3]      diffuse RGB albedo; 0 for emitters
    flags   uint8   [T]         bit 0 = emitter
    light   dict(kind=0 point | 1 quad, pos, edge_u, edge_v, power)  float32
    camera  dict(eye, target, up, vfov_deg, width, height)
    params  dict of generation / gather constants
"""
from __future__ import annotations

import math

import numpy as np

EMITTER = 1

# ---------------------------------------------------------------------------
# geometry builders (vertex placement only)
# ---------------------------------------------------------------------------


def _quad_grid(p0, u, v, front, nu, nv):
    """Triangles of a parallelogram p0 + s*u + t*v split into nu x nv cells.

    The winding is chosen so that the front side faces ``front``: if
    (u x v) points away from ``front`` the two edge vectors are swapped.
    Grid points are computed once so shared edges have identical floats.
    """
    p0 = np.asarray(p0, np.float64)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    if np.dot(np.cross(u, v), np.asarray(front, np.float64)) < 0:
        u, v = v, u
        nu, nv = nv, nu
    s = np.arange(nu + 1, dtype=np.float64) / nu
    t = np.arange(nv + 1, dtype=np.float64) / nv
    grid = (p0[None, None, :] + s[:, None, None] * u[None, None, :]
            + t[None, :, None] * v[None, None, :]).astype(np.float32)
    a = grid[:-1, :-1].reshape(-1, 3)
    b = grid[1:, :-1].reshape(-1, 3)
    c = grid[1:, 1:].reshape(-1, 3)
    d = grid[:-1, 1:].reshape(-1, 3)
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    return np.concatenate([t1, t2], axis=0)


def _rot_y(deg):
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _rot_uniform(rng):
    """Uniform random rotation (Shoemake 1992, unit quaternion from 3 uniforms)."""
    u1, u2, u3 = rng.random(3)
    q = np.array([
        math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
        math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
        math.sqrt(u1) * math.sin(2 * math.pi * u3),
        math.sqrt(u1) * math.cos(2 * math.pi * u3),
    ])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _box_faces(center, half, R, subdiv, skip_bottom=False):
    """Faces of an oriented box with outward fronts; one list entry per face."""
    center = np.asarray(center, np.float64)
    faces = []
    for axis in range(3):
        for sign in (-1.0, 1.0):
            if skip_bottom and axis == 1 and sign < 0:
                continue
            i, j = [k for k in range(3) if k != axis]
            e = np.zeros(3)
            e[axis] = sign * half[axis]
            ei = np.zeros(3)
            ei[i] = 2 * half[i]
            ej = np.zeros(3)
            ej[j] = 2 * half[j]
            fc = center + R @ e
            u = R @ ei
            v = R @ ej
            p0 = fc - 0.5 * u - 0.5 * v
            faces.append(_quad_grid(p0, u, v, R @ (e / half[axis]), subdiv, subdiv))
    return faces


def _icosphere(center, radius, level):
    """Icosphere of 20 * 4**level triangles, fronts facing outward."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.array(p, np.float64) / np.linalg.norm(p) for p in verts]
    cache = {}

    def mid(i, j):
        key = (min(i, j), max(i, j))
        if key not in cache:
            m = v[i] + v[j]
            v.append(m / np.linalg.norm(m))
            cache[key] = len(v) - 1
        return cache[key]

    for _ in range(level):
        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = (np.asarray(center, np.float64)[None, :] + radius * np.stack(v)).astype(np.float32)
    F = np.asarray(faces, np.int64)
    tri = V[F]
    # orient every triangle so that its front faces away from the centre
    a, b, c = (tri[:, k].astype(np.float64) for k in range(3))
    outward = np.einsum('ij,ij->i', np.cross(b - a, c - a), (a + b + c) / 3 - center)
    flip = outward < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


class _Builder:
    def __init__(self):
        self.tris, self.alb, self.flags = [], [], []

    def add(self, tris, albedo, flag=0):
        tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
        self.tris.append(tris)
        self.alb.append(np.broadcast_to(np.asarray(albedo, np.float32), (len(tris), 3)))
        self.flags.append(np.full(len(tris), flag, np.uint8))

    def arrays(self):
        return (np.ascontiguousarray(np.concatenate(self.tris)),
                np.ascontiguousarray(np.concatenate(self.alb)),
                np.ascontiguousarray(np.concatenate(self.flags)))


def _f32(x):
    return np.asarray(x, np.float32)


def make_camera(eye, target, up, vfov_deg, width, height):
    return dict(eye=_f32(eye), target=_f32(target), up=_f32(up),
                vfov_deg=float(np.float32(vfov_deg)), width=int(width), height=int(height))


def point_light(pos, power):
    return dict(kind=0, pos=_f32(pos), edge_u=_f32([0, 0, 0]), edge_v=_f32([0, 0, 0]),
                power=_f32(power))


def quad_light(corner, edge_u, edge_v, power):
    return dict(kind=1, pos=_f32(corner), edge_u=_f32(edge_u), edge_v=_f32(edge_v),
                power=_f32(power))


def default_params(**kw):
    p = dict(k_near=64, n_far=192, max_bounces=3, d_near=1.8, patch_h=0.1,
             g_clamp=10.0, t_eps=1e-4)
    p.update(kw)
    # cap on walk paths: 64 per VPL of the budget (reaching it is flagged)
    p.setdefault("max_paths", 64 * (p["k_near"] + p["n_far"]) + 1024)
    return p


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------


def cornell(seed=0, width=128, height=128, light="quad", **params):
    """Cornell-style box: 5 walls + 2 boxes (5 faces each) + 2 light triangles = 32.

    Unit room [0,1]^3 open at z = 0, one 0.25 x 0.25 one-sided quad light just
    below the ceiling facing down, per-face RGB albedo U[0.5, 0.8].
    light="point": the light-model ablation -- an isotropic point light of the
    same power at the quad's centre, lowered to y = 0.9 (one patch size below
    the ceiling) and without the emitter triangles (30 triangles).
    """
    rng = np.random.default_rng(seed)
    b = _Builder()
    walls = [  # (corner, u, v, front)
        ((0, 0, 0), (1, 0, 0), (0, 0, 1), (0, 1, 0)),    # floor y = 0
        ((0, 1, 0), (1, 0, 0), (0, 0, 1), (0, -1, 0)),   # ceiling y = 1
        ((0, 0, 1), (1, 0, 0), (0, 1, 0), (0, 0, -1)),   # back z = 1
        ((0, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 0)),    # left x = 0
        ((1, 0, 0), (0, 1, 0), (0, 0, 1), (-1, 0, 0)),   # right x = 1
    ]
    for p0, u, v, n in walls:
        b.add(_quad_grid(p0, u, v, n, 1, 1), rng.uniform(0.5, 0.8, 3))
    boxes = [((0.32, 0.15, 0.38), (0.15, 0.15, 0.15)),
             ((0.66, 0.30, 0.66), (0.14, 0.30, 0.14))]
    for c, h in boxes:
        R = _rot_y(rng.uniform(-25.0, 25.0))
        for face in _box_faces(c, np.asarray(h), R, 1, skip_bottom=True):
            b.add(face, rng.uniform(0.5, 0.8, 3))
    corner, eu, ev = (0.375, 0.999, 0.375), (0.25, 0, 0), (0, 0, 0.25)
    if light == "point":
        lt = point_light((0.5, 0.9, 0.5), (1, 1, 1))
    else:
        b.add(_quad_grid(corner, eu, ev, (0, -1, 0), 1, 1), (0, 0, 0), EMITTER)
        lt = quad_light(corner, eu, ev, (1, 1, 1))
    tri, alb, flags = b.arrays()
    return dict(name="cornell" if light != "point" else "cornell_point", tri=tri, albedo=alb, flags=flags,
                light=lt,
                camera=make_camera((0.5, 0.5, -1.0), (0.5, 0.5, 0.5), (0, 1, 0), 40.0, width, height),
                params=default_params(**params))


ROOM = (10.0, 3.0, 10.0)
ROOM_LIGHT = (5.0, 2.7, 5.0)
ROOM_EYE = (6.0, 1.6, 6.0)
ROOM_TARGET = (0.0, 0.8, 0.0)


def _room_walls(b, rng, cells, alb_lo, alb_hi):
    X, Y, Z = ROOM
    walls = [
        ((0, 0, 0), (X, 0, 0), (0, 0, Z), (0, 1, 0)),
        ((0, Y, 0), (X, 0, 0), (0, 0, Z), (0, -1, 0)),
        ((0, 0, 0), (X, 0, 0), (0, Y, 0), (0, 0, 1)),
        ((0, 0, Z), (X, 0, 0), (0, Y, 0), (0, 0, -1)),
        ((0, 0, 0), (0, Y, 0), (0, 0, Z), (1, 0, 0)),
        ((X, 0, 0), (0, Y, 0), (0, 0, Z), (-1, 0, 0)),
    ]
    for p0, u, v, n in walls:
        b.add(_quad_grid(p0, u, v, n, cells, cells), rng.uniform(alb_lo, alb_hi, 3))


def _place(rng, radius, avoid):
    """Uniform centre inside the room, at least `clear + radius` from each avoid point."""
    X, Y, Z = ROOM
    for _ in range(10000):
        c = np.array([rng.uniform(0.5, X - 0.5), rng.uniform(0.3, Y - 0.3), rng.uniform(0.5, Z - 0.5)])
        if all(np.linalg.norm(c - np.asarray(p)) >= clear + radius for p, clear in avoid):
            return c
    raise RuntimeError("could not place object")


def procedural_room(seed, n_boxes, box_subdiv, n_spheres, sphere_level, eye=ROOM_EYE,
                    target=ROOM_TARGET, vfov=60.0, width=512, height=512, name="room",
                    alb_lo=0.2, alb_hi=0.9, **params):
    """Closed 10 x 3 x 10 room (walls 15 x 15 quads) with boxes and spheres.

    The default camera frames the corner at the origin; with d_near = 7 its
    near region holds about 15% of the scene's surface area.

    Boxes: sizes U[0.3, 1.5]^3, uniform centres, uniform random rotations,
    every face subdivided box_subdiv^2 quads.  Spheres: icospheres of radius
    U[0.2, 0.8].  Objects keep >= 1 from the point light and >= 0.3 from the eye.
    """
    rng = np.random.default_rng(seed)
    b = _Builder()
    _room_walls(b, rng, 15, alb_lo, alb_hi)
    avoid = [(ROOM_LIGHT, 1.0), (tuple(eye), 0.3)]
    for _ in range(n_boxes):
        size = rng.uniform(0.3, 1.5, 3)
        half = size / 2
        R = _rot_uniform(rng)
        c = _place(rng, float(np.linalg.norm(half)), avoid)
        for face in _box_faces(c, half, R, box_subdiv):
            b.add(face, rng.uniform(alb_lo, alb_hi, 3))
    for _ in range(n_spheres):
        r = rng.uniform(0.2, 0.8)
        c = _place(rng, r, avoid)
        b.add(_icosphere(c, r, sphere_level), rng.uniform(alb_lo, alb_hi, 3))
    tri, alb, flags = b.arrays()
    return dict(name=name, tri=tri, albedo=alb, flags=flags,
                light=point_light(ROOM_LIGHT, (100, 100, 100)),
                camera=make_camera(eye, target, (0, 1, 0), vfov, width, height),
                params=default_params(**params))


def room20k(seed=1, width=512, height=512, **params):
    """About 20k triangles: 2,700 wall + 40 boxes x 6 faces x 6 x 6 x 2 = 19,980."""
    p = dict(k_near=2048, n_far=2048, d_near=7.0)
    p.update(params)
    return procedural_room(seed, 40, 6, 0, 0, width=width, height=height, name="room20k", **p)


def room200k(seed=2, width=1920, height=1080, **params):
    """About 200k triangles: walls + 60 boxes (8 x 8 faces) + 30 icospheres (level 4)."""
    p = dict(k_near=12288, n_far=4096, d_near=7.0)
    p.update(params)
    return procedural_room(seed, 60, 8, 30, 4, width=width, height=height, name="room200k", **p)


def cornell_point(**kw):
    """The Cornell box lit by an isotropic point light instead of the quad (light-model ablation)."""
    return cornell(light="point", **kw)


WORKLOADS = {"cornell": cornell, "cornell_point": cornell_point, "room20k": room20k, "room200k": room200k}


def make_scene(name, **kw):
    return WORKLOADS[name](**kw)


# ---------------------------------------------------------------------------
# batched views and served requests
# ---------------------------------------------------------------------------

RESOLUTIONS = ((256, 256), (512, 512), (1024, 1024), (1920, 1080))


def batch_scene(seed, n_tris):
    """Procedural room whose triangle count is close to n_tris (boxes 6x6, spheres level 3)."""
    rest = max(0, n_tris - 2700)
    n_box = max(1, int(round(0.4 * rest / 432)))
    n_sph = max(0, int(round(0.6 * rest / 1280)))
    return procedural_room(seed, n_box, 6, n_sph, 3, name=f"batch{seed}")


def batch_scenes(first_seed=100, count=8, seed=100):
    rng = np.random.default_rng(seed + 10_000)
    counts = np.exp(rng.uniform(math.log(5000), math.log(200000), count))
    return [batch_scene(first_seed + i, int(counts[i])) for i in range(count)]


def _view_camera(rng, scene, width, height):
    X, Y, Z = ROOM
    for _ in range(1000):
        cx, cz = rng.choice([0.0, X]), rng.choice([0.0, Z])
        target = np.array([cx, rng.uniform(0.3, 1.5), cz])
        dist = rng.uniform(2.5, 5.0)
        toward = np.array([X / 2 - cx, 0.0, Z / 2 - cz])
        toward /= np.linalg.norm(toward)
        ang = rng.uniform(-0.4, 0.4)
        ca, sa = math.cos(ang), math.sin(ang)
        toward = np.array([ca * toward[0] + sa * toward[2], 0.0, -sa * toward[0] + ca * toward[2]])
        eye = target + dist * toward
        eye[1] = rng.uniform(1.0, 2.5)
        # keep the eye clear of every object: no vertex within 0.3 of it
        if np.min(np.linalg.norm(scene["tri"].reshape(-1, 3) - eye[None, :].astype(np.float32), axis=1)) > 0.3:
            return make_camera(eye, target, (0, 1, 0), 60.0, width, height)
    raise RuntimeError("no camera found")


def batch_views(scenes, n_views=64, seed=200, m_lo=1024, m_hi=16384):
    """Views: scene uniform, camera looking at a room corner, resolution from RESOLUTIONS,
    VPL count log-uniform in [m_lo, m_hi] rounded to a multiple of 64, split 1:1."""
    rng = np.random.default_rng(seed)
    views = []
    for _ in range(n_views):
        si = int(rng.integers(len(scenes)))
        w, h = RESOLUTIONS[int(rng.integers(len(RESOLUTIONS)))]
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi))) / 64.0)) * 64
        m = max(64, m)
        cam = _view_camera(rng, scenes[si], w, h)
        views.append(dict(scene=si, camera=cam,
                          params=default_params(k_near=m // 2, n_far=m - m // 2, d_near=7.0)))
    return views
