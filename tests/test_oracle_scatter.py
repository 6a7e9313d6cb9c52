"""Pins of the oracle's direction sampling and of the two rules that excuse GPU/oracle disagreements.

* The quasi-random walk (Section "Close-Range VPL Sampling", flow step (3), instant radiosity) scatters
  at every hit with a cosine-weighted direction about the face normal, and the quad light emits
  cosine-weighted directions about its normal.  In a closed box every ray hits, so the walk's own VPLs
  show the sampled directions: the cosine to the normal has mean 2/3 and mean square 1/2 (a
  uniform-hemisphere sampler gives 1/2 and 1/3), the azimuth is isotropic, and the share of directions
  reaching the opposite face is the point-to-parallel-rectangle form factor (a uniform-hemisphere sampler
  gives the solid angle over 2 pi instead: 0.128 against 0.239 from the floor's centre).
* oracle_grazing flags a pair iff moving one endpoint by delta along a coordinate axis flips its
  visibility: segments passing an occluder's edge within the band are flagged, segments through the
  interior, far outside, or through the shared edge of two triangles are not.
* oracle_gbuffer_edges flags a pixel iff tilting its ray changes the hit triangle: its flags on a
  two-triangle square facing the camera equal the analytic set of pixels within the tilt of the square's
  outline or its diagonal.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2203_11484_amd import scenes
from tests import helpers as H


def _ri(b, i):
    """Radical inverse of i in base b, exact."""
    f, r = Fraction(1, b), Fraction(0)
    while i > 0:
        r += f * (i % b)
        i //= b
        f /= b
    return r


# a generic rotation (unit quaternion), so that the faces' normals are not coordinate axes
_Q = np.array([0.8, 0.3, -0.4, 0.33])
_Q /= np.linalg.norm(_Q)


def _rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _box_walk(light, n_far, flags=None, extra_tri=None, rotate=False):
    tri = H.closed_box((0, 0, 0), (1, 1, 1), cells=2)
    fl = np.zeros(len(tri), np.uint8)
    if extra_tri is not None:
        tri = np.concatenate([tri, extra_tri])
        fl = np.concatenate([fl, flags])
    if rotate:
        R = _rot(_Q)
        tri = (tri.astype(np.float64) - 0.5) @ R.T + 0.5
        light = dict(light)
        light["pos"] = ((light["pos"].astype(np.float64) - 0.5) @ R.T + 0.5).astype(np.float32)
        for k in ("edge_u", "edge_v"):
            light[k] = (light[k].astype(np.float64) @ R.T).astype(np.float32)
    cam = scenes.make_camera((0.5, 0.5, 0.05), (0.5, 0.5, 1.0), (0, 1, 0), 60.0, 32, 32)
    params = scenes.default_params(k_near=0, n_far=n_far, d_near=0.0)
    alb = np.full((len(tri), 3), 0.5, np.float32)
    alb[fl == 1] = 0.0
    sc = H.scene_dict(tri, alb, flags=fl, light=light, camera=cam, params=params)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    return sc, S.generate(sc["camera"], sc["light"], sc["params"])


def _tangent_frame(n):
    """An orthonormal pair orthogonal to the unit vector n (any one: the moments below do not depend on it)."""
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.6 else np.array([0.0, 1.0, 0.0])
    t1 = a - np.dot(a, n) * n
    t1 /= np.linalg.norm(t1)
    return t1, np.cross(n, t1)


def _direction_moments(origins, normals, hits):
    """Cosine of each direction to its normal and its components along a tangent frame of the normal."""
    d = hits - origins
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    n = normals / np.linalg.norm(normals, axis=1, keepdims=True)
    c = np.einsum("ij,ij->i", d, n)
    ta = np.array([[np.dot(d[i], t) for t in _tangent_frame(n[i])] for i in range(len(d))])
    return c, ta


def _corner_ff(a, b, h):
    """Form factor from a differential area to a parallel a x b rectangle at height h, the foot of the
    normal at one corner of the rectangle (Howell's catalogue, C-11)."""
    A, B = a / h, b / h
    sa, sb = math.sqrt(1 + A * A), math.sqrt(1 + B * B)
    return (A / sa * math.atan(B / sa) + B / sb * math.atan(A / sb)) / (2 * math.pi)


def _ff_parallel_unit_square(px, pz, h):
    """Form factor from a point (px, pz) below the unit square [0,1]^2 at height h (four corner pieces)."""
    return sum(_corner_ff(a, b, h) for a in (px, 1 - px) for b in (pz, 1 - pz) if a > 0 and b > 0)


def test_ff_parallel_square_closed_forms():
    # centre of the floor to the ceiling of a unit cube: 4 corner pieces of 0.5 x 0.5 at height 1
    assert abs(_ff_parallel_unit_square(0.5, 0.5, 1.0) - 0.23938) < 1e-4
    # a point under a huge square sees all of the hemisphere
    assert abs(4 * _corner_ff(1e6, 1e6, 1.0) - 1.0) < 1e-5
    # reciprocity-free check against a brute-force cosine-weighted integral over the square
    n = 400
    g = (np.arange(n) + 0.5) / n
    X, Z = np.meshgrid(g - 0.2, g - 0.7)
    r2 = X * X + Z * Z + 0.8 ** 2
    brute = float((0.8 * 0.8 / (math.pi * r2 * r2)).sum() / (n * n))
    assert abs(_ff_parallel_unit_square(0.2, 0.7, 0.8) - brute) < 1e-4


def test_walk_scatter_is_cosine_weighted():
    """Every walk segment after the first leaves its hit point with a cosine-weighted direction."""
    sc, g = _box_walk(scenes.point_light((0.4, 0.55, 0.45), (1, 1, 1)), n_far=4500, rotate=True)
    assert g["stats"]["n_paths"] == 1500 and g["n"] == 4500
    src, dst = np.nonzero(g["bounce"] < 3)[0], np.nonzero(g["bounce"] > 1)[0]
    assert np.array_equal(g["path"][src], g["path"][dst]) and np.array_equal(g["bounce"][src] + 1, g["bounce"][dst])
    c, ta = _direction_moments(g["pos"][src], g["nrm"][src], g["pos"][dst])
    assert c.min() > 0.0, "a scattered direction leaves the hemisphere"
    assert abs(c.mean() - 2 / 3) < 5e-3, c.mean()
    assert abs((c * c).mean() - 1 / 2) < 5e-3, (c * c).mean()
    # isotropic azimuth: each tangential axis carries half of the mean square sin^2 = 1/2, and the two
    # are uncorrelated
    assert np.all(np.abs((ta * ta).mean(0) - 1 / 4) < 5e-3), (ta * ta).mean(0)
    assert abs((ta[:, 0] * ta[:, 1]).mean()) < 5e-3
    assert np.all(np.abs(ta.mean(0)) < 1e-2), ta.mean(0)


def test_walk_scatter_from_floor_reaches_ceiling_by_form_factor():
    """From the floor's bounce-1 points, the share of bounce-2 hits on the ceiling is the mean
    point-to-parallel-square form factor of those points."""
    sc, g = _box_walk(scenes.point_light((0.4, 0.55, 0.45), (1, 1, 1)), n_far=18000)
    b1 = np.nonzero(g["bounce"] == 1)[0]
    floor = b1[g["pos"][b1, 1] < 1e-6]
    nxt = floor + 1
    assert np.array_equal(g["bounce"][nxt], np.full(len(nxt), 2))
    on_ceiling = g["pos"][nxt, 1] > 1 - 1e-6
    expect = sum(_ff_parallel_unit_square(g["pos"][i, 0], g["pos"][i, 2], 1.0) for i in floor)
    got = int(on_ceiling.sum())
    assert len(floor) > 800
    assert abs(got - expect) < 0.05 * expect, (got, expect, len(floor))


def test_quad_light_emits_cosine_weighted():
    """The quad light's path i starts at corner + phi_2(i) edge_u + phi_3(i) edge_v and leaves along a
    cosine-weighted direction about the light's normal: its first hit shows both."""
    corner, eu, ev = (0.3, 0.999, 0.35), (0.4, 0.0, 0.0), (0.0, 0.0, 0.3)
    lt = scenes.quad_light(corner, eu, ev, (1, 1, 1))
    quad = scenes._quad_grid(corner, eu, ev, (0, -1, 0), 1, 1)
    for rotate in (False, True):
        sc, g = _box_walk(lt, n_far=4500, flags=np.ones(len(quad), np.uint8), extra_tri=quad, rotate=rotate)
        L = sc["light"]
        b1 = np.nonzero(g["bounce"] == 1)[0]
        u = L["edge_u"].astype(np.float64)
        v = L["edge_v"].astype(np.float64)
        n_l = np.cross(u, v)
        n_l /= np.linalg.norm(n_l)
        c0 = L["pos"].astype(np.float64)
        paths = g["path"][b1]
        org = np.array([c0 + float(_ri(2, int(p))) * u + float(_ri(3, int(p))) * v for p in paths])
        c, ta = _direction_moments(org, np.tile(n_l, (len(b1), 1)), g["pos"][b1])
        assert len(b1) > 1400 and c.min() > 0.0
        assert abs(c.mean() - 2 / 3) < 5e-3, c.mean()
        assert abs((c * c).mean() - 1 / 2) < 5e-3, (c * c).mean()
        assert np.all(np.abs((ta * ta).mean(0) - 1 / 4) < 5e-3), (ta * ta).mean(0)
        assert abs((ta[:, 0] * ta[:, 1]).mean()) < 5e-3
        if not rotate:
            # share of first hits on the floor: the mean form factor from the emission points to it
            on_floor = g["pos"][b1, 1] < 1e-6
            expect = sum(_ff_parallel_unit_square(o[0], o[2], o[1]) for o in org)
            assert abs(on_floor.sum() - expect) < 0.05 * expect, (on_floor.sum(), expect)


# ---------------------------------------------------------------------------
# the grazing rule


def _square_occluder(s=1.0, z=0.5, x0=0.0):
    A, B, C, D = (x0 - s, -s, z), (x0 + s, -s, z), (x0 + s, s, z), (x0 - s, s, z)
    return np.array([[A, B, C], [A, C, D]], np.float32)


@pytest.mark.parametrize("delta_rel", [1e-5, 1e-6, 1e-7])
def test_grazing_flags_only_pairs_within_the_band(delta_rel):
    """At the GPU parity protocol's band (1e-6 of the diagonal), a wider and a narrower one.  The square spans x in
    [-2, 0], so the points near its edge x = 0 are exact in float32 even 0.2 band widths from it."""
    tri = _square_occluder(x0=-1.0)
    S = orc.Scene(tri, np.full((2, 3), 0.5, np.float32), np.zeros(2, np.uint8), use_bvh=False)
    delta = delta_rel * S.diag
    # vertical segments z: 0 -> 1 crossing the occluder's plane at s = 1/2, where moving one endpoint
    # by delta along x moves the crossing by delta / 2
    xs = [(-1.0, 0.0, 0, 0),                     # interior: blocked, robust
          (0.5, 0.0, 1, 0),                      # far outside: visible, robust
          (0.2 * delta, 0.3, 1, 1),              # just outside the edge x = 0: flips
          (-0.2 * delta, 0.3, 0, 1),             # just inside: flips
          (3.0 * delta, 0.3, 1, 0),              # outside the band
          (-3.0 * delta, 0.3, 0, 0),             # inside, beyond the band
          (-0.75, 0.25 + 0.1 * delta, 0, 0),     # next to the shared diagonal: blocked either way
          (-0.75, 0.25, 0, 0)]                   # on the shared diagonal (watertight)
    x = np.array([[px, py, 0.0] for px, py, _, _ in xs], np.float32)
    y = np.array([[px, py, 1.0] for px, py, _, _ in xs], np.float32)
    # segments z: -8.5 -> 1 crossing at s = 0.947, where moving the far endpoint moves the crossing by
    # 0.947 delta and moving the near one by 0.053 delta: only the far endpoint can flip them
    ys = [(0.3 * delta, -0.2, 1, 1), (-0.3 * delta, -0.2, 0, 1)]
    xs += ys
    x = np.concatenate([x, np.array([[px, py, -8.5] for px, py, _, _ in ys], np.float32)])
    y = np.concatenate([y, np.array([[px, py, 1.0] for px, py, _, _ in ys], np.float32)])
    none = np.full(len(xs), -1, np.int32)
    vis = S.visibility(x, none, y, none)
    graz = S.grazing(x, none, y, none, delta_rel=delta_rel)
    assert vis.tolist() == [v for _, _, v, _ in xs]
    assert graz.tolist() == [g for _, _, _, g in xs]


@pytest.mark.parametrize("delta_rel", [1e-5, 1e-6, 1e-7])
def test_grazing_flags_crossings_at_the_segment_ends(delta_rel):
    """A crossing just inside the shadow segment's end range s > t_eps flips under the perturbation; one
    in the middle does not."""
    tri = _square_occluder(z=0.0)  # in the plane z = 0: the near endpoints z = -a are exact in float32
    S = orc.Scene(tri, np.full((2, 3), 0.5, np.float32), np.zeros(2, np.uint8), use_bvh=False)
    eps = 1e-4
    delta = delta_rel * S.diag
    cases = [(eps + 0.3 * delta, 0, 1), (eps - 0.3 * delta, 1, 1), (0.5, 0, 0), (eps + 3 * delta, 0, 0)]
    x = np.array([[0.1, 0.2, -a] for a, _, _ in cases], np.float32)
    y = x + np.array([0, 0, 1.0], np.float32)
    none = np.full(len(cases), -1, np.int32)
    assert S.visibility(x, none, y, none, eps=eps).tolist() == [v for _, v, _ in cases]
    assert S.grazing(x, none, y, none, eps=eps, delta_rel=delta_rel).tolist() == [g for _, _, g in cases]


# ---------------------------------------------------------------------------
# the G-buffer edge rule


def test_gbuffer_edges_match_the_analytic_band():
    """A square of two triangles at depth D facing the camera, turned by 0.3 rad in its plane so that the
    pixel centres sample every offset from its edges."""
    D, s, W, Hh, vfov, delta, ang = 2.0, 0.7, 256, 192, 60.0, 0.01, 0.3
    ca, sa = math.cos(ang), math.sin(ang)

    def world(x, y):
        return (ca * x - sa * y, sa * x + ca * y, D)

    A, B, C, Dd = world(-s, -s), world(s, -s), world(s, s), world(-s, s)
    tri = np.array([[A, B, C], [A, C, Dd]], np.float32)
    S = orc.Scene(tri, np.full((2, 3), 0.5, np.float32), np.zeros(2, np.uint8), use_bvh=False)
    cam = scenes.make_camera((0, 0, 0), (0, 0, 1), (0, 1, 0), vfov, W, Hh)
    flags = S.gbuffer_edges(cam, delta=delta).astype(bool)
    gb = S.gbuffer(cam)
    # camera basis: f = +z, r = f x up = -x, u = +y; the ray through pixel (i, j) is f + sx r + sy u and
    # meets the plane z = D at (-D sx, D sy); a tilt of delta |d| along r or u moves that point by
    # D delta |d| along x or y
    th = math.tan(math.radians(vfov) / 2)
    tx = th * W / Hh

    def local(X, Y):
        return ca * X + sa * Y, -sa * X + ca * Y

    def region(X, Y):
        x, y = local(X, Y)
        if abs(x) > s or abs(y) > s:
            return -1
        return 0 if y < x else 1

    def near_boundary(X, Y, tol=1e-7):
        x, y = local(X, Y)
        inside_ext = abs(x) <= s + tol and abs(y) <= s + tol
        return (inside_ext and (abs(abs(x) - s) < tol or abs(abs(y) - s) < tol)) or (inside_ext and abs(x - y) < tol)

    expect = np.zeros(W * Hh, bool)
    ambiguous = np.zeros(W * Hh, bool)
    for j in range(Hh):
        for i in range(W):
            sx = (2 * (i + 0.5) / W - 1) * tx
            sy = (1 - 2 * (j + 0.5) / Hh) * th
            X, Y = -D * sx, D * sy
            m = D * delta * math.sqrt(1 + sx * sx + sy * sy)
            pts = [(X, Y), (X + m, Y), (X - m, Y), (X, Y + m), (X, Y - m)]
            p = j * W + i
            ambiguous[p] = any(near_boundary(*q) for q in pts)
            expect[p] = any(region(*q) != region(X, Y) for q in pts[1:])
    ok = ~ambiguous
    assert ambiguous.sum() <= 4
    assert np.array_equal(flags[ok], expect[ok]), np.nonzero(flags[ok] != expect[ok])
    # the band is there and is narrow: outline and diagonal flagged, interior and outside not
    hit = gb["tri"] >= 0
    assert 0.05 < flags[hit].mean() < 0.5 and flags[~hit].mean() < 0.2
    assert (hit & ~flags).sum() > 2000 and (~hit & ~flags).sum() > 2000
