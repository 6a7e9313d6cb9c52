"""Pins of the oracle's direct term L_e(y) of eq. (1) (light model of eq. (2)).

Closed forms: a point light over a plane (E = Phi h / (4 pi r^3)), the shadow of a square occluder
(similar triangles), Lambert's polygon irradiance for the quad light, plus the zero cases
(back-facing receiver, no hit) and exact linearity in the light power.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2203_11484_amd import scenes
from tests import helpers as H


def _floor_points(xs, zs, y=0.0):
    pts = np.array([[x, y, z] for x in xs for z in zs], np.float32)
    return pts


def _direct(S, pos, nrm, alb, tri, light):
    n = len(pos)
    return S.direct(pos, np.broadcast_to(np.asarray(nrm, np.float32), (n, 3)),
                    np.broadcast_to(np.asarray(alb, np.float32), (n, 3)), np.asarray(tri, np.int32), light)


def test_direct_point_light_over_plane():
    """L = (rho / pi) Phi h / (4 pi r^3) for a floor point under a point light at height h."""
    tri = H.floor_quad(-10, 10, -10, 10)
    sc = H.scene_dict(tri, 0.5)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    h = 2.0
    light = scenes.point_light((0.25, h, -0.5), (3.0, 5.0, 7.0))
    pts = _floor_points(np.linspace(-4, 4, 9), np.linspace(-3, 3, 7))
    L = _direct(S, pts, (0, 1, 0), (0.5, 0.25, 0.125), np.zeros(len(pts), np.int32), light)
    for i, p in enumerate(pts.astype(np.float64)):
        w = np.array([0.25, h, -0.5]) - p
        r = np.linalg.norm(w)
        E = h / (4.0 * math.pi * r ** 3)
        ref = np.array([0.5, 0.25, 0.125]) / math.pi * np.array([3.0, 5.0, 7.0]) * E
        assert np.allclose(L[i], ref, rtol=1e-12, atol=0)


def test_direct_square_occluder_shadow():
    """A square occluder of half-size s at height a under a point light at height h casts a square
    shadow of half-size s h / (h - a) on the floor: zero inside it, the closed form outside."""
    h, a, s = 3.0, 1.0, 0.5
    floor = H.floor_quad(-10, 10, -10, 10)
    occ = scenes._quad_grid((-s, a, -s), (2 * s, 0, 0), (0, 0, 2 * s), (0, -1, 0), 1, 1)
    tri = np.concatenate([floor, occ])
    sc = H.scene_dict(tri, 0.5)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    light = scenes.point_light((0, h, 0), (1, 1, 1))
    half = s * h / (h - a)  # 0.75
    inside = _floor_points(np.linspace(-0.7, 0.7, 5), np.linspace(-0.7, 0.7, 5))
    outside = _floor_points([-2.0, -0.8, 0.8, 2.0], [0.0, 1.5])
    Li = _direct(S, inside, (0, 1, 0), (1, 1, 1), np.zeros(len(inside), np.int32), light)
    Lo = _direct(S, outside, (0, 1, 0), (1, 1, 1), np.zeros(len(outside), np.int32), light)
    assert (Li == 0).all()
    for i, p in enumerate(outside.astype(np.float64)):
        assert max(abs(p[0]), abs(p[2])) > half
        r = np.linalg.norm(np.array([0, h, 0]) - p)
        assert np.allclose(Lo[i], 1 / math.pi * h / (4 * math.pi * r ** 3), rtol=1e-12, atol=0)


def _lambert_polygon_irradiance(poly, x, n, radiance):
    """E = (L / 2) sum_edges theta_e (n . g_e) (Lambert's formula), the sign making E >= 0."""
    E = 0.0
    m = len(poly)
    for i in range(m):
        a = poly[i] - x
        b = poly[(i + 1) % m] - x
        th = math.acos(np.clip(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)), -1, 1))
        g = np.cross(a, b)
        g /= np.linalg.norm(g)
        E += th * np.dot(n, g)
    return abs(0.5 * radiance * E)


def test_direct_quad_light_lambert_polygon():
    """Quad light (one-sided, radiance Phi / (pi A), facing down) over a floor: the 16-cell rule agrees
    with Lambert's polygon irradiance within its O((size / distance)^2) midpoint error."""
    tri = H.floor_quad(-10, 10, -10, 10)
    sc = H.scene_dict(tri, 1.0)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    corner, eu, ev = np.array([-0.25, 1.5, -0.25]), np.array([0.5, 0, 0]), np.array([0, 0, 0.5])
    light = scenes.quad_light(corner, eu, ev, (2.0, 2.0, 2.0))
    assert np.cross(eu, ev)[1] < 0  # the emitting side (edge_u x edge_v) faces the floor
    poly = [corner, corner + ev, corner + ev + eu, corner + eu]
    area = 0.25
    pts = _floor_points(np.linspace(-2, 2, 5), np.linspace(-2, 2, 5))
    L = _direct(S, pts, (0, 1, 0), (1, 1, 1), np.zeros(len(pts), np.int32), light)
    centre = corner + 0.5 * eu + 0.5 * ev
    for i, p in enumerate(pts.astype(np.float64)):
        E_ref = 2.0 * _lambert_polygon_irradiance(poly, p, np.array([0, 1.0, 0]), 1.0 / (math.pi * area))
        E = L[i, 0] * math.pi
        dist = np.linalg.norm(p - centre)
        assert abs(E - E_ref) <= 0.1 * (0.5 / dist) ** 2 * E_ref, (p, E, E_ref)


def test_direct_zero_cases_and_linearity():
    """Back-facing receivers and pixels without a hit get 0; L is exactly linear in the power."""
    tri = H.floor_quad(-10, 10, -10, 10)
    sc = H.scene_dict(tri, 1.0)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    pts = _floor_points([0.0, 1.0], [0.0, -1.0])
    l1 = scenes.point_light((0, 2, 0), (1, 1, 1))
    back = _direct(S, pts, (0, -1, 0), (1, 1, 1), np.zeros(4, np.int32), l1)
    miss = _direct(S, pts, (0, 1, 0), (1, 1, 1), np.full(4, -1, np.int32), l1)
    assert (back == 0).all() and (miss == 0).all()
    base = _direct(S, pts, (0, 1, 0), (1, 1, 1), np.zeros(4, np.int32), l1)
    for k in (1, 3, 7):
        lk = scenes.point_light((0, 2, 0), (2.0 ** k,) * 3)
        assert (_direct(S, pts, (0, 1, 0), (1, 1, 1), np.zeros(4, np.int32), lk) == base * 2.0 ** k).all()


@pytest.mark.parametrize("name", ["cornell", "room20k"])
def test_direct_is_eq2_irradiance(name):
    """The direct term at a patch VPL is the irradiance its eq. (2) flux was made from:
    I_k = rho E D / pi with E = pi L_e / rho (same light model, same visibility)."""
    sc = scenes.make_scene(name, width=32, height=32)
    S = orc.Scene.from_dict(sc)
    prm = dict(sc["params"], k_near=min(sc["params"]["k_near"], 256), n_far=0)
    g = S.generate(sc["camera"], sc["light"], prm)
    k = np.nonzero(g["bounce"] == 0)[0][:64]
    t = g["tri"][k]
    L = S.direct(g["pos"][k].astype(np.float32), g["nrm"][k].astype(np.float32),
                 np.ones((len(k), 3), np.float32), t, sc["light"], eps=prm["t_eps"])
    D = g["stats"]["Q"] * (0.1 * 0.1 * 2.0 ** -24) / prm["k_near"]
    I_from_direct = sc["albedo"][t].astype(np.float64) * (math.pi * L) * D / math.pi
    lit = g["I"][k].max(axis=1) > 0
    assert lit.sum() >= 8
    # positions enter the direct term rounded to float32: relative differences of a few 1e-7
    assert np.allclose(I_from_direct[lit], g["I"][k][lit], rtol=2e-5, atol=0)
