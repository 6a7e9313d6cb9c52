"""Pins of the oracle's VPL generation (Section "Close-Range VPL Sampling").

Closed forms for eq. (2) (point-to-plane irradiance, the solid angle of a
rectangle, Lambert's polygon irradiance for the quad light), an independent
projection-matrix formulation of the near test, brute-force point-in-patch
searches for the patch of every VPL, exact rational Halton values, and the
furnace identity of the quasi-random walk.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2203_11484_amd import scenes
from tests import helpers as H

UNIT_SHIFT = 24


def _unit(h):
    return h * h * 2.0 ** -UNIT_SHIFT


def _top_camera(center, height, vfov=120.0, w=64, hh=64):
    c = np.asarray(center, np.float64)
    return scenes.make_camera(c + [0, height, 0], c, (0, 0, 1), vfov, w, hh)


def _floor_scene(x0, x1, z0, z1, light_pos, power=(1, 1, 1), rho=1.0, k=64, cells=1, d_near=100.0):
    tri = H.floor_quad(x0, x1, z0, z1, nu=cells, nv=cells)
    cam = _top_camera(((x0 + x1) / 2, 0, (z0 + z1) / 2), 2.0 * max(x1 - x0, z1 - z0), vfov=90.0)
    params = scenes.default_params(k_near=k, n_far=0, d_near=d_near)
    return H.scene_dict(tri, rho, light=scenes.point_light(light_pos, power), camera=cam, params=params)


# ---------------------------------------------------------------------------
# eq. (2)
# ---------------------------------------------------------------------------

def test_eq2_point_to_plane_irradiance():
    """A patch VPL under a point light at height h: E = Phi h / (4 pi r^3), I = rho E D / pi."""
    h = 1.5
    sc = _floor_scene(-1, 1, -1, 1, (0.2, h, -0.1), power=(2.0, 3.0, 4.0), rho=0.5, k=8)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    g = S.generate(sc["camera"], sc["light"], sc["params"])
    st = g["stats"]
    assert st["k_eff"] == 8 and st["n_far"] == 0
    D = st["Q"] * _unit(0.1) / 8
    lp = sc["light"]["pos"].astype(np.float64)
    for k in range(8):
        y = g["pos"][k]
        r = np.linalg.norm(lp - y)
        hh = lp[1] - y[1]
        E = np.array([2.0, 3.0, 4.0]) * hh / (4 * math.pi * r ** 3)
        expect = 0.5 * E * D / math.pi
        np.testing.assert_allclose(g["I"][k], expect, rtol=1e-12)


def _rect_solid_angle(x0, x1, z0, z1, h):
    """Solid angle of the rectangle [x0,x1] x [z0,z1] seen from height h above the origin."""
    def f(x, z):
        return math.atan(x * z / (h * math.sqrt(x * x + z * z + h * h)))
    return f(x1, z1) - f(x0, z1) - f(x1, z0) + f(x0, z0)


def test_eq2_total_flux_solid_angle():
    """With rho = 1 the patch VPLs carry the flux the rectangle intercepts, Phi Omega / (4 pi);
    the midpoint strata make the error fall as K grows, below 1e-3 at K = 4096."""
    x0, x1, z0, z1, h = -0.7, 1.3, -1.1, 0.6, 0.9
    expect = _rect_solid_angle(x0, x1, z0, z1, h) / (4 * math.pi)
    errs = []
    for K in (16, 64, 256, 1024, 4096):
        sc = _floor_scene(x0, x1, z0, z1, (0, h, 0), k=K, cells=3)
        S = orc.Scene.from_dict(sc, use_bvh=False)
        g = S.generate(sc["camera"], sc["light"], sc["params"])
        assert g["stats"]["n_eligible"] == g["stats"]["n_patches"]
        total = (g["I"][:, 0] * math.pi).sum()
        errs.append(abs(total - expect) / expect)
    assert errs[-1] < 1e-3, errs
    assert errs[-1] < errs[0] / 10, errs


def test_eq2_cube_face_one_sixth():
    """Point light at the centre of a cube: one face intercepts exactly 1/6 of the flux
    (solid angle 2 pi / 3, closed form)."""
    tri = H.floor_quad(-1, 1, -1, 1, nu=4, nv=4)
    cam = _top_camera((0, 0, 0), 1.0, vfov=150.0)
    params = scenes.default_params(k_near=4096, n_far=0, d_near=100.0)
    sc = H.scene_dict(tri, 1.0, light=scenes.point_light((0, 1, 0), (6, 6, 6)), camera=cam, params=params)
    g = orc.Scene.from_dict(sc, use_bvh=False).generate(cam, sc["light"], params)
    golden = [ln.split() for ln in open(os.path.join(os.path.dirname(__file__), "golden", "solid_angle.txt"))
              if ln.strip() and ln[0] != "#"]
    frac = float(Fraction(golden[0][1]))
    assert abs((g["I"][:, 0] * math.pi).sum() - 6.0 * frac) < 6.0 * frac * 1e-3


def _lambert_polygon_irradiance(poly, x, n, radiance):
    """E = (L / 2) sum_edges theta_e (n . g_e), g_e the unit normal of the plane through x and edge e
    (Lambert's formula for a uniform polygonal emitter), with the sign that makes E >= 0."""
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


def test_eq2_quad_light_lambert_polygon():
    """The Cornell quad light seen from near patch VPLs: the 16-cell rule of eq. (2) agrees with
    Lambert's polygon irradiance (one-sided emitter of radiance Phi / (pi A)).  The 4 x 4 midpoint
    rule has an O((size / distance)^2) error: below 1% for VPLs more than 0.4 from the light."""
    sc = scenes.make_scene("cornell")
    S = orc.Scene.from_dict(sc)
    g = S.generate(sc["camera"], sc["light"], sc["params"])
    st = g["stats"]
    lt = sc["light"]
    c = lt["pos"].astype(np.float64)
    eu, ev = lt["edge_u"].astype(np.float64), lt["edge_v"].astype(np.float64)
    poly = [c, c + eu, c + eu + ev, c + ev]
    area = np.linalg.norm(np.cross(eu, ev))
    D = st["Q"] * _unit(0.1) / sc["params"]["k_near"]
    normals = S.normals()
    checked = 0
    errs = []
    for k in range(st["k_eff"]):
        t = g["tri"][k]
        y = g["pos"][k]
        if np.linalg.norm(y - (c + 0.5 * eu + 0.5 * ev)) < 0.4 or g["I"][k, 0] == 0:
            continue
        # only VPLs that see every light cell (no box in between): compare unoccluded irradiance
        cells = [c + (i + 0.5) / 4 * eu + (j + 0.5) / 4 * ev for j in range(4) for i in range(4)]
        vis = S.visibility(np.tile(y.astype(np.float32), (16, 1)), np.full(16, t), np.array(cells, np.float32),
                           np.full(16, -1))
        if not vis.all():
            continue
        E_ref = _lambert_polygon_irradiance(poly, y, normals[t], 1.0 / (math.pi * area))
        E = g["I"][k, 0] * math.pi / (sc["albedo"][t, 0] * D)
        rel = abs(E - E_ref) / E_ref
        dist = np.linalg.norm(y - (c + 0.5 * eu + 0.5 * ev))
        assert rel < 0.1 * (0.25 / dist) ** 2, (k, E, E_ref)
        errs.append(rel)
        checked += 1
    assert checked >= 10
    assert np.median(errs) < 2e-3


# ---------------------------------------------------------------------------
# patches, near test, Morton order, strata
# ---------------------------------------------------------------------------

def _level_exact(A, B, C, h):
    """Smallest n >= 1 with n h >= the longest edge, in exact rational arithmetic."""
    A, B, C = ([Fraction(float(v)) for v in p] for p in (A, B, C))

    def sq(p, q):
        return sum((a - b) ** 2 for a, b in zip(p, q))
    m2 = max(sq(B, A), sq(C, B), sq(A, C))
    hf = Fraction(h)
    n = 1
    while (n * hf) ** 2 < m2:
        n += 1
    return n


def _patch_vertices(tri, n, local):
    """Patch `local` of a triangle on the n x n barycentric grid: rows b, then a, up before down."""
    A, B, C = (tri[k].astype(np.float64) for k in range(3))
    r = 0
    while (r + 1) * (2 * n - (r + 1)) <= local:
        r += 1
    rem = local - r * (2 * n - r)
    a, b, down = rem // 2, r, rem & 1

    def G(i, j):
        return A + (B - A) * (i / n) + (C - A) * (j / n)
    if down:
        return np.array([G(a + 1, b), G(a + 1, b + 1), G(a, b + 1)])
    return np.array([G(a, b), G(a + 1, b), G(a, b + 1)])


def _project_ndc(cam, p):
    """Perspective projection with a look-at view matrix (independent of the oracle's dot-product test)."""
    eye = cam["eye"].astype(np.float64)
    f = cam["target"].astype(np.float64) - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, cam["up"].astype(np.float64))
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    view = np.eye(4)
    view[0, :3], view[1, :3], view[2, :3] = s, u, -f
    view[:3, 3] = -view[:3, :3] @ eye
    aspect = cam["width"] / cam["height"]
    t = 1.0 / math.tan(math.radians(cam["vfov_deg"]) / 2)
    proj = np.array([[t / aspect, 0, 0, 0], [0, t, 0, 0], [0, 0, -1, -0.02], [0, 0, -1, 0]])
    clip = proj @ view @ np.append(p, 1.0)
    return clip[:2] / clip[3], clip[3]


@pytest.fixture(scope="module")
def cornell_gen():
    sc = scenes.make_scene("cornell")
    S = orc.Scene.from_dict(sc)
    return sc, S, S.generate(sc["camera"], sc["light"], sc["params"])


def test_patch_levels_exact(cornell_gen):
    sc, S, g = cornell_gen
    off = g["patch_off"]
    for t in range(len(sc["tri"])):
        n = _level_exact(*sc["tri"][t], 0.1)
        assert off[t + 1] - off[t] == n * n


def test_near_flags_match_projection(cornell_gen):
    """Near = centroid inside the view frustum and closer than d_near (Section "Close-Range VPL
    Sampling", first step), checked with a projection matrix; emitters are never near."""
    sc, S, g = cornell_gen
    cam, dn = sc["camera"], sc["params"]["d_near"]
    off = g["patch_off"]
    rng = np.random.default_rng(1)
    n_checked = 0
    for t in range(len(sc["tri"])):
        n = int(round(math.sqrt(off[t + 1] - off[t])))
        for loc in rng.choice(n * n, min(n * n, 40), replace=False):
            P = _patch_vertices(sc["tri"][t], n, int(loc))
            c = P.mean(0)
            ndc, w = _project_ndc(cam, c)
            dist = np.linalg.norm(c - cam["eye"].astype(np.float64))
            margin = min(abs(abs(ndc[0]) - 1), abs(abs(ndc[1]) - 1), abs(dist - dn))
            if margin < 1e-9:
                continue
            near = (w > 0) and abs(ndc[0]) <= 1 and abs(ndc[1]) <= 1 and dist < dn and not (sc["flags"][t] & 1)
            assert bool(g["pflags"][off[t] + loc] & 1) == near, (t, loc)
            n_checked += 1
    assert n_checked > 300
    assert 0 < (g["pflags"] & 1).sum() < len(g["pflags"])


def test_eligible_faces_the_light(cornell_gen):
    sc, S, g = cornell_gen
    nrm = S.normals()
    lt = sc["light"]
    lc = lt["pos"].astype(np.float64) + 0.5 * lt["edge_u"] + 0.5 * lt["edge_v"]
    off = g["patch_off"]
    for gi in g["sorted"]:
        t = int(np.searchsorted(off, gi, side="right") - 1)
        n = int(round(math.sqrt(off[t + 1] - off[t])))
        c = _patch_vertices(sc["tri"][t], n, int(gi - off[t])).mean(0)
        assert np.dot(nrm[t], lc - c) > 0
        assert g["pflags"][gi] & 3 == 3


def _part1by2(x):
    x &= 0x3FF
    x = (x | (x << 16)) & 0x030000FF
    x = (x | (x << 8)) & 0x0300F00F
    x = (x | (x << 4)) & 0x030C30C3
    x = (x | (x << 2)) & 0x09249249
    return x


def test_morton_order_and_cdf(cornell_gen):
    """Eligible patches sorted by (Morton key of the centroid on the h grid, index); the fixed-point
    prefix is strictly increasing; each stratum midpoint target lies in its patch's CDF interval."""
    sc, S, g = cornell_gen
    off = g["patch_off"]
    lo = sc["tri"].reshape(-1, 3).astype(np.float64).min(0)
    keys = []
    for gi in g["sorted"]:
        t = int(np.searchsorted(off, gi, side="right") - 1)
        n = int(round(math.sqrt(off[t + 1] - off[t])))
        c = _patch_vertices(sc["tri"][t], n, int(gi - off[t])).mean(0)
        cell = np.clip(np.floor((c - lo) / 0.1), 0, 1023).astype(int)
        keys.append(_part1by2(cell[0]) | (_part1by2(cell[1]) << 1) | (_part1by2(cell[2]) << 2))
    assert np.array_equal(np.array(keys, np.uint32), g["keys"])
    pairs = list(zip(g["keys"].tolist(), g["sorted"].tolist()))
    assert pairs == sorted(pairs)
    F = g["F"]
    assert np.all(np.diff(F) > 0) and F[-1] == g["stats"]["Q"]
    K = sc["params"]["k_near"]
    Q = g["stats"]["Q"]
    for k, m in enumerate(g["m"]):
        u = ((2 * k + 1) * Q) // (2 * K)
        lo_f = F[m - 1] if m > 0 else 0
        assert lo_f <= u < F[m]


def _point_in_tri(P, y, tol=1e-9):
    A, B, C = P
    e1, e2, w = B - A, C - A, y - A
    n = np.cross(e1, e2)
    nn = np.dot(n, n)
    bu = np.dot(np.cross(w, e2), n) / nn
    bv = np.dot(np.cross(e1, w), n) / nn
    off_plane = abs(np.dot(w, n)) / math.sqrt(nn)
    return bu >= -tol and bv >= -tol and bu + bv <= 1 + tol and off_plane < 1e-9


def test_patch_vpls_lie_in_their_stratum_patch(cornell_gen):
    sc, S, g = cornell_gen
    off = g["patch_off"]
    for k, m in enumerate(g["m"]):
        gi = g["sorted"][m]
        t = int(np.searchsorted(off, gi, side="right") - 1)
        assert g["tri"][k] == t
        n = int(round(math.sqrt(off[t + 1] - off[t])))
        assert _point_in_tri(_patch_vertices(sc["tri"][t], n, int(gi - off[t])), g["pos"][k])


def test_far_vpls_lie_in_far_patches(cornell_gen):
    """Every walk VPL sits on a patch that is not near (hits on near patches are discarded)."""
    sc, S, g = cornell_gen
    off = g["patch_off"]
    K = g["stats"]["k_eff"]
    for i in range(K, g["n"]):
        t = g["tri"][i]
        n = int(round(math.sqrt(off[t + 1] - off[t])))
        owners = [loc for loc in range(n * n) if _point_in_tri(_patch_vertices(sc["tri"][t], n, loc), g["pos"][i],
                                                                tol=1e-12)]
        assert owners, i
        assert any(not (g["pflags"][off[t] + loc] & 1) for loc in owners), i


# ---------------------------------------------------------------------------
# quasi-random walk
# ---------------------------------------------------------------------------

def _closed_box_scene(rho, n_far, k_near=0, d_near=0.0, light=(0.4, 0.55, 0.45)):
    tri = H.closed_box((0, 0, 0), (1, 1, 1), cells=2)
    cam = scenes.make_camera((0.5, 0.5, 0.05), (0.5, 0.5, 1.0), (0, 1, 0), 60.0, 32, 32)
    params = scenes.default_params(k_near=k_near, n_far=n_far, d_near=d_near)
    return H.scene_dict(tri, rho, light=scenes.point_light(light, (3.0, 2.0, 1.0)), camera=cam, params=params)


def test_walk_furnace_identity():
    """Closed box, uniform albedo, no near region: every walk VPL carries Phi_L rho^b / N_paths, and
    since every ray hits, the bounce-1 VPLs sum to Phi_L rho."""
    rho = 0.625
    sc = _closed_box_scene(rho, n_far=300)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    g = S.generate(sc["camera"], sc["light"], sc["params"])
    st = g["stats"]
    assert st["n_near"] == 0 and st["k_eff"] == 0 and st["n_far"] == 300
    assert st["n_paths"] == 100 and st["far_b1"] == st["far_b2"] == st["far_b3"] == 100
    PL = np.array([3.0, 2.0, 1.0])
    phi = g["I"] * math.pi * st["n_paths"]
    for i in range(g["n"]):
        np.testing.assert_allclose(phi[i], PL * rho ** g["bounce"][i], rtol=1e-12)
    b1 = g["bounce"] == 1
    np.testing.assert_allclose((g["I"][b1] * math.pi).sum(0), PL * rho, rtol=1e-12)
    # paths are numbered from 1 and each deposits at bounces 1, 2, 3 in order
    assert g["path"].tolist() == [p for p in range(1, 101) for _ in range(3)]
    assert g["bounce"].tolist() == [1, 2, 3] * 100


def test_walk_truncates_last_path():
    sc = _closed_box_scene(0.5, n_far=301)
    g = orc.Scene.from_dict(sc, use_bvh=False).generate(sc["camera"], sc["light"], sc["params"])
    st = g["stats"]
    assert st["n_far"] == 301 and st["n_paths"] == 101
    assert st["far_b1"] == 101 and st["far_b2"] == 100
    np.testing.assert_allclose(g["I"][-1] * math.pi * 101, np.array([3.0, 2.0, 1.0]) * 0.5, rtol=1e-12)


def test_walk_first_direction_is_halton_sphere():
    """The first segment of path i leaves the point light along the uniform-sphere direction built
    from (phi_2(i), phi_3(i)); its first hit lies on that ray."""
    sc = _closed_box_scene(0.5, n_far=60)
    g = orc.Scene.from_dict(sc, use_bvh=False).generate(sc["camera"], sc["light"], sc["params"])
    lp = sc["light"]["pos"].astype(np.float64)
    for i in np.nonzero(g["bounce"] == 1)[0]:
        p = int(g["path"][i])
        u1, u2 = float(_ri(2, p)), float(_ri(3, p))
        z = 1 - 2 * u1
        r = math.sqrt(max(0.0, 1 - z * z))
        d = np.array([r * math.cos(2 * math.pi * u2), r * math.sin(2 * math.pi * u2), z])
        w = g["pos"][i] - lp
        np.testing.assert_allclose(w / np.linalg.norm(w), d, atol=1e-12)


def _ri(b, i):
    f, r = Fraction(1, b), Fraction(0)
    while i > 0:
        r += f * (i % b)
        i //= b
        f /= b
    return r


def test_reduction_no_near_region_is_plain_ir():
    """d_near = 0: no near patch exists, the near budget moves to the walk and nothing is discarded."""
    sc = scenes.make_scene("cornell", d_near=0.0)
    g = orc.Scene.from_dict(sc).generate(sc["camera"], sc["light"], sc["params"])
    st = g["stats"]
    assert st["n_near"] == 0 and st["k_eff"] == 0
    assert st["n_far_target"] == 256 and st["n_far"] == 256 and st["near_discarded"] == 0


def test_cornell_bounce1_flux_uses_host_albedo(cornell_gen):
    """Quad light walk: a bounce-1 VPL carries Phi_L rho_t / N_paths of its own triangle."""
    sc, S, g = cornell_gen
    n_paths = g["stats"]["n_paths"]
    for i in np.nonzero(g["bounce"] == 1)[0]:
        t = g["tri"][i]
        np.testing.assert_allclose(g["I"][i] * math.pi * n_paths, sc["albedo"][t].astype(np.float64), rtol=1e-12)


def test_room_generation_counts():
    sc = scenes.make_scene("room20k", width=64, height=64)
    g = orc.Scene.from_dict(sc).generate(sc["camera"], sc["light"], sc["params"])
    st = g["stats"]
    assert st["k_eff"] == 2048 and st["n_far"] == 2048 and st["flags"] == 0
    assert g["n"] == 4096
    tri = sc["tri"].astype(np.float64)
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1).sum()
    near_area = st["Q"] * _unit(0.1)
    assert 0.08 < near_area / area < 0.2


# ---------------------------------------------------------------------------
# walk variant: near hits kept after the first bounce
# ---------------------------------------------------------------------------

def _walk_vpl_patch_flags(sc, g):
    """For each VPL, by brute-force point-in-patch over its triangle's patches: whether some owning patch
    is far, and whether every owning patch is near (a point on a patch edge has several owners)."""
    off, pf = g["patch_off"], g["pflags"]
    any_far = np.zeros(g["n"], bool)
    all_near = np.zeros(g["n"], bool)
    for i in range(g["n"]):
        if g["bounce"][i] == 0:
            continue
        t = g["tri"][i]
        n = int(round(math.sqrt(off[t + 1] - off[t])))
        owners = [loc for loc in range(n * n)
                  if _point_in_tri(_patch_vertices(sc["tri"][t], n, loc), g["pos"][i], tol=1e-12)]
        assert owners, i
        near = [bool(pf[off[t] + loc] & 1) for loc in owners]
        any_far[i] = not all(near)
        all_near[i] = all(near)
    return any_far, all_near


def test_walk_near_variant_reduces_to_plain_ir_without_near_region():
    """With no near region (d_near = 0) the variant changes nothing: the same VPLs bit for bit."""
    sc = scenes.make_scene("cornell", d_near=0.0)
    S = orc.Scene.from_dict(sc)
    g0 = S.generate(sc["camera"], sc["light"], sc["params"])
    g1 = S.generate(sc["camera"], sc["light"], dict(sc["params"], walk_near=1))
    for k in ("pos", "nrm", "I", "tri", "path", "bounce"):
        assert np.array_equal(g0[k], g1[k]), k


def test_walk_near_variant_keeps_later_near_hits():
    """Variant walk_near = 1: first-bounce walk VPLs are all on far patches, near hits are discarded only at
    the first bounce, some later-bounce VPLs lie on near patches, and every walk VPL still carries
    Phi_L times the albedo product along its path over N_paths (the furnace identity)."""
    sc = _closed_box_scene(0.625, n_far=300, k_near=64, d_near=1.2)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    p1 = dict(sc["params"], walk_near=1)
    g = S.generate(sc["camera"], sc["light"], p1)
    g0 = S.generate(sc["camera"], sc["light"], sc["params"])
    st, st0 = g["stats"], g0["stats"]
    assert st["k_eff"] == st0["k_eff"] == 64
    assert st["n_far"] == st["n_far_target"]
    walk = g["bounce"] > 0
    any_far, all_near = _walk_vpl_patch_flags(sc, g)
    assert any_far[walk & (g["bounce"] == 1)].all()
    assert all_near[walk & (g["bounce"] >= 2)].any()
    # the paper's reading never keeps a near hit, and discards more
    any_far0, _ = _walk_vpl_patch_flags(sc, g0)
    assert any_far0[g0["bounce"] > 0].all()
    assert st["near_discarded"] < st0["near_discarded"]
    PL = np.array([3.0, 2.0, 1.0])
    phi = g["I"][walk] * math.pi * st["n_paths"]
    for i, b in enumerate(g["bounce"][walk]):
        np.testing.assert_allclose(phi[i], PL * 0.625 ** b, rtol=1e-12)
