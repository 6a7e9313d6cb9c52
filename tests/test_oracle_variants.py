"""Pins of the oracle's generation variants (readings of the paper's patch-sampling passage and flow
step (3) that the text leaves open).

* walk_near = 2: a walk hit on a near patch is discarded and ends its path.  Pinned against the
  paper's walk (walk_near = 0) on the same Halton paths: every path keeps exactly its far hits up to
  its first near hit.
* jitter = 1: stratum k's target is B_k + floor(xi_k (B_{k+1} - B_k)) with B_k = floor(k f(N) / K)
  and xi_k the base-5 radical inverse of k + 1.  Pinned with exact rational arithmetic.
* brightness = 1: a patch VPL's flux is eq. (2) summed over the patches of its stratum, each at its
  centroid with the part of its area inside the stratum.  Pinned by closed-form point-light
  irradiance at independently computed patch centroids: conservation of the total for any K, the
  one-patch-per-stratum case, and large patches shared among several VPLs.
"""
import math
from bisect import bisect_right
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2203_11484_amd import scenes
from tests import helpers as H
from tests.test_oracle_generation import _closed_box_scene, _floor_scene, _patch_vertices, _unit


# ---------------------------------------------------------------------------
# terminate at the first near hit
# ---------------------------------------------------------------------------

def _paths(g):
    """path -> list of (bounce, pos, tri, flux * n_paths) of its walk VPLs, in bounce order."""
    out = {}
    n_paths = g["stats"]["n_paths"]
    for i in np.nonzero(g["bounce"] > 0)[0]:
        out.setdefault(int(g["path"][i]), []).append(
            (int(g["bounce"][i]), g["pos"][i].copy(), int(g["tri"][i]), g["I"][i] * math.pi * n_paths))
    for v in out.values():
        v.sort(key=lambda e: e[0])
    return out


def test_terminate_at_near_keeps_the_far_prefix_of_each_path():
    sc = _closed_box_scene(0.625, n_far=300, k_near=64, d_near=1.2)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    g0 = S.generate(sc["camera"], sc["light"], sc["params"])
    g2 = S.generate(sc["camera"], sc["light"], dict(sc["params"], walk_near=2))
    st0, st2 = g0["stats"], g2["stats"]
    assert st2["n_far"] == st2["n_far_target"] == st0["n_far_target"]
    # ending paths early needs more of them
    assert st2["n_paths"] > st0["n_paths"]
    p0, p2 = _paths(g0), _paths(g2)
    last = min(st0["n_paths"], st2["n_paths"]) - 1  # the last path of a run is cut by the far target
    checked = stopped = 0
    for path in range(1, last + 1):
        a, b = p0.get(path, []), p2.get(path, [])
        m = len(b)
        # the kept bounces are 1..m: a near hit ends the path, so there are no gaps
        assert [e[0] for e in b] == list(range(1, m + 1)), path
        # they are the paper's walk's VPLs of the same path up to bounce m, bit for bit
        assert [e[0] for e in a[:m]] == list(range(1, m + 1)), path
        for e0, e2 in zip(a[:m], b):
            assert np.array_equal(e0[1], e2[1]) and e0[2] == e2[2]
            np.testing.assert_allclose(e0[3], e2[3], rtol=1e-12)
        # after the prefix the paper's walk has no VPL at bounce m + 1 (that hit was near, or the path ended)
        assert all(e[0] != m + 1 for e in a), path
        stopped += len(a) > m
        checked += 1
    assert checked > 100 and stopped > 0
    # the furnace identity still holds: flux = Phi_L * rho^bounce over N_paths
    PL = np.array([3.0, 2.0, 1.0])
    for v in p2.values():
        for bnc, _, _, phi in v:
            np.testing.assert_allclose(phi, PL * 0.625 ** bnc, rtol=1e-12)


def test_terminate_at_near_without_near_region_is_plain_ir():
    sc = scenes.make_scene("cornell", d_near=0.0)
    S = orc.Scene.from_dict(sc)
    g0 = S.generate(sc["camera"], sc["light"], sc["params"])
    g2 = S.generate(sc["camera"], sc["light"], dict(sc["params"], walk_near=2))
    for k in ("pos", "nrm", "I", "tri", "path", "bounce"):
        assert np.array_equal(g0[k], g2[k]), k


# ---------------------------------------------------------------------------
# jittered strata
# ---------------------------------------------------------------------------

def _radical_inverse(b, i):
    f, x = Fraction(1), Fraction(0)
    while i:
        f /= b
        x += f * (i % b)
        i //= b
    return x


def test_jittered_targets_exact():
    sc = _floor_scene(-0.7, 1.3, -1.1, 0.6, (0, 0.9, 0), k=300, cells=3)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    g = S.generate(sc["camera"], sc["light"], dict(sc["params"], jitter=1))
    g_mid = S.generate(sc["camera"], sc["light"], sc["params"])
    F = [int(x) for x in g["F"][: g["stats"]["n_eligible"]]]
    Q, K = g["stats"]["Q"], 300
    assert Q == F[-1]
    ties = 0
    for k in range(K):
        Bk, Bk1 = k * Q // K, (k + 1) * Q // K
        x = _radical_inverse(5, k + 1) * (Bk1 - Bk)
        u = Bk + min(math.floor(x), Bk1 - Bk - 1)
        m = bisect_right(F, u)  # smallest j with F[j] > u
        if x.denominator == 1:  # an exact integer: FP64 may land on either side
            ties += 1
            assert g["m"][k] in (m, bisect_right(F, u - 1))
        else:
            assert g["m"][k] == m, k
        # the target's patch overlaps the stratum
        assert F[g["m"][k]] > Bk and (g["m"][k] == 0 or F[g["m"][k] - 1] < Bk1)
    assert ties < K // 10
    # the jitter moves targets: some strata pick another patch than their midpoint
    assert (g["m"] != g_mid["m"]).sum() > K // 10
    # placement within the patch and eq. (2) are unchanged: same Halton point formula, D = f(N) / K
    assert np.all(np.diff(g["m"]) >= 0)


def test_jittered_strata_total_flux_converges():
    """With rho = 1 the jittered patch VPLs still carry the flux the rectangle intercepts."""
    x0, x1, z0, z1, h = -0.7, 1.3, -1.1, 0.6, 0.9

    def f(x, z):
        return math.atan(x * z / (h * math.sqrt(x * x + z * z + h * h)))
    expect = (f(x1, z1) - f(x0, z1) - f(x1, z0) + f(x0, z0)) / (4 * math.pi)
    errs = []
    for K in (64, 4096):
        sc = _floor_scene(x0, x1, z0, z1, (0, h, 0), k=K, cells=3)
        g = orc.Scene.from_dict(sc, use_bvh=False).generate(sc["camera"], sc["light"], dict(sc["params"], jitter=1))
        errs.append(abs((g["I"][:, 0] * math.pi).sum() - expect) / expect)
    assert errs[-1] < 2e-3 and errs[-1] < errs[0], errs


# ---------------------------------------------------------------------------
# brightness from the stratum's set of patches
# ---------------------------------------------------------------------------

def _patch_table(sc, g):
    """Per eligible patch in sorted order: centroid (FP64, from the patch's own vertices), triangle,
    fixed-point area q (recomputed here), from the oracle's sorted ids and patch offsets."""
    off = g["patch_off"]
    ne = g["stats"]["n_eligible"]
    h = sc["params"]["patch_h"]
    cents, tris, qs = [], [], []
    for j in range(ne):
        gid = int(g["sorted"][j])
        t = int(np.searchsorted(off, gid, side="right") - 1)
        n = int(round(math.sqrt(off[t + 1] - off[t])))
        P = _patch_vertices(sc["tri"][t], n, gid - off[t])
        cents.append(((P[0] + P[1]) + P[2]) / 3.0)
        tris.append(t)
        A, B, C = (sc["tri"][t][i].astype(np.float64) for i in range(3))
        area = 0.5 * np.linalg.norm(np.cross(B - A, C - A)) / (n * n)
        qs.append(int(round(area / _unit(h))))
    return np.array(cents), np.array(tris), np.array(qs, np.int64)


def _point_factor(light_pos, c):
    """Irradiance per unit power at a floor point (normal +y), unoccluded point light: h / (4 pi r^3)."""
    w = np.asarray(light_pos, np.float64) - c
    r = np.linalg.norm(w)
    return w[1] / (4 * math.pi * r ** 3)


def test_set_sum_conserves_the_near_flux_for_any_K():
    lp = (0.3, 0.8, -0.2)
    rho, PL = 0.5, np.array([2.0, 3.0, 4.0])
    totals = []
    for K in (1, 7, 64, 1000):
        sc = _floor_scene(-0.7, 1.3, -1.1, 0.6, lp, power=tuple(PL), rho=rho, k=K, cells=3)
        S = orc.Scene.from_dict(sc, use_bvh=False)
        g = S.generate(sc["camera"], sc["light"], dict(sc["params"], brightness=1))
        assert g["stats"]["k_eff"] == K
        totals.append(g["I"].sum(axis=0) * math.pi)
    cents, tris, qs = _patch_table(sc, g)
    assert qs.sum() == g["stats"]["Q"]
    unit = _unit(sc["params"]["patch_h"])
    lp = sc["light"]["pos"].astype(np.float64)  # as stored (float32)
    expect = sum(rho * PL * _point_factor(lp, c) * (q * unit) for c, q in zip(cents, qs))
    for tot in totals:
        np.testing.assert_allclose(tot, expect, rtol=1e-12)


def test_set_sum_one_patch_per_stratum():
    """A floor of equal patches and K = their number: stratum k is exactly patch k, and the VPL carries
    that patch's eq. (2) flux at its centroid."""
    lp = (0.1, 0.7, 0.2)
    sc0 = _floor_scene(-0.5, 0.5, -0.5, 0.5, lp, rho=0.8, k=1, cells=1)
    g0 = orc.Scene.from_dict(sc0, use_bvh=False).generate(sc0["camera"], sc0["light"], sc0["params"])
    K = g0["stats"]["n_eligible"]
    sc = _floor_scene(-0.5, 0.5, -0.5, 0.5, lp, rho=0.8, k=K, cells=1)
    g = orc.Scene.from_dict(sc, use_bvh=False).generate(sc["camera"], sc["light"], dict(sc["params"], brightness=1))
    cents, tris, qs = _patch_table(sc, g)
    lp = sc["light"]["pos"].astype(np.float64)
    assert len(set(qs.tolist())) == 1, "equal patches expected"
    assert np.array_equal(g["m"][:K], np.arange(K))
    unit = _unit(sc["params"]["patch_h"])
    for k in range(K):
        expect = float(np.float32(0.8)) * _point_factor(lp, cents[k]) * qs[k] * unit / math.pi
        np.testing.assert_allclose(g["I"][k], expect, rtol=1e-12)


def test_set_sum_shares_large_patches():
    """Patches larger than a stratum: each VPL gets eq. (2) of the patches it overlaps, weighted by the
    exact integer overlap of [F_{j-1}, F_j) with [B_k, B_{k+1})."""
    lp = (0.2, 1.1, -0.3)
    sc = _floor_scene(-1, 1, -1, 1, lp, rho=1.0, k=37, cells=2)
    sc["params"] = dict(sc["params"], patch_h=2.0)  # each triangle is one patch: 8 patches, 37 strata
    S = orc.Scene.from_dict(sc, use_bvh=False)
    g = S.generate(sc["camera"], sc["light"], dict(sc["params"], brightness=1))
    cents, tris, qs = _patch_table(sc, g)
    lp = sc["light"]["pos"].astype(np.float64)
    assert len(qs) == 8
    F = np.cumsum(qs)
    Q, K = int(F[-1]), 37
    unit = _unit(2.0)
    shared = 0
    for k in range(K):
        Bk, Bk1 = k * Q // K, (k + 1) * Q // K
        acc = 0.0
        parts = 0
        for j in range(8):
            f0 = int(F[j - 1]) if j else 0
            ov = min(int(F[j]), Bk1) - max(f0, Bk)
            if ov > 0:
                acc += _point_factor(lp, cents[j]) * ov * unit
                parts += 1
        shared += parts > 1
        np.testing.assert_allclose(g["I"][k, 0], acc / math.pi, rtol=1e-12)
    assert shared > 0
    # the flux of each patch is split among its strata without loss
    np.testing.assert_allclose(g["I"][:, 0].sum() * math.pi,
                               sum(_point_factor(lp, c) * q * unit for c, q in zip(cents, qs)), rtol=1e-12)


def test_set_sum_skips_occluded_patches():
    """A square occluder between the point light and the floor: patches whose centroid is in its shadow
    contribute nothing, the rest their closed-form share."""
    h, a, s = 2.0, 1.0, 0.3
    floor = H.floor_quad(-1, 1, -1, 1, nu=4, nv=4)
    occ = scenes._quad_grid((-s, a, -s), (2 * s, 0, 0), (0, 0, 2 * s), (0, -1, 0), 1, 1)
    tri = np.concatenate([floor, occ])
    cam = scenes.make_camera((0, 0.5, -0.01), (0, 0, 0), (0, 0, 1), 170.0, 64, 64)
    params = scenes.default_params(k_near=1, n_far=0, d_near=100.0)
    sc = H.scene_dict(tri, 1.0, light=scenes.point_light((0, h, 0), (1, 1, 1)), camera=cam, params=params)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    g = S.generate(cam, sc["light"], dict(params, brightness=1))
    cents, tris, qs = _patch_table(sc, g)
    floor_ids = tris < len(floor)
    assert floor_ids.all(), "the occluder faces away from the light: not eligible"
    half = s * h / (h - a)
    unit = _unit(params["patch_h"])
    lit = np.array([max(abs(c[0]), abs(c[2])) > half for c in cents])
    assert (~lit).sum() > 0 and lit.sum() > 0
    expect = sum(_point_factor((0, h, 0), c) * q * unit for c, q, L in zip(cents, qs, lit) if L)
    np.testing.assert_allclose(g["I"][0, 0] * math.pi, expect, rtol=1e-12)


# ---------------------------------------------------------------------------
# Keller's path schedule
# ---------------------------------------------------------------------------

def test_keller_mean_albedo():
    """Area-weighted mean over the faces that do not emit, of the channel mean: quads of area 1 and 3 with
    grey albedo 0.25 and 0.75 give (0.25 + 2.25) / 4 = 0.625; an emitting face does not count."""
    a = H.floor_quad(0, 1, 0, 1)             # area 1
    b = H.floor_quad(2, 5, 0, 1)             # area 3
    e = H.floor_quad(0, 1, 2, 3, y=1.0)      # emitter
    tri = np.concatenate([a, b, e])
    alb = np.array([[0.25] * 3] * 2 + [[0.75] * 3] * 2 + [[1.0, 0.5, 0.0]] * 2, np.float32)
    flags = np.array([0, 0, 0, 0, 1, 1], np.uint8)
    S = orc.Scene.from_dict(H.scene_dict(tri, alb, flags=flags), use_bvh=False)
    assert S.rho_bar() == 0.625


def _keller_expect(rb, n_far, maxb=3):
    S, r = 0.0, 1.0
    for _ in range(maxb):
        S += r
        r *= rb
    N = math.floor(n_far / S)
    T, r = [], 1.0
    for _ in range(maxb):
        T.append(math.floor(r * N))
        r *= rb
    return N, T


def test_keller_schedule_counts_and_path_limits():
    """Closed box, every hit deposits (no near region): N = floor(n_far / (1 + rb + rb^2)) paths; path i
    deposits at bounces 1..b with b the last bounce whose limit floor(rb^(b-1) N) admits it, so
    bounce b holds exactly that many VPLs."""
    sc = _closed_box_scene(0.625, n_far=500)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    rb = S.rho_bar()
    assert abs(rb - 0.625) < 1e-15
    g = S.generate(sc["camera"], sc["light"], dict(sc["params"], walk_schedule=1))
    N, T = _keller_expect(rb, 500)
    st = g["stats"]
    assert st["n_paths"] == N and st["flags"] == 0
    assert [st["far_b1"], st["far_b2"], st["far_b3"]] == T
    assert st["n_far"] == sum(T) <= 500
    p = _paths(g)
    assert sorted(p) == list(range(1, N + 1))
    for path, v in p.items():
        bmax = max(b for b in (1, 2, 3) if path <= T[b - 1])
        assert [e[0] for e in v] == list(range(1, bmax + 1)), path


def test_keller_schedule_flux_weights():
    """A deposit at bounce b carries Phi rho^b / (N rb^(b-1)); each bounce's VPLs together carry about
    Phi rho^b, the reflected power of that bounce (off by the floor of the path limit only)."""
    sc = _closed_box_scene(0.625, n_far=500)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    rb = S.rho_bar()
    g = S.generate(sc["camera"], sc["light"], dict(sc["params"], walk_schedule=1))
    N, T = _keller_expect(rb, 500)
    PL = np.array([3.0, 2.0, 1.0])
    phi = g["I"] * math.pi
    for i in range(g["n"]):
        b = int(g["bounce"][i])
        np.testing.assert_allclose(phi[i] * N, PL * 0.625 ** b / rb ** (b - 1), rtol=1e-12)
    for b in (1, 2, 3):
        tot = phi[g["bounce"] == b].sum(axis=0)
        np.testing.assert_allclose(tot, PL * 0.625 ** b, rtol=1.0 / (rb ** (b - 1) * N) + 1e-12)


def test_keller_schedule_white_box_is_the_default_walk():
    """Albedo 1: rb = 1, every path runs all its bounces as in the default walk, and the VPLs of each path
    are the default walk's, bit for bit (fluxes times the path count equal)."""
    sc = _closed_box_scene(1.0, n_far=300)
    S = orc.Scene.from_dict(sc, use_bvh=False)
    assert S.rho_bar() == 1.0
    g0 = S.generate(sc["camera"], sc["light"], sc["params"])
    gk = S.generate(sc["camera"], sc["light"], dict(sc["params"], walk_schedule=1))
    assert gk["stats"]["n_paths"] == 100  # floor(300 / 3)
    p0, pk = _paths(g0), _paths(gk)
    for path in range(1, 100):
        a, b = p0[path], pk[path]
        assert [e[0] for e in a] == [e[0] for e in b] == [1, 2, 3]
        for e0, ek in zip(a, b):
            assert np.array_equal(e0[1], ek[1]) and e0[2] == ek[2]
            np.testing.assert_allclose(e0[3], ek[3], rtol=1e-12)
