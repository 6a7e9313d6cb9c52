"""Degenerate inputs and size limits of the C ABI on the GPU path, against the oracle.

* Degenerate triangles (a repeated vertex, three collinear vertices) inside the Cornell box: they
  bound no area, so they occlude nothing and get no patches that face the light; the gather, the
  G-buffer and every integer output of the generation still match the oracle.
* The scene away from the origin (all coordinates shifted): parity at the same bar.
* One VPL; a VPL on the receivers' own triangle (its segments lie in the plane: geometry term 0);
  a VPL of zero intensity.
* Size limits and invalid values rejected before any device work: triangle counts above 2^25,
  non-finite vertices, G-buffers above 2^28 pixels.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc  # noqa: E402
from paper_2203_11484_amd import scenes  # noqa: E402
from tests import helpers as H  # noqa: E402
from tests.test_gpu_parity import _check_gather, _gather_gpu  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vplg():
    from paper_2203_11484_amd import vplg as v
    v.lib()
    return v


@pytest.fixture(scope="module")
def ctx(vplg):
    c = vplg.context_create(0)
    yield c
    vplg.context_destroy(c)


def _with_degenerates(sc):
    """The scene plus two zero-area triangles across the room's middle (albedo 0.5, not emitters)."""
    deg = np.array([[[0.2, 0.5, 0.3], [0.8, 0.5, 0.7], [0.8, 0.5, 0.7]],     # repeated vertex
                    [[0.125, 0.25, 0.5], [0.5, 0.5, 0.5], [0.875, 0.75, 0.5]]],  # collinear (exact in binary)
                   np.float32)
    out = dict(sc)
    out["tri"] = np.concatenate([sc["tri"], deg])
    out["albedo"] = np.concatenate([sc["albedo"], np.full((2, 3), 0.5, np.float32)])
    out["flags"] = np.concatenate([sc["flags"], np.zeros(2, np.uint8)])
    return out


def _oracle_inputs(sc):
    S = orc.Scene.from_dict(sc)
    gbo = {k: (v.astype(np.float32) if v.dtype == np.float64 else v) for k, v in S.gbuffer(sc["camera"]).items()}
    g = S.generate(sc["camera"], sc["light"], sc["params"])
    vp = dict(pos=g["pos"].astype(np.float32), nrm=g["nrm"].astype(np.float32), I=g["I"].astype(np.float32),
              tri=g["tri"])
    return S, gbo, vp, g


def test_degenerate_triangles_gather_parity(vplg, ctx):
    sc = _with_degenerates(scenes.make_scene("cornell", width=96, height=72))
    S, gbo, vp, _ = _oracle_inputs(sc)
    # no pixel sees a degenerate triangle, and no VPL lies on one
    assert (gbo["tri"] < len(sc["tri"]) - 2).all() and (vp["tri"] < len(sc["tri"]) - 2).all()
    _check_gather(vplg, ctx, sc, S, gbo, vp, np.arange(96 * 72), sc["params"], "cornell + degenerate")


def test_degenerate_triangles_generation_parity(vplg, ctx):
    sc = _with_degenerates(scenes.make_scene("cornell"))
    S = orc.Scene.from_dict(sc)
    ref = S.generate(sc["camera"], sc["light"], sc["params"])
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    vid = vplg.vpls_generate(ctx, sid, sc["camera"], sc["params"])
    st = vplg.vplset_stats(ctx, vid)
    assert (st["n_patches"], st["n_eligible"], st["q_total"], st["n_paths"]) == \
        (ref["stats"]["n_patches"], ref["stats"]["n_eligible"], ref["stats"]["Q"], ref["stats"]["n_paths"])
    for name, key in (("pflags", "pflags"), ("sorted", "sorted"), ("prefix", "F"), ("strata", "m"),
                      ("path", "path"), ("bounce", "bounce")):
        assert np.array_equal(vplg.vplset_debug(ctx, vid, name), ref[key]), name
    # the degenerate triangles' patches never face the light (their normal is undefined)
    off = ref["patch_off"]
    T = len(sc["tri"])
    assert not (ref["pflags"][off[T - 2]:off[T]] & 2).any()
    d = vplg.vpls_download(ctx, vid)
    assert np.array_equal(d["tri"], ref["tri"])
    vplg.vplset_release(ctx, vid)
    vplg.scene_release(ctx, sid)


def test_scene_away_from_the_origin(vplg, ctx):
    sc = scenes.make_scene("cornell", width=80, height=60)
    shift = np.array([5.0, 3.0, -7.0], np.float32)
    sc = dict(sc, tri=(sc["tri"] + shift).astype(np.float32))
    light = dict(sc["light"])
    light["pos"] = (np.asarray(light["pos"], np.float32) + shift).astype(np.float32)
    cam = dict(sc["camera"])
    for k in ("eye", "target"):
        cam[k] = (np.asarray(cam[k], np.float64) + shift).astype(np.float64)
    sc.update(light=light, camera=cam)
    S, gbo, vp, _ = _oracle_inputs(sc)
    _check_gather(vplg, ctx, sc, S, gbo, vp, np.arange(80 * 60), sc["params"], "cornell shifted")


def test_single_and_special_vpls(vplg, ctx):
    sc = scenes.make_scene("cornell", width=48, height=40)
    S, gbo, vp, _ = _oracle_inputs(sc)
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    gb = vplg.GBuffer.from_arrays(gbo["pos"], gbo["nrm"], gbo["alb"], gbo["tri"], 48, 40)
    f = gb.to_numpy()

    def gather(pos, nrm, I, tri):
        vid = vplg.vpls_upload(ctx, pos, nrm, I, tri)
        L = _gather_gpu(vplg, ctx, sid, vid, gb, sc["params"])
        vplg.vplset_release(ctx, vid)
        ref = S.gather(f["pos"], f["nrm"], f["alb"], f["tri"], np.asarray(pos, np.float32),
                       np.asarray(nrm, np.float32), np.asarray(I, np.float32), np.asarray(tri, np.int32))
        return L, ref

    # one VPL
    L, ref = gather(vp["pos"][:1], vp["nrm"][:1], vp["I"][:1], vp["tri"][:1])
    assert H.radiance_close(L, ref).all() and (ref > 0).any()
    # a VPL on the floor, in the floor's plane: every floor pixel's segment lies in the plane (cos = 0)
    floor_px = np.nonzero(f["nrm"][:, 1] > 0.99)[0]
    t_floor = int(f["tri"][floor_px[0]])
    on = np.array([[0.5, float(f["pos"][floor_px[0], 1]), 0.5]], np.float32)
    L, ref = gather(on, [[0, 1, 0]], [[1, 1, 1]], [t_floor])
    assert H.radiance_close(L, ref).all()
    assert np.all(L[floor_px] == 0)
    # zero intensity: exact zeros everywhere
    L, ref = gather(vp["pos"][:5], vp["nrm"][:5], np.zeros((5, 3), np.float32), vp["tri"][:5])
    assert np.all(L == 0) and np.all(ref == 0)
    vplg.scene_release(ctx, sid)


def test_size_limits_rejected_before_device_work(vplg, ctx):
    lib = vplg.lib()
    sc = scenes.make_scene("cornell", width=8, height=8)
    tri = np.ascontiguousarray(sc["tri"], np.float32)
    alb = np.ascontiguousarray(sc["albedo"], np.float32)
    fl = np.ascontiguousarray(sc["flags"], np.uint8)
    L = vplg.make_light(sc["light"])
    sid = C.c_uint64()
    # triangle count above 2^25 (checked before the arrays are read)
    rc = lib.vplg_scene_upload(ctx, tri.ctypes.data, alb.ctypes.data, fl.ctypes.data, (1 << 25) + 1, C.byref(L),
                               None, C.byref(sid))
    assert rc == vplg.EINVAL
    # a non-finite vertex
    bad = tri.copy()
    bad[3, 1, 2] = np.nan
    with pytest.raises(vplg.VplgError) as e:
        vplg.scene_upload(ctx, bad, alb, fl, sc["light"])
    assert e.value.code == vplg.EINVAL
    # a G-buffer above 2^28 pixels (no plane is touched: the size is checked first)
    s2 = vplg.scene_upload(ctx, tri, alb, fl, sc["light"])
    vid = vplg.vpls_upload(ctx, np.zeros((1, 3)), np.array([[0, 1, 0]]), np.ones((1, 3)), np.zeros(1, np.int32))
    small = vplg.GBuffer(8, 8)
    big = vplg.GBufferStruct()
    C.memmove(C.byref(big), C.byref(small.struct), C.sizeof(big))
    big.width, big.height = 1 << 15, 1 << 14
    rad = torch.zeros((3, 8, 8), dtype=torch.float32, device="cuda")
    gp = vplg.make_gather_params(sc["params"])
    rc = lib.vplg_gather(ctx, s2, vid, C.byref(big), vplg.radiance_planes(rad), C.byref(gp), None)
    assert rc == vplg.EINVAL
    cam = vplg.make_camera(sc["camera"])
    rc = lib.vplg_gbuffer_render(ctx, s2, C.byref(cam), C.byref(big), None)
    assert rc == vplg.EINVAL
    torch.cuda.synchronize()
    vplg.vplset_release(ctx, vid)
    vplg.scene_release(ctx, s2)


@pytest.mark.parametrize("name", ["cornell", "room20k"])
def test_scene_describe(vplg, ctx, name):
    """The resident scene's description: its triangle count, its bounds (the float32 vertex extremes,
    exactly), a BVH2 with both children present (inner nodes = leaves - 1, or one root over a single
    leaf), the depth limit, and device bytes that the context's usage accounts for."""
    sc = scenes.make_scene(name, width=8, height=8)
    used0 = vplg.context_usage(ctx)[0]
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    d = vplg.scene_describe(ctx, sid)
    assert d["n_tris"] == len(sc["tri"])
    v = sc["tri"].reshape(-1, 3)
    assert d["lo"] == v.min(axis=0).tolist() and d["hi"] == v.max(axis=0).tolist()
    assert 1 <= d["n_leaves"] <= d["n_tris"]
    assert d["n_nodes"] == max(1, d["n_leaves"] - 1)
    assert 1 <= d["max_depth"] <= 47
    assert d["device_bytes"] > 64 * d["n_tris"]
    assert vplg.context_usage(ctx)[0] - used0 >= d["device_bytes"]
    vplg.scene_release(ctx, sid)
    assert vplg.context_usage(ctx)[0] == used0
    with pytest.raises(vplg.VplgError) as e:
        vplg.scene_describe(ctx, sid)
    assert e.value.code == vplg.ENOTFOUND
