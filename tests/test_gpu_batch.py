"""Batched gather (one persistent, graph-replayed launch over many views), the tile autotuner, and how a lone
gather's work is dealt out: its split tail equals whole tiles, a captured gather replays bit for bit, and
gathers on two streams at once keep to their own work memory."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc  # noqa: E402
from paper_2203_11484_amd import scenes  # noqa: E402
from tests import oracle_check as OC  # noqa: E402

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


def _views(vplg, ctx):
    """Seven views over two scenes: ragged sizes, different VPL budgets and tile shapes (1 to 16 waves per
    tile, pixel blocks of 1, 2 and 4 tiles, so the batch runs in 16-wave workgroups; a subset whose blocks
    take at most 8 waves runs in 8-wave ones)."""
    sc_a = scenes.make_scene("cornell")
    sc_b = scenes.procedural_room(11, 6, 6, 2, 2, k_near=192, n_far=320, d_near=7.0)
    ids = {}
    for key, sc in (("a", sc_a), ("b", sc_b)):
        ids[key] = (sc, vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"]))
    specs = [("a", 40, 36, 1, 256), ("b", 64, 64, 8, 64), ("a", 100, 75, 4, 128), ("b", 72, 40, 2, 256),
             ("b", 33, 17, 8, 0), ("a", 128, 96, 0, 0), ("b", 56, 48, 16, 0)]
    views = []
    for key, w, h, tv, px in specs:
        sc, sid = ids[key]
        cam = dict(sc["camera"])
        cam["width"], cam["height"] = w, h
        gb = vplg.GBuffer(w, h)
        vplg.gbuffer_render(ctx, sid, cam, gb)
        vid = vplg.vpls_generate(ctx, sid, cam, sc["params"])
        rad = torch.full((3, h, w), -1.0, dtype=torch.float32, device="cuda")
        gp = vplg.make_gather_params(sc["params"])
        gp.tile_vpl = tv
        gp.tile_px = px
        views.append(dict(scene=sid, vplset=vid, gb=gb, radiance=rad, params=gp, sc=sc, cam=cam))
    return views


def test_batch_equals_per_view_and_replays(vplg, ctx):
    views = _views(vplg, ctx)
    refs = []
    for v in views:
        # tile_vpl 0 resolves to 8 in a batch (untuned); a lone gather's rule would pick 16 for these sizes
        gp = vplg.make_gather_params(v["sc"]["params"])
        gp.tile_vpl = v["params"].tile_vpl or 8
        gp.tile_px = v["params"].tile_px
        r = torch.zeros_like(v["radiance"])
        vplg.gather(ctx, v["scene"], v["vplset"], v["gb"], r, gp)
        refs.append(r)
    torch.cuda.synchronize()
    for rep in range(3):
        for v in views:
            v["radiance"].fill_(-1.0)
        vplg.gather_batch(ctx, views)
        torch.cuda.synchronize()
        for i, v in enumerate(views):
            assert torch.equal(v["radiance"], refs[i]), f"replay {rep}: view {i} differs from its single gather"
        # eager work between replays
        _ = (torch.ones(1 << 20, device="cuda") * 2).sum().item()
    # a different subset and order in the next replay (blocks of at most 8 waves: 8-wave workgroups)
    sub = [views[4], views[0], views[3]]
    for v in sub:
        v["radiance"].fill_(-1.0)
    vplg.gather_batch(ctx, sub)
    torch.cuda.synchronize()
    for v in sub:
        i = views.index(v)
        assert torch.equal(v["radiance"], refs[i])


@pytest.mark.parametrize("size,tile_vpl", [((512, 512), 16), ((1024, 1024), 8)])
def test_split_tail_equals_whole_tiles(vplg, ctx, size, tile_vpl):
    """A lone gather of a view with at least four rounds of tiles claims its last two rounds as
    quarter-tile round-group items (summed by a second kernel); a batch never splits.  The two must
    agree bit for bit, since a tile's sum is fixed as chunk, round-group, wave and group order."""
    w, h = size
    tiles = ((w + 7) // 8) * ((h + 7) // 8)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    per_cu = 2 if tile_vpl == 16 else 4  # resident workgroups of that size (8 waves per SIMD)
    assert tiles >= 4 * per_cu * cus, "the view must be large enough for the lone gather to split tiles"
    sc = scenes.make_scene("cornell", width=w, height=h)
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    gb = vplg.GBuffer(w, h)
    vplg.gbuffer_render(ctx, sid, sc["camera"], gb)
    vid = vplg.vpls_generate(ctx, sid, sc["camera"], sc["params"])
    gp = vplg.make_gather_params(sc["params"])
    gp.tile_vpl = tile_vpl
    lone = torch.full((3, h, w), -1.0, dtype=torch.float32, device="cuda")
    vplg.gather(ctx, sid, vid, gb, lone, gp)
    view = dict(scene=sid, vplset=vid, gb=gb, radiance=torch.full_like(lone, -1.0), params=gp)
    vplg.gather_batch(ctx, [view])
    torch.cuda.synchronize()
    assert (lone >= 0).all() and (lone > 0).any()
    assert torch.equal(view["radiance"], lone)
    vplg.vplset_release(ctx, vid)
    vplg.scene_release(ctx, sid)


@pytest.mark.parametrize("size", [(512, 512), (100, 75)])
def test_pixel_blocks_equal_single_tiles(vplg, ctx, size):
    """Every tile shape of a lone gather: pixel blocks of 2 (16 x 8) and 4 (16 x 16) tiles give, bit for bit,
    the single-tile result at the same waves per tile, with (512 x 512: at least four rounds of blocks) and
    without (100 x 75, ragged: blocks hang over the edges) the split tail; and so does the batch."""
    w, h = size
    sc = scenes.make_scene("cornell", width=w, height=h)
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    gb = vplg.GBuffer(w, h)
    vplg.gbuffer_render(ctx, sid, sc["camera"], gb)
    vid = vplg.vpls_generate(ctx, sid, sc["camera"], sc["params"])
    for tv in (1, 2, 4, 8):
        outs = {}
        for px in (64, 128, 256):
            if px // 64 * tv > 16:
                continue
            gp = vplg.make_gather_params(sc["params"])
            gp.tile_vpl, gp.tile_px = tv, px
            outs[px] = torch.full((3, h, w), -1.0, dtype=torch.float32, device="cuda")
            vplg.gather(ctx, sid, vid, gb, outs[px], gp)
            view = dict(scene=sid, vplset=vid, gb=gb, radiance=torch.full_like(outs[px], -1.0), params=gp)
            vplg.gather_batch(ctx, [view])
            torch.cuda.synchronize()
            assert torch.equal(view["radiance"], outs[px]), f"tile_vpl {tv} tile_px {px}: batch != lone"
        assert (outs[64] >= 0).all() and (outs[64] > 0).any()
        for px, o in outs.items():
            assert torch.equal(o, outs[64]), f"tile_vpl {tv}: tile_px {px} differs from 64"
    vplg.vplset_release(ctx, vid)
    vplg.scene_release(ctx, sid)


def test_gather_graph_replays(vplg, ctx):
    """A lone gather (with its split tail: 512 x 512) captured into a HIP graph on a stream that has
    already run a gather (its work memory exists), replayed three times with eager work and
    synchronisation between replays; every replay equals the eager gather bit for bit."""
    w = h = 512
    sc = scenes.make_scene("cornell", width=w, height=h)
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    gb = vplg.GBuffer(w, h)
    vplg.gbuffer_render(ctx, sid, sc["camera"], gb)
    vid = vplg.vpls_generate(ctx, sid, sc["camera"], sc["params"])
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    eager = torch.zeros((3, h, w), dtype=torch.float32, device="cuda")
    vplg.gather(ctx, sid, vid, gb, eager, sc["params"], s)
    s.synchronize()
    out = torch.full_like(eager, -1.0)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        vplg.gather(ctx, sid, vid, gb, out, sc["params"], s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"
        _ = (torch.ones(1 << 20, device="cuda") * 2).sum().item()
    del g
    vplg.vplset_release(ctx, vid)
    vplg.scene_release(ctx, sid)


def test_concurrent_gathers_on_two_streams(vplg, ctx):
    """Two lone gathers with split tails (512 x 512) running at once on two streams, over different VPL
    sets: each stream has its own work memory (tile counter, round-group sums), so each result equals
    the same gather run alone, bit for bit."""
    w = h = 512
    sc = scenes.make_scene("cornell", width=w, height=h)
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    gb = vplg.GBuffer(w, h)
    vplg.gbuffer_render(ctx, sid, sc["camera"], gb)
    vids = [vplg.vpls_generate(ctx, sid, sc["camera"], sc["params"]),
            vplg.vpls_generate(ctx, sid, sc["camera"], dict(sc["params"], k_near=128, n_far=384))]
    torch.cuda.synchronize()
    refs = []
    for vid in vids:
        r = torch.zeros((3, h, w), dtype=torch.float32, device="cuda")
        vplg.gather(ctx, sid, vid, gb, r, sc["params"])
        torch.cuda.synchronize()
        refs.append(r)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(2):
        outs = [torch.full_like(refs[0], -1.0) for _ in vids]
        torch.cuda.synchronize()
        for i in range(2):
            vplg.gather(ctx, sid, vids[i], gb, outs[i], sc["params"], streams[i])
        torch.cuda.synchronize()
        for i in range(2):
            assert torch.equal(outs[i], refs[i]), f"rep {rep} stream {i}"
    for vid in vids:
        vplg.vplset_release(ctx, vid)
    vplg.scene_release(ctx, sid)


def test_untuned_tile_vpl_rule(vplg, ctx):
    """tile_vpl 0 on an untuned shape: a lone gather takes 16 waves per tile below 32 tiles per compute
    unit (bit for bit the explicit 16), a view in a batch takes 8."""
    v = _views(vplg, ctx)[5]
    assert v["params"].tile_vpl == 0
    out = {}
    for tv in (0, 8, 16):
        gp = vplg.make_gather_params(v["sc"]["params"])
        gp.tile_vpl = tv
        out[tv] = torch.zeros_like(v["radiance"])
        vplg.gather(ctx, v["scene"], v["vplset"], v["gb"], out[tv], gp)
    v["radiance"].fill_(-1.0)
    vplg.gather_batch(ctx, [v])
    torch.cuda.synchronize()
    assert torch.equal(out[0], out[16])
    assert torch.equal(v["radiance"], out[8])
    assert torch.allclose(out[8], out[16], rtol=1e-5, atol=1e-7)


def test_batch_view_matches_oracle(vplg, ctx):
    """Batched views against the oracle under the gather's parity protocol (tests/oracle_check.py), every
    pixel: one view on the oracle's own G-buffer and VPLs, batched beside two others, and two of the batch's
    views on the G-buffers and VPL sets the GPU made (downloaded for the oracle)."""
    sc = scenes.make_scene("cornell", width=48, height=40)
    S = orc.Scene.from_dict(sc)
    gbo = S.gbuffer(sc["camera"])
    g = S.generate(sc["camera"], sc["light"], sc["params"])
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    gb = vplg.GBuffer.from_arrays(gbo["pos"], gbo["nrm"], gbo["alb"], gbo["tri"], 48, 40)
    vid = vplg.vpls_upload(ctx, g["pos"], g["nrm"], g["I"], g["tri"])
    views = _views(vplg, ctx)
    other = [views[1], views[3]]
    rad = torch.zeros((3, 40, 48), dtype=torch.float32, device="cuda")
    vplg.gather_batch(ctx, other + [dict(scene=sid, vplset=vid, gb=gb, radiance=rad, params=sc["params"])])
    torch.cuda.synchronize()
    L_gpu = rad.cpu().numpy().reshape(3, -1).T
    OC.check_gather(vplg, ctx, S, sid, vid, gb, L_gpu, np.arange(48 * 40), sc["params"], "batched cornell view")
    for j, v in enumerate(other):
        Sv = orc.Scene.from_dict(v["sc"])
        P = v["gb"].width * v["gb"].height
        Lv = v["radiance"].cpu().numpy().reshape(3, -1).T
        OC.check_gather(vplg, ctx, Sv, v["scene"], v["vplset"], v["gb"], Lv, np.arange(P), v["sc"]["params"],
                        f"batched room view {j}", min_lit=0.1)


def test_batch_rejects_bad_views(vplg, ctx):
    views = _views(vplg, ctx)[:2]
    bad = dict(views[1])
    bad["vplset"] = 123456789
    with pytest.raises(vplg.VplgError) as e:
        vplg.gather_batch(ctx, [views[0], bad])
    assert e.value.code == vplg.ENOTFOUND
    for tv, px in ((3, 0), (2, 96), (8, 256), (16, 128)):
        gp = vplg.make_gather_params()
        gp.tile_vpl, gp.tile_px = tv, px
        big = dict(views[0])
        big["params"] = gp
        with pytest.raises(vplg.VplgError) as e:
            vplg.gather_batch(ctx, [big])
        assert e.value.code == vplg.EINVAL, (tv, px)
        with pytest.raises(vplg.VplgError) as e:
            vplg.gather(ctx, big["scene"], big["vplset"], big["gb"], big["radiance"], gp)
        assert e.value.code == vplg.EINVAL, (tv, px)


def test_autotune_roundtrip(vplg, ctx, tmp_path):
    v = _views(vplg, ctx)[1]
    best = vplg.autotune(ctx, v["scene"], v["vplset"], v["gb"], v["radiance"], v["params"])
    assert best[0] in (1, 2, 4, 8, 16) and best[1] in (64, 128, 256) and best[1] // 64 * best[0] <= 16
    n = vplg.vplset_count(ctx, v["vplset"])
    assert vplg.autotune_lookup(ctx, v["gb"].width, v["gb"].height, n) == best
    path = os.path.join(tmp_path, "tune.txt")
    vplg.autotune_save(ctx, path)
    c2 = vplg.context_create(0)
    try:
        # untuned: 8 x 8 blocks and the tile-count rule (16 waves below 32 tiles per compute unit, else 8);
        # in a batch, 8
        tiles = ((v["gb"].width + 7) // 8) * ((v["gb"].height + 7) // 8)
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        assert vplg.autotune_lookup(c2, v["gb"].width, v["gb"].height, n) == (16 if tiles < 32 * cus else 8, 64)
        assert vplg.autotune_lookup(c2, 1920, 1080, n) == (16 if 240 * 135 < 32 * cus else 8, 64)
        assert vplg.autotune_lookup(c2, 1920, 1080, n, batched=True) == (8, 64)
        vplg.autotune_load(c2, path)
        assert vplg.autotune_lookup(c2, v["gb"].width, v["gb"].height, n) == best
    finally:
        vplg.context_destroy(c2)


def test_autotune_batch(vplg, ctx, tmp_path):
    """The batch autotuner on open views (tile shape left to it): each bucket's shape comes from timing that
    bucket's views as a batch; the tuned shapes are kept only if the whole batch is faster with them.  Either
    way every view then equals a lone gather at the shape the batch resolved for it, and the batched table
    survives a save and load."""
    views = _views(vplg, ctx)
    for v in views:
        v["params"] = vplg.make_gather_params(v["sc"]["params"])  # open: tile_vpl 0, tile_px 0
    c = ctx  # the views' scenes and VPL sets live in this context
    kept = vplg.autotune_batch(c, views)
    assert 0 <= kept <= len(views)
    for v in views:
        v["radiance"].fill_(-1.0)
    vplg.gather_batch(c, views)
    torch.cuda.synchronize()
    shapes = set()
    for i, v in enumerate(views):
        n = vplg.vplset_count(c, v["vplset"])
        w, px = vplg.autotune_lookup(c, v["gb"].width, v["gb"].height, n, batched=True)
        shapes.add((w, px))
        assert px // 64 * w <= 16
        gp = vplg.make_gather_params(v["sc"]["params"])
        gp.tile_vpl, gp.tile_px = w, px
        r = torch.zeros_like(v["radiance"])
        vplg.gather(c, v["scene"], v["vplset"], v["gb"], r, gp)
        torch.cuda.synchronize()
        assert torch.equal(v["radiance"], r), f"view {i}"
    print(f"batch autotuner kept {kept} buckets; shapes {sorted(shapes)}", flush=True)
    path = os.path.join(tmp_path, "tune_batch.txt")
    vplg.autotune_save(c, path)
    c2 = vplg.context_create(0)
    try:
        vplg.autotune_load(c2, path)
        for v in views:
            n = vplg.vplset_count(c, v["vplset"])
            assert (vplg.autotune_lookup(c2, v["gb"].width, v["gb"].height, n, batched=True) ==
                    vplg.autotune_lookup(c, v["gb"].width, v["gb"].height, n, batched=True))
    finally:
        vplg.context_destroy(c2)
