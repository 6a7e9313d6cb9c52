"""vplg_gather_noalloc (work memory in the library's fixed per-device array) against vplg_gather (work
memory allocated per stream): the same kernels and summation order, so the radiance must agree bit for
bit.  Two calls in a row, the second on a smaller view; the first view is large enough that its last
tiles are split into round-group items, whose sums go through the array."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2203_11484_amd import scenes  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vplg():
    from paper_2203_11484_amd import vplg as v
    v.lib()
    return v


def _view(vplg, ctx, name, size):
    sc = scenes.make_scene(name, width=size[0], height=size[1])
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"])
    gb = vplg.GBuffer(*size)
    vplg.gbuffer_render(ctx, sid, sc["camera"], gb)
    vid = vplg.vpls_generate(ctx, sid, sc["camera"], sc["params"])
    torch.cuda.synchronize()
    return sc, sid, gb, vid


def test_noalloc_equals_gather(vplg):
    ctx = vplg.context_create(0)
    try:
        big = _view(vplg, ctx, "room20k", (512, 512))
        small = _view(vplg, ctx, "cornell", (100, 75))
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        # 4,096 tiles at 16 waves per tile (2 resident workgroups per CU): at least four rounds, so the
        # lone gather splits its last two rounds into round-group items
        assert 64 * 64 >= 4 * 2 * cus
        for label, (sc, sid, gb, vid) in (("room20k 512x512", big), ("cornell 100x75", small)):
            print(f"noalloc: {label}", flush=True)
            ref = torch.full((3, gb.height, gb.width), -1.0, dtype=torch.float32, device="cuda")
            out = torch.full_like(ref, -2.0)
            vplg.gather(ctx, sid, vid, gb, ref, sc["params"])
            vplg.gather_noalloc(ctx, sid, vid, gb, out, sc["params"])
            torch.cuda.synchronize()
            assert (ref > 0).any()
            assert torch.equal(out, ref), f"{label}: {(out != ref).sum().item()} values differ"
        # every explicit tile shape on the small view, one after another on the shared array
        sc, sid, gb, vid = small
        for tv in (1, 2, 4, 8, 16):
            gp = vplg.make_gather_params(sc["params"])
            gp.tile_vpl = tv
            ref = torch.zeros((3, gb.height, gb.width), dtype=torch.float32, device="cuda")
            out = torch.full_like(ref, -2.0)
            vplg.gather(ctx, sid, vid, gb, ref, gp)
            vplg.gather_noalloc(ctx, sid, vid, gb, out, gp)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), f"tile_vpl {tv}"
        for sc, sid, gb, vid in (big, small):
            vplg.vplset_release(ctx, vid)
            vplg.scene_release(ctx, sid)
    finally:
        vplg.context_destroy(ctx)


def test_noalloc_rejects_bad_arguments(vplg):
    ctx = vplg.context_create(0)
    try:
        sc, sid, gb, vid = _view(vplg, ctx, "cornell", (16, 8))
        rad = torch.zeros((3, 8, 16), dtype=torch.float32, device="cuda")
        with pytest.raises(vplg.VplgError) as e:
            vplg.gather_noalloc(ctx, sid, 123456789, gb, rad, sc["params"])
        assert e.value.code == vplg.ENOTFOUND
        gp = vplg.make_gather_params(sc["params"])
        gp.tile_vpl = 3
        with pytest.raises(vplg.VplgError) as e:
            vplg.gather_noalloc(ctx, sid, vid, gb, rad, gp)
        assert e.value.code == vplg.EINVAL
        vplg.gather_noalloc(ctx, sid, vid, gb, rad, sc["params"])
        torch.cuda.synchronize()
        assert np.isfinite(rad.cpu().numpy()).all()
    finally:
        vplg.context_destroy(ctx)
