"""Render server: continuous admission under an HBM budget; every result equals the same request run alone,
and that lone run meets the oracle under the gather's parity protocol (tests/oracle_check.py), so the served
image does too."""
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
def env(vplg):
    ctx = vplg.context_create(0)
    scs = [scenes.make_scene("cornell"), scenes.procedural_room(21, 5, 6, 2, 2, d_near=7.0),
           scenes.procedural_room(22, 8, 6, 0, 0, d_near=7.0)]
    sids = [vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"]) for sc in scs]
    yield vplg, ctx, scs, sids
    vplg.context_destroy(ctx)


def _requests(scs, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        si = int(rng.integers(len(scs)))
        sc = scs[si]
        cam = dict(sc["camera"])
        cam["width"], cam["height"] = [(48, 40), (64, 64), (96, 72), (33, 29)][int(rng.integers(4))]
        m = int(rng.choice([128, 256, 512]))
        prm = scenes.default_params(k_near=m // 2, n_far=m - m // 2, d_near=sc["params"]["d_near"])
        out.append((si, cam, prm))
    return out


def _alone(vplg, ctx, sid, cam, prm, oracle=None):
    """The request run alone through the plain calls.  With oracle = (scene dict, pixels, label), its image is
    also checked against the oracle on the G-buffer and VPL set this run made."""
    gb = vplg.GBuffer(cam["width"], cam["height"])
    vplg.gbuffer_render(ctx, sid, cam, gb)
    vid = vplg.vpls_generate(ctx, sid, cam, prm)
    rad = torch.zeros((3, cam["height"], cam["width"]), dtype=torch.float32, device="cuda")
    vplg.gather(ctx, sid, vid, gb, rad, prm)
    torch.cuda.synchronize()
    if oracle is not None:
        sc, pixels, label = oracle
        L = rad.cpu().numpy().reshape(3, -1).T
        nd, n = OC.check_gather(vplg, ctx, orc.Scene.from_dict(sc), sid, vid, gb, L, pixels, prm, label,
                                min_lit=0.1)
        print(f"{label}: {nd} grazing disagreements of {n} cast pairs", flush=True)
    vplg.vplset_release(ctx, vid)
    return rad


@pytest.mark.parametrize("budget_mb,inflight", [(512, 8), (24, 8)])
def test_server_results_equal_alone(env, budget_mb, inflight):
    """Twelve mixed requests submitted at once; a 24 MB budget forces admission to wait for memory."""
    vplg, ctx, scs, sids = env
    reqs = _requests(scs, 12, seed=budget_mb)
    srv = vplg.server_start(ctx, budget_mb << 20, max_inflight=inflight, n_streams=4)
    try:
        outs, tickets, keep = [], [], []
        for si, cam, prm in reqs:
            rad = torch.full((3, cam["height"], cam["width"]), -1.0, dtype=torch.float32, device="cuda")
            r = vplg.make_request(sids[si], cam, prm, rad)
            keep.append(r)
            outs.append(rad)
            tickets.append(vplg.server_submit(srv, r))
        times = [vplg.server_wait(srv, t, timeout_ms=120000) for t in tickets]
        st = vplg.server_query(srv)
    finally:
        vplg.server_stop(srv)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_bytes"] <= budget_mb << 20
    if budget_mb == 512:
        assert st["peak_running"] >= 2, "requests should overlap on the device"
    for t in times:
        assert t["state"] == vplg.REQ_DONE and t["submit_ns"] <= t["admit_ns"] <= t["done_ns"]
    # the largest request of the mix is also held to the oracle, every pixel
    big = max(range(len(reqs)), key=lambda i: reqs[i][1]["width"] * reqs[i][1]["height"] *
              (reqs[i][2]["k_near"] + reqs[i][2]["n_far"]))
    for i, ((si, cam, prm), rad) in enumerate(zip(reqs, outs)):
        orq = None
        if i == big:
            orq = (scs[si], np.arange(cam["width"] * cam["height"]), f"served request {i} ({budget_mb} MB)")
        assert torch.equal(rad, _alone(vplg, ctx, sids[si], cam, prm, orq))


def test_server_large_view_equals_alone(env):
    """A 512 x 512 request: alone, its gather splits the last tiles into round-group items (at least four
    rounds of tiles); the server's gathers claim whole tiles.  The images must agree bit for bit."""
    vplg, ctx, scs, sids = env
    sc = scs[0]
    cam = dict(sc["camera"])
    cam["width"], cam["height"] = 512, 512
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert 64 * 64 >= 4 * 2 * cus, "the lone gather must split tiles for this view"
    prm = scenes.default_params(k_near=128, n_far=128, d_near=sc["params"]["d_near"])
    rad = torch.full((3, 512, 512), -1.0, dtype=torch.float32, device="cuda")
    srv = vplg.server_start(ctx, 512 << 20, max_inflight=2, n_streams=2)
    try:
        r = vplg.make_request(sids[0], cam, prm, rad)
        t = vplg.server_submit(srv, r)
        assert vplg.server_wait(srv, t, timeout_ms=120000)["state"] == vplg.REQ_DONE
    finally:
        vplg.server_stop(srv)
    pixels = np.sort(np.random.default_rng(17).choice(512 * 512, 4096, replace=False))
    alone = _alone(vplg, ctx, sids[0], cam, prm, (scs[0], pixels, "served 512x512 request"))
    assert (alone > 0).any()
    assert torch.equal(rad, alone)


def test_server_rejects_and_cancels(env):
    vplg, ctx, scs, sids = env
    si, cam, prm = _requests(scs, 1, seed=5)[0]
    rad = torch.zeros((3, cam["height"], cam["width"]), dtype=torch.float32, device="cuda")
    srv = vplg.server_start(ctx, 1 << 16, max_inflight=1, n_streams=1)
    try:
        with pytest.raises(vplg.VplgError) as e:
            vplg.server_submit(srv, vplg.make_request(sids[si], cam, prm, rad))
        assert e.value.code == vplg.EBUDGET
        bad = vplg.make_request(987654, cam, prm, rad)
        with pytest.raises(vplg.VplgError) as e:
            vplg.server_submit(srv, bad)
        assert e.value.code == vplg.ENOTFOUND
    finally:
        vplg.server_stop(srv)
    # a queue behind one slot: cancel the last request before it is admitted
    srv = vplg.server_start(ctx, 256 << 20, max_inflight=1, n_streams=1)
    try:
        keep, tickets = [], []
        for _ in range(6):
            r = vplg.make_request(sids[si], cam, prm, rad)
            keep.append(r)
            tickets.append(vplg.server_submit(srv, r))
        try:
            vplg.server_cancel(srv, tickets[-1])
            cancelled = True
        except vplg.VplgError as e:
            assert e.code == vplg.EBUSY
            cancelled = False
        for t in tickets[:-1]:
            assert vplg.server_wait(srv, t, timeout_ms=120000)["state"] == vplg.REQ_DONE
        if cancelled:
            assert vplg.server_poll(srv, tickets[-1])["state"] == vplg.REQ_CANCELLED
    finally:
        vplg.server_stop(srv)
