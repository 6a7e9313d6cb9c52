"""The gather's parity protocol against the FP64 oracle, for any G-buffer and VPL set on the device.

The oracle evaluates eq. (1) (indirect part) on the very inputs the GPU gather read: the G-buffer planes and
the VPL set are downloaded from the device, whoever made them (the oracle's own arrays uploaded, the GPU's
G-buffer render and VPL generation, a served request's lone twin).  Then:

* visibility: the GPU's bits (the gather's own shadow-ray code, through the visibility dump) against the
  oracle's plain definition, pair by pair; every disagreement must be grazing (moving an endpoint by BAND =
  1e-6 of the scene diagonal along a coordinate axis flips the oracle's answer: 1.5e-5 in the rooms, about
  fifteen FP32 ulps of their coordinates; a segment between two points of one flat face lies in the face's
  plane, where the face's own triangles, rounded to FP32, sit a few 1e-7 off it and cross it: the GPU's
  parallel cut passes them, the oracle meets them, and only moves of about 1e-6 of the diagonal flip that)
  and, over the pairs whose shadow ray the gather casts, at most 1e-4 of them;
* radiance: per channel within 1e-4 relative (floor 1e-3 of the channel mean, exact zeros stay zero), with
  the oracle re-evaluated on the GPU's bit for the disagreeing pairs.
"""
import numpy as np

from tests import helpers as H

# grazing band of the visibility protocol, relative to the scene's bounding-box diagonal
BAND = 1e-6


def dump_visibility(vplg, ctx, sid, vid, gb, pixels, M, prm):
    import torch

    words = (M + 31) // 32
    pix = torch.from_numpy(np.ascontiguousarray(pixels, np.int32)).cuda()
    bits = torch.zeros((len(pixels), max(words, 1)), dtype=torch.int32, device="cuda")
    vplg.gather_visibility_dump(ctx, sid, vid, gb, pix, bits, prm)
    torch.cuda.synchronize()
    b = bits.cpu().numpy().view(np.uint32)
    k = np.arange(M)
    return ((b[:, k // 32] >> (k % 32).astype(np.uint32)) & 1).astype(np.uint8)


def check_gather(vplg, ctx, S, sid, vid, gb, L_gpu, pixels, prm, label, min_lit=0.3):
    """L_gpu: the GPU radiance of the whole view, [P, 3]; pixels: the pixel indices to check.
    Returns (cast-pair disagreements, cast pairs)."""
    pixels = np.asarray(pixels)
    f = gb.to_numpy()
    vp = vplg.vpls_download(ctx, vid)
    M = int(vp["n"])
    gpos, gnrm, galb, gtri = f["pos"][pixels], f["nrm"][pixels], f["alb"][pixels], f["tri"][pixels]
    vpos, vnrm, vI, vtri = vp["pos"][:M], vp["nrm"][:M], vp["I"][:M], vp["tri"][:M]
    L = np.asarray(L_gpu, np.float64)[pixels]
    vis_gpu = dump_visibility(vplg, ctx, sid, vid, gb, pixels, M, prm)
    vis_ref = S.vis_matrix(gpos, gtri, vpos, vtri, eps=prm["t_eps"])
    dis = np.nonzero(vis_gpu != vis_ref)
    # pairs whose shadow ray the gather casts: both cosines above the 1e-5 grazing epsilon
    dvec = vpos.astype(np.float64)[None, :, :] - gpos.astype(np.float64)[:, None, :]
    dlen = np.maximum(np.linalg.norm(dvec, axis=2), 1e-300)
    cp = np.einsum("pkc,pc->pk", dvec, gnrm.astype(np.float64)) / dlen
    ck = -np.einsum("pkc,kc->pk", dvec, vnrm.astype(np.float64)) / dlen
    cast = (cp > 1e-5) & (ck > 1e-5) & (gtri[:, None] >= 0)
    n_pairs = int(cast.sum())
    n_dis_cast = int(cast[dis].sum())
    print(f"{label}: {len(dis[0])} disagreements over all {vis_ref.size} pairs, {n_dis_cast} over {n_pairs} "
          f"cast pairs", flush=True)
    if len(dis[0]):
        xi, ki = dis
        graz = S.grazing(gpos[xi], gtri[xi], vpos[ki], vtri[ki], eps=prm["t_eps"], delta_rel=BAND)
        # reported, not asserted: how many would still be excused by a band ten times narrower
        finer = int(S.grazing(gpos[xi], gtri[xi], vpos[ki], vtri[ki], eps=prm["t_eps"], delta_rel=BAND / 10).sum())
        print(f"{label}: {int(graz.sum())} of {len(xi)} disagreements grazing at {BAND:g} of the diagonal, "
              f"{finer} at {BAND / 10:g}", flush=True)
        for j in np.nonzero(graz == 0)[0][:20]:
            print(f"{label}: non-grazing pair px={pixels[xi[j]]} tri_p={gtri[xi[j]]} x={gpos[xi[j]].tolist()} "
                  f"vpl={ki[j]} tri_k={vtri[ki[j]]} y={vpos[ki[j]].tolist()} "
                  f"gpu={vis_gpu[xi[j], ki[j]]} ref={vis_ref[xi[j], ki[j]]}", flush=True)
        assert graz.all(), f"{label}: {(graz == 0).sum()} non-grazing visibility disagreements"
    assert n_dis_cast <= 1e-4 * n_pairs + 0.5, f"{label}: {n_dis_cast} disagreements of {n_pairs} cast pairs"
    ov = (dis[0].astype(np.int32), dis[1].astype(np.int32), vis_gpu[dis]) if len(dis[0]) else None
    L_ref = S.gather(gpos, gnrm, galb, gtri, vpos, vnrm, vI, vtri, C=prm["g_clamp"], eps=prm["t_eps"], overrides=ov)
    ok = H.radiance_close(L, L_ref, rel=1e-4)
    assert ok.all(), f"{label}: {(~ok).sum()} of {len(ok)} pixels outside 1e-4"
    if min_lit is not None:
        assert (L_ref > 0).mean() > min_lit, f"{label}: too few lit pixels to be a check"
    return n_dis_cast, n_pairs
