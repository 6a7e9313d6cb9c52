"""Image-quality harness of the paper's Section "Results", on the library's own GPU path.

The paper measures the root mean square error of indirect-lighting images against a reference
rendered by densely sampled instant radiosity (more than 200k VPLs), and compares its hybrid VPL
generation with plain instant radiosity at equal VPL counts.  Here:

* the reference is the gather of eq. (1) over a plain instant-radiosity VPL set of `ref_vpls`
  VPLs: the generation with d_near = 0 has no near patches, so every walk hit becomes a VPL;
* "plain IR at M" is the same with M VPLs; "hybrid at M" is the paper's method with the workload's
  near:far split of M, with the paper's walk (every near hit discarded) and with the variant that
  keeps near hits after the first bounce (`walk_near` = 1);
* the hybrid at a large count (`converged_vpls`) shows where each reading converges: the paper's
  walk loses the near-field light of the second and later bounces, the variant does not;
* RMSE is taken over the pixels with a hit, all three channels, of the indirect images only
  (the direct term is left out, as in the paper's statistics).

Everything runs through the C-ABI library (scene upload, G-buffer, generation, gather); nothing
here computes the method.
"""
import math

import numpy as np


def rmse(a, b, mask=None):
    """Root mean square difference of two [3, H, W] (or [n, 3]) images over the pixels in `mask`."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.ndim == 3:
        a = a.reshape(3, -1).T
        b = b.reshape(3, -1).T
    if mask is not None:
        m = np.asarray(mask, bool).reshape(-1)
        a, b = a[m], b[m]
    if len(a) == 0:
        return 0.0
    return float(math.sqrt(np.mean((a - b) ** 2)))


def plain_ir_params(params, n_vpls):
    """Plain instant radiosity with n_vpls VPLs: no near region, every walk hit deposits."""
    p = dict(params)
    p.update(k_near=0, n_far=int(n_vpls), d_near=0.0)
    p["max_paths"] = 64 * int(n_vpls) + 1024
    return p


def hybrid_params(params, n_vpls, walk_near=0):
    """The hybrid method with n_vpls VPLs, split near:far as in `params`."""
    p = dict(params, walk_near=walk_near)
    k, f = params["k_near"], params["n_far"]
    near = int(round(n_vpls * k / float(k + f)))
    p.update(k_near=near, n_far=int(n_vpls) - near)
    p["max_paths"] = 64 * int(n_vpls) + 1024
    return p


class Renderer:
    """Indirect images of one scene and camera through the library (one resident scene, one G-buffer)."""

    def __init__(self, vplg, ctx, scene, stream=None):
        import torch

        self.vplg, self.ctx, self.sc = vplg, ctx, scene
        cam = scene["camera"]
        self.W, self.H = cam["width"], cam["height"]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.sid = vplg.scene_upload(ctx, scene["tri"], scene["albedo"], scene["flags"], scene["light"],
                                     self.stream)
        self.gb = vplg.GBuffer(self.W, self.H)
        vplg.gbuffer_render(ctx, self.sid, cam, self.gb, self.stream)
        torch.cuda.synchronize()
        self.mask = (self.gb.tri >= 0).cpu().numpy().reshape(-1)

    def indirect(self, params):
        """Indirect radiance [3, H, W] (numpy float64) for generation parameters `params`, and its VPL count."""
        import torch

        v = self.vplg
        vid = v.vpls_generate(self.ctx, self.sid, self.sc["camera"], params, self.stream)
        rad = torch.zeros((3, self.H, self.W), dtype=torch.float32, device="cuda")
        v.gather(self.ctx, self.sid, vid, self.gb, rad, params, self.stream)
        torch.cuda.synchronize()
        n = v.vplset_count(self.ctx, vid)
        v.vplset_release(self.ctx, vid)
        return rad.cpu().numpy().astype(np.float64), n

    def direct(self, t_eps=1e-4):
        import torch

        rad = torch.zeros((3, self.H, self.W), dtype=torch.float32, device="cuda")
        self.vplg.direct(self.ctx, self.sid, self.gb, rad, t_eps, self.stream)
        torch.cuda.synchronize()
        return rad.cpu().numpy().astype(np.float64)

    def release(self):
        self.vplg.scene_release(self.ctx, self.sid)


def equal_sample_study(vplg, ctx, scene, counts=(1024, 5120), ref_vpls=262144, converged_vpls=65536):
    """RMSE of the hybrid (paper's walk and variant) and plain-IR indirect images at each VPL count against
    the dense-IR reference, plus the hybrid's RMSE at `converged_vpls` (its bias floor)."""
    r = Renderer(vplg, ctx, scene)
    try:
        ref, n_ref = r.indirect(plain_ir_params(scene["params"], ref_vpls))
        ref_rms = rmse(ref, np.zeros_like(ref), r.mask)
        rows = []
        for m in list(counts) + [converged_vpls]:
            hy, n_hy = r.indirect(hybrid_params(scene["params"], m))
            hv, _ = r.indirect(hybrid_params(scene["params"], m, walk_near=1))
            ir, n_ir = r.indirect(plain_ir_params(scene["params"], m))
            e_hy, e_hv, e_ir = rmse(hy, ref, r.mask), rmse(hv, ref, r.mask), rmse(ir, ref, r.mask)
            rows.append(dict(vpls=int(m), hybrid_vpls=int(n_hy), ir_vpls=int(n_ir), hybrid_rmse=e_hy,
                             hybrid_walk_near_rmse=e_hv, ir_rmse=e_ir,
                             ratio_ir_over_hybrid=e_ir / e_hy if e_hy > 0 else float("inf"),
                             ratio_ir_over_hybrid_walk_near=e_ir / e_hv if e_hv > 0 else float("inf")))
        return dict(scene=scene.get("name", "?"), reference_vpls=int(n_ref), ref_rms=ref_rms, rows=rows[:-1],
                    converged=rows[-1])
    finally:
        r.release()
