"""Image-quality harness of the paper's Section "Results", on the library's own GPU path.

The paper measures the root mean square error of indirect-lighting images against a reference
rendered by densely sampled instant radiosity (more than 200k VPLs), compares its hybrid VPL
generation with plain instant radiosity at equal VPL counts, and claims the hybrid reaches a
given quality 2-5 times faster.  Here:

* the reference is the gather of eq. (1) over a plain instant-radiosity VPL set of `ref_vpls`
  VPLs: the generation with d_near = 0 has no near patches, so every walk hit becomes a VPL;
* "plain IR at M" is the same with M VPLs (`ir`; `ir_keller`: Keller's path schedule, at most M
  VPLs); "hybrid at M" is the paper's method with the workload's near:far split of M, in the paper's
  reading (`paper`) and in the variants of the generation (`VARIANTS`: near walk hits kept after the
  first bounce, a near hit ending its path, brightness summed over the stratum's patches, jittered
  strata, Keller's path schedule with the near hits kept after the first bounce);
* RMSE is taken over the pixels with a hit, all three channels, of the indirect images only
  (the direct term is left out, as in the paper's statistics);
* a sweep renders every method at a geometric grid of VPL counts, timing generation and gather with
  HIP events on the rendering stream; the equal-sample table reads its rows, and the equal-RMSE
  study interpolates, per method, the VPL count and gather time that reach a target RMSE
  (log-log between grid points).

Everything runs through the C-ABI library (scene upload, G-buffer, generation, gather); nothing
here computes the method.
"""
import math

import numpy as np

# hybrid generation variants compared against plain IR (vplg_gen_params switches)
VARIANTS = {
    "paper": {},
    "walk_near1": {"walk_near": 1},
    "walk_near2": {"walk_near": 2},
    "set_sum": {"brightness": 1},
    "set_sum_walk_near1": {"brightness": 1, "walk_near": 1},
    "jitter": {"jitter": 1},
    "keller": {"walk_schedule": 1, "walk_near": 1},
}

DEFAULT_COUNTS = (256, 512, 1024, 2048, 4096, 5120, 8192, 16384, 32768, 65536)


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


def plain_ir_params(params, n_vpls, walk_schedule=0):
    """Plain instant radiosity with n_vpls VPLs: no near region, every walk hit deposits (with
    walk_schedule = 1 in Keller's path schedule, at most n_vpls VPLs)."""
    p = dict(params)
    p.update(k_near=0, n_far=int(n_vpls), d_near=0.0, walk_near=0, jitter=0, brightness=0,
             walk_schedule=int(walk_schedule))
    p["max_paths"] = 64 * int(n_vpls) + 1024
    return p


def hybrid_params(params, n_vpls, walk_near=0, **variant):
    """The hybrid method with n_vpls VPLs, split near:far as in `params`, with generation switches."""
    p = dict(params, walk_near=walk_near, jitter=0, brightness=0, walk_schedule=0)
    p.update(variant)
    k, f = params["k_near"], params["n_far"]
    near = int(round(n_vpls * k / float(k + f)))
    p.update(k_near=near, n_far=int(n_vpls) - near)
    p["max_paths"] = 64 * int(n_vpls) + 1024
    return p


def count_for_rmse(counts, errs, target):
    """Smallest VPL count at which a method reaches RMSE <= target, interpolated log-log between the
    last grid point above the target and the first at or below it.  Returns (count, exact) with
    exact False when the first grid point is already below the target (the count is an upper
    bound), or (None, False) when no grid point reaches it."""
    counts = [float(c) for c in counts]
    for i, e in enumerate(errs):
        if e <= target:
            if i == 0:
                return counts[0], False
            c0, c1, e0, e1 = counts[i - 1], counts[i], errs[i - 1], e
            if e0 <= e1 or e1 <= 0.0:
                return c1, True
            f = (math.log(e0) - math.log(target)) / (math.log(e0) - math.log(e1))
            return math.exp(math.log(c0) + f * (math.log(c1) - math.log(c0))), True
    return None, False


def interp_loglog(xs, ys, x):
    """y at x from the piecewise log-log line through (xs, ys) (xs increasing; clamped to the ends)."""
    if x <= xs[0]:
        return float(ys[0]) * x / float(xs[0]) if ys[0] > 0 else float(ys[0])
    for i in range(1, len(xs)):
        if x <= xs[i]:
            lx0, lx1 = math.log(xs[i - 1]), math.log(xs[i])
            ly0, ly1 = math.log(ys[i - 1]), math.log(ys[i])
            return math.exp(ly0 + (math.log(x) - lx0) / (lx1 - lx0) * (ly1 - ly0))
    return float(ys[-1]) * x / float(xs[-1])


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

    def indirect(self, params, timed=False):
        """Indirect radiance [3, H, W] (numpy float64) for generation parameters `params` and its VPL
        count; with timed=True also the generation and gather times in ms (HIP events on the stream)."""
        import torch

        v = self.vplg
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(self.stream)
        vid = v.vpls_generate(self.ctx, self.sid, self.sc["camera"], params, self.stream)
        ev[1].record(self.stream)
        rad = torch.zeros((3, self.H, self.W), dtype=torch.float32, device="cuda")
        v.gather(self.ctx, self.sid, vid, self.gb, rad, params, self.stream)
        ev[2].record(self.stream)
        torch.cuda.synchronize()
        n = v.vplset_count(self.ctx, vid)
        v.vplset_release(self.ctx, vid)
        img = rad.cpu().numpy().astype(np.float64)
        if timed:
            return img, n, ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
        return img, n

    def direct(self, t_eps=1e-4):
        import torch

        rad = torch.zeros((3, self.H, self.W), dtype=torch.float32, device="cuda")
        self.vplg.direct(self.ctx, self.sid, self.gb, rad, t_eps, self.stream)
        torch.cuda.synchronize()
        return rad.cpu().numpy().astype(np.float64)

    def release(self):
        self.vplg.scene_release(self.ctx, self.sid)


def sweep(vplg, ctx, scene, counts=DEFAULT_COUNTS, ref_vpls=262144, variants=VARIANTS, log=None):
    """Every method (plain IR and the hybrid variants) at every VPL count of `counts`: RMSE against the
    dense-IR reference, VPLs made, generation and gather ms.  Returns a dict with the reference's
    RMS and, per method, lists aligned with `counts`."""
    r = Renderer(vplg, ctx, scene)
    try:
        # a first gather outside the measurements (code loading, first-touch allocations)
        r.indirect(plain_ir_params(scene["params"], counts[0]))
        ref, n_ref, _, ref_ms = r.indirect(plain_ir_params(scene["params"], ref_vpls), timed=True)
        ref_rms = rmse(ref, np.zeros_like(ref), r.mask)
        methods = {"ir": lambda m: plain_ir_params(scene["params"], m),
                   "ir_keller": lambda m: plain_ir_params(scene["params"], m, walk_schedule=1)}
        for name, var in variants.items():
            methods[name] = (lambda m, var=var: hybrid_params(scene["params"], m, **var))
        out = {"scene": scene.get("name", "?"), "reference_vpls": int(n_ref), "reference_gather_ms": ref_ms,
               "ref_rms": ref_rms, "counts": [int(c) for c in counts], "methods": {}}
        for name, mk in methods.items():
            rows = {"rmse": [], "vpls": [], "gen_ms": [], "gather_ms": []}
            for m in counts:
                img, n, gms, tms = r.indirect(mk(m), timed=True)
                rows["rmse"].append(rmse(img, ref, r.mask))
                rows["vpls"].append(int(n))
                rows["gen_ms"].append(gms)
                rows["gather_ms"].append(tms)
            out["methods"][name] = rows
            if log:
                log(f"{out['scene']} {name}: " + " ".join(f"{c}:{e:.3g}" for c, e in zip(counts, rows["rmse"])))
        return out
    finally:
        r.release()


def equal_sample_table(sw, at=(1024, 5120)):
    """Rows of the equal-sample comparison (the paper's table): RMSE of every method at the counts `at`."""
    rows = []
    for m in at:
        i = sw["counts"].index(m)
        row = {"vpls": m}
        for name, d in sw["methods"].items():
            row[name] = d["rmse"][i]
        rows.append(row)
    return rows


def equal_rmse_table(sw, fractions=(0.2, 0.1, 0.05, 0.02, 0.01)):
    """The equal-RMSE time study: for targets = fraction x the reference's RMS, the VPL count and gather
    ms each method needs (None when its errors never reach the target on the grid), and plain IR's
    gather time over each hybrid method's."""
    counts = sw["counts"]
    rows = []
    for fr in fractions:
        target = fr * sw["ref_rms"]
        row = {"fraction": fr, "target_rmse": target, "methods": {}}
        for name, d in sw["methods"].items():
            c, exact = count_for_rmse(counts, d["rmse"], target)
            t = interp_loglog(counts, d["gather_ms"], c) if c is not None else None
            tg = interp_loglog(counts, d["gen_ms"], c) if c is not None else None
            row["methods"][name] = {"vpls": c, "exact": exact, "gather_ms": t, "gen_ms": tg}
        ir = row["methods"]["ir"]
        row["time_ratio_ir_over"] = {
            name: (ir["gather_ms"] / v["gather_ms"] if ir["gather_ms"] and v["gather_ms"] else None)
            for name, v in row["methods"].items() if name != "ir"}
        rows.append(row)
    return rows


def equal_sample_study(vplg, ctx, scene, counts=(1024, 5120), ref_vpls=262144, converged_vpls=65536,
                       variants=None):
    """RMSE of plain IR and of the hybrid variants at each of `counts` and at `converged_vpls` (where
    each reading ends up) against the dense-IR reference."""
    variants = variants if variants is not None else {k: VARIANTS[k] for k in ("paper", "walk_near1")}
    grid = tuple(counts) + (converged_vpls,)
    sw = sweep(vplg, ctx, scene, counts=grid, ref_vpls=ref_vpls, variants=variants)
    rows = equal_sample_table(sw, at=grid)
    return dict(scene=sw["scene"], reference_vpls=sw["reference_vpls"], ref_rms=sw["ref_rms"], rows=rows[:-1],
                converged=rows[-1], sweep=sw)
