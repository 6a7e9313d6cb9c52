#!/usr/bin/env python
"""Benchmark of the hybrid-VPL hot path on one MI355X.

One step = G-buffer render + VPL generation (near patch VPLs + far walk) +
the VPL gather (eq. (1), indirect part) for one view of the workload, with
the scene (and its BVH) resident in HBM before the timed region.  The metric
is VPL-pixel shading pairs per second including visibility: P * M pairs per
step divided by the step time.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload room200k] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak (published)
# algorithmic FLOPs (FMA = 2; min, max and compares not counted): per pair of
# the shading formula; per cast shadow ray its slab set-up (3 reciprocals, 3
# products) and watertight set-up (reciprocal, 2 shear products, |d|^2/d_kz^2);
# per BVH2 node the ray's own segment entered (two slab tests of 6 FMAs); per
# triangle of a leaf the ray's own segment entered, one watertight
# test (9 differences, 6 shear FMAs, 3 edge functions, determinant, T, t and
# the parallel cut)
FLOP_PAIR, FLOP_RAY, FLOP_NODE, FLOP_TRI = 27, 13, 24, 44


def measured_traffic(workload):
    """HBM bytes per gather launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, scaled by
    the same counters' reading of a 1 GiB copy; None unless the gather source and the BVH builder (whose tree
    the gather walks) are the ones measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_gather_{workload}_hbm.json")
    csrc = os.path.join(ROOT, "paper_2203_11484_amd", "csrc")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    for name, key in (("k_gather.hip", "kernel_source_sha256"), ("bvh_build.cpp", "builder_source_sha256")):
        if hashlib.sha256(open(os.path.join(csrc, name), "rb").read()).hexdigest() != d.get(key):
            return None
    return d["traffic_bytes_per_launch"]


def cpu_baseline(sc, target_s, seed=0):
    """The FP64 oracle's gather timed on the host cores on a bounded pixel sample of the workload."""
    import numpy as np
    from oracle import oracle as orc

    S = orc.Scene.from_dict(sc)
    gb = S.gbuffer(sc["camera"])
    g = S.generate(sc["camera"], sc["light"], sc["params"])
    f32 = lambda a: a.astype(np.float32)  # noqa: E731
    P = len(gb["tri"])
    rng = np.random.default_rng(seed)
    order = rng.permutation(P)
    threads = orc.num_threads()

    def run(n):
        idx = np.sort(order[:n])
        t = time.perf_counter()
        S.gather(f32(gb["pos"][idx]), f32(gb["nrm"][idx]), f32(gb["alb"][idx]), gb["tri"][idx], f32(g["pos"]),
                 f32(g["nrm"]), f32(g["I"]), g["tri"], C=sc["params"]["g_clamp"], eps=sc["params"]["t_eps"],
                 nthreads=threads)
        return time.perf_counter() - t

    probe = min(P, max(threads * 4, 64))
    dt = run(probe)
    n = int(min(P, max(probe, probe * target_s / max(dt, 1e-6))))
    dt = run(n)
    pairs = n * g["n"]
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=pairs / dt, unit="pairs/s", cores=threads, kind="oracle", cpu=model,
                host_cpus=os.cpu_count(),
                sample=f"{n} seeded random pixels of the {sc['camera']['width']}x{sc['camera']['height']} image x "
                       f"{g['n']} VPLs ({pairs} pairs, FP64, {dt:.1f} s); the full frame's pairs/s is extrapolated "
                       f"from this sample")


def bench_batch(args):
    """64 views over 8 seeded rooms of 5k-200k triangles, resolutions from {256^2, 512^2, 1024^2, 1920x1080},
    VPL budgets log-uniform in [1024, 16384]: one persistent batched launch against 64 plain launches."""
    import numpy as np
    import torch

    from paper_2203_11484_amd import scenes, vplg

    scs = scenes.batch_scenes()
    vs = scenes.batch_views(scs)
    torch.cuda.init()
    ctx = vplg.context_create(0)
    stream = torch.cuda.current_stream()
    sids = [vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"], stream) for sc in scs]
    views = []
    pairs = 0
    for v in vs:
        cam = v["camera"]
        gb = vplg.GBuffer(cam["width"], cam["height"])
        vplg.gbuffer_render(ctx, sids[v["scene"]], cam, gb, stream)
        vid = vplg.vpls_generate(ctx, sids[v["scene"]], cam, v["params"], stream)
        rad = torch.zeros((3, cam["height"], cam["width"]), dtype=torch.float32, device="cuda")
        views.append(dict(scene=sids[v["scene"]], vplset=vid, gb=gb, radiance=rad, params=dict(v["params"])))
    torch.cuda.synchronize()
    for v in views:
        pairs += v["gb"].width * v["gb"].height * vplg.vplset_count(ctx, v["vplset"])
    print(f"bench: batch of {len(views)} views, {pairs:.3e} pairs", file=sys.stderr, flush=True)
    def time_batch():
        vplg.gather_batch(ctx, views, stream)  # warm-up (the first call captures the graph)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            vplg.gather_batch(ctx, views, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps / 1e3

    t_untuned = time_batch()
    print(f"bench: untuned batch {t_untuned * 1e3:.1f} ms", file=sys.stderr, flush=True)
    tuned = {}
    t_batch = t_untuned
    if args.autotune:
        kept = vplg.autotune_batch(ctx, views, stream)
        for v in views:
            n = vplg.vplset_count(ctx, v["vplset"])
            key = f"{v['gb'].width}x{v['gb'].height}_{n}"
            tuned[key] = vplg.autotune_lookup(ctx, v["gb"].width, v["gb"].height, n, batched=True)
        print(f"bench: batch autotuner kept {kept} buckets: {tuned}", file=sys.stderr, flush=True)
        t_batch = time_batch()
        print(f"bench: tuned batch {t_batch * 1e3:.1f} ms", file=sys.stderr, flush=True)
    ref = [v["radiance"].clone() for v in views]
    # the plain one-frame-per-launch gather of the same views, each in the tile shape the batch resolved for it
    plain = []
    for v in views:
        w, px = vplg.autotune_lookup(ctx, v["gb"].width, v["gb"].height, vplg.vplset_count(ctx, v["vplset"]),
                                     batched=True)
        plain.append(dict(v["params"], tile_vpl=w, tile_px=px))
    for v, p in zip(views, plain):  # warm
        vplg.gather(ctx, v["scene"], v["vplset"], v["gb"], v["radiance"], p, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for v, p in zip(views, plain):
        vplg.gather(ctx, v["scene"], v["vplset"], v["gb"], v["radiance"], p, stream)
    ev[1].record(stream)
    torch.cuda.synchronize()
    same = all(torch.equal(a, v["radiance"]) for a, v in zip(ref, views))
    t_plain = ev[0].elapsed_time(ev[1]) / 1e3
    out = {
        "metric": "VPL-pixel shading pairs/sec incl. visibility (1 GPU), batched",
        "value": pairs / t_batch, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64", "views": len(views), "scenes": len(scs),
                   "triangles": [int(len(sc["tri"])) for sc in scs], "pairs": int(pairs)},
        "untuned_batch": {"value": pairs / t_untuned, "unit": "pairs/s", "ms": t_untuned * 1e3},
        "plain_launches": {"value": pairs / t_plain, "unit": "pairs/s", "ms": t_plain * 1e3},
        "batched_equals_plain": bool(same),
        "autotuned": {k: {"tile_vpl": w, "tile_px": px} for k, (w, px) in tuned.items()},
    }
    vplg.context_destroy(ctx)
    print(json.dumps(out), flush=True)


def serve_requests(n, seed=300):
    """Seeded request stream over the 8 batch scenes: resolution from {256^2, 512^2, 1024^2, 1920x1080},
    VPL budget log-uniform in [1024, 32768] (multiple of 64, split 1:1)."""
    import numpy as np

    from paper_2203_11484_amd import scenes

    scs = scenes.batch_scenes()
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        si = int(rng.integers(len(scs)))
        w, h = scenes.RESOLUTIONS[int(rng.integers(len(scenes.RESOLUTIONS)))]
        m = max(64, int(round(math.exp(rng.uniform(math.log(1024), math.log(32768))) / 64.0)) * 64)
        cam = scenes._view_camera(rng, scs[si], w, h)
        reqs.append((si, cam, scenes.default_params(k_near=m // 2, n_far=m - m // 2, d_near=7.0)))
    return scs, reqs


def bench_serve(args):
    """Poisson request stream at 0.7 x the plain path's capacity: the continuous-batching server against the
    plain FIFO one-frame-per-launch loop on the same arrival trace; p50 / p99 latency and throughput."""
    import numpy as np
    import torch

    from paper_2203_11484_amd import vplg

    n_warm, n = args.warm_requests, args.requests
    scs, reqs = serve_requests(n_warm + n)
    torch.cuda.init()
    ctx = vplg.context_create(0)
    stream = torch.cuda.current_stream()
    sids = [vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"], stream) for sc in scs]
    outs = [torch.zeros((3, c["height"], c["width"]), dtype=torch.float32, device="cuda") for _, c, _ in reqs]

    def plain(i):
        si, cam, prm = reqs[i]
        gb = vplg.GBuffer(cam["width"], cam["height"])
        vplg.gbuffer_render(ctx, sids[si], cam, gb, stream)
        vid = vplg.vpls_generate(ctx, sids[si], cam, prm, stream)
        vplg.gather(ctx, sids[si], vid, gb, outs[i], prm, stream)
        torch.cuda.synchronize()
        vplg.vplset_release(ctx, vid)

    t = time.perf_counter()
    for i in range(n_warm):
        plain(i)
    service = (time.perf_counter() - t) / n_warm
    rate = 0.7 / service
    rng = np.random.default_rng(301)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    print(f"bench: serve {n} requests, mean plain service {service * 1e3:.1f} ms, rate {rate:.2f}/s",
          file=sys.stderr, flush=True)
    pairs = sum(c["width"] * c["height"] * (p["k_near"] + p["n_far"]) for _, c, p in reqs[n_warm:])
    out = {
        "metric": "VPL-pixel shading pairs/sec incl. visibility (1 GPU), served; p99 frame latency",
        "value": None, "unit": "pairs/s", "n_gpus": 1, "steps": n, "warmup": n_warm,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serve", "requests": n, "warm_requests": n_warm, "arrival_rate_per_s": rate,
                   "budget_bytes": 2 << 30, "max_inflight": 8, "streams": 4, "loops": args.serve_loop},
    }
    ref = None
    if args.serve_loop in ("both", "fifo"):
        # plain FIFO loop on the arrival trace
        lat_plain = []
        t0 = time.perf_counter()
        for j in range(n):
            while time.perf_counter() - t0 < arrivals[j]:
                time.sleep(0.0005)
            plain(n_warm + j)
            lat_plain.append(time.perf_counter() - t0 - arrivals[j])
            if (j + 1) % 64 == 0:
                print(f"bench: plain FIFO loop, {j + 1}/{n} requests done", file=sys.stderr, flush=True)
        span_plain = time.perf_counter() - t0
        out["plain_fifo"] = {"p50_ms": float(np.percentile(lat_plain, 50) * 1e3),
                             "p99_ms": float(np.percentile(lat_plain, 99) * 1e3),
                             "throughput_req_per_s": n / span_plain, "pairs_per_s": pairs / span_plain}
        if args.serve_loop == "fifo":
            out["value"] = pairs / span_plain
            out["ms_per_step"] = span_plain / n * 1e3
            vplg.context_destroy(ctx)
            print(json.dumps(out), flush=True)
            return
        ref = [outs[n_warm + j].clone() for j in range(n)]
        for j in range(n):
            outs[n_warm + j].fill_(-1.0)
        torch.cuda.synchronize()
    # the server on the same trace
    srv = vplg.server_start(ctx, 2 << 30, max_inflight=8, n_streams=4)
    keep, tickets = [], []
    t0 = time.perf_counter()
    base_ns = time.monotonic_ns()
    for j in range(n):
        while time.perf_counter() - t0 < arrivals[j]:
            time.sleep(0.0005)
        si, cam, prm = reqs[n_warm + j]
        r = vplg.make_request(sids[si], cam, prm, outs[n_warm + j])
        keep.append(r)
        tickets.append(vplg.server_submit(srv, r))
        if (j + 1) % 64 == 0:
            print(f"bench: server, {j + 1}/{n} requests submitted", file=sys.stderr, flush=True)
    times = [vplg.server_wait(srv, tk, timeout_ms=600000) for tk in tickets]
    print("bench: server, every request done", file=sys.stderr, flush=True)
    st = vplg.server_query(srv)
    vplg.server_stop(srv)
    torch.cuda.synchronize()
    lat_srv = [(tm["done_ns"] - tm["submit_ns"]) / 1e9 for tm in times]
    span_srv = (max(tm["done_ns"] for tm in times) - min(tm["submit_ns"] for tm in times)) / 1e9
    if ref is not None:
        same = all(torch.equal(ref[j], outs[n_warm + j]) for j in range(n))
        checked = n
    else:
        # server loop alone: a seeded sample of served requests against the same requests run alone
        pick = np.random.default_rng(302).choice(n, min(n, 64), replace=False)
        same = True
        for j in pick:
            served = outs[n_warm + j].clone()
            plain(n_warm + j)
            same = same and torch.equal(served, outs[n_warm + j])
        checked = len(pick)
    out["value"] = pairs / span_srv
    out["ms_per_step"] = span_srv / n * 1e3
    out["server"] = {"p50_ms": float(np.percentile(lat_srv, 50) * 1e3),
                     "p99_ms": float(np.percentile(lat_srv, 99) * 1e3), "throughput_req_per_s": n / span_srv,
                     "peak_running": st["peak_running"], "peak_bytes": st["peak_bytes"]}
    out["served_equals_alone"] = bool(same)
    out["served_equals_alone_checked"] = int(checked)
    vplg.context_destroy(ctx)
    print(json.dumps(out), flush=True)


def bench_quality(args):
    """The paper's quality studies (Section "Results") on the library's GPU path, per scene: every method
    (plain instant radiosity and the hybrid generation in the paper's reading and its variants) at a
    geometric grid of VPL counts against a dense instant-radiosity reference (262,144 VPLs), with
    generation and gather timed by HIP events.  Reports the equal-sample RMSE table (1,024 and 5,120
    VPLs) and the equal-RMSE time study (VPLs and gather time each method needs for a target RMSE)."""
    import torch

    from paper_2203_11484_amd import quality, scenes, vplg

    torch.cuda.init()
    ctx = vplg.context_create(0)
    names = args.scenes.split(",")
    studies = []
    ratios = []
    t0 = time.perf_counter()

    def log(msg):
        print(f"bench: quality {msg}", file=sys.stderr, flush=True)

    for name in names:
        sc = scenes.make_scene(name)
        sw = quality.sweep(vplg, ctx, sc, counts=quality.DEFAULT_COUNTS, ref_vpls=args.ref_vpls, log=log)
        es = quality.equal_sample_table(sw, at=(1024, 5120))
        er = quality.equal_rmse_table(sw)
        log(f"{name}: ref RMS {sw['ref_rms']:.4g}; equal-sample " +
            "; ".join(f"M={r['vpls']}: " + " ".join(f"{k} {v:.4g}" for k, v in r.items() if k != "vpls") for r in es))
        for r in er:
            log(f"{name}: target {r['fraction']:g} x RMS: IR/hybrid gather time " +
                " ".join(f"{k} {v:.3g}" if v else f"{k} -" for k, v in r["time_ratio_ir_over"].items()))
        studies.append({"scene": name, "sweep": sw, "equal_sample": es, "equal_rmse": er})
        ratios += [r["ir"] / r["paper"] for r in es]
    vplg.context_destroy(ctx)
    gm = math.exp(sum(math.log(x) for x in ratios) / len(ratios))
    out = {
        "metric": "indirect-image RMSE of plain instant radiosity / hybrid (paper's reading), equal VPL count "
                  "(geometric mean)",
        "value": gm, "unit": "ratio", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": (time.perf_counter() - t0) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "quality", "scenes": names, "reference_vpls": args.ref_vpls,
                   "counts": list(quality.DEFAULT_COUNTS), "variants": quality.VARIANTS},
        "studies": studies,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="room200k")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile-vpl", type=int, default=0, help="waves (VPL slices) per 8x8 pixel tile, 0 = default")
    ap.add_argument("--autotune", action="store_true",
                    help="batch64: autotune the tile shape per view-shape bucket with the batched launch as objective")
    ap.add_argument("--requests", type=int, default=64, help="serve: requests after the warm-ups")
    ap.add_argument("--warm-requests", type=int, default=8,
                    help="serve: plain runs first (they set the mean service time the arrival rate is scaled by)")
    ap.add_argument("--serve-loop", choices=("both", "server", "fifo"), default="both",
                    help="serve: run the server and the plain FIFO loop on the same trace, or one of them")
    ap.add_argument("--scenes", default="cornell,cornell_point,room20k,room200k",
                    help="quality: workloads of the study")
    ap.add_argument("--ref-vpls", type=int, default=262144, help="quality: VPLs of the dense-IR reference")
    ap.add_argument("--in-flight", type=int, default=1,
                    help="frames in flight (2: the next frame's G-buffer and VPLs are made while the current one "
                         "gathers; 1: one frame at a time)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "quality":
        return bench_quality(args)

    import numpy as np
    import torch

    from paper_2203_11484_amd import scenes, vplg

    sc = scenes.make_scene(args.workload)
    cam, prm = sc["camera"], sc["params"]
    W, H = cam["width"], cam["height"]
    P = W * H
    print(f"bench: {args.workload} {len(sc['tri'])} triangles, {W}x{H}, K={prm['k_near']} N_far={prm['n_far']}",
          file=sys.stderr, flush=True)
    torch.cuda.init()
    ctx = vplg.context_create(0)
    stream = torch.cuda.current_stream()
    sid = vplg.scene_upload(ctx, sc["tri"], sc["albedo"], sc["flags"], sc["light"], stream)
    gb = vplg.GBuffer(W, H)
    rad = torch.zeros((3, H, W), dtype=torch.float32, device="cuda")
    vid = vplg.vpls_generate(ctx, sid, cam, prm, stream)
    M = vplg.vplset_count(ctx, vid)
    gp = vplg.make_gather_params(prm)
    gp.tile_vpl = args.tile_vpl

    if args.in_flight >= 2:
        # Two frames in flight: one stream renders the G-buffer and generates the VPLs of the next
        # frame into the other of two buffer slots while the second stream gathers the current one,
        # so the next frame's generation runs in the gather's tail.  Every step still runs the whole
        # path on its own frame; a slot is rewritten only after the gather that read it is done.
        gen_s, gat_s = torch.cuda.Stream(), torch.cuda.Stream()
        slots = [(gb, vid)]
        for _ in range(1, args.in_flight):
            g2 = vplg.GBuffer(W, H)
            slots.append((g2, vplg.vpls_generate(ctx, sid, cam, prm, stream)))
        torch.cuda.synchronize()
        gen_done = [torch.cuda.Event() for _ in slots]
        free = [torch.cuda.Event() for _ in slots]
        for e in free:
            e.record(gat_s)

        def step_i(i, ev=None):
            k = i % len(slots)
            g_k, v_k = slots[k]
            gen_s.wait_event(free[k])
            vplg.gbuffer_render(ctx, sid, cam, g_k, gen_s)
            vplg.vpls_regenerate(ctx, v_k, cam, prm, gen_s)
            gen_done[k].record(gen_s)
            gat_s.wait_event(gen_done[k])
            if ev:
                ev[0].record(gat_s)
            vplg.gather(ctx, sid, v_k, g_k, rad, gp, gat_s)
            if ev:
                ev[1].record(gat_s)
            free[k].record(gat_s)

        t_stream = gat_s
    else:
        # the G-buffer does not depend on the VPLs: it renders on a second stream (default priority)
        # while the generation runs on the first, and the gather waits for both
        side = torch.cuda.Stream()
        go, gb_done = torch.cuda.Event(), torch.cuda.Event()

        def step_i(i, ev=None):
            go.record(stream)
            side.wait_event(go)
            vplg.gbuffer_render(ctx, sid, cam, gb, side)
            gb_done.record(side)
            vplg.vpls_regenerate(ctx, vid, cam, prm, stream)
            stream.wait_event(gb_done)
            if ev:
                ev[0].record(stream)
            vplg.gather(ctx, sid, vid, gb, rad, gp, stream)
            if ev:
                ev[1].record(stream)

        t_stream = stream

    for i in range(args.warmup):
        step_i(i)
    torch.cuda.synchronize()
    print(f"bench: warmup done, M={M}, frames in flight {max(1, args.in_flight)}", file=sys.stderr, flush=True)

    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    g_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start.record(t_stream)
    if args.in_flight >= 2:
        gen_s.wait_event(t_start)
    for i in range(args.steps):
        step_i(args.warmup + i, g_ev[i])
    t_end.record(t_stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    # frame intervals: from one gather's end to the next (the first from the start)
    ends = [t_start.elapsed_time(b) for _, b in g_ev]
    frame_ms = np.diff(np.array([0.0] + ends))
    gather_ms = np.array([a.elapsed_time(b) for a, b in g_ev])
    print(f"bench: {args.steps} steps, {ms_step:.3f} ms/step, gather {gather_ms.mean():.3f} ms",
          file=sys.stderr, flush=True)

    # instrumented launch (untimed): pairs, shadow rays, BVH nodes, triangle tests
    cnt = torch.zeros(vplg.N_COUNTERS, dtype=torch.int64, device="cuda")
    vplg.gather_counted(ctx, sid, vid, gb, rad, cnt, gp, stream)
    torch.cuda.synchronize()
    (pairs_c, rays, nodes, tris, packets, psteps, plane, ptris, rides, both, pops, pk_blocked, pk_clear,
     blocked) = (int(x) for x in cnt.cpu().tolist())
    stats = vplg.vplset_stats(ctx, vid)
    valid = int((gb.tri >= 0).sum().item())

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    flops = FLOP_PAIR * pairs_c + FLOP_RAY * rays + FLOP_NODE * nodes + FLOP_TRI * tris
    g_mean_s = gather_ms.mean() / 1e3
    achieved = flops / g_mean_s / 1e12
    pairs_step = P * M
    out = {
        "metric": "VPL-pixel shading pairs/sec incl. visibility (1 GPU)",
        "value": pairs_step / (ms_step / 1e3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "triangles": int(len(sc["tri"])), "width": W, "height": H,
                   "vpls": M, "near_vpls": int(stats["k_eff"]), "far_vpls": int(stats["n_far"]),
                   "light": "point" if sc["light"]["kind"] == 0 else "quad", "g_clamp": prm["g_clamp"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(args.workload),
                     "kernel": "k_gather", "flop_per_launch": flops, "gather_ms": float(gather_ms.mean())},
        "gather_pairs_per_s": pairs_step / g_mean_s,
        "frames_in_flight": max(1, args.in_flight),
        "p50_frame_ms": float(np.percentile(frame_ms, 50)),
        "p99_frame_ms": float(np.percentile(frame_ms, 99)),
        "valid_pixel_frac": valid / P,
        "shadow_ray_frac": rays / max(pairs_c, 1),
        "blocked_ray_frac": blocked / max(rays, 1),
        "nodes_per_ray": nodes / max(rays, 1),
        "tris_per_ray": tris / max(rays, 1),
        "ray_tri_tests_per_s": tris / g_mean_s,
        "packets": {"count": packets, "lanes_per_packet": plane / max(packets, 1),
                    "steps_per_packet": psteps / max(packets, 1), "tri_steps_per_packet": ptris / max(packets, 1),
                    "lane_efficiency_nodes": nodes / max(64 * psteps, 1),
                    "rider_frac": (rides - nodes) / max(rides, 1),
                    "both_children_frac": both / max(psteps, 1), "pop_frac": pops / max(psteps, 1),
                    "all_blocked_frac": pk_blocked / max(packets, 1), "none_blocked_frac": pk_clear / max(packets, 1)},
        "generation": {k: int(stats[k]) for k in ("n_patches", "n_near", "n_eligible", "n_paths")},
    }
    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
    vplg.context_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
