"""Host-side pieces of the image-quality harness: the RMSE and the parameter sets it compares."""
import math

import numpy as np

from paper_2203_11484_amd import quality, scenes


def test_rmse_definition():
    rng = np.random.default_rng(3)
    a = rng.random((3, 8, 6))
    assert quality.rmse(a, a) == 0.0
    # a constant offset c on every pixel and channel gives |c|
    assert math.isclose(quality.rmse(a + 0.25, a), 0.25, rel_tol=1e-12)
    # masked pixels do not count; [n, 3] and [3, H, W] layouts agree
    mask = np.zeros(48, bool)
    mask[:10] = True
    b = a.copy()
    b.reshape(3, -1)[:, 10:] += 5.0
    assert quality.rmse(b, a, mask) == 0.0
    flat_a, flat_b = a.reshape(3, -1).T, (a + 0.5).reshape(3, -1).T
    assert math.isclose(quality.rmse(flat_b, flat_a), 0.5, rel_tol=1e-12)
    # one channel of one pixel off by d among n pixels: d / sqrt(3 n)
    c = a.copy()
    c[1, 2, 3] += 6.0
    assert math.isclose(quality.rmse(c, a), 6.0 / math.sqrt(3 * 48), rel_tol=1e-12)


def test_compared_parameter_sets():
    base = scenes.make_scene("room200k")["params"]
    ir = quality.plain_ir_params(base, 5120)
    assert (ir["k_near"], ir["n_far"], ir["d_near"]) == (0, 5120, 0.0)
    hy = quality.hybrid_params(base, 5120)
    assert hy["k_near"] + hy["n_far"] == 5120 and hy["k_near"] == 3840  # the workload's 3:1 split
    assert hy["d_near"] == base["d_near"]
    c1 = quality.hybrid_params(scenes.make_scene("cornell")["params"], 1024)
    assert (c1["k_near"], c1["n_far"]) == (256, 768)  # 64:192


def test_count_for_rmse_interpolates_loglog():
    counts = [100, 400, 1600]
    # errors falling as 1 / sqrt(count): 0.1, 0.05, 0.025
    errs = [0.1, 0.05, 0.025]
    c, exact = quality.count_for_rmse(counts, errs, 0.05 / math.sqrt(2))
    assert exact and math.isclose(c, 800.0, rel_tol=1e-12)
    assert quality.count_for_rmse(counts, errs, 0.2) == (100.0, False)  # already below at the first count
    assert quality.count_for_rmse(counts, errs, 0.01) == (None, False)  # never reached
    c, exact = quality.count_for_rmse(counts, errs, 0.05)
    assert exact and math.isclose(c, 400.0, rel_tol=1e-12)


def test_interp_loglog_power_law():
    xs = [1.0, 10.0, 100.0]
    ys = [2.0, 20.0, 200.0]
    assert math.isclose(quality.interp_loglog(xs, ys, 31.6227766), 63.2455532, rel_tol=1e-9)
    ys2 = [3.0, 300.0, 30000.0]  # y = 3 x^2
    assert math.isclose(quality.interp_loglog(xs, ys2, 5.0), 75.0, rel_tol=1e-12)


def test_equal_rmse_table_from_a_synthetic_sweep():
    """Two methods on power laws: IR err = 1 / sqrt(M), a method with half the error at equal M needs a
    quarter of the VPLs, so at equal time per VPL its time ratio is 4 at every reachable target; a
    method with an error floor never reaches targets below it."""
    counts = [256, 1024, 4096, 16384]
    t = [c * 0.01 for c in counts]
    sw = {"counts": counts, "ref_rms": 1.0, "methods": {
        "ir": {"rmse": [1 / math.sqrt(c) for c in counts], "gather_ms": t, "gen_ms": t},
        "half": {"rmse": [0.5 / math.sqrt(c) for c in counts], "gather_ms": t, "gen_ms": t},
        "floor": {"rmse": [max(0.02, 1 / math.sqrt(c)) for c in counts], "gather_ms": t, "gen_ms": t}}}
    rows = quality.equal_rmse_table(sw, fractions=(0.03, 0.015, 0.01))
    for r in rows:
        assert math.isclose(r["time_ratio_ir_over"]["half"], 4.0, rel_tol=1e-9)
    assert rows[0]["methods"]["floor"]["vpls"] is not None
    assert rows[1]["methods"]["floor"]["vpls"] is None and rows[1]["time_ratio_ir_over"]["floor"] is None
    assert quality.equal_sample_table(sw, at=(1024,))[0]["half"] == 0.5 / 32
