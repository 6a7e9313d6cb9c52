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
