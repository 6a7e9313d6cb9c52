"""The BVH builder on the host (`csrc/bvh_build.cpp`, no GPU): binned SAH, then insertion-based optimisation of
the inner nodes over the fixed leaves.

`tests/native/bvh_check.cpp` builds the device arrays and checks their structure (leaf ranges partition the
triangles, records hold their triangles, each inner node reached once, depth within the traversal stack, boxes
nesting and holding their leaves' vertices, the split word's axis, child order and key) and their
conservativeness: for random segments (a third starting on a triangle, as shadow rays do), every triangle the
segment crosses in FP64 lies in a leaf that an FP64 slab walk of the tree reaches.  Visibility through the tree
is then the brute-force definition the oracle uses, which the GPU parity tests rely on.  The same check also
runs with the host code under AddressSanitizer and UndefinedBehaviorSanitizer.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2203_11484_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_11484_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
SRC = os.path.join(ROOT, "tests", "native", "bvh_check.cpp")


def _hipcc():
    hipcc = shutil.which("hipcc") or (os.path.exists("/opt/rocm/bin/hipcc") and "/opt/rocm/bin/hipcc")
    if not hipcc:
        pytest.skip("no hipcc for the builder's headers")
    return hipcc


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("bvh") / "bvh_check")
    subprocess.run([_hipcc(), "-O2", "-std=c++17", "-I", CSRC, "-I", INCLUDE, SRC, os.path.join(CSRC, "bvh_build.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def _run(checker, tmp_path, tri, segments):
    tri = np.ascontiguousarray(tri, np.float32).reshape(-1, 9)
    path = tmp_path / "tri.bin"
    with open(path, "wb") as f:
        f.write(np.int32(len(tri)).tobytes())
        f.write(tri.tobytes())
    out = subprocess.run([checker, str(path), str(segments)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    return out.stdout


@pytest.mark.parametrize("name,segments", [("cornell", 20000), ("room20k", 1500)])
def test_workload_scenes(checker, tmp_path, name, segments):
    sc = scenes.make_scene(name)
    s = _run(checker, tmp_path, sc["tri"], segments)
    assert "crossings=0" not in s, "the segments should cross some triangles"


def test_batch_scene(checker, tmp_path):
    _run(checker, tmp_path, scenes.batch_scene(101, 6000)["tri"], 3000)


def test_rooms_where_a_picked_node_becomes_the_root(checker, tmp_path):
    """In these rooms an optimisation pass moves one of the nodes it picked to the root before reaching it
    (a root has no parent to remove: the pass must skip it)."""
    _run(checker, tmp_path, scenes.procedural_room(11, 6, 6, 2, 2)["tri"], 2000)
    _run(checker, tmp_path, scenes.procedural_room(22, 8, 6, 0, 0)["tri"], 2000)


def test_degenerate_inputs(checker, tmp_path):
    rng = np.random.default_rng(7)
    one = np.array([[0, 0, 0, 1, 0, 0, 0, 1, 0]], np.float32)
    _run(checker, tmp_path, one, 500)                               # one leaf: a root over it twice
    _run(checker, tmp_path, np.repeat(one, 3, axis=0), 500)         # identical centroids
    _run(checker, tmp_path, np.repeat(one, 40, axis=0), 500)        # identical centroids, more than a leaf
    _run(checker, tmp_path, rng.uniform(-1, 1, (5, 9)), 2000)
    # slivers along one axis and a large/small mix
    t = rng.uniform(-1, 1, (3000, 9)).astype(np.float32)
    t[:, 1::3] *= 1e-3
    _run(checker, tmp_path, t, 500)
    big = rng.uniform(-50, 50, (20, 9))
    small = rng.uniform(-1, 1, (2000, 3))[:, None, :] + rng.uniform(-0.01, 0.01, (2000, 3, 3))
    _run(checker, tmp_path, np.concatenate([big, small.reshape(-1, 9)]), 500)


def test_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "bvh_check_asan")
    subprocess.run([_hipcc(), "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined", "-I", CSRC, "-I", INCLUDE,
                    SRC, os.path.join(CSRC, "bvh_build.cpp"), "-o", exe], check=True, capture_output=True)
    rng = np.random.default_rng(7)
    t = rng.uniform(-1, 1, (3000, 9)).astype(np.float32)
    t[:, 1::3] *= 1e-3
    for tri in (scenes.make_scene("cornell")["tri"], scenes.procedural_room(22, 8, 6, 0, 0)["tri"], t):
        out = _run(exe, tmp_path, tri, 200)
        assert "runtime error" not in out
