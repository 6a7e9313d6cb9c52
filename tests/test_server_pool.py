"""Render-server pool bookkeeping on the host (`server_pool.h`, no GPU).

A request reuses an idle pooled VPL set of its shape and an idle G-buffer block, and the server evicts
other idle entries so that the rest fits its HBM budget.  The entries it reuses must never be among
those evicted: a freed G-buffer block would leave the request's G-buffer planes at a null base, and its
kernels would write there.  `tests/native/server_pool_check.cpp` runs the server's FIFO admission over
request mixes with requests finishing in random orders, and checks after every admission that reused
entries are live, evictions take only idle entries that no request holds, pooled bytes match the live
entries and the budget, and every request that fits alone is admitted.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_11484_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "server_pool_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("pool") / "server_pool_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wall", "-I", CSRC, SRC, "-o", exe], check=True)
    return exe


def test_random_mixes(checker):
    out = subprocess.run([checker, "random", "4000"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr


def test_serving_mix_under_a_tight_budget(checker):
    """The twelve requests of the GPU serving test under its 24 MB budget (the same seeded generator:
    scene, resolution, VPL count), with set sizes of the order the library plans for them (about 7.8 MB
    for the rooms' ~2e5 patches, 0.85 MB for the Cornell box's ~3e3)."""
    rng = np.random.default_rng(24)
    lines = [f"{24 << 20} 8"]
    for _ in range(12):
        si = int(rng.integers(3))
        w, h = [(48, 40), (64, 64), (96, 72), (33, 29)][int(rng.integers(4))]
        m = int(rng.choice([128, 256, 512]))
        k, n = m // 2, m - m // 2
        set_bytes = (850_000 if si == 0 else 7_800_000) + 150 * m
        lines.append(f"{si} {k} {n} {40 * w * h} {set_bytes}")
    out = subprocess.run([checker, "mix", "2000"], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
