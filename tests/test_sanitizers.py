"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

The FP64 oracle (`oracle/oracle.c`) is rebuilt with -fsanitize=address,undefined and driven through its
ctypes front end on a small Cornell box in a child process with the ASan runtime preloaded: G-buffer and its
edge rule, generation (patches, Morton sort, strata, walk), visibility with the grazing rule, the gather and
the direct term.  The server's pool bookkeeping check (`tests/native/server_pool_check.cpp`) runs the same
way.  Any sanitizer report fails the test.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc(name):
    exe = shutil.which(name)
    if not exe:
        pytest.skip(f"no {name}")
    return exe


def _asan_runtime(gcc):
    path = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not path or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("no ASan runtime")
    return path


def _clean(out):
    for bad in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer"):
        assert bad not in out, out[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    gcc = _gcc("gcc")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run([gcc, "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"],
                   check=True)
    script = textwrap.dedent("""
        import sys
        sys.path.insert(0, %r)
        import numpy as np
        from oracle import oracle as orc
        from paper_2203_11484_amd import scenes
        sc = scenes.make_scene("cornell", width=24, height=20)
        S = orc.Scene.from_dict(sc)
        cam, prm = sc["camera"], sc["params"]
        gb = S.gbuffer(cam)
        edge = S.gbuffer_edges(cam)
        g = S.generate(cam, sc["light"], prm)
        f32 = lambda a: a.astype(np.float32)
        pix = np.arange(0, 24 * 20, 7)
        vis = S.vis_matrix(f32(gb["pos"][pix]), gb["tri"][pix], f32(g["pos"]), g["tri"])
        graz = S.grazing(f32(gb["pos"][pix[:8]]), gb["tri"][pix[:8]], f32(g["pos"][:8]), g["tri"][:8])
        L = S.gather(f32(gb["pos"]), f32(gb["nrm"]), f32(gb["alb"]), gb["tri"], f32(g["pos"]), f32(g["nrm"]),
                     f32(g["I"]), g["tri"])
        D = S.direct(f32(gb["pos"]), f32(gb["nrm"]), f32(gb["alb"]), gb["tri"], sc["light"])
        assert np.isfinite(L).all() and np.isfinite(D).all() and vis.shape == (len(pix), g["n"])
        assert orc.lib()._name == %r, orc.lib()._name  # the sanitized build, not the plain one
        print("sanitized oracle ok", int(edge.sum()), int(g["n"]), float(L.sum()))
    """) % (ROOT, lib)
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(gcc), ASAN_OPTIONS="detect_leaks=0", ORACLE_LIB=lib,
               OMP_NUM_THREADS="2")
    out = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=300)
    _clean(out.stdout + out.stderr)
    assert out.returncode == 0 and "sanitized oracle ok" in out.stdout, out.stdout + out.stderr[-4000:]


def test_server_pool_under_sanitizers(tmp_path):
    gxx = _gcc("g++")
    exe = str(tmp_path / "server_pool_check_asan")
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "paper_2203_11484_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "server_pool_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe, "random", "800"], capture_output=True, text=True, timeout=300)
    _clean(out.stdout + out.stderr)
    assert out.returncode == 0, out.stdout + out.stderr[-4000:]
