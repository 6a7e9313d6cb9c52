"""Build the gfx950 shared library libvplg.so (HIP kernels + C-ABI runtime) in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libvplg.so")
BUILD = os.path.join(HERE, "_build")

ARCH = "gfx950"
COMMON = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC,
          # packed FP32 instructions stay off (v_pk_* f32 forms are not trusted here)
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
# sources and their extra flags; generation and the host runtime take FP64
# decisions whose operation order must be kept exactly (no contraction)
SOURCES = [
    # the FP32 ray kernels never see NaN box or triangle inputs (degenerate
    # determinants fail the parallel-ray cut), so min/max need no NaN quieting;
    # no contraction: the watertight edge functions need separately rounded
    # products (fused forms are written out as fmaf); the packet traversal's
    # wave-uniform branches stay plain scalar branches (no structurisation)
    ("k_gather.hip", ["-fno-honor-nans", "-ffp-contract=off", "-mllvm", "-structurizecfg-skip-uniform-regions=true"]),
    ("k_generate.hip", ["-ffp-contract=off"]),
    ("bvh_build.cpp", []),
    ("runtime.cpp", ["-ffp-contract=off"]),
    ("server.cpp", []),
]


def _compile(src, extra, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = ["hipcc", *COMMON, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln
                    and "is not a recognized feature" not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if msg.strip() and verbose:
        print(msg)
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda s: _compile(s[0], s[1], verbose), SOURCES))
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
