"""Compile the HIP library libga.so in-tree for gfx950 (hipcc, no torch)."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libga.so")
SOURCES = ["ops3d.hip", "ops3d_lowp.hip", "spline1d.cpp", "ops2d.hip", "vec.hip", "pinv.hip", "pinv_band.hip", "pinv_mfma.hip", "mixed.hip", "gnet.hip",
           "api.hip", "noalloc.hip", "api_gnet.hip", "batch.hip", "wave1d.hip"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def _compile(src, extra=(), build=None):
    build = build or BUILD
    obj = os.path.join(build, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = ["hipcc", *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build_library(verbose=False, extra=(), out=None, build=None):
    """Compile every source and link; `extra` adds compiler flags, `out` and
    `build` redirect the library and object files (defaults: in-tree)."""
    out = out or LIB
    build = build or BUILD
    os.makedirs(build, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, tuple(extra), build), SOURCES))
    tmp = out + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build_library(verbose=True)
