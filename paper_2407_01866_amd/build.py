"""Build libimagegs.so (hand-written HIP for gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only.  Packed FP32 instructions are disabled
(``-target-feature -packed-fp32-ops``) and floating-point contraction is left to the explicit
``fma`` calls in the sources.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libimagegs.so")
# the bounds-checked build (IGS_BOUNDS_CHECK): every checked index is validated on the device and
# reported through igs_bounds_violations; for tests and debugging, not for speed
LIB_DEBUG = os.path.join(PKG, "libimagegs_debug.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["binning.hip", "scan.hip", "radix_sort.hip", "raster_fwd.hip", "raster_bwd.hip",
           "raster_fit.hip", "loss_adam.hip", "ssim.hip", "place.hip", "query.hip", "timing.cpp",
           "api.cpp"]

FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-fvisibility=hidden",
         "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]


# Per-file extra flags.  The forward rasterizer, the single-pass fitting kernel and the point
# queries rank candidates with FP64 min/max on packed keys that are never NaN; -fno-honor-nans
# stops the compiler from quieting their inputs.
EXTRA = {"raster_fwd.hip": ["-fno-honor-nans"], "raster_fit.hip": ["-fno-honor-nans"],
         "query.hip": ["-fno-honor-nans"]}


def _compile(src: str, verbose: bool, debug: bool) -> str:
    out = os.path.join(BUILD, "debug") if debug else BUILD
    obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), *(["-DIGS_BOUNDS_CHECK"] if debug else []), "-x",
           "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
    if msgs and verbose:
        print("\n".join(msgs))
    return obj


def build(verbose: bool = False, debug: bool = False) -> str:
    """Builds libimagegs.so, or with debug=True the bounds-checked libimagegs_debug.so."""
    os.makedirs(os.path.join(BUILD, "debug") if debug else BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, debug), SOURCES))
    lib = LIB_DEBUG if debug else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, debug="--debug" in sys.argv))
