"""Host-side memory and undefined-behaviour checks (CPU only, no GPU needed).

* The FP64 oracle (oracle/oracle.c) is built with AddressSanitizer and UndefinedBehaviorSanitizer
  (gcc) and driven through every entry point on small seeded inputs and with invalid arguments
  (tests/sanitize/oracle_driver.c).
* libimagegs's host code (argument validation, buffer carving, size queries) is built with the
  same sanitizers on the host side only (each -fsanitize behind -Xarch_host: the gfx950 device
  code is compiled as usual) and driven through its size queries and through every compute entry
  point with arguments that must be rejected before any device work
  (tests/sanitize/abi_driver.c).

Builds go to _build/sanitize and are reused while the sources are unchanged.  Any sanitizer
report aborts the driver (-fno-sanitize-recover=all), which fails the test.
"""
import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
CSRC = os.path.join(ROOT, "paper_2407_01866_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SOURCES = ["binning.hip", "scan.hip", "radix_sort.hip", "raster_fwd.hip", "raster_bwd.hip",
           "raster_fit.hip", "loss_adam.hip", "ssim.hip", "place.hip", "query.hip", "timing.cpp",
           "api.cpp"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _digest(paths, extra=""):
    h = hashlib.sha256(extra.encode())
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def _fresh(stamp, digest):
    return os.path.exists(stamp) and open(stamp).read() == digest


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]
    return r


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(ROOT, "oracle", "oracle.c"),
            os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")]
    exe = os.path.join(OUT, "oracle_driver")
    stamp = exe + ".stamp"
    dig = _digest(srcs)
    if not (_fresh(stamp, dig) and os.path.exists(exe)):
        _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-fopenmp",
              "-ffp-contract=off", *srcs, "-lm", "-o", exe])
        open(stamp, "w").write(dig)
    r = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
                         "OMP_NUM_THREADS": "2"})
    assert "oracle driver ok" in r.stdout


def test_abi_host_code_under_address_and_undefined_behaviour_sanitizers():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    headers = [os.path.join(CSRC, h) for h in sorted(os.listdir(CSRC)) if h.endswith(".hpp")]
    driver = os.path.join(ROOT, "tests", "sanitize", "abi_driver.c")
    exe = os.path.join(OUT, "abi_driver")
    stamp = exe + ".stamp"
    dig = _digest(srcs + headers + [driver, os.path.join(INCLUDE, "imagegs.h")], " ".join(HOST_SAN))
    if not (_fresh(stamp, dig) and os.path.exists(exe)):
        def compile_one(s):
            obj = os.path.join(OUT, os.path.splitext(os.path.basename(s))[0] + ".o")
            _run([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
                  "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  *HOST_SAN, f"-I{INCLUDE}", "-x", "hip", "-c", s, "-o", obj])
            return obj
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(compile_one, srcs))
        dobj = os.path.join(OUT, "abi_driver.o")
        _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              f"-I{INCLUDE}", "-c", driver, "-o", dobj])
        _run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, dobj, *objs, "-o", exe])
        open(stamp, "w").write(dig)
    # leaks are not checked here: the HIP runtime keeps its own allocations until exit
    r = _run([exe], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1"})
    assert "abi driver ok" in r.stdout
