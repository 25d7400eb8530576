"""Build librtw.so (the gfx950 HIP library behind include/rtw.h) in-tree.

    python -m paper_2403_13856_amd.build

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are
disabled for the device code (``-target-feature -packed-fp32-ops``); hipcc's
host pass warns that it does not know the feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIB_DIR, "librtw.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("rtw_lib.hip", "rtw_mlp.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("rtw_device.hpp", "rtw_raster.hpp")] + \
    [os.path.join(ROOT, "include", f) for f in ("rtw.h", "rtw_surrogate.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build librtw.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
