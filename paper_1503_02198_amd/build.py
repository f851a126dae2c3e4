"""Builds libssd.so (the HIP library behind include/ssd.h) for gfx950, in-tree.

    python -m paper_1503_02198_amd.build
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libssd.so")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("ssd_host.hip", "ssd_kernels.hip", "ssd_batch.hip", "ssd_mlp.hip",
                     "ssd_iface.hip", "ssd_probe.hip")]
HEADERS = [os.path.join(ROOT, "include", "ssd.h")] + [
    os.path.join(HERE, "csrc", f) for f in ("ssd_internal.h", "ssd_launch.h", "ssd_device.h", "ssd_tiles.h")]


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def command(out=LIB, extra=()):
    return [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions stay disabled on this target
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            *extra, "-o", out, *SOURCES]


def build(verbose=False):
    """Compile every source into paper_1503_02198_amd/libssd.so (always)."""
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libssd.so")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
