"""Build the gfx950 shared library libfelbm.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libfelbm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions stay disabled in every device compile
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    obj_host = os.path.join(LIBDIR, "mesh_prep.o")
    obj_dev = os.path.join(LIBDIR, "felbm.o")
    obj_dev3 = os.path.join(LIBDIR, "felbm3d.o")
    _run(["g++", *COMMON, "-c", os.path.join(CSRC, "mesh_prep.cpp"), "-o", obj_host], verbose)
    for src, obj in (("felbm.hip", obj_dev), ("felbm3d.hip", obj_dev3)):
        _run([HIPCC, *COMMON, f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj],
             verbose)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", obj_dev, obj_dev3, obj_host, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
