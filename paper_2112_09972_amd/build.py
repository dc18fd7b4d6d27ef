"""Build step of the HIP library: compiles ``csrc/sclbm.hip`` (lattice Boltzmann
solver) and ``csrc/sclmlp.hip`` (droplet-shape surrogate) for gfx950 into one
``libsclbm.so`` next to this file (in-tree, so it travels with the source tree).

Usage: ``python -m paper_2112_09972_amd.build`` or ``build_library()``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRCS = [os.path.join(PKG, "csrc", "sclbm.hip"), os.path.join(PKG, "csrc", "sclmlp.hip")]
LIB = os.path.join(PKG, "libsclbm.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


DEBUG_LIB = os.path.join(PKG, "libsclbm_debug.so")


def build_library(verbose: bool = False, debug: bool = False) -> str:
    """Compile the library (always recompiles).  debug=True builds
    libsclbm_debug.so, whose step kernels fill the LDS cells they are about to
    write with NaN at every plane (reads of unwritten cells become visible)."""
    lib = DEBUG_LIB if debug else LIB
    tmp = lib + ".tmp%d" % os.getpid()
    extra = ["-DSCLBM_DEBUG_FILL=1"] if debug else []
    cmd = [hipcc()] + HIPCC_FLAGS + extra + ["-I" + os.path.join(ROOT, "include"), "-o", tmp] + SRCS
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout)
    if verbose and out:
        print(out)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv, debug="--debug" in sys.argv))
