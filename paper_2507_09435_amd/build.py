"""Compile the HIP library for gfx950 into the package directory."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmpm_hip.so")
SOURCES = ["mpm_prepare.hip", "mpm_assemble.hip", "mpm_krylov.hip", "mpm_mg.hip", "mpm_mg3.hip", "mpm_adjoint.hip",
           "mpm_api.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Always recompiles (the build check must compile every time)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
