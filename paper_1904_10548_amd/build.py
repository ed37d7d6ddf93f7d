"""Build the tapg C-ABI library (HIP for gfx950) in-tree.

``python -m paper_1904_10548_amd.build`` compiles ``csrc/*.cpp`` and
``csrc/*.hip`` with hipcc into ``paper_1904_10548_amd/libtapg.so``.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libtapg.so")

# Packed FP32 instructions are disabled for all device code (the compiler is
# free to form them from ordinary float code otherwise).
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    c = os.path.join(PKG, "csrc")
    return sorted(glob.glob(os.path.join(c, "*.cpp"))) + sorted(glob.glob(os.path.join(c, "*.hip")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(line for line in proc.stderr.splitlines()
                    if "packed-fp32-ops" not in line and line.strip())
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed ({proc.returncode}):\n{err}")
    if verbose and err:
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
