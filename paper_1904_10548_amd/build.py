"""Build the tapg C-ABI library (HIP for gfx950) in-tree.

``python -m paper_1904_10548_amd.build`` compiles ``csrc/*.cpp`` and
``csrc/*.hip`` with hipcc (one object per source, in parallel, under
``_build/``) and links them into ``paper_1904_10548_amd/libtapg.so``, then
builds the command-line front-end ``paper_1904_10548_amd/tapg_control`` from
``csrc/app/`` against that library.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libtapg.so")
CLI = os.path.join(PKG, "tapg_control")
OBJ_DIR = os.path.join(ROOT, "_build", "tapg")

# Packed FP32 instructions are disabled for all device code (the compiler is
# free to form them from ordinary float code otherwise).
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    c = os.path.join(PKG, "csrc")
    return sorted(glob.glob(os.path.join(c, "*.cpp"))) + sorted(glob.glob(os.path.join(c, "*.hip")))


def _hipcc():
    return os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _filter(stderr: str) -> str:
    return "\n".join(line for line in stderr.splitlines()
                     if "packed-fp32-ops" not in line and line.strip())


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    err = _filter(proc.stderr)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({proc.returncode}):\n{err}")
    if verbose and err:
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"link failed ({proc.returncode}):\n{_filter(proc.stderr)}")
    os.replace(tmp, LIB)
    _build_cli(verbose)
    return LIB


def _build_cli(verbose: bool) -> str:
    """The front-end executable: host code only, linked to libtapg.so next to it."""
    src = os.path.join(PKG, "csrc", "app", "tapg_control.cpp")
    tmp = CLI + ".tmp"
    cmd = [_hipcc(), "-O2", "-std=c++17", "-x", "c++", "-I", os.path.join(ROOT, "include"), src,
           "-x", "none", "-L", PKG, "-l:libtapg.so", "-Wl,-rpath,$ORIGIN", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"tapg_control build failed ({proc.returncode}):\n{_filter(proc.stderr)}")
    os.replace(tmp, CLI)
    return CLI


if __name__ == "__main__":
    print(build(verbose=True))
