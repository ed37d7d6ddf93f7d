"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer
and under ThreadSanitizer (CPU only).

Every host source of the library (validation, JSON reader, factor step, sweep
planner, forest builder, request server, closed loop) is compiled with g++ and
the sanitizer, linked with a stand-in device layer
(``tests/host_sanitize/mock_device.cpp``: no GPU, no arithmetic of the
method) and driven by ``tests/host_sanitize/driver.cpp`` through the C ABI,
including concurrent clients of the request server and fuzzed JSON input.
Any sanitizer report fails the run."""

import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

import dwn_synth as ds
from dwn_synth import json_files as jf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1904_10548_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_sanitize")

VARIANTS = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "tsan": ["-fsanitize=thread"],
}


def _gxx():
    return shutil.which("g++")


def _build(variant, out_dir):
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
             "-I" + CSRC] + VARIANTS[variant]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.cpp"))) + [
        os.path.join(HERE, "mock_device.cpp"), os.path.join(HERE, "driver.cpp")]
    os.makedirs(out_dir, exist_ok=True)

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        r = subprocess.run([_gxx(), *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, f"{src}:\n{r.stderr[-3000:]}"
        return obj

    with ThreadPoolExecutor(min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    exe = os.path.join(out_dir, "driver")
    r = subprocess.run([_gxx(), *flags, *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.skipif(_gxx() is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_host_code_under_sanitizer(tmp_path, variant):
    P = ds.config_problem("small")
    inst = tmp_path / "instance"
    jf.write_instance(P, str(inst), tol=1e-4, max_iter=1000)
    exe = _build(variant, str(tmp_path / "build"))
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    r = subprocess.run([exe, str(inst), str(scratch)], capture_output=True, text=True, env=env,
                       timeout=600)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert "failed: 0" in r.stdout
