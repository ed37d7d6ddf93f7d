"""Host checks of bench.py: the one-GPU contract, and which committed counter
summary a bench line may cite for its dominant sweep."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the 128-scenario tree's profiled schedule (light upper levels, forward
# launch on single leaves)
PROFILED = "TAPG_SCAN=1 TAPG_LEVELS=0:1,1:1,4:1,6:1 TAPG_FWD_GROUP=1 TAPG_TOP=1"


def _summary_spec():
    path = os.path.join(ROOT, "profiles", "scan_sweeps_dwn128_fp64_hbm_counters.md")
    line = next(l for l in open(path) if l.startswith("traffic-json:"))
    return json.loads(line.split(":", 1)[1])


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_traffic_is_cited_only_under_the_launches_it_was_taken_on():
    data = _summary_spec()
    assert sorted(data["spec"].split()) == sorted(PROFILED.split())
    bwd = bench.measured_traffic("dwn128", "fp64", "scan", PROFILED, kind="bwd")
    fwd = bench.measured_traffic("dwn128", "fp64", "scan", PROFILED, kind="fwd")
    if bwd is None:  # kernel sources changed since the counters were taken
        assert data["kernel_sources_sha256"] != _sources_sha()
        return
    assert bwd == data["bytes_per_launch"]["bwd"] and fwd == data["bytes_per_launch"]["fwd"]
    # another forward grouping: the backward launches are the same ones
    other_fg = PROFILED.replace("TAPG_FWD_GROUP=1", "TAPG_FWD_GROUP=0")
    assert bench.measured_traffic("dwn128", "fp64", "scan", other_fg, kind="bwd") == bwd
    assert bench.measured_traffic("dwn128", "fp64", "scan", other_fg, kind="fwd") is None
    # other levels or no light upper levels: other backward launches
    other_lv = PROFILED.replace("0:1,1:1,4:1,6:1", "0:1,2:1,4:1,6:1")
    assert bench.measured_traffic("dwn128", "fp64", "scan", other_lv, kind="bwd") is None
    no_top = PROFILED.replace(" TAPG_TOP=1", "")
    assert bench.measured_traffic("dwn128", "fp64", "scan", no_top, kind="bwd") is None
    assert bench.measured_traffic("dwn128", "fp64", "scan", no_top, kind="fwd") == fwd
    # another workload, precision or form: no summary
    assert bench.measured_traffic("dwn128", "fp32", "scan", PROFILED, kind="bwd") is None
    assert bench.measured_traffic("dwn128", "fp64", "projector", PROFILED, kind="bwd") is None


def _sources_sha():
    import hashlib
    sha = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            sha.update(fh.read())
    return sha.hexdigest()
