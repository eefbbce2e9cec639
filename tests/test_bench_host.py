"""Host-side logic of bench.py (no GPU): the one-GPU rule and the rule that
ties the reported HBM traffic to the kernel source it was measured on."""

from __future__ import annotations

import importlib.util
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_profiled_kernel_source(tmp_path):
    b = _bench()
    for d in ("profiles", os.path.join("paper_2102_10768_amd", "csrc")):
        os.makedirs(tmp_path / d)
    src = os.path.join("paper_2102_10768_amd", "csrc", "enumerate_global.hip")
    prof = os.path.join("profiles", "c2_power_law_hbm_counters.md")
    shutil.copy(os.path.join(ROOT, src), tmp_path / src)
    shutil.copy(os.path.join(ROOT, prof), tmp_path / prof)
    b.ROOT = str(tmp_path)
    want = None
    for line in open(tmp_path / prof):
        if line.startswith("traffic_bytes_per_launch:"):
            want = float(line.split(":")[1])
    cur = b.measured_traffic("c2")
    # the committed summary either matches the committed source (a number) or
    # is stale (None); a changed source must always give None
    assert cur in (want, None)
    assert b.measured_traffic("c3") is None
    with open(tmp_path / src, "a") as f:
        f.write("\n// changed\n")
    assert b.measured_traffic("c2") is None
    os.remove(tmp_path / prof)
    assert b.measured_traffic("c2") is None
