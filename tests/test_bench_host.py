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
    prof = os.path.join("profiles", "c5_rmat26_hbm_counters.md")
    shutil.copy(os.path.join(ROOT, src), tmp_path / src)
    shutil.copy(os.path.join(ROOT, prof), tmp_path / prof)
    b.ROOT = str(tmp_path)
    want = None
    for line in open(tmp_path / prof):
        if line.startswith("traffic_bytes_per_launch:"):
            want = float(line.split(":")[1])
    cur = b.measured_traffic("c5")
    # the committed summary either matches the committed source (a number) or
    # is stale (None); a changed source must always give None
    assert cur in (want, None)
    assert b.measured_traffic("c3") is None
    with open(tmp_path / src, "a") as f:
        f.write("\n// changed\n")
    assert b.measured_traffic("c5") is None
    os.remove(tmp_path / prof)
    assert b.measured_traffic("c5") is None


def _st(mode, ms, N=0, M=0, F=0, summed=0, image_bytes=0, launches=1):
    return {"mode": mode, "kernel_ms": ms, "launches": launches, "extensions": N, "edge_checks": M, "pushed": F,
            "summed": summed, "image_bytes": image_bytes}


def test_roofline_prices_the_enumeration_kernel():
    b = _bench()
    # device-memory mode: CST bytes + 4 per read candidate + 4 per check + 8 per push, per launch
    counted = [({"bytes": 1000}, _st(2, 0, N=100, M=10, F=5, summed=40)),
               ({"bytes": 3000}, _st(2, 0, N=50, M=0, F=1))]
    r = b.roofline_of(40.0, 2, counted, "c3")
    alg = (1000 + 3000 + 4 * (150 - 40) + 4 * 10 + 8 * 6) / 2
    assert r["kernel"] == "k_enumerate_global" and r["algorithmic_bytes_per_launch"] == alg
    assert abs(r["avg_launch_ms"] - 20.0) < 1e-12
    assert abs(r["achieved"] - alg / 0.020 / 1e9) < 1e-12
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-15 and "on_chip" not in r
    assert r["traffic"] is None and r["hbm_gbs"] is None  # no counter summary for this workload
    assert "lane_utilisation" not in r  # no round counts given
    counted[0][1]["chunks"], counted[1][1]["chunks"] = 2, 1
    r = b.roofline_of(40.0, 2, counted, "c3")
    assert abs(r["lane_utilisation"] - (150 - 40) / (64 * 3)) < 1e-15 and r["work"]["chunks"] == 3
    # LDS images: HBM bytes are the images, the list work is on chip
    counted = [({"bytes": 1000}, _st(1, 0, N=100, M=10, F=5, image_bytes=7000))]
    r = b.roofline_of(50.0, 1, counted, "c3")
    assert r["kernel"] == "k_enumerate" and r["algorithmic_bytes_per_launch"] == 7000
    assert r["on_chip"]["bytes_per_launch"] == 4 * 100 + 4 * 10 + 8 * 5
    assert abs(r["on_chip"]["peak"] - 128 * 256 * 2.4) < 1e-9
    assert b.roofline_of(0.0, 0, [], "c3")["achieved"] == 0.0


def test_workload_queries_skip_inf_and_carry_limits():
    b = _bench()
    W = {"workload": {"queries": {"limit": 7}},
         "queries": [{"qlabel": [0, 1], "qedges": [[0, 1]], "count": 3, "limit": 7},
                     {"qlabel": [0, 1], "qedges": [[0, 1]], "count": None, "limit": 7},
                     {"qlabel": [2], "qedges": [], "count": 5}]}
    qs, exp, lim, inf = b.workload_queries(W)
    assert exp == [3, 5] and lim == [7, 7] and inf == 1 and [q.k for q in qs] == [2, 1]
    qs, exp, lim, inf = b.workload_queries(W, max_queries=1)
    assert exp == [3] and inf == 1
    # exact totals only: a count that reached its limit is not a total
    W["queries"].append({"qlabel": [0], "qedges": [], "count": 7, "limit": 7})
    W["queries"].append({"qlabel": [1], "qedges": [], "count": 2, "limit": 0})
    qs, exp, lim, inf = b.workload_queries(W, exact_only=True)
    assert exp == [3, 5, 2] and lim == [0, 0, 0] and inf == 1
    qs, exp, lim, inf = b.workload_queries(W)
    assert exp == [3, 5, 7, 2] and lim == [7, 7, 7, 0]


def test_cpu_baseline_samples_stored_queries_and_checks_finished_counts():
    """The oracle baseline runs the stored queries of a small workload to their
    stored counts (every one finishes here) and reports the rate it found."""
    import types

    b = _bench()
    from synth import make_graph

    W = b.load_workload("c1")
    qs, exp, lim, _ = b.workload_queries(W)
    S = types.SimpleNamespace(g=make_graph(W["workload"]["graph"]), queries=qs, limits=lim, expected=exp)
    allc, one = b.cpu_baselines(S, types.SimpleNamespace(cpu_seconds=20.0), n_sample=4)
    assert one["cores"] == 1 and allc["cores"] >= 1
    for r in (allc, one):
        assert r["value"] > 0 and r["kind"] == "oracle" and "4 finished" in r["sample"]


def test_pipelined_step_traffic_is_read_for_the_profiled_kernel_source(tmp_path):
    b = _bench()
    for d in ("profiles", os.path.join("paper_2102_10768_amd", "csrc")):
        os.makedirs(tmp_path / d)
    src = os.path.join("paper_2102_10768_amd", "csrc", "enumerate_global.hip")
    prof = os.path.join("profiles", "c5_rmat26_pipelined_hbm_counters.md")
    shutil.copy(os.path.join(ROOT, src), tmp_path / src)
    shutil.copy(os.path.join(ROOT, prof), tmp_path / prof)
    b.ROOT = str(tmp_path)
    want = None
    for line in open(tmp_path / prof):
        if line.startswith("traffic_bytes_per_step:"):
            want = float(line.split(":")[1])
    assert b.measured_step_traffic("c5_pipelined") in (want, None)
    assert b.measured_step_traffic("c5") is None  # the single-launch summary has no per-step figure
    with open(tmp_path / src, "a") as f:
        f.write("\n// changed\n")
    assert b.measured_step_traffic("c5_pipelined") is None
    # an explicit traffic figure replaces the profile; None means not measured
    counted = [({"bytes": 1000}, _st(2, 0, N=100, M=10, F=5, summed=40))]
    assert b.roofline_of(10.0, 1, counted, "c5", traffic=None)["traffic"] is None
    assert b.roofline_of(10.0, 1, counted, "c5", traffic=123.0)["traffic_bytes_per_launch"] == 123.0
