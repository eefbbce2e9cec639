"""Launch-parameter search for batched enumeration.

A batch of CSTs is enumerated by one persistent launch (``batch_count``).  How
fast that launch runs depends on knobs that leave every count unchanged:

* where the CST is read from and how it is cut (``enum_mode``; in LDS mode the
  partition budget delta_S of Section V-B follows from ``wgs_per_cu``),
* the matching order the CSTs are built with (``order_rule``: the path-based
  order of Section V-B, or non-tree constraints first),
* how many wavefronts share a task (``waves_per_wg``, ``hbm_wgs_per_cu``),
* how often and how deep work is handed to idle wavefronts
  (``hbm_donate_period``, ``hbm_donate_last_min``) and from what frontier
  size the last level is expanded flat (``hbm_flat_max``).

:func:`tune` times candidate settings on a seeded calibration subset of the
batch (by default 20 %, seed 301; a smaller subset cannot fill the GPU, so it
favours narrower grids) by coordinate descent: first the mode, then
each knob of that mode over a short list of values, keeping the best so far.
Every candidate's counts must equal those of the first setting tried; a
candidate that changes a count is rejected and reported.  After the first,
each candidate runs under a launch deadline of a few times the best time so
far, so a setting that suits the batch badly costs little.  The chosen setting
is left applied to the context and returned with the timings.
"""

from __future__ import annotations

import time

import numpy as np

from . import cstm

# knob -> values tried, per enumeration mode
HBM_KNOBS = {
    "order_rule": [0, 1],
    "hbm_wgs_per_cu": [2, 3, 4],
    "hbm_donate_min": [4, 16, 32],
    "hbm_donate_period": [64, 256],
    "hbm_flat_max": [-1, 2048, 16384],
    "hbm_donate_last_min": [1024, 4096, 65536],
}
LDS_KNOBS = {
    "wgs_per_cu": [2, 4, 8],
    "waves_per_wg": [4, 8, 16],
}
MODE_START = {
    "hbm": {"enum_mode": cstm.MODE_HBM},
    "lds": {"enum_mode": cstm.MODE_LDS, "part_budget_bytes": 0},
}


def calibration_subset(n: int, frac: float = 0.2, seed: int = 301, min_n: int = 8) -> list[int]:
    """Sorted indices of a seeded random subset of ``max(min_n, frac * n)`` of ``n`` items."""
    m = min(n, max(min_n, int(round(frac * n))))
    rng = np.random.Generator(np.random.PCG64(seed))
    return sorted(int(i) for i in rng.choice(n, size=m, replace=False))


def _time_setting(ctx, graph, queries, setting: dict, repeats: int, stream, limits=None):
    """Fresh CSTs (an LDS setting partitions them on its first launch), one
    untimed launch, then ``repeats`` timed launches; returns (best seconds, counts)."""
    ctx.tune = setting
    csts = [cstm.CST(ctx, graph, q.qlabel, q.qedges, stream=stream) for q in queries]
    try:
        counts = cstm.batch_count(ctx, csts, stream=stream, limits=limits)
        best = float("inf")
        for _ in range(repeats):
            t = time.perf_counter()
            got = cstm.batch_count(ctx, csts, stream=stream, limits=limits)
            best = min(best, time.perf_counter() - t)
            if got != counts:
                raise RuntimeError("counts changed between launches of one setting")
    finally:
        for c in csts:
            c.close()
    return best, counts


def tune(ctx, graph, queries, *, frac: float = 0.2, seed: int = 301, repeats: int = 2,
         modes=("hbm", "lds"), stream=None, log=None, limits=None) -> dict:
    """Choose launch parameters for ``batch_count`` over ``queries`` (see the module docstring).

    ``queries`` are objects with ``qlabel`` and ``qedges``; ``limits`` (optional,
    one per query) are the per-query result limits of the batch.  Returns a
    record with the chosen setting, the subset used and every timing."""
    idx = calibration_subset(len(queries), frac, seed)
    sub = [queries[i] for i in idx]
    sub_limits = None if limits is None else [int(limits[i]) for i in idx]
    base = dict(ctx.tune)
    base["collect_stats"] = 0
    trials = []
    ref_counts = None

    def run(setting):
        nonlocal ref_counts
        full = {**base, **setting}
        if best_sec < float("inf"):
            full["deadline_ms"] = max(100, int(4e3 * best_sec) + 1)
        try:
            sec, counts = _time_setting(ctx, graph, sub, full, repeats, stream, sub_limits)
        except cstm.CstmError as e:
            why = "slower than the deadline" if e.status == cstm.ETIMEOUT else str(e)
            trials.append({"setting": setting, "error": why})
            if log:
                log(f"autotune {setting}: {why}")
            return float("inf")
        if ref_counts is None:
            ref_counts = counts
        if counts != ref_counts:
            trials.append({"setting": setting, "error": "counts differ from the first setting"})
            return float("inf")
        trials.append({"setting": setting, "seconds": sec})
        if log:
            log(f"autotune {setting}: {sec * 1e3:.2f} ms")
        return sec

    best_setting, best_sec = None, float("inf")  # read by run() for the deadline
    for mode in modes:
        s = dict(MODE_START[mode])
        sec = run(s)
        if sec < best_sec:
            best_setting, best_sec = s, sec
    if best_setting is None:
        ctx.tune = base
        raise RuntimeError("no candidate setting ran")
    knobs = HBM_KNOBS if best_setting["enum_mode"] == cstm.MODE_HBM else LDS_KNOBS
    for knob, values in knobs.items():
        for v in values:
            if base.get(knob) == v and knob not in best_setting:
                continue  # the current value was timed already
            if best_setting.get(knob) == v:
                continue
            s = {**best_setting, knob: v}
            if knob == "wgs_per_cu":
                s["part_budget_bytes"] = 0  # the LDS budget follows the workgroups per CU
            sec = run(s)
            if sec < best_sec:
                best_setting, best_sec = s, sec
    ctx.tune = {**base, **best_setting}
    return {
        "choice": best_setting,
        "seconds": best_sec,
        "subset": {"frac": frac, "seed": seed, "indices": idx},
        "trials": trials,
    }
