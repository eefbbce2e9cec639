"""Write the screened query sets and their expected counts for the named workloads.

    python tests/golden/make_workloads.py c1
    python tests/golden/make_workloads.py c2 [--budget 200000000] [--count-cap 20000000000]
    python tests/golden/make_workloads.py c3|c5 [--budget N] [--threads 0] [--unlimited-s 2]

Expected values come from the CPU oracle (``oracle``); inputs come only
from ``synth``.  For the sparse class of c2 the expected count is the exact
labelled tree DP of ``closed_forms`` (see below).

Screen (deterministic and host-independent but for the dense deadline): walks are drawn in order from the
seeded query stream and join their class (sparse: average query degree below
3, dense: 3 or more) while it has room.
  sparse: the query must be a tree with pairwise-distinct labels and have at
          most count_cap embeddings; its exact count is the labelled tree
          homomorphism DP (injectivity is automatic for such queries), a pin
          independent of the oracle that is exact at any graph size;
  dense:  the oracle must reach min(#embeddings, dense_limit) within the
          workload's dense_budget visited partial embeddings and
          dense_deadline_s seconds (at most dense_tries attempts); the stored
          count is that minimum, and the query carries the limit.
On the power-law graph almost every random-walk query has 10^9 to 10^25
embeddings; the screen keeps the ones an exact reference can still count.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import closed_forms as cf  # noqa: E402
from synth import make_graph, query_set  # noqa: E402
from synth.graphs import _rng  # noqa: E402
from synth.queries import STREAM_QUERIES, random_walk_query  # noqa: E402
from synth.workloads import ALL  # noqa: E402


def write(name: str, payload: dict):
    path = os.path.join(HERE, f"{name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(payload, f, indent=1)
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


def make_small(w: dict):
    g = make_graph(w["graph"])
    qs = query_set(g, w["queries"]["sizes"], w["queries"]["seed"])
    out = []
    for q in qs:
        r = oracle.match(g, q, list_rows=True, cap=1 << 20)
        assert r.status == oracle.OK
        d = q.to_dict()
        d.update(count=r.count, nodes=r.nodes)
        out.append(d)
    write(w["name"], {"workload": w, "graph_summary": g.summary(), "oracle": {"threads": r.threads},
                      "queries": out})


def make_screened(w: dict, budget: int, max_draws: int, threads: int, count_cap: int, dense_tries: int,
                  dense_seconds: float):
    """Screen random walks into the sparse and dense classes (see the module docstring).
    Dense tries stop after dense_tries attempts or once they have used
    dense_seconds of oracle time (0: no time cap)."""
    g = make_graph(w["graph"])
    print("graph", g.summary(), flush=True)
    lcol = oracle.label_grouped_col(g, threads=threads)
    dense_spent = 0.0
    exact = cf.ExactTreeCounter(g)
    spec = w["queries"]
    quota = {"sparse": int(spec["sparse"]), "dense": int(spec["dense"])}
    dense_limit = int(spec.get("dense_limit", 0))
    dense_deadline = float(spec.get("dense_deadline_s", 0.0))
    dense_budget = int(spec.get("dense_budget", budget))
    got = {"sparse": [], "dense": []}
    rng = _rng(spec["seed"], STREAM_QUERIES)
    stats = {"draws": 0, "skipped_full": 0, "sparse_not_distinct_label_tree": 0, "sparse_over_cap": 0,
             "dense_tried": 0, "dense_over_budget": 0, "dense_not_tried": 0}
    t_start = time.time()
    for draw in range(max_draws):
        if all(len(got[c]) >= quota[c] for c in quota):
            break
        q = random_walk_query(g, int(spec["k"]), rng)
        stats["draws"] += 1
        cls = "dense" if q.avg_degree >= 3.0 else "sparse"
        if len(got[cls]) >= quota[cls]:
            stats["skipped_full"] += 1
            continue
        d = q.to_dict()
        if cls == "sparse":
            if not cf.is_tree_with_distinct_labels(q):
                stats["sparse_not_distinct_label_tree"] += 1
                continue
            try:
                c = exact.count(q)
            except OverflowError:
                c = None
            if c is None or c > count_cap:
                stats["sparse_over_cap"] += 1
                continue
            d.update(draw=draw, kind=cls, count=c, expected_from="tree_dp")
        else:
            if stats["dense_tried"] >= dense_tries or (dense_seconds and dense_spent >= dense_seconds):
                stats["dense_not_tried"] += 1
                continue
            stats["dense_tried"] += 1
            t = time.time()
            r = oracle.match(g, q, node_budget=dense_budget, deadline_s=dense_deadline, threads=threads, lcol=lcol,
                             limit=dense_limit)
            dt = time.time() - t
            dense_spent += dt
            if r.status != oracle.OK:
                stats["dense_over_budget"] += 1
                print(f"draw {draw} dense m_q={q.m_q} over budget ({dt:.1f}s)", flush=True)
                continue
            d.update(draw=draw, kind=cls, count=r.count, nodes=r.nodes, oracle_s=round(dt, 3), expected_from="oracle")
            if dense_limit:
                d["limit"] = dense_limit
        got[cls].append(d)
        print(f"draw {draw} {cls} m_q={q.m_q} count={d['count']} "
              f"[{len(got['sparse'])}/{quota['sparse']} sparse, {len(got['dense'])}/{quota['dense']} dense]",
              flush=True)
    queries = sorted(got["sparse"] + got["dense"], key=lambda d: d["draw"])
    for i, d in enumerate(queries):
        d["qid"] = i
    stats["seconds"] = round(time.time() - t_start, 1)
    write(w["name"], {
        "workload": w,
        "graph_summary": g.summary(),
        "screen": {"sparse_rule": "tree query with pairwise-distinct labels and at most count_cap embeddings "
                                  "(exact count: labelled tree homomorphism DP)",
                   "dense_rule": "oracle (label-grouped rows) reaches min(total, dense_limit) within dense_budget "
                                 "work units and dense_deadline_s seconds",
                   "dense_limit": dense_limit, "dense_budget": dense_budget, "dense_deadline_s": dense_deadline,
                   "count_cap": count_cap, "max_draws": max_draws,
                   "dense_tries": dense_tries, "dense_seconds_cap": dense_seconds,
                   "dense_oracle_seconds": round(dense_spent, 1), **stats,
                   "short": {c: quota[c] - len(got[c]) for c in quota}},
        "oracle": {"threads": threads or oracle.num_cores()},
        "queries": queries,
    })


def make_batch(w: dict, budget: int, max_draws: int, threads: int):
    """Batch / serving workload: query sizes uniform in [k_min, k_max]; each draw
    is kept when the oracle finishes it within the work budget (the same
    deterministic screen).  With a result limit L in the recipe, the stored
    count is min(#embeddings, L) and the oracle may stop once it found L."""
    g = make_graph(w["graph"])
    print("graph", g.summary(), flush=True)
    lcol = oracle.label_grouped_col(g)
    spec = w["queries"]
    rng = _rng(spec["seed"], STREAM_QUERIES)
    want = int(spec["count"])
    limit = int(spec.get("limit", 0))
    out = []
    stats = {"draws": 0, "over_budget": 0}
    t_start = time.time()
    for draw in range(max_draws):
        if len(out) >= want:
            break
        k = int(rng.integers(int(spec["k_min"]), int(spec["k_max"]) + 1))
        q = random_walk_query(g, k, rng)
        stats["draws"] += 1
        t = time.time()
        r = oracle.match(g, q, node_budget=budget, threads=threads, lcol=lcol, limit=limit)
        dt = time.time() - t
        if (draw + 1) % 250 == 0:
            print(f"{draw + 1} draws, {len(out)} kept ({time.time() - t_start:.0f}s)", flush=True)
        if r.status != oracle.OK:
            stats["over_budget"] += 1
            continue
        d = q.to_dict()
        d.update(draw=draw, qid=len(out), count=r.count, nodes=r.nodes, oracle_s=round(dt, 4),
                 expected_from="oracle")
        if limit:
            d["limit"] = limit
        out.append(d)
        if len(out) % 50 == 0:
            print(f"{len(out)}/{want} after {draw + 1} draws ({time.time() - t_start:.0f}s)", flush=True)
    stats["seconds"] = round(time.time() - t_start, 1)
    write(w["name"], {
        "workload": w,
        "graph_summary": g.summary(),
        "screen": {"rule": "oracle (label-grouped rows) finishes within node_budget work units"
                           + (f" or finds {limit} embeddings (stored count = min(total, {limit}))" if limit else ""),
                   "node_budget": budget, "sizes_kept": {str(k): sum(1 for d in out if len(d["qlabel"]) == k)
                                                         for k in range(int(spec["k_min"]), int(spec["k_max"]) + 1)},
                   "max_draws": max_draws, **stats, "short": want - len(out)},
        "oracle": {"threads": threads or oracle.num_cores()},
        "queries": out,
    })


def make_fixed_draws(w: dict, budget: int, threads: int, unlimited_s: float, deadline_s: float):
    """Batch and billion-edge workloads: exactly the configured number of random walks
    (sizes uniform in [k_min, k_max]), every one kept, none redrawn.  Each
    asks for min(#embeddings, limit); the oracle (label-grouped rows) screens
    each within node_budget work units and deadline_s seconds.  Queries it
    finishes get their stored count; the others are recorded as INF (no
    count) and stay out of parity.  Progress is appended to
    <name>.partial.jsonl next to the output, and a rerun skips the queries
    already there (the file is removed once the set is written)."""
    t_start = time.time()
    g = make_graph(w["graph"], log=lambda m: print(m, flush=True))
    print("graph", g.summary(), f"({time.time() - t_start:.0f}s)", flush=True)
    lcol = oracle.label_grouped_col(g, threads=threads)
    spec = w["queries"]
    rng = _rng(spec["seed"], STREAM_QUERIES)
    limit = int(spec["limit"])
    qs = []
    for _ in range(int(spec["count"])):
        k = int(rng.integers(int(spec["k_min"]), int(spec["k_max"]) + 1))
        qs.append(random_walk_query(g, k, rng))
    partial = os.path.join(HERE, f"{w['name']}.partial.jsonl")
    done, unl = {}, {}
    if os.path.exists(partial):
        for line in open(partial):
            d = json.loads(line)
            (unl if d.get("unlimited") else done)[int(d["qid"])] = d
        print(f"resuming: {len(unl)} unlimited and {len(done)} limited runs already made", flush=True)
    out, inf = [], []
    oracle_s = 0.0
    with open(partial, "a") as pf:
        # first, without the limit: does any query finish within unlimited_s seconds?
        unlimited = []
        for i, q in enumerate(qs):
            if unlimited_s <= 0:
                break
            if i not in unl:
                r = oracle.match(g, q, deadline_s=unlimited_s, threads=threads, lcol=lcol)
                unl[i] = {"qid": i, "unlimited": True, "finished": r.status == oracle.OK, "count_at_stop": r.count}
                pf.write(json.dumps(unl[i]) + "\n")
                pf.flush()
            unlimited.append(unl[i])
            print(f"unlimited query {i}: {'finished' if unl[i]['finished'] else 'INF'} {unl[i]['count_at_stop']}",
                  flush=True)
        for i, q in enumerate(qs):
            if i in done:
                d = q.to_dict()
                d.update(done[i])
            else:
                t = time.time()
                r = oracle.match(g, q, node_budget=budget, deadline_s=deadline_s, threads=threads, lcol=lcol,
                                 limit=limit)
                dt = time.time() - t
                d = q.to_dict()
                d.update(draw=i, qid=i, nodes=r.nodes, oracle_s=round(dt, 3), limit=limit)
                if r.status == oracle.OK:
                    d.update(count=r.count, expected_from="oracle")
                else:
                    d.update(count=None, partial=r.count, expected_from="INF")
                pf.write(json.dumps(d) + "\n")
                pf.flush()
            oracle_s += float(d["oracle_s"])
            if d["count"] is None:
                inf.append(i)
            out.append(d)
            print(f"query {i} k={q.k} m_q={q.m_q}: {'INF' if d['count'] is None else d['count']} "
                  f"in {d['oracle_s']:.1f}s ({len(inf)} INF so far)", flush=True)
    screen = {"rule": f"every drawn query kept; the oracle (label-grouped rows) must reach min(total, {limit}) "
                      "within node_budget work units and deadline_s seconds, else the query is INF and has no "
                      "stored count",
              "node_budget": budget, "deadline_s": deadline_s, "inf": inf, "oracle_seconds": round(oracle_s, 1),
              "sizes": {str(k): sum(1 for d in out if len(d["qlabel"]) == k)
                        for k in range(int(spec["k_min"]), int(spec["k_max"]) + 1)},
              "sizes_with_count": {str(k): sum(1 for d in out if len(d["qlabel"]) == k and d["count"] is not None)
                                   for k in range(int(spec["k_min"]), int(spec["k_max"]) + 1)},
              "seconds": round(time.time() - t_start, 1)}
    if unlimited:
        screen["unlimited_screen"] = {
            "seconds_per_query": unlimited_s, "finished": sum(u["finished"] for u in unlimited),
            "tried": len(unlimited),
            "min_count_at_stop": min(u["count_at_stop"] for u in unlimited),
            "max_count_at_stop": max(u["count_at_stop"] for u in unlimited)}
    write(w["name"], {
        "workload": w,
        "graph_summary": g.summary(),
        "screen": screen,
        "oracle": {"threads": threads or oracle.num_cores()},
        "queries": out,
    })
    os.remove(partial)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(ALL))
    ap.add_argument("--budget", type=int, default=200_000_000)
    ap.add_argument("--max-draws", type=int, default=200_000)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--count-cap", type=int, default=20_000_000_000)
    ap.add_argument("--dense-tries", type=int, default=100)
    ap.add_argument("--dense-seconds", type=float, default=0.0,
                    help="c2: stop trying dense draws after this much oracle time (0: no cap)")
    ap.add_argument("--deadline-s", type=float, default=300.0,
                    help="c3/c5: oracle seconds per query before it counts as INF")
    ap.add_argument("--unlimited-s", type=float, default=2.0,
                    help="c5: seconds of an unlimited oracle run per query before the limited screen (0: skip)")
    a = ap.parse_args()
    w = ALL[a.name]
    if w["queries"].get("fixed_draws"):
        default_budget = int(w["queries"].get("screen_budget", 150_000_000_000))
        make_fixed_draws(w, a.budget if a.budget != 200_000_000 else default_budget, a.threads, a.unlimited_s,
                         a.deadline_s)
    elif "sizes" in w["queries"]:
        make_small(w)
    elif "k_min" in w["queries"]:
        make_batch(w, a.budget, a.max_draws, a.threads)
    else:
        make_screened(w, a.budget, a.max_draws, a.threads, a.count_cap, a.dense_tries, a.dense_seconds)


if __name__ == "__main__":
    main()
