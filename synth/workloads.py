"""Named synthetic workloads (graph recipe + query recipe), shaped like the paper's.

The paper measures on LDBC-SNB social graphs (Section VII, Table III) with
queries from LDBC tasks; neither is available, so these seeded synthetic
stand-ins take their place.  Only recipes live here; which drawn queries make
up a screened set, and their expected counts, are written by
``tests/golden/make_workloads.py`` (from the CPU oracle) into
``tests/golden/<name>.json``.
"""

from __future__ import annotations

SMALL = {
    "name": "c1",
    "title": "ER G(3000, 10/2999), 20 uniform labels, 8 random-walk queries of 4 vertices",
    "graph": {"kind": "er", "n": 3000, "p": 10 / 2999, "seed": 11, "labels": {"kind": "uniform", "L": 20}},
    "queries": {"sizes": [4] * 8, "seed": 21},
}

POWER_LAW_1M = {
    "name": "c2",
    "title": "Chung-Lu 1M vertices, 16M edges, gamma 2.3, 32 Zipf(1.0) labels; screened 8-vertex random-walk queries "
             "(sparse: exact counts; dense: min(#embeddings, 10^9))",
    "graph": {"kind": "chung_lu", "n": 1_000_000, "m": 16_000_000, "gamma": 2.3, "seed": 12,
              "labels": {"kind": "zipf", "L": 32, "s": 1.0}},
    # 50 sparse (average query degree < 3) and 50 dense (>= 3) random-walk
    # queries; a dense query counts min(#embeddings, dense_limit), since on this
    # graph nearly every dense walk has more embeddings than an exact reference
    # can enumerate
    "queries": {"k": 8, "sparse": 50, "dense": 50, "seed": 22, "dense_limit": 1_000_000_000,
                "dense_deadline_s": 120.0, "dense_budget": 15_000_000_000},
}

RMAT_22 = {
    "name": "c3",
    "title": "R-MAT scale 22 (a,b,c = .57,.19,.19), 64 uniform labels; 1000 random-walk queries of 4..16 vertices, "
             "each counting min(#embeddings, 10^8)",
    "graph": {"kind": "rmat", "scale": 22, "edge_factor": 16, "a": 0.57, "b": 0.19, "c": 0.19, "seed": 13,
              "labels": {"kind": "uniform", "L": 64}},
    # exactly the 1,000 drawn walks (sizes uniform in 4..16); most walks of six or
    # more vertices have 10^9 to 10^17 embeddings here, so each asks for
    # min(#embeddings, limit), which the oracle counts exactly
    "queries": {"k_min": 4, "k_max": 16, "count": 1000, "seed": 23, "limit": 100_000_000, "fixed_draws": True,
                "screen_budget": 15_000_000_000},
}

SERVE_16M = {
    "name": "c4",
    "title": "Chung-Lu 16M vertices, 256M edges, gamma 2.1 (native generator), 100 Zipf(0.8) labels; "
             "screened pool of random-walk queries of 4..24 vertices, results limited to 10^6, Poisson arrivals",
    # generated natively (counter-based SplitMix64, alias sampling, all host threads)
    "graph": {"kind": "chung_lu_native", "n": 16_000_000, "m": 256_000_000, "gamma": 2.1, "seed": 14,
              "labels": {"kind": "zipf", "L": 100, "s": 0.8}},
    # each request asks for min(#embeddings, limit): on this graph almost every
    # random-walk query has far more embeddings than any search can visit
    "queries": {"k_min": 4, "k_max": 24, "count": 200, "seed": 24, "limit": 1_000_000},
    # request streams: 2,000 arrivals per rate, one seed per rate; admission budget
    "serve": {"rates": [50, 200, 800], "arrivals": 2000, "seeds": [201, 202, 203], "mem_budget_gb": 64},
}

BILLION = {
    "name": "c5",
    "title": "R-MAT scale 26 (a,b,c = .57,.19,.19; native SplitMix64 generator), 128 uniform labels; "
             "200 random-walk queries of 12..32 vertices, each counting min(#embeddings, 10^9)",
    "graph": {"kind": "rmat_native", "scale": 26, "edge_factor": 16, "a": 0.57, "b": 0.19, "c": 0.19, "seed": 15,
              "labels": {"kind": "uniform", "L": 128}},
    # every one of these random walks has far more embeddings than any search
    # can visit (the oracle's partial counts pass 10^8 within seconds), so each
    # query asks for min(#embeddings, limit); the stored counts come from the oracle
    "queries": {"k_min": 12, "k_max": 32, "count": 200, "seed": 25, "limit": 1_000_000_000, "fixed_draws": True,
                "screen_budget": 150_000_000_000},
}

ALL = {w["name"]: w for w in (SMALL, POWER_LAW_1M, RMAT_22, SERVE_16M, BILLION)}
