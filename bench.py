#!/usr/bin/env python3
"""Throughput benchmark of the GPU subgraph matcher on one MI355X.

Workload (default): the medium synthetic knowledge graph (300,000 vertices,
1.6M directed edges, 64 vertex types, 32 Zipf relations) resident in HBM and
100 random-walk queries of 6-10 vertices (paths and trees, 0-2 pinned
vertices), matched one query at a time with full sorted embedding tables
copied back to the host. One step = the 100 queries. ``value`` = queries/s.

Also reported: embeddings/s, per-query latency p50/p99, the same 100 queries
through sgm_match_batch, the roofline of the dominant kernel class (HIP
events on the library's stream, algorithmic bytes per launch) and the CPU
oracle on a bounded sample of the same queries.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the matcher "
              "has no multi-GPU path in this build.", file=sys.stderr)
        sys.exit(2)

    import kggen
    import paper_1807_08804_amd as P

    t0 = time.time()
    kg = kggen.named_graph("medium")
    queries, rejected = kggen.medium_queries(kg, args.queries)
    log(f"inputs ready in {time.time() - t0:.1f}s (rejected {rejected})")

    g = P.Graph.from_kg(kg)
    gp = P.Graph.from_kg(kg, profile=1)

    def one_step(graph, lat=None, stats=None):
        rows = 0
        for q in queries:
            a = time.perf_counter_ns()
            if stats is None:
                r = graph.match_query(q)
            else:
                r, st = graph.match_query(q, with_stats=True)
                stats.append(st)
            if lat is not None:
                lat.append(time.perf_counter_ns() - a)
            rows += len(r)
        return rows

    for i in range(args.warmup):
        one_step(g)
        log(f"warmup {i + 1}/{args.warmup} done")
    lat = []
    t = time.perf_counter()
    rows = 0
    for i in range(args.steps):
        rows += one_step(g, lat)
    el = time.perf_counter() - t
    log(f"timed {args.steps} steps in {el:.3f}s")
    nq = len(queries) * args.steps
    qps = nq / el
    lat_ms = sorted(x / 1e6 for x in lat)
    p50 = lat_ms[len(lat_ms) // 2]
    p99 = lat_ms[min(len(lat_ms) - 1, int(round(0.99 * (len(lat_ms) - 1))))]

    # the same queries through sgm_match_batch
    g.match_batch(queries)
    t = time.perf_counter()
    for i in range(args.steps):
        g.match_batch(queries)
    el_b = time.perf_counter() - t
    batch_qps = nq / el_b
    log(f"batch path {el_b:.3f}s")

    # per-phase device times of the persistent kernel (one pass)
    stl = []
    one_step(g, stats=stl)
    narrow = [st for st in stl if st["path"] == P.SGM_PATH_NARROW]
    phases = {k: round(statistics.mean(st[k] for st in narrow) / 1e3, 2) if narrow else None
              for k in ("ns_filter", "ns_collect", "ns_join", "ns_finish")}
    phases["queries_on_persistent_kernel"] = len(narrow)

    # roofline: every launch timed with HIP events on the library stream
    one_step(gp)
    gp.reset_kernel_stats()
    t = time.perf_counter()
    for i in range(args.steps):
        one_step(gp)
    el_p = time.perf_counter() - t
    ks = gp.kernel_stats()
    log("kernel classes (profiled region): " + json.dumps(
        {k: dict(launches=v["launches"], ms=round(v["ms"], 3)) for k, v in ks.items()}))
    dom = max((k for k in ks if ks[k]["bytes"] > 0), key=lambda k: ks[k]["ms"])
    d = ks[dom]
    achieved = d["bytes"] / (d["ms"] / 1e3) / 1e9 if d["ms"] > 0 else 0.0
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": None, "launches": d["launches"],
            "avg_launch_us": round(d["ms"] * 1e3 / max(d["launches"], 1), 3),
            "bytes_per_launch": round(d["bytes"] / max(d["launches"], 1), 1)}

    cpu = None
    if not args.no_cpu:
        import oracle
        og = oracle.graph_from_kg(kg)
        cores = os.cpu_count() or 1
        cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
        done, t = 0, time.perf_counter()
        while done < len(queries) and time.perf_counter() - t < args.cpu_seconds:
            og.match_query(queries[done], nthreads=cores)
            done += 1
        el_c = time.perf_counter() - t
        cpu = {"value": round(done / el_c, 3), "unit": "queries/s", "cores": cores,
               "kind": "oracle",
               "sample": f"first {done} of the {len(queries)} medium queries, one at a time, "
                         f"{el_c:.1f}s wall"}

    out = {
        "metric": "queries/s (single-query, medium KG, 100 walk queries)",
        "value": round(qps, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "medium KG 300K V / 1.6M E, 64 types, 32 Zipf relations; "
                               "100 random-walk queries of 6-10 vertices (paths+trees, 0-2 pins), "
                               "one at a time, sorted tables to host",
                   "queries_per_step": len(queries)},
        "embeddings_per_s": round(rows / el, 1),
        "latency_ms": {"p50": round(p50, 3), "p99": round(p99, 3)},
        "batch_api_queries_per_s": round(batch_qps, 3),
        "persistent_kernel_phase_us": phases,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
