#!/usr/bin/env python3
"""Throughput benchmark of the GPU subgraph matcher on one MI355X.

Default workload ("large"): the large synthetic knowledge graph (4M
vertices, 20M directed edges, 64 vertex types, 32 Zipf relations, int32 CSR)
resident in HBM and the stored 1,024-query mixed batch (3-16 vertices;
paths, stars, trees, cyclic; 0-50% pinned). One step = the 1,024 queries as
one sgm_match_batch call (one persistent-kernel launch in a HIP graph, full
sorted embedding tables copied back to the host); ``value`` = batched
queries/s. Beside it: embeddings/s, the same 1,024 queries one at a time on
the same GPU (queries/s, p50/p99 latency), the served form on the same
graph at 200 / 1,000 / 5,000 Poisson arrivals per second (sustained qps,
p50/p99 of completion minus arrival, admission stalls), the roofline of the
persistent kernel and of the batch's root sweep, and the CPU oracle on a
bounded sample of the same batch.

``--workload medium``: the medium graph (300,000 vertices, 1.6M edges) and
100 random-walk queries of 6-10 vertices matched one at a time (plus the
same queries as one batch and served at 1,000 / 5,000 / 20,000 qps).

``--workload large-cyclic``: 50 cyclic unpinned 8-16-vertex queries on the
large graph (intermediate tables up to ~1e8 rows, chunked joins), one at a
time: exact counts for all, sorted tables to host below a row cap.

``--workload sweep``: query-size and average-degree sweeps on 1M-vertex
graphs and graph-size scaling (0.1M-16M vertices) with the graph in device
memory and in host memory; a record per point, batched and one at a time.

``--workload compressed``: multi-level compression of graphs with similar
vertices (size per level), and queries matched directly and through the
weighted graph, the original graph in device or in host memory.
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


def recorded_traffic(key):
    """HBM bytes per launch measured with rocprofv3 counters for this
    workload and kernel (profiles/hbm_traffic.json), or None when there is no
    record or the kernel sources changed since it was taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
            rec = json.load(f)
        from paper_1807_08804_amd.prof_summary import kernel_source_hash
    except (OSError, ValueError, ImportError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    e = rec.get("entries", {}).get(key)
    return e["bytes_per_launch"] if e else None


def roofline(ks, kernel=None, traffic_key=None):
    """Roofline of one kernel class (the dominant one with byte accounting
    if not named) from HIP-event times and algorithmic bytes."""
    if kernel is None:
        kernel = max((k for k in ks if ks[k]["bytes"] > 0), key=lambda k: ks[k]["ms"])
    d = ks[kernel]
    achieved = d["bytes"] / (d["ms"] / 1e3) / 1e9 if d["ms"] > 0 else 0.0
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": recorded_traffic(traffic_key) if traffic_key else None,
            "launches": d["launches"],
            "avg_launch_us": round(d["ms"] * 1e3 / max(d["launches"], 1), 3),
            "bytes_per_launch": round(d["bytes"] / max(d["launches"], 1), 1)}


def served_leg(P, kggen, g, queries, rates, arrivals):
    """Each rate gets at least `arrivals` Poisson arrivals and at least two
    seconds of them (at most 10,000), so that draining the last batch is a
    small part of the wall time; sustained = arrivals / wall time."""
    out = {}
    for rate in rates:
        n = min(10_000, max(arrivals, int(2 * rate)))
        stream = [queries[i % len(queries)] for i in range(n)]
        arr = kggen.poisson_arrivals(len(stream), rate, seed=int(rate))
        srv = P.Server(g)
        t = time.perf_counter()
        lat, _ = srv.replay(stream, arr, keep_results=False)
        wall = time.perf_counter() - t
        sst = srv.stats()
        srv.close()
        warm = len(lat) // 20  # the first 5% of arrivals are warm-up
        lt = np.sort(lat[warm:]) / 1e6
        out[str(int(rate))] = {
            "sustained_qps": round(len(stream) / wall, 1),
            "p50_ms": round(float(np.percentile(lt, 50)), 3),
            "p99_ms": round(float(np.percentile(lt, 99)), 3),
            "arrivals": n, "batches": sst["batches"], "max_in_flight": sst["max_in_flight"],
            "admission_stalls": sst["admission_stalls"], "wide_fallbacks": sst["wide_fallbacks"]}
        log(f"served at {rate:.0f} qps: {out[str(int(rate))]}")
    return out


def phase_rates(stats, P, resident):
    """Per-phase bytes and workgroup time of the persistent kernel over a
    batch: the rate one workgroup sustains in each phase, and that rate
    times the workgroups resident at once (the launch's slots) against the
    HBM peak, i.e. the fraction the phase would reach if every slot were in
    it at the same time."""
    names = ("filter", "collect", "join", "finish")
    keys = ("ns_filter", "ns_collect", "ns_join", "ns_finish")
    narrow = [st for st in stats if st["path"] == P.SGM_PATH_NARROW]
    out = {"queries": len(narrow), "resident_workgroups": resident}
    tot_ns = sum(st[k] for st in narrow for k in keys)
    for i, (nm, k) in enumerate(zip(names, keys)):
        b = sum(st["phase_bytes"][i] for st in narrow)
        ns = sum(st[k] for st in narrow)
        per_wg = b / ns if ns else 0.0  # bytes per ns = GB/s
        out[nm] = {"bytes": int(b), "workgroup_ms": round(ns / 1e6, 3),
                   "share_of_device_time": round(ns / tot_ns, 4) if tot_ns else None,
                   "per_workgroup_gbs": round(per_wg, 3),
                   "frac_if_all_slots": round(per_wg * resident / HBM_PEAK_GBS, 5)}
    return out


def cold_leg(P, g, queries):
    """Single queries with cold caches: before each, 1 GiB of device memory
    is written (hipMemset through the HIP runtime the library itself uses),
    which evicts the graph's lines from the L2s and the last-level cache;
    then the query runs alone. Per-phase device time and algorithmic bytes
    come from the persistent kernel's own clocks."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    junk, size = ctypes.c_void_p(), ctypes.c_size_t(1 << 30)
    if hip.hipMalloc(ctypes.byref(junk), size) != 0:
        raise RuntimeError("hipMalloc of the 1 GiB eviction buffer failed")
    lat, ph_ns, ph_b = [], np.zeros(4), np.zeros(4)
    for i, q in enumerate(queries):
        if hip.hipMemset(junk, ctypes.c_int(i & 255), size) != 0 or hip.hipDeviceSynchronize() != 0:
            raise RuntimeError("eviction write failed")
        t = time.perf_counter_ns()
        _, st = g.match_query(q, with_stats=True)
        lat.append((time.perf_counter_ns() - t) / 1e6)
        ph_ns += [st["ns_filter"], st["ns_collect"], st["ns_join"], st["ns_finish"]]
        ph_b += list(st["phase_bytes"])
    hip.hipFree(junk)
    lat = np.sort(np.asarray(lat))
    names = ["filter", "collect", "join", "finish"]
    return {"queries": len(queries),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "phases": {n: {"us_per_query": round(ph_ns[k] / len(queries) / 1e3, 2),
                           "bytes_per_query": round(ph_b[k] / len(queries), 1),
                           "gbs": round(ph_b[k] / max(ph_ns[k], 1), 3)}
                       for k, n in enumerate(names)}}


# the thesis's four refinement variants (Ch. 3, Sec. "Effect of Optimization
# Techniques"): (name, refine_rounds, refine_reversed)
ABLATION_VARIANTS = [("converge", -1, 0), ("converge_reversed", -1, 1),
                     ("one_round_reversed", 1, 1), ("none", 0, 1)]


def ablation_leg(P, kg, queries):
    """Each refinement variant with both graph representations and with the
    outgoing graph alone, on the multi-kernel path (the one that runs both),
    counting only. Intermediate bytes of a query: its candidate lists (4 B
    per candidate), its candidate-edge tables (4 B per candidate edge) and
    its largest join table; time is the host wall time per query."""
    per = {}
    for out_only in (0, 1):
        for name, rounds, rev in ABLATION_VARIANTS:
            key = f"{'out_only' if out_only else 'in_out'}/{name}"
            g = P.Graph.from_kg(kg, path=P.SGM_PATH_WIDE, out_only=out_only,
                                refine_rounds=rounds, refine_reversed=rev)
            for q in queries[:4]:
                g.match_query(q, count_only=True)
            ms, inter, peak, cand, counts = [], [], [], [], []
            for q in queries:
                t = time.perf_counter()
                n, st = g.match_query(q, count_only=True, with_stats=True)
                ms.append((time.perf_counter() - t) * 1e3)
                inter.append(4 * sum(st["cand"][:q.n]) + 4 * sum(st["ec"][:q.m]) + st["peak_bytes"])
                peak.append(st["peak_rows"])
                cand.append(sum(st["cand"][:q.n]))
                counts.append(int(n))
            g.close()
            per[key] = dict(ms=ms, inter=inter, peak=peak, cand=cand, counts=counts)
            log(f"ablation {key}: {np.mean(ms):.2f} ms/query, intermediate "
                f"{np.mean(inter) / 2**20:.2f} MiB mean")
    base = per["in_out/one_round_reversed"]
    for k, v in per.items():
        if v["counts"] != base["counts"]:
            raise RuntimeError(f"ablation variant {k} changed a result count")
    out = {}
    for k, v in per.items():
        ratio = np.asarray(v["inter"], np.float64) / np.maximum(np.asarray(base["inter"]), 1)
        out[k] = {"ms_per_query": round(float(np.mean(v["ms"])), 3),
                  "intermediate_mib_mean": round(float(np.mean(v["inter"])) / 2**20, 3),
                  "intermediate_mib_max": round(float(np.max(v["inter"])) / 2**20, 3),
                  "peak_rows_max": int(np.max(v["peak"])),
                  "candidates_mean": round(float(np.mean(v["cand"])), 1),
                  "intermediate_ratio_to_default_max": round(float(np.max(ratio)), 2),
                  "intermediate_ratio_to_default_median": round(float(np.median(ratio)), 3)}
    return {"queries": len(queries), "max_vertices": int(max(q.n for q in queries)),
            "default": "in_out/one_round_reversed", "variants": out}


def cpu_leg(kg, queries, seconds):
    """The oracle on a bounded sample of the same workload: the queries in
    order, cycling, until `seconds` of wall time have passed (queries that
    hit the oracle's work budget are counted as skipped, not as done)."""
    import oracle
    og = oracle.graph_from_kg(kg)
    cores = os.cpu_count() or 1
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    done, skipped, i, t = 0, 0, 0, time.perf_counter()
    while time.perf_counter() - t < seconds:
        try:
            og.match_query(queries[i % len(queries)], nthreads=cores, max_steps=200_000_000)
            done += 1
        except oracle.OracleError:
            skipped += 1
        i += 1
    el = time.perf_counter() - t
    passes = f"{i / len(queries):.1f} passes over" if i >= len(queries) else f"the first {i} of"
    return {"value": round(done / el, 3), "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{passes} the {len(queries)} queries one at a time, {i} calls "
                      f"({skipped} stopped by the oracle's work budget of 2e8 candidate tests), "
                      f"{el:.1f}s wall"}


def bench_medium(args, P, kggen):
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
    lat_ms = sorted(x / 1e6 for x in lat)
    p50 = lat_ms[len(lat_ms) // 2]
    p99 = lat_ms[min(len(lat_ms) - 1, int(round(0.99 * (len(lat_ms) - 1))))]

    g.match_batch(queries)
    t = time.perf_counter()
    for i in range(args.steps):
        g.match_batch(queries)
    el_b = time.perf_counter() - t
    log(f"batch path {el_b:.3f}s")
    # the same batches with separate launches instead of one HIP graph
    gd = P.Graph.from_kg(kg, graphs=0)
    gd.match_batch(queries)
    t = time.perf_counter()
    for i in range(args.steps):
        gd.match_batch(queries)
    el_bd = time.perf_counter() - t
    gd.close()

    served = None if args.no_serve else served_leg(
        P, kggen, g, queries, [float(x) for x in args.serve_rates.split(",") if x],
        args.serve_arrivals)

    stl = []
    one_step(g, stats=stl)
    narrow = [st for st in stl if st["path"] == P.SGM_PATH_NARROW]
    phases = {k: round(statistics.mean(st[k] for st in narrow) / 1e3, 2) if narrow else None
              for k in ("ns_filter", "ns_collect", "ns_join", "ns_finish")}
    phases["queries_on_persistent_kernel"] = len(narrow)

    one_step(gp)
    gp.reset_kernel_stats()
    for i in range(args.steps):
        one_step(gp)
    ks = gp.kernel_stats()
    log("kernel classes (profiled region): " + json.dumps(
        {k: dict(launches=v["launches"], ms=round(v["ms"], 3)) for k, v in ks.items()}))

    cpu = None if args.no_cpu else cpu_leg(kg, queries, args.cpu_seconds)
    return {
        "metric": "queries/s (single-query, medium KG, 100 walk queries)",
        "value": round(nq / el, 3),
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
        "batch_api_queries_per_s": round(nq / el_b, 3),
        "batch_api_queries_per_s_no_graph": round(nq / el_bd, 3),
        "served": served,
        "persistent_kernel_phase_us": phases,
        "roofline": roofline(ks, "persist", "medium:persist"),
        "cpu_baseline": cpu,
    }


def bench_large(args, P, kggen):
    t0 = time.time()
    kg = kggen.named_graph("large")
    queries, rejected = kggen.load_large_batch(args.batch)
    log(f"batch inputs ready in {time.time() - t0:.1f}s (rejected {rejected})")
    t = time.time()
    g = P.Graph.from_kg(kg)
    gp = P.Graph.from_kg(kg, profile=1)
    log(f"graph resident in {time.time() - t:.1f}s")

    # tune the persistent kernel's work division and join schedule on a
    # sample of the batch (outside the timed region), then time the batch
    default_tuning = g.tuning()
    g.match_batch(queries)
    t = time.perf_counter()
    for i in range(args.steps):
        g.match_batch(queries)
    el_default = time.perf_counter() - t
    t = time.perf_counter()
    tuned = g.autotune(queries[::4], reps=1)
    log(f"autotune in {time.perf_counter() - t:.1f}s: {tuned}")
    for i in range(args.warmup):
        g.match_batch(queries)
    log(f"{args.warmup} warmup batches done")
    t = time.perf_counter()
    rows = 0
    for i in range(args.steps):
        rows = sum(len(r) for r in g.match_batch(queries))
    el_b = time.perf_counter() - t
    log(f"batched: {args.steps} x {len(queries)} in {el_b:.3f}s (default tuning {el_default:.3f}s)")
    gp.set_tuning(**tuned)
    # one query at a time with the library's default tuning (its work
    # sharing serves single queries; the batch's pick may switch it off)
    g.set_tuning(**default_tuning)
    for q in queries[:32]:
        g.match_query(q)
    lat = []
    rows_1 = 0
    t = time.perf_counter()
    for q in queries:
        a = time.perf_counter_ns()
        rows_1 += len(g.match_query(q))
        lat.append(time.perf_counter_ns() - a)
    el_1 = time.perf_counter() - t
    lat_ms = np.sort(np.asarray(lat, np.float64)) / 1e6
    log(f"one at a time: {len(queries)} in {el_1:.3f}s")
    cold = None if args.no_cold else cold_leg(P, g, queries[:64])
    if cold:
        log(f"cold caches, one at a time: p50 {cold['p50_ms']} ms, p99 {cold['p99_ms']} ms")

    # per-phase algorithmic bytes and device time of the persistent kernel
    # (filter = root candidates, explore and refine; collect = candidate
    # edges; join; finish = ordering and output), summed over the batch
    _, bstats = g.match_batch(queries, count_only=True, with_stats=True)
    phases = phase_rates(bstats, P, resident=min(tuned["slots"], len(queries)))

    gp.match_batch(queries)
    gp.reset_kernel_stats()
    for i in range(args.steps):
        gp.match_batch(queries)
    ks = gp.kernel_stats()
    log("kernel classes (profiled region): " + json.dumps(
        {k: dict(launches=v["launches"], ms=round(v["ms"], 3)) for k, v in ks.items()}))

    served = None
    if not args.no_serve:
        sq, _ = kggen.load_large_serve(args.serve_queries)
        served = served_leg(P, kggen, g, sq, [200.0, 1000.0, 5000.0], args.serve_arrivals)
    ablation = None
    if not args.no_ablation:
        t = time.time()
        # the 24 largest queries and the 24 with the largest join tables
        # under the default settings (from the batch's own statistics)
        big = sorted(range(len(queries)), key=lambda i: (-queries[i].n, i))[:24]
        heavy = sorted((i for i in range(len(queries)) if i not in set(big)),
                       key=lambda i: (-bstats[i]["peak_rows"], i))[:24]
        lq = [queries[i] for i in big + heavy]
        mkg = kggen.named_graph("medium")
        mq, _ = kggen.medium_queries(mkg, 40)
        ablation = {"large": ablation_leg(P, kg, lq), "medium": ablation_leg(P, mkg, mq)}
        log(f"ablation legs in {time.time() - t:.1f}s")
    cpu = None if args.no_cpu else cpu_leg(kg, queries, args.cpu_seconds)
    nq = args.steps * len(queries)
    return {
        "metric": "queries/s (batched: 1024 mixed queries on the large KG as one call)",
        "value": round(nq / el_b, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el_b * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "large KG 4M V / 20M E (64 types, 32 Zipf relations); batch of "
                               "1024 queries, 3-16 vertices, paths/stars/trees/cyclic, 0-50% "
                               "pinned, H <= 1e6 (kggen/fixtures/large_batch.json); sorted "
                               "tables to host",
                   "queries_per_step": len(queries)},
        "embeddings_per_s": round(rows * args.steps / el_b, 1),
        "single_query": {"queries_per_s": round(len(queries) / el_1, 3),
                         "embeddings_per_s": round(rows_1 / el_1, 1),
                         "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                         "cold_caches": cold},
        "batched_over_single": round((nq / el_b) / (len(queries) / el_1), 2),
        "tuning": tuned,
        "default_tuning": {"tuning": default_tuning,
                           "queries_per_s": round(args.steps * len(queries) / el_default, 3)},
        "served": served,
        "roofline": roofline(ks, "persist", "large:persist"),
        "roofline_root_sweep": roofline(ks, "check", "large:check"),
        "persistent_kernel_phases": phases,
        "refinement_ablation": ablation,
        "cpu_baseline": cpu,
    }


def bench_large_cyclic(args, P, kggen):
    """50 cyclic 8-16-vertex unpinned queries on the large graph, one at a
    time: exact counts for all (all join levels on the device, chunked to
    the join budget) and full sorted tables to host for those up to the row
    cap (above it the library answers SGM_ETOOBIG with the exact count)."""
    t0 = time.time()
    kg = kggen.named_graph("large")
    kg.ensure_in()
    queries = kggen.load_large_cyclic()
    g = P.Graph.from_kg(kg)
    gc = P.Graph.from_kg(kg, result_cap_rows=args.row_cap)
    log(f"inputs ready in {time.time() - t0:.1f}s")
    for q in queries[:3]:
        g.match_query(q, count_only=True)
    counts, peaks, chunks, t_count = [], [], [], []
    for i, q in enumerate(queries):
        t = time.perf_counter()
        n, st = g.match_query(q, count_only=True, with_stats=True)
        t_count.append(time.perf_counter() - t)
        counts.append(n)
        peaks.append(st["peak_rows"])
        chunks.append(st["n_chunks"])
    el_c = sum(t_count)
    log(f"count-only: {len(queries)} queries in {el_c:.2f}s, {sum(counts)} embeddings")
    done, rows, capped, t = 0, 0, 0, time.perf_counter()
    for q, n in zip(queries, counts):
        try:
            r = gc.match_query(q)
            rows += len(r)
            done += 1
            del r
        except P.SGMError as e:
            if e.code != P.SGM_ETOOBIG:
                raise
            capped += 1
    el_m = time.perf_counter() - t
    log(f"materialized: {done} tables, {rows} rows in {el_m:.2f}s ({capped} above the cap)")
    return {
        "metric": "queries/s (large KG, 50 cyclic unpinned queries, exact counts, one at a time)",
        "value": round(len(queries) / el_c, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 3,
        "ms_per_step": round(el_c * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "large KG 4M V / 20M E; 50 queries of 8-16 vertices with 1-3 "
                               "cycles, no pins, 1e7 <= H <= 2e9 (kggen/fixtures/large_cyclic.json)",
                   "queries_per_step": len(queries)},
        "embeddings_per_s": round(sum(counts) / el_c, 1),
        "embeddings": int(sum(counts)),
        "peak_intermediate_rows": int(max(peaks)),
        "max_chunks": int(max(chunks)),
        "materialized": {"row_cap": args.row_cap, "queries": done, "above_cap": capped,
                         "rows": rows, "seconds": round(el_m, 3),
                         "rows_per_s": round(rows / el_m, 1) if el_m > 0 else None},
        "per_query_ms": {"p50": round(1e3 * float(np.percentile(t_count, 50)), 2),
                         "max": round(1e3 * max(t_count), 2)},
        "roofline": None,
        "cpu_baseline": None,
    }


def _point(P, g, qs, batches=3):
    """One sweep point: the queries as one batch (warm once, then the mean
    of ``batches`` calls) and one at a time, on graph g."""
    g.match_batch(qs)
    t = time.perf_counter()
    for _ in range(batches):
        res = g.match_batch(qs)
    el_b = (time.perf_counter() - t) / batches
    rows = [len(r) for r in res]
    for q in qs[:4]:
        g.match_query(q)
    lat = []
    for q in qs:
        a = time.perf_counter_ns()
        g.match_query(q)
        lat.append(time.perf_counter_ns() - a)
    lat_ms = np.asarray(lat, np.float64) / 1e6
    return {"queries": len(qs), "batched_qps": round(len(qs) / el_b, 1),
            "single_qps": round(len(qs) / (lat_ms.sum() / 1e3), 1),
            "single_p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
            "single_p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
            "rows_mean": round(float(np.mean(rows)), 1), "rows_max": int(max(rows))}


def bench_sweep(args, P, kggen):
    """Query-size and average-degree sweeps (thesis Ch. 3, Sec. "Comparison
    with state-of-the-art CPU algorithms": 6..14 query vertices at degree 16,
    degree 8..24 at 10 query vertices, 1M-vertex graphs) and graph-size
    scaling with the graph in device memory and in pinned host memory (Sec.
    "Scalability Test": 6-vertex queries). Stored queries, 64 per point."""
    pts = kggen.load_sweep()
    out = {"metric": "size / degree / graph-size sweeps", "unit": "queries/s",
           "n_gpus": 1, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "power-law KGs (64 types, 32 Zipf relations, out-degree "
                                  "<= V/32): 1M vertices at average degree 8-24; 0.1M-16M "
                                  "vertices at degree 5; one pinned vertex per query, other "
                                  "labels 'any' with p 0.5 (vertices) / 0.25 (edges), H <= 1e6 "
                                  "(kggen/fixtures/sweep.json)"},
           "degree": {}, "size": {}, "scale": {}}
    graphs = {}
    # grouped by graph so that each graph is drawn once
    for key, kind, param, n in sorted(kggen.sweep_points(), key=lambda p: (p[1], p[2])):
        t = time.time()
        gk = (kind, param)
        if gk not in graphs:
            graphs.clear()
            graphs[gk] = kggen.sweep_point_graph(kind, param)
        kg = graphs[gk]
        qs = pts[key]
        grp, val = key.split("/")
        if kind == "scale":
            rec = {"vertices": kg.V, "edges": kg.E}
            for hg in (0, 1):
                g = P.Graph.from_kg(kg, host_graph=hg)
                rec["host_memory" if hg else "device_memory"] = _point(P, g, qs)
                g.close()
            rec["host_over_device_batched"] = round(rec["host_memory"]["batched_qps"] /
                                                    rec["device_memory"]["batched_qps"], 3)
        else:
            g = P.Graph.from_kg(kg)
            rec = dict(_point(P, g, qs), vertices=kg.V, edges=kg.E, query_vertices=n)
            g.close()
        out[grp][val] = rec
        log(f"{key}: {json.dumps(rec)} ({time.time() - t:.1f}s)")
    return out


def _one_at_a_time(f, qs):
    for q in qs[:4]:
        f(q)
    lat = []
    for q in qs:
        a = time.perf_counter_ns()
        f(q)
        lat.append(time.perf_counter_ns() - a)
    lat_ms = np.asarray(lat, np.float64) / 1e6
    return {"queries_per_s": round(len(qs) / (lat_ms.sum() / 1e3), 1),
            "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
            "p99_ms": round(float(np.percentile(lat_ms, 99)), 3)}


def bench_compressed(args, P, kggen):
    """Multi-level compression (thesis Ch. 3, Sec. "Multi-level Graph
    Compression", Table 3.4) on graphs with similar vertices: the size of
    each level, and the same queries matched directly and through the
    weighted graph (expansion on the device), with the original graph in
    device memory and in host memory (the thesis' setting: the original
    graph in main memory, the compressed one on the GPU)."""
    out = {"metric": "multi-level compression: size per level and queries/s one at a time",
           "unit": "queries/s", "n_gpus": 1, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "twin graphs (kggen.twin_graph: power-law base, two rounds of "
                                  "twins keeping 90 % of the edges), 64 queries of 2-8 vertices "
                                  "(kggen.twin_queries; kggen/fixtures/twin_large.json), levels at "
                                  "delta 0.8 / 0.7 / 0.7"},
           "graphs": {}}
    for name in ("twin-medium", "twin-large"):
        t = time.time()
        kg = kggen.twin_named(name)
        # the large graph's queries are stored (drawing them takes ~30 s)
        qs = (kggen.load_twin_large() if name == "twin-large"
              else kggen.twin_queries(kg, 64, kggen.BASE_SEED + 930))
        log(f"{name}: {kg.V} vertices, {kg.E} edges, queries in {time.time() - t:.1f}s")
        t = time.perf_counter()
        comp = P.Compressed.from_kg(kg)
        t_comp = time.perf_counter() - t
        rec = {"vertices": kg.V, "edges": kg.E, "compress_s": round(t_comp, 2),
               "levels": comp.levels,
               "size_ratio_per_level": [round(x / comp.level_size[0], 4) for x in comp.level_size],
               "weighted_vertices": comp.n_vertices, "weighted_edges": comp.n_edges,
               "largest_mapping_list": int(np.diff(comp.map_off).max())}
        g = P.Graph.from_kg(kg)
        rows = [g.match_query(q, count_only=True) for q in qs]
        rec["rows_mean"] = round(float(np.mean(rows)), 1)
        rec["direct_device_graph"] = _one_at_a_time(lambda q: g.match_query(q), qs)
        cg = P.CompressedGraph(g, comp)
        wrows = [cg.match_weighted(q, count_only=True) for q in qs]
        rec["weighted_rows_mean"] = round(float(np.mean(wrows)), 1)
        rec["compressed_device_graph"] = _one_at_a_time(lambda q: cg.match_query(q), qs)
        cg.close()
        g.close()
        gh = P.Graph.from_kg(kg, host_graph=1)
        rec["direct_host_graph"] = _one_at_a_time(lambda q: gh.match_query(q), qs)
        cgh = P.CompressedGraph(gh, comp)
        rec["compressed_host_graph"] = _one_at_a_time(lambda q: cgh.match_query(q), qs)
        cgh.close()
        gh.close()
        comp.close()
        out["graphs"][name] = rec
        log(f"{name}: {json.dumps(rec)}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["medium", "large", "large-cyclic", "sweep", "compressed"],
                    default="large")
    ap.add_argument("--row-cap", type=int, default=250_000_000,
                    help="large-cyclic: row cap for materialized tables")
    ap.add_argument("--queries", type=int, default=100)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--serve-queries", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-rates", default="1000,5000,20000",
                    help="arrival rates (qps) of the medium served-form measurement")
    ap.add_argument("--serve-arrivals", type=int, default=2000)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form legs")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the cold-cache single-query leg")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the refinement / two-graph ablation legs")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (torch), the known-size "
                         "reference for HBM byte counters, and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe << 18  # int32 elements
        x = torch.ones(n, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the matcher "
              "has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import kggen
    import paper_1807_08804_amd as P
    run = {"medium": bench_medium, "large": bench_large, "large-cyclic": bench_large_cyclic,
           "sweep": bench_sweep, "compressed": bench_compressed}
    out = run[args.workload](args, P, kggen)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
