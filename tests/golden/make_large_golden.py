"""Writes tests/golden/large_golden.json: for every query of the large-graph
workloads, the number of embeddings and the SHA-256 of the sorted int32 row
table, both computed by the CPU oracle (oracle/) alone. Inputs come from the
seeded generator (kggen) and its stored query fixtures; nothing here touches
the GPU library.

Workloads (all on named_graph("large"), 4M vertices / 20M edges):
* batch:  the 1,024-query mixed batch (kggen.load_large_batch);
* serve:  the 512 served-stream queries (kggen.load_large_serve);
* cyclic: the 50 cyclic unpinned queries (kggen.load_large_cyclic).

Each query runs under a budget of candidate tests (``--budget``, per
workload); a query whose table would exceed ``--row-cap`` rows is counted
without materialising its rows (count only, no hash). Queries that hit the
budget are recorded as unfinished: their GPU tables stay parity-unpinned
against the oracle. ``--retry-unfinished --retry-budget B`` runs those
entries again under a larger budget B, which the entry then records. The file is rewritten after every query, and a rerun
keeps the entries already computed with the same budgets.

    python tests/golden/make_large_golden.py [batch] [serve] [cyclic]
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import kggen  # noqa: E402
import oracle  # noqa: E402

PATH = os.path.join(HERE, "large_golden.json")


def table_sha256(rows: np.ndarray) -> str:
    """SHA-256 of a row table as C-ordered little-endian int32 bytes."""
    return hashlib.sha256(np.ascontiguousarray(rows, dtype="<i4").tobytes()).hexdigest()


def graph_sha256(kg) -> str:
    h = hashlib.sha256()
    for a in (kg.row_ptr, kg.col, kg.rel, kg.vtype):
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def workloads():
    return {
        "batch": (kggen.LARGE_BATCH_RECIPE, lambda: kggen.load_large_batch()[0]),
        "serve": (kggen.LARGE_SERVE_RECIPE, lambda: kggen.load_large_serve()[0]),
        "cyclic": (kggen.LARGE_CYCLIC_RECIPE, kggen.load_large_cyclic),
    }


def one(og, q, budget, row_cap):
    """(entry dict, seconds) for one query."""
    t = time.perf_counter()
    try:
        rows = og.match_query(q, max_steps=budget, max_rows=row_cap)
        e = {"count": int(len(rows)), "sha256": table_sha256(rows)}
    except oracle.OracleError as err:
        if err.code == oracle.OR_EBUDGET:
            e = {"unfinished": "budget"}
        elif err.code == oracle.OR_ETOOBIG:
            try:
                e = {"count": int(og.match_query(q, max_steps=budget, count_only=True)),
                     "sha256": None}
            except oracle.OracleError as err2:
                if err2.code != oracle.OR_EBUDGET:
                    raise
                e = {"unfinished": "budget"}
        else:
            raise
    return e, time.perf_counter() - t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["batch", "serve", "cyclic"])
    ap.add_argument("--budget", type=float, default=2e11,
                    help="candidate tests per query (batch and serve)")
    ap.add_argument("--cyclic-budget", type=float, default=1e9,
                    help="candidate tests per query (cyclic)")
    ap.add_argument("--row-cap", type=int, default=100_000_000,
                    help="largest table materialised and hashed")
    ap.add_argument("--retry-unfinished", action="store_true",
                    help="compute again the entries recorded as unfinished")
    ap.add_argument("--retry-budget", type=float, default=0,
                    help="candidate tests per query for the retried entries (default: the "
                         "workload's budget); the entry records the budget it ran under")
    args = ap.parse_args()
    doc = {}
    if os.path.exists(PATH):
        with open(PATH) as f:
            doc = json.load(f)
    kg = kggen.named_graph("large")
    gsha = graph_sha256(kg)
    if doc.get("graph_sha256") != gsha:
        doc = {}
    doc.update({"source": "oracle/ (CPU backtracking enumerator) on kggen named_graph('large'); "
                          "written by tests/golden/make_large_golden.py",
                "graph": "named_graph('large'): 4,000,000 vertices, 20,000,000 edges",
                "graph_sha256": gsha,
                "table_hash": "sha256 of the sorted [rows][n] table as little-endian int32"})
    og = oracle.graph_from_kg(kg)
    for name in args.which:
        recipe, load = workloads()[name]
        budget = int(args.cyclic_budget if name == "cyclic" else args.budget)
        qs = load()
        sec = doc.get(name, {})
        if sec.get("recipe") != recipe or sec.get("budget") != budget or \
                sec.get("row_cap") != args.row_cap:
            sec = {"recipe": recipe, "budget": budget, "row_cap": args.row_cap, "entries": {}}
        doc[name] = sec
        t0 = time.time()
        for i, q in enumerate(qs):
            e = sec["entries"].get(str(i))
            if e is not None and not (args.retry_unfinished and "unfinished" in e):
                continue
            retry = e is not None and args.retry_budget > 0
            eb = int(args.retry_budget) if retry else budget
            e, el = one(og, q, eb, args.row_cap)
            e["oracle_s"] = round(el, 3)
            if eb != budget:
                e["budget"] = eb
            sec["entries"][str(i)] = e
            print(f"{name} {i}: {e}", flush=True)
            tmp = PATH + ".tmp"
            with open(tmp, "w") as f:
                json.dump(doc, f, indent=0, sort_keys=True)
            os.replace(tmp, PATH)
        done = sum("count" in e for e in sec["entries"].values())
        print(f"{name}: {done} of {len(qs)} finished in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
