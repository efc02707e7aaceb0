"""Writes the stored query workloads of the large graph under
kggen/fixtures/. Drawing them takes minutes (every candidate query needs its
spanning-tree bound on the 20M-edge graph), so the bench and the tests read
the stored copies; each loader checks that its file was drawn from the same
recipe.

* large_cyclic.json: the 50 cyclic queries (8-16 vertices, 1-3 cycles, no
  pins, 10^7 <= H <= 2*10^9), ``large_queries`` with its default seed;
* large_batch.json: the 1,024-query mixed batch (3-16 vertices; paths,
  stars, trees, cyclic; 0-50% pinned; H <= 10^6), ``batch_queries``;
* large_serve.json: 512 served-stream queries (3-12 vertices, tree plus 0-1
  extra edge, 0-2 pins, H <= 10^6), ``serve_queries``;
* sweep.json: 64 queries per query-size / degree / graph-size point
  (``sweep_points``, ``sweep_queries``), each point drawn on its own graph
  in a worker process;
* twin_large.json: 64 queries of the large graph with similar vertices
  (``twin_queries`` on ``twin_named('twin-large')``).

    python -m kggen.make_fixtures [cyclic] [batch] [serve] [sweep] [twin]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import kggen  # noqa: E402


def _write(name, recipe, qs, rejected):
    path = os.path.join(HERE, "fixtures", name)
    doc = {"recipe": recipe, "rejected": rejected, "queries": [q.as_dict() for q in qs]}
    with open(path, "w") as f:
        json.dump(doc, f, separators=(",", ":"))


def _sweep_point(arg):
    k, (key, kind, param, n) = arg
    g = kggen.sweep_point_graph(kind, param)
    qs, rej = kggen.sweep_queries(g, n, kggen.SWEEP_COUNT, seed=kggen.BASE_SEED + 600 + k)
    return key, [q.as_dict() for q in qs], rej


def write_sweep(workers=6):
    import multiprocessing as mp
    pts = list(enumerate(kggen.sweep_points()))
    # the largest graphs first so that they overlap the rest
    pts.sort(key=lambda kp: -(kp[1][2] if kp[1][1] == "scale" else kp[1][2] * kggen.SWEEP_V // 5))
    with mp.get_context("spawn").Pool(workers) as pool:
        got = pool.map(_sweep_point, pts, chunksize=1)
    order = [key for key, *_ in kggen.sweep_points()]
    by = {key: (qs, rej) for key, qs, rej in got}
    doc = {"recipe": kggen.SWEEP_RECIPE, "rejected": {k: by[k][1] for k in order},
           "points": {k: by[k][0] for k in order}}
    with open(os.path.join(HERE, "fixtures", "sweep.json"), "w") as f:
        json.dump(doc, f, separators=(",", ":"))


def main(which):
    t = time.time()
    if "twin" in which:
        qs = kggen.twin_queries(kggen.twin_named("twin-large"), 64, seed=kggen.BASE_SEED + 930)
        _write("twin_large.json", kggen.TWIN_LARGE_RECIPE, qs, 0)
        print(f"twin_large: {len(qs)} queries at {time.time() - t:.0f}s")
        which = [w for w in which if w != "twin"]
        if not which:
            return
    if "sweep" in which:
        write_sweep()
        print(f"sweep: {len(kggen.sweep_points())} points at {time.time() - t:.0f}s")
        which = [w for w in which if w != "sweep"]
        if not which:
            return
    kg = kggen.named_graph("large")
    kg.ensure_in()
    if "cyclic" in which:
        qs, rej = kggen.large_queries(kg, 50)
        _write("large_cyclic.json", kggen.LARGE_CYCLIC_RECIPE, qs, rej)
        print(f"large_cyclic: {len(qs)} queries ({rej} rejected) at {time.time() - t:.0f}s")
    if "batch" in which:
        qs, rej = kggen.batch_queries(kg, 1024)
        _write("large_batch.json", kggen.LARGE_BATCH_RECIPE, qs, rej)
        print(f"large_batch: {len(qs)} queries ({rej} rejected) at {time.time() - t:.0f}s")
    if "serve" in which:
        qs, rej = kggen.serve_queries(kg, 512)
        _write("large_serve.json", kggen.LARGE_SERVE_RECIPE, qs, rej)
        print(f"large_serve: {len(qs)} queries ({rej} rejected) at {time.time() - t:.0f}s")


if __name__ == "__main__":
    main(sys.argv[1:] or ["cyclic", "batch", "serve", "sweep", "twin"])
