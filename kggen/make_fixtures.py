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
  extra edge, 0-2 pins, H <= 10^6), ``serve_queries``.

    python -m kggen.make_fixtures [cyclic] [batch] [serve]
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


def main(which):
    t = time.time()
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
    main(sys.argv[1:] or ["cyclic", "batch", "serve"])
