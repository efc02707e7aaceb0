"""Writes kggen/fixtures/large_cyclic.json: the 50 cyclic queries of the
large-graph workload (8-16 vertices, 1-3 cycles, no pins, 10^7 <= H <= 2*10^9),
drawn by ``large_queries`` on ``named_graph("large")`` with its default seed.
Drawing them takes minutes (every candidate needs its tree bound on the
20M-edge graph), so the bench and the tests read the stored copy;
``load_large_cyclic`` checks that the file was drawn from the same recipe.

    python -m kggen.make_fixtures
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import kggen  # noqa: E402

PATH = os.path.join(HERE, "fixtures", "large_cyclic.json")


def main():
    t = time.time()
    kg = kggen.named_graph("large")
    kg.ensure_in()
    qs, rejected = kggen.large_queries(kg, 50)
    doc = {"recipe": kggen.LARGE_CYCLIC_RECIPE, "rejected": rejected,
           "queries": [q.as_dict() for q in qs]}
    with open(PATH, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {len(qs)} queries ({rejected} rejected) in {time.time() - t:.0f}s")


if __name__ == "__main__":
    main()
