"""Writes the stored expected tables under tests/golden/ from the CPU oracle
(inputs from the seeded generator). Run: python tests/golden/make_golden.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import kggen  # noqa: E402
import oracle  # noqa: E402


def main():
    g = kggen.named_graph("tiny")
    q = kggen.tiny_query(g)
    rows = oracle.graph_from_kg(g).match_query(q)
    with open(os.path.join(HERE, "tiny_query.json"), "w") as f:
        json.dump({"source": "oracle/ on kggen tiny graph (2000 V, 8000 E, seed 180708804) "
                             "and kggen.tiny_query", "query": q.as_dict(),
                   "rows": rows.tolist()}, f, indent=1)


if __name__ == "__main__":
    main()
