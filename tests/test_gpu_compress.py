"""GpSense over a compressed graph (thesis Ch. 3, Sec. "Multi-level Graph
Compression" and Sec. "GpSense Framework"): queries matched on the weighted
graph and expanded on the device through the mapping lists give exactly the
oracle's tables on the original graph, with the original graph in device or
in host memory."""
import sys

import numpy as np
import pytest

import kggen
import oracle
import paper_1807_08804_amd as P
from tests.micro import random_graph, random_query

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(got, want, what):
    assert isinstance(got, np.ndarray), (what, got)
    assert got.shape == want.shape and np.array_equal(got, want), what


@pytest.fixture(scope="module")
def small_case():
    kg = kggen.twin_named("twin-small")
    qs = kggen.twin_queries(kg, 40, kggen.BASE_SEED + 910)
    og = oracle.graph_from_kg(kg)
    return kg, qs, [og.match_query(q) for q in qs]


PATHS = [P.SGM_PATH_AUTO, P.SGM_PATH_WIDE, P.SGM_PATH_NARROW]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("host_graph", [0, 1])
def test_compressed_small(small_case, host_graph, path):
    """40 queries on the small graph with similar vertices (three levels of
    compression), full tables and counts, against the oracle, with the
    weighted graph matched on each execution path."""
    kg, qs, want = small_case
    comp = P.Compressed.from_kg(kg)
    g = P.Graph.from_kg(kg, host_graph=host_graph)
    cg = P.CompressedGraph(g, comp, path=path)
    say(f"case: compressed twin-small host_graph={host_graph} path={path} levels={comp.levels} "
        f"|Vw|={comp.n_vertices}")
    for i, (q, w) in enumerate(zip(qs, want)):
        same(cg.match_query(q), w, i)
        assert cg.match_query(q, count_only=True) == len(w)
    cg.close()
    g.close()


def test_weighted_matches_cover_the_original(small_case):
    """Thm. 3.2 on the device's own weighted matches: every oracle match,
    read through the mapping lists, is among the weighted graph's matches."""
    kg, qs, want = small_case
    comp = P.Compressed.from_kg(kg)
    g = P.Graph.from_kg(kg)
    cg = P.CompressedGraph(g, comp)
    for i, (q, w) in enumerate(zip(qs, want)):
        wm = cg.match_weighted(q)
        have = set(map(tuple, wm.tolist()))
        for row in w.tolist():
            assert tuple(int(comp.hyper_of[x]) for x in row) in have, i
    cg.close()
    g.close()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(8))
def test_compressed_micro(seed, path):
    """Micro graphs (repeated triples, self-loops, two types) compressed at
    a low threshold, queries with "any" labels and pins, against the oracle
    (weighted matches with self-loops and repeated weighted vertices)."""
    rng = np.random.default_rng(1400 + seed)
    V = int(rng.integers(3, 50))
    mg = random_graph(rng, V, int(rng.integers(V, 5 * V)), n_types=2, n_rels=2)
    rp, col, rel, typ = mg.csr()
    og = oracle.Graph(V, mg.src, mg.dst, mg.rel, mg.vtype)
    comp = P.Compressed(rp, col, rel, typ, max_levels=4, delta=0.3)
    g = P.Graph(rp, col, rel, typ)
    cg = P.CompressedGraph(g, comp, path=path)
    say(f"case: compressed micro seed={seed} path={path} V={V} |Vw|={comp.n_vertices}")
    for _ in range(12):
        q = random_query(rng, int(rng.integers(1, 6)), 2, 2, V, p_pin=0.15, extra=3)
        want = og.match_query(q)
        try:
            same(cg.match_query(q), want, q)
        except P.SGMError as e:
            # the persistent path alone refuses what fits no slot
            assert path == P.SGM_PATH_NARROW and e.code == P.SGM_EUNSUPPORTED
    cg.close()
    g.close()


def test_compressed_medium():
    """The medium graph with similar vertices (676K vertices, 5.8M edges;
    three levels leave 29 %), 24 queries, original graph in host memory as
    in the thesis' setting, against the oracle."""
    kg = kggen.twin_named("twin-medium")
    qs = kggen.twin_queries(kg, 24, kggen.BASE_SEED + 920)
    og = oracle.graph_from_kg(kg)
    want = [og.match_query(q) for q in qs]
    comp = P.Compressed.from_kg(kg)
    g = P.Graph.from_kg(kg, host_graph=1)
    cg = P.CompressedGraph(g, comp)
    say(f"case: compressed twin-medium |Vw|={comp.n_vertices}")
    for i, (q, w) in enumerate(zip(qs, want)):
        same(cg.match_query(q), w, i)
    cg.close()
    g.close()


def test_compressed_large_bench_workload():
    """The compressed-graph bench workload at its full size: the large
    graph with similar vertices (4.5M vertices, 36.9M edges) compressed in
    three levels, its 64 stored queries matched through the weighted graph
    with the original graph in host memory, against the oracle."""
    kg = kggen.twin_named("twin-large")
    qs = kggen.load_twin_large()
    og = oracle.graph_from_kg(kg)
    want = [og.match_query(q) for q in qs]
    comp = P.Compressed.from_kg(kg)
    g = P.Graph.from_kg(kg, host_graph=1)
    cg = P.CompressedGraph(g, comp)
    say(f"case: compressed twin-large |Vw|={comp.n_vertices} levels={comp.levels}")
    for i, (q, w) in enumerate(zip(qs, want)):
        same(cg.match_query(q), w, i)
    cg.close()
    g.close()
    comp.close()


def test_compressed_entry_points_checked(small_case):
    kg, qs, _ = small_case
    comp = P.Compressed.from_kg(kg)
    g = P.Graph.from_kg(kg)
    # no outgoing-graph-only form of a compressed graph
    with pytest.raises(P.SGMError) as e:
        P.CompressedGraph(g, comp, out_only=1, path=P.SGM_PATH_WIDE)
    assert e.value.code == P.SGM_EINVAL
    # a mapping made from a graph of another size
    tiny = P.Compressed(np.array([0, 1, 1], np.int32), np.array([1], np.int32),
                        np.array([0], np.int32), np.array([0, 0], np.int32))
    with pytest.raises(P.SGMError) as e:
        P.CompressedGraph(g, tiny)
    assert e.value.code == P.SGM_EINVAL
    g.close()
