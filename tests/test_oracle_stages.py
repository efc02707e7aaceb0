"""Pins of the stage oracles (query plan, filtering phase, candidate-edge
counts) and agreement of the library's host planner with the oracle's.

The hand-worked cases below apply the thesis' rules (Ch. 3, Sec. "Query Plan
Generation", Alg. 3.2, Sec. "Candidate Nodes Refinement", Sec. "Joining
Phase") step by step; every expected set is derived in the comments.
"""
import numpy as np
import pytest

import oracle
import paper_1807_08804_amd as P
from tests.micro import MicroGraph, MicroQuery, brute_force, random_graph, random_query


def og_of(g: MicroGraph):
    return oracle.Graph(g.V, g.src, g.dst, g.rel, g.vtype)


def sets(cand):
    return [set(np.nonzero(c)[0].tolist()) for c in cand]


def test_hand_path_explore_push():
    # data: 0->1, 0->2, 1->3, 2->4, 5->3 (relation 0), 6 vertices, one type
    g = og_of(MicroGraph(6, [0, 0, 1, 2, 5], [1, 2, 3, 4, 3], [0] * 5, [0] * 6))
    # query a->b->c, any types, relation 0 on both edges
    q = MicroQuery(3, [-1] * 3, [-1] * 3, [0, 1], [1, 2], [0, 0])
    # f = deg/6: f0 = 1/6, f1 = 2/6, f2 = 1/6; both edges sum to 3/6 -> edge 0;
    # its endpoint of larger f is 1 -> root 1; expanding 1 reaches 0 and 2
    p = g.plan(q)
    assert p["visit_order"] == [1] and p["init_order"] == [1, 0, 2]
    assert p["parent"] == [1, -1, 1] and p["parent_edge"] == [0, -1, 1]
    # kernel_check(1): out >= 1 and in >= 1 -> {1, 2}; explore keeps both
    # (in-neighbour 0 has an out-edge; out-neighbours 3, 4 have in-edges);
    # pushes: C(0) = in-neighbours {0}, C(2) = out-neighbours {3, 4};
    # refinement skips degree-1 vertices and vertex 1 has no other edges
    for rounds in (0, 1, -1):
        assert sets(g.filter(q, rounds=rounds)) == [{0}, {1, 2}, {3, 4}]
    cand = g.filter(q)
    assert g.edge_candidates(q, cand).tolist() == [2, 2]
    assert g.match_query(q).tolist() == [[0, 1, 3], [0, 2, 4]]


def test_hand_plan_concept_node_first():
    # concept nodes 0, 1 (degree 2, adjacent) and 4 (degree 3): the
    # commonsense rule of Sec. "GpSense" starts at the concept node of
    # maximum degree, 4 (the edge rule would take edge (0, 1): f sum 2 + 2);
    # expanding 4 reaches 2, 3, 5; 2 and 3 each have one unreached neighbour
    # and equal f (2/13): 2 (lower id) reaches 0; then 3 and 0 each have one
    # (vertex 1), and the concept node 0 has the larger f (2/1): 0 reaches 1
    g = og_of(MicroGraph(13, [0], [1], [0], [0] * 13))
    q = MicroQuery(6, [-1] * 6, [10, 11, -1, -1, 12, -1], [0, 0, 1, 4, 4, 4],
                   [1, 2, 3, 2, 3, 5], [-1] * 6)
    p = g.plan(q)
    assert p["visit_order"] == [4, 2, 0]
    assert p["init_order"] == [4, 2, 3, 5, 0, 1]
    assert p["parent"] == [2, 0, 4, 4, -1, 4]


def test_hand_prune_by_relation():
    # 0->1 r0, 1->3 r1, 0->2 r0, 2->4 r0; query a -r0-> b -r1-> c
    g = og_of(MicroGraph(5, [0, 1, 0, 2], [1, 3, 2, 4], [0, 1, 0, 0], [0] * 5))
    q = MicroQuery(3, [-1] * 3, [-1] * 3, [0, 1], [1, 2], [0, 1])
    # root 1 again; candidate 2 has no r1 out-edge -> pruned by explore
    assert sets(g.filter(q)) == [{0}, {1}, {3}]
    assert g.edge_candidates(q, g.filter(q)).tolist() == [1, 1]


def test_hand_parent_intersection_and_refinement():
    # data (8 vertices, one type): 0->1 r0, 1->2 r0, 2->3 r1, 5->6 r0, 6->7 r0,
    # 7->5 r0; query a -r0-> b -r0-> c -r1-> d, any types
    g = og_of(MicroGraph(8, [0, 1, 2, 5, 6, 7], [1, 2, 3, 6, 7, 5], [0, 0, 1, 0, 0, 0], [0] * 8))
    q = MicroQuery(4, [-1] * 4, [-1] * 4, [0, 1, 2], [1, 2, 3], [0, 0, 1])
    # f = deg/8 = (1, 2, 2, 1)/8: edge 1 has the largest sum; f1 = f2 -> root
    # 1 (lower id); expand 1 -> {0, 2}; then 2 (one unreached neighbour) -> 3
    p = g.plan(q)
    assert p["visit_order"] == [1, 2] and p["init_order"] == [1, 0, 2, 3]
    # kernel_check(1): out >= 1, in >= 1 -> {1, 2, 5, 6, 7}
    # explore(1): 2 has no r0 out-edge -> pruned; C(1) = {1, 5, 6, 7};
    #   push C(0) = r0 in-neighbours {0, 7, 5, 6}, C(2) = r0 out-neighbours
    #   passing out >= 1, in >= 1: {2, 6, 7, 5}
    # explore(2): parent 1 tested on its set, child 3 on in >= 1; 5, 6, 7
    #   have no r1 out-edge -> C(2) = {2}; C(3) = {3}; the parent is
    #   intersected with the r0 in-neighbours of {2}: C(1) = {1}
    # refinement (vertices of degree > 1, reversed: 2 then 1) removes nothing
    for rounds in (0, 1, -1):
        assert sets(g.filter(q, rounds=rounds)) == [{0, 5, 6, 7}, {1}, {2}, {3}]
    # with threshold 0 every vertex is refined (order 3, 2, 0, 1): 5, 6, 7
    # have no r0 out-neighbour in C(1) = {1} -> C(0) = {0}
    assert sets(g.filter(q, low_conn=0)) == [{0}, {1}, {2}, {3}]
    # forward order (1, 2 for threshold 1) gives the same sets here
    assert sets(g.filter(q, reversed=0)) == [{0, 5, 6, 7}, {1}, {2}, {3}]
    assert g.edge_candidates(q, g.filter(q)).tolist() == [1, 1, 1]
    assert g.match_query(q).tolist() == [[0, 1, 2, 3]]


def test_pinned_vertex_first_and_complete_graph():
    m = 5
    src, dst = zip(*[(i, j) for i in range(m) for j in range(m) if i != j])
    g = og_of(MicroGraph(m, src, dst, [0] * len(src), [0] * m))
    q = MicroQuery(3, [-1] * 3, [-1, 4, -1], [0, 1], [1, 2], [-1, -1])
    # the pinned vertex has frequency 1: f1 = 2 dominates -> root 1
    assert g.plan(q)["visit_order"] == [1]
    # C(1) = {4}; explore pushes its in- and out-neighbours {0, 1, 2, 3}
    # (no self-loops); refinement skips both degree-1 neighbours
    assert sets(g.filter(q)) == [{0, 1, 2, 3}, {4}, {0, 1, 2, 3}]
    # candidate edges: (x, 4) for the first edge, (4, y) for the second
    assert g.edge_candidates(q, g.filter(q)).tolist() == [4, 4]


@pytest.mark.parametrize("seed", range(30))
def test_filter_is_sound_and_monotone(seed):
    """Every match survives every filter stage (filtering only drops
    vertices that cannot be matched); refinement only removes candidates;
    edge counts bound the matches' projections."""
    rng = np.random.default_rng(2000 + seed)
    V = int(rng.integers(3, 9))
    mg = random_graph(rng, V, int(rng.integers(V, 3 * V)), n_types=2, n_rels=2)
    g = og_of(mg)
    for _ in range(5):
        q = random_query(rng, int(rng.integers(1, 5)), 2, 2, V, p_pin=0.15)
        rows = brute_force(mg, q)
        c0 = g.filter(q, rounds=0)
        c1 = g.filter(q, rounds=1)
        cf = g.filter(q, rounds=-1)
        c_all = g.filter(q, rounds=-1, low_conn=0)
        assert np.all(c1 <= c0) and np.all(cf <= c1) and np.all(c_all <= cf)
        for f in rows:
            for u in range(q.n):
                assert c_all[u, f[u]], (q, f, u)
        if q.m:
            ec = g.edge_candidates(q, c1)
            for e in range(q.m):
                a, b = int(q.esrc[e]), int(q.edst[e])
                assert ec[e] >= len({(f[a], f[b]) for f in rows})


@pytest.mark.parametrize("seed", range(40))
def test_library_plan_matches_oracle_plan(seed):
    rng = np.random.default_rng(3000 + seed)
    V = int(rng.integers(4, 12))
    mg = random_graph(rng, V, 3 * V, n_types=3, n_rels=2)
    g = og_of(mg)
    tf = np.bincount(mg.vtype, minlength=3)
    for _ in range(5):
        q = random_query(rng, int(rng.integers(1, 12)), 3, 2, V, p_pin=0.2, extra=4)
        want = g.plan(q)
        got = P.sgm_plan_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel, V, tf)
        assert got == want, (q, got, want)
