"""Pins of the CPU oracle against facts that do not come from the oracle:
brute-force enumeration, closed-form counts, networkx's monomorphism matcher,
sparse-matrix identities on the generated graphs, and a stored golden table.
"""
import json
import math
import os

import numpy as np
import pytest

import kggen
import oracle
from tests.micro import MicroGraph, MicroQuery, brute_force, random_graph, random_query

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def og_of(g: MicroGraph):
    return oracle.Graph(g.V, g.src, g.dst, g.rel, g.vtype)


def rows_of(a):
    return [tuple(int(x) for x in r) for r in a]


# --------------------------------------------------------------------------
# P1: brute force on micro graphs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_micro(seed):
    rng = np.random.default_rng(1000 + seed)
    V = int(rng.integers(3, 8))
    g = random_graph(rng, V, int(rng.integers(V, 3 * V)), n_types=2, n_rels=2)
    og = og_of(g)
    for _ in range(6):
        n = int(rng.integers(1, 5))
        q = random_query(rng, n, 2, 2, V)
        want = brute_force(g, q)
        got = rows_of(og.match_query(q, nthreads=2))
        assert got == want, (q, got, want)


def test_bruteforce_hypothesis():
    hyp = pytest.importorskip("hypothesis")
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=150, deadline=None, derandomize=True)
    @given(st.integers(0, 2**31 - 1), st.integers(2, 7), st.integers(1, 4))
    def check(seed, V, n):
        rng = np.random.default_rng(seed)
        g = random_graph(rng, V, int(rng.integers(1, 3 * V)), n_types=3, n_rels=3)
        q = random_query(rng, n, 3, 3, V, p_pin=0.25)
        assert rows_of(og_of(g).match_query(q)) == brute_force(g, q)

    check()


def test_rows_sorted_unique_and_satisfy_definition():
    rng = np.random.default_rng(7)
    g = random_graph(rng, 12, 60, n_types=2, n_rels=2)
    og = og_of(g)
    E = g.edge_set()
    for _ in range(30):
        q = random_query(rng, int(rng.integers(2, 5)), 2, 2, 12)
        rows = rows_of(og.match_query(q))
        assert rows == sorted(set(rows))
        for f in rows:
            assert len(set(f)) == q.n
            for a, b, r in zip(q.esrc, q.edst, q.elabel):
                assert any(s == f[a] and d == f[b] and (r < 0 or rr == r) for s, d, rr in E)


# --------------------------------------------------------------------------
# P2: closed forms
# --------------------------------------------------------------------------

def complete_digraph(m):
    src, dst = zip(*[(i, j) for i in range(m) for j in range(m) if i != j])
    return MicroGraph(m, src, dst, [0] * len(src), [0] * m)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_complete_digraph_counts(k):
    m = 6
    g = complete_digraph(m)
    og = og_of(g)
    rng = np.random.default_rng(k)
    for _ in range(5):
        q = random_query(rng, k, 1, 1, m, p_pin=0.0, extra=3)
        # every query vertex/edge label 0 or -1 matches: m!/(m-k)!
        assert og.match_query(q, count_only=True) == math.perm(m, k)


@pytest.mark.parametrize("m", [5, 7, 9])
def test_directed_cycle_counts(m):
    src = list(range(m))
    dst = [(i + 1) % m for i in range(m)]
    g = og_of(MicroGraph(m, src, dst, [0] * m, [0] * m))
    for k in range(2, m):
        path = MicroQuery(k, [-1] * k, [-1] * k, list(range(k - 1)), list(range(1, k)), [0] * (k - 1))
        assert g.match_query(path, count_only=True) == m
    for k in range(3, m + 1):
        cyc = MicroQuery(k, [-1] * k, [-1] * k, list(range(k)), [(i + 1) % k for i in range(k)],
                         [-1] * k)
        assert g.match_query(cyc, count_only=True) == (m if k == m else 0)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_out_star_counts(k):
    d = 6
    g = og_of(MicroGraph(d + 1, [0] * d, list(range(1, d + 1)), [1] * d, [0] * (d + 1)))
    star = MicroQuery(k + 1, [-1] * (k + 1), [-1] * (k + 1), [0] * k, list(range(1, k + 1)), [1] * k)
    assert g.match_query(star, count_only=True) == math.perm(d, k)
    pinned = MicroQuery(k + 1, [-1] * (k + 1), [0] + [-1] * k, [0] * k, list(range(1, k + 1)), [-1] * k)
    assert g.match_query(pinned, count_only=True) == math.perm(d, k)
    wrong_pin = MicroQuery(k + 1, [-1] * (k + 1), [3] + [-1] * k, [0] * k, list(range(1, k + 1)),
                           [-1] * k)
    assert g.match_query(wrong_pin, count_only=True) == 0
    wrong_rel = MicroQuery(2, [-1, -1], [-1, -1], [0], [1], [0])
    assert g.match_query(wrong_rel, count_only=True) == 0


@pytest.mark.parametrize("pin", [True, False])
def test_hub_row_with_repeated_destinations(pin):
    """A hub with 5,000 out-neighbours, all but one reached by two relations,
    so its row (9,999 entries) is longer than the oracle's work pieces and runs of
    one destination cross piece boundaries: a one-edge variable query from
    the hub has exactly one row per neighbour (out-star, k = 1), and a
    two-leaf query with one leaf typed d!/(d-2)! restricted as counted."""
    d = 5000
    # neighbour 1 by one relation, the others by two: runs start at odd entries
    dst = [1] + [2 + i // 2 for i in range(2 * (d - 1))]
    rel = [1] + [i % 2 for i in range(2 * (d - 1))]
    src = [0] * len(dst)
    vtype = [1] + [0] * d
    vtype[7] = 2
    g = og_of(MicroGraph(d + 1, src, dst, rel, vtype))
    vpin = [0, -1] if pin else [-1, -1]
    vlab = [-1, -1] if pin else [1, -1]
    rows = g.match_query(MicroQuery(2, vlab, vpin, [0], [1], [-1]))
    assert rows.tolist() == [[0, x] for x in range(1, d + 1)]
    assert g.match_query(MicroQuery(2, vlab, vpin, [0], [1], [1]), count_only=True) == d
    # centre, a typed-2 leaf (vertex 7 only) and any other leaf
    q3 = MicroQuery(3, vlab + [2], vpin + [-1], [0, 0], [1, 2], [-1, -1])
    assert g.match_query(q3, count_only=True) == d - 1


def test_disjoint_labels_zero():
    g = complete_digraph(5)
    og = og_of(g)
    q = MicroQuery(2, [0, 7], [-1, -1], [0], [1], [-1])
    assert og.match_query(q, count_only=True) == 0


# --------------------------------------------------------------------------
# P3: networkx monomorphisms on small simple digraphs
# --------------------------------------------------------------------------

def test_networkx_monomorphisms():
    nx = pytest.importorskip("networkx")
    from networkx.algorithms import isomorphism as iso

    rng = np.random.default_rng(42)
    for trial in range(25):
        V = int(rng.integers(8, 40))
        E = int(rng.integers(V, 4 * V))
        g = random_graph(rng, V, E, n_types=3, n_rels=2, self_loops=False)
        G = nx.DiGraph()
        for v in range(V):
            G.add_node(v, t=int(g.vtype[v]), vid=v)
        for s, d, r in g.edge_set():
            if G.has_edge(s, d):
                G[s][d]["rels"].add(r)
            else:
                G.add_edge(s, d, rels={r})
        og = og_of(g)
        for _ in range(4):
            q = random_query(rng, int(rng.integers(2, 5)), 3, 2, V, p_pin=0.1)
            Q = nx.DiGraph()
            for u in range(q.n):
                Q.add_node(u, t=int(q.vlabel[u]), pin=int(q.vpin[u]))
            # a simple digraph cannot hold two query edges on one ordered
            # pair: fold their relation constraints into one set
            for a, b, r in zip(q.esrc.tolist(), q.edst.tolist(), q.elabel.tolist()):
                if Q.has_edge(a, b):
                    Q[a][b]["need"].append(r)
                else:
                    Q.add_edge(a, b, need=[r])

            def node_match(gn, qn):
                return (qn["t"] < 0 or qn["t"] == gn["t"]) and (qn["pin"] < 0 or qn["pin"] == gn["vid"])

            def edge_match(ge, qe):
                return all(r < 0 or r in ge["rels"] for r in qe["need"])

            gm = iso.DiGraphMatcher(G, Q, node_match=node_match, edge_match=edge_match)
            want = sorted(tuple(inv[u] for u in range(q.n)) for inv in
                          ({v: k for k, v in mp.items()} for mp in gm.subgraph_monomorphisms_iter()))
            assert rows_of(og.match_query(q)) == want, (trial, q)


# --------------------------------------------------------------------------
# P6: sparse-matrix identities on the medium generated graph
# --------------------------------------------------------------------------

def _adj(kg, mask_rel=None, V=None):
    import scipy.sparse as sp
    src = kg.src()
    keep = np.ones(len(src), bool) if mask_rel is None else (kg.rel == mask_rel)
    return sp.csr_matrix((np.ones(int(keep.sum()), np.int64), (src[keep], kg.col[keep])),
                         shape=(kg.V, kg.V))


def q_of(n, edges, vlabel=None, vpin=None):
    vlabel = [-1] * n if vlabel is None else vlabel
    vpin = [-1] * n if vpin is None else vpin
    return MicroQuery(n, vlabel, vpin, [e[0] for e in edges], [e[1] for e in edges],
                      [e[2] for e in edges])


def test_sparse_identities_medium(medium_kg, oracle_medium):
    import scipy.sparse as sp
    kg, og = medium_kg, oracle_medium
    A = _adj(kg)
    A2 = A @ A
    # one labelled edge
    for r in (0, 5, 31):
        assert og.match_query(q_of(2, [(0, 1, r)]), count_only=True) == int((kg.rel == r).sum())
    assert og.match_query(q_of(2, [(0, 1, -1)]), count_only=True) == kg.E
    # 2-cycle
    assert og.match_query(q_of(2, [(0, 1, -1), (1, 0, -1)]), count_only=True) == \
        int(A.multiply(A.T).sum())
    # 2-path a->b->c with a != c
    assert og.match_query(q_of(3, [(0, 1, -1), (1, 2, -1)]), count_only=True) == \
        int(A2.sum() - A2.diagonal().sum())
    # directed 3-cycle
    assert og.match_query(q_of(3, [(0, 1, -1), (1, 2, -1), (2, 0, -1)]), count_only=True) == \
        int((A2 @ A).diagonal().sum())
    # transitive triangle
    assert og.match_query(q_of(3, [(0, 1, -1), (1, 2, -1), (0, 2, -1)]), count_only=True) == \
        int(A2.multiply(A).sum())
    # typed out-star with 2 leaves of type t: sum_v d_t(v) (d_t(v) - 1)
    t = 5
    At = A @ sp.diags((kg.vtype == t).astype(np.int64))
    dt = np.asarray(At.sum(axis=1)).ravel()
    star = q_of(3, [(0, 1, -1), (0, 2, -1)], vlabel=[-1, t, t])
    assert og.match_query(star, count_only=True) == int((dt * (dt - 1)).sum())
    # labelled 2-path with types on every vertex and one relation
    t0, t1, t2, r = 3, 7, 11, 0
    D = lambda tt: sp.diags((kg.vtype == tt).astype(np.int64))
    Ar = _adj(kg, mask_rel=r)
    M = D(t0) @ Ar @ D(t1) @ A @ D(t2)
    path = q_of(3, [(0, 1, r), (1, 2, -1)], vlabel=[t0, t1, t2])
    expect = int(M.sum() - (M.diagonal().sum() if t0 == t2 else 0))
    assert og.match_query(path, count_only=True) == expect


# --------------------------------------------------------------------------
# walk queries contain their own walk; golden table
# --------------------------------------------------------------------------

def test_walk_query_contains_walk(medium_kg, oracle_medium):
    qs, _ = kggen.medium_queries(medium_kg, 12)
    for q in qs:
        rows = oracle_medium.match_query(q)
        assert len(rows) >= 1
        assert tuple(q.walk.tolist()) in set(rows_of(rows))


def test_golden_tiny(tiny_kg, oracle_tiny):
    with open(os.path.join(GOLDEN, "tiny_query.json")) as f:
        gold = json.load(f)
    q = kggen.Query.from_dict(gold["query"])
    assert rows_of(oracle_tiny.match_query(q)) == [tuple(r) for r in gold["rows"]]
    assert q.as_dict()["esrc"] == kggen.tiny_query(tiny_kg).as_dict()["esrc"]


def test_oracle_rejects_bad_queries(oracle_tiny):
    with pytest.raises(oracle.OracleError):
        oracle_tiny.match(2, [-1, -1], [-1, -1], [0], [0], [-1])  # self-loop
    with pytest.raises(oracle.OracleError):
        oracle_tiny.match(3, [-1] * 3, [-1] * 3, [0], [1], [-1])  # disconnected
    with pytest.raises(oracle.OracleError) as e:
        oracle_tiny.match(2, [-1, -1], [-1, -1], [0], [1], [-1], max_rows=10)
    assert e.value.code == oracle.OR_ETOOBIG


# --------------------------------------------------------------------------
# P4: metamorphic invariants (the definition is invariant under renaming)
# --------------------------------------------------------------------------

def _permuted_graph(g: MicroGraph, perm):
    """Data vertex v becomes perm[v]."""
    vtype = np.empty_like(g.vtype)
    vtype[perm] = g.vtype
    return MicroGraph(g.V, perm[g.src], perm[g.dst], g.rel, vtype)


@pytest.mark.parametrize("seed", range(12))
def test_vertex_renaming_permutes_rows(seed):
    """Renaming data vertices renames the values of every row; renumbering
    query vertices permutes the columns. Rows are then re-sorted."""
    rng = np.random.default_rng(5000 + seed)
    V = int(rng.integers(4, 10))
    g = random_graph(rng, V, 3 * V, n_types=2, n_rels=2)
    perm = rng.permutation(V).astype(np.int32)
    gp = _permuted_graph(g, perm)
    og, ogp = og_of(g), og_of(gp)
    for _ in range(4):
        q = random_query(rng, int(rng.integers(2, 5)), 2, 2, V, p_pin=0.2)
        base = og.match_query(q)
        # data renaming: pins follow the renaming
        qp = MicroQuery(q.n, q.vlabel, np.where(q.vpin >= 0, perm[np.maximum(q.vpin, 0)], -1),
                        q.esrc, q.edst, q.elabel)
        got = ogp.match_query(qp)
        want = np.array(sorted(tuple(int(perm[x]) for x in r) for r in base), np.int32)
        assert np.array_equal(got.reshape(-1, q.n), want.reshape(-1, q.n))
        # query renumbering: query vertex u becomes sigma[u]
        sigma = rng.permutation(q.n)
        inv = np.argsort(sigma)
        qs = MicroQuery(q.n, q.vlabel[inv], q.vpin[inv], sigma[q.esrc], sigma[q.edst], q.elabel)
        got = og.match_query(qs)
        want = np.array(sorted(tuple(int(r[inv[c]]) for c in range(q.n)) for r in base), np.int32)
        assert np.array_equal(got.reshape(-1, q.n), want.reshape(-1, q.n))


@pytest.mark.parametrize("seed", range(12))
def test_more_constraints_give_subsets(seed):
    """Adding a query edge between matched vertices, or pinning a vertex,
    keeps exactly the rows that satisfy the new constraint."""
    rng = np.random.default_rng(6000 + seed)
    V = int(rng.integers(4, 9))
    g = random_graph(rng, V, 3 * V, n_types=2, n_rels=2)
    og = og_of(g)
    E = g.edge_set()
    for _ in range(4):
        q = random_query(rng, int(rng.integers(2, 5)), 2, 2, V, p_pin=0.0)
        base = rows_of(og.match_query(q))
        # a pin on vertex u to x keeps the rows with f(u) = x
        u, x = int(rng.integers(0, q.n)), int(rng.integers(0, V))
        qp = MicroQuery(q.n, q.vlabel, np.where(np.arange(q.n) == u, x, q.vpin), q.esrc, q.edst,
                        q.elabel)
        assert rows_of(og.match_query(qp)) == [r for r in base if r[u] == x]
        # a new edge a -> b (any relation) keeps the rows with a data edge f(a) -> f(b)
        a, b = (int(t) for t in rng.choice(q.n, 2, replace=False))
        if any(int(s) == a and int(d) == b and int(r) == -1
               for s, d, r in zip(q.esrc, q.edst, q.elabel)):
            continue
        qe = MicroQuery(q.n, q.vlabel, q.vpin, np.append(q.esrc, a), np.append(q.edst, b),
                        np.append(q.elabel, -1))
        pairs = {(s, d) for s, d, _ in E}
        assert rows_of(og.match_query(qe)) == [r for r in base if (r[a], r[b]) in pairs]


# --------------------------------------------------------------------------
# projection (the distinct projected tuples of all matches)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_projection_bruteforce_micro(seed):
    """The oracle's projection of its table equals the set of projected
    tuples of the brute-force matches, sorted, for every non-empty subset of
    a micro query's vertices."""
    rng = np.random.default_rng(1000 + seed)
    g = random_graph(rng, V=int(rng.integers(4, 9)), E=int(rng.integers(4, 20)), n_types=2,
                     n_rels=2)
    q = random_query(rng, int(rng.integers(2, 5)), 2, 2, g.V, p_pin=0.1)
    og = og_of(g)
    full = og.match_query(q)
    bf = brute_force(g, q)
    for mask in range(1, 1 << q.n):
        cols = [u for u in range(q.n) if (mask >> u) & 1]
        want = sorted({tuple(r[u] for u in cols) for r in bf})
        got = oracle.project_rows(full, cols)
        assert got.shape == (len(want), len(cols))
        assert [tuple(r) for r in got.tolist()] == want


def test_projection_closed_forms_medium(medium_kg, oracle_medium):
    """On the medium graph (simple, no self-loops): projecting an unlabelled
    edge a -> b onto a gives the vertices of out-degree >= 1, onto b those of
    in-degree >= 1; a star with a type-5 centre and leaves of types 3 and 7,
    onto its centre, gives the type-5 vertices with an out-neighbour of each
    type; a 2-path a -> b -> c with typed ends onto (a, c) gives the ordered
    pairs at distance two through some b with a != c (sparse A^2 off the
    diagonal)."""
    import scipy.sparse as sp
    kg = medium_kg
    outdeg = np.diff(kg.row_ptr)
    indeg = np.bincount(kg.col, minlength=kg.V)
    src = kg.src()
    e = MicroQuery(2, [-1, -1], [-1, -1], [0], [1], [-1])
    rows = oracle_medium.match_query(e)
    assert np.array_equal(oracle.project_rows(rows, [0])[:, 0], np.nonzero(outdeg >= 1)[0])
    assert np.array_equal(oracle.project_rows(rows, [1])[:, 0], np.nonzero(indeg >= 1)[0])
    star = MicroQuery(3, [5, 3, 7], [-1, -1, -1], [0, 0], [1, 2], [-1, -1])
    got = oracle.project_rows(oracle_medium.match_query(star), [0])
    has3 = np.zeros(kg.V, bool)
    has7 = np.zeros(kg.V, bool)
    has3[src[kg.vtype[kg.col] == 3]] = True
    has7[src[kg.vtype[kg.col] == 7]] = True
    assert np.array_equal(got[:, 0], np.nonzero(has3 & has7 & (kg.vtype == 5))[0])
    p2 = MicroQuery(3, [3, -1, 7], [-1, -1, -1], [0, 1], [1, 2], [-1, -1])
    got = oracle.project_rows(oracle_medium.match_query(p2), [0, 2])
    A = sp.csr_matrix((np.ones(kg.E), kg.col, kg.row_ptr), shape=(kg.V, kg.V))
    A2 = (A @ A).tocoo()
    keep = (A2.row != A2.col) & (kg.vtype[A2.row] == 3) & (kg.vtype[A2.col] == 7)
    want = np.stack([A2.row[keep], A2.col[keep]], axis=1)
    want = want[np.lexsort((want[:, 1], want[:, 0]))]
    assert np.array_equal(got, want)
