"""GPU parity: the HIP library's embedding tables against the CPU oracle,
element by element (bit-exact: all work is integer)."""
import sys

import numpy as np
import pytest

import kggen
import oracle
import paper_1807_08804_amd as P
from tests.micro import MicroQuery, random_graph, random_query

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(gpu_rows, want):
    assert gpu_rows.shape == want.shape, (gpu_rows.shape, want.shape)
    assert np.array_equal(gpu_rows, want)


@pytest.fixture(scope="module")
def g_tiny(tiny_kg):
    return P.Graph.from_kg(tiny_kg)


@pytest.fixture(scope="module")
def g_medium(medium_kg):
    return P.Graph.from_kg(medium_kg)


@pytest.fixture(scope="module")
def medium_queries(medium_kg):
    qs, _ = kggen.medium_queries(medium_kg, 100)
    return qs


def test_tiny_config(tiny_kg, g_tiny, oracle_tiny):
    say("case: tiny config query")
    q = kggen.tiny_query(tiny_kg)
    same(g_tiny.match_query(q), oracle_tiny.match_query(q))


def test_graph_info(tiny_kg, g_tiny):
    info = g_tiny.info()
    assert info["n_vertices"] == tiny_kg.V and info["n_edges"] == tiny_kg.E
    assert info["max_out"] == int(np.diff(tiny_kg.row_ptr).max())


PATHS = [P.SGM_PATH_AUTO, P.SGM_PATH_WIDE, P.SGM_PATH_NARROW]


def match_or_unsupported(g, q):
    """Rows, or None when the narrow-only path reports the query too big."""
    try:
        return g.match_query(q)
    except P.SGMError as e:
        if e.code == P.SGM_EUNSUPPORTED:
            return None
        raise


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(16))
def test_micro_random(seed, path):
    """Micro graphs with repeated triples, self-loops and multi-relation
    pairs; queries with any-type vertices, variable edges, pins, 2-cycles."""
    rng = np.random.default_rng(500 + seed)
    V = int(rng.integers(2, 40))
    mg = random_graph(rng, V, int(rng.integers(1, 4 * V)), n_types=3, n_rels=3)
    rp, col, rel, typ = mg.csr()
    say(f"case: micro seed={seed} path={path} V={V} E={len(col)}")
    g = P.Graph(rp, col, rel, typ, path=path)
    og = oracle.Graph(V, mg.src, mg.dst, mg.rel, mg.vtype)
    qs = [random_query(rng, int(rng.integers(1, 6)), 3, 3, V, p_pin=0.15, extra=3)
          for _ in range(10)]
    for q in qs:
        got = match_or_unsupported(g, q)
        if got is not None or path != P.SGM_PATH_NARROW:
            same(got, og.match_query(q))
    # the same queries as one batch
    for q, b in zip(qs, g.match_batch(qs)):
        if isinstance(b, P.SGMError):
            assert path == P.SGM_PATH_NARROW and b.code == P.SGM_EUNSUPPORTED
        else:
            same(b, og.match_query(q))
    g.close()


@pytest.fixture(scope="module")
def medium_expected(oracle_medium, medium_queries):
    return [oracle_medium.match_query(q) for q in medium_queries]


@pytest.mark.parametrize("path", PATHS)
def test_medium_config(path, medium_kg, medium_queries, medium_expected):
    """100 random-walk queries of 6-10 vertices (paths and trees, <= 2 pins),
    one at a time, on each execution path."""
    g = P.Graph.from_kg(medium_kg, path=path)
    tot = 0
    narrow_done = 0
    for i, (q, want) in enumerate(zip(medium_queries, medium_expected)):
        say(f"case: medium query {i} path={path} n={q.n} m={q.m} pins={(q.vpin >= 0).sum()}")
        got = match_or_unsupported(g, q)
        if got is None:
            assert path == P.SGM_PATH_NARROW
            continue
        narrow_done += 1
        same(got, want)
        assert tuple(q.walk) in set(map(tuple, got.tolist()))
        tot += len(got)
    assert tot > 0
    assert narrow_done >= 90
    g.close()


def test_medium_batch(medium_kg, g_medium, medium_queries, medium_expected):
    """The 100 queries as one sgm_match_batch call (one persistent launch)."""
    say("case: medium batch")
    for q, got, want in zip(medium_queries, g_medium.match_batch(medium_queries), medium_expected):
        same(got, want)


def test_batch_graph_replays(medium_kg, medium_queries, medium_expected):
    """Batches launched as HIP graphs (options.graphs = 1, the default) equal
    separate launches (graphs = 0) and the oracle on every replay, with
    batches of different sizes and root-sweep needs (node parameters change
    on each replay) and eager work on the same graph between replays."""
    say("case: batch graph replays")
    gg = P.Graph.from_kg(medium_kg, graphs=1)
    gd = P.Graph.from_kg(medium_kg, graphs=0)
    pinned_root = [i for i, q in enumerate(medium_queries) if (np.asarray(q.vpin) >= 0).any()]
    subsets = [list(range(100)), list(range(7)), pinned_root[:10], list(range(50, 100)), [3],
               list(range(100))]
    for rep, idx in enumerate(subsets):
        qs = [medium_queries[i] for i in idx]
        got = gg.match_batch(qs)
        direct = gd.match_batch(qs)
        for i, a, b in zip(idx, got, direct):
            same(a, medium_expected[i])
            same(b, medium_expected[i])
        # eager work between replays: a multi-kernel query and a count-only
        # single query on the graph that replays
        q = medium_queries[rep]
        same(gg.match_query(q), medium_expected[rep])
        wide = P.Graph.from_kg(medium_kg, path=P.SGM_PATH_WIDE)
        same(wide.match_query(q), medium_expected[rep])
        wide.close()
    gg.close()
    gd.close()


def test_vertex_renaming_medium(medium_kg, medium_queries, medium_expected):
    """The medium graph with its vertices renamed by a random permutation (a
    different CSR layout, root sweep and hub placement): every result, renamed
    back and re-sorted, equals the oracle's on the original graph."""
    say("case: medium graph with renamed vertices")
    kg = medium_kg
    rng = np.random.default_rng(77)
    perm = rng.permutation(kg.V).astype(np.int32)
    inv = np.argsort(perm).astype(np.int32)
    ns, nd = perm[kg.src()], perm[kg.col]
    order = np.lexsort((kg.rel, nd, ns))
    row_ptr = np.zeros(kg.V + 1, np.int64)
    np.cumsum(np.bincount(ns, minlength=kg.V), out=row_ptr[1:])
    vt = np.empty_like(kg.vtype)
    vt[perm] = kg.vtype
    gp = P.Graph(row_ptr.astype(np.int32), nd[order], kg.rel[order], vt)
    qs = medium_queries[:40]
    renamed = [MicroQuery(q.n, q.vlabel, np.where(q.vpin >= 0, perm[np.maximum(q.vpin, 0)], -1),
                          q.esrc, q.edst, q.elabel) for q in qs]
    for got, want in zip(gp.match_batch(renamed), medium_expected[:40]):
        back = inv[got]
        back = back[np.lexsort(back.T[::-1])] if len(back) else back
        same(back, want)
    gp.close()


def any_query(n, edges, vlabel=None, vpin=None):
    return MicroQuery(n, [-1] * n if vlabel is None else vlabel,
                      [-1] * n if vpin is None else vpin,
                      [e[0] for e in edges], [e[1] for e in edges], [e[2] for e in edges])


@pytest.mark.parametrize("name,q", [
    ("edge-any", any_query(2, [(0, 1, -1)])),
    ("path3-reversed-cols", any_query(3, [(2, 1, -1), (1, 0, -1)])),
    ("triangle", any_query(3, [(0, 1, -1), (1, 2, -1), (0, 2, -1)])),
    ("2cycle+tail", any_query(3, [(0, 1, -1), (1, 0, -1), (2, 1, 0)])),
    ("star3-typed", any_query(4, [(1, 0, -1), (1, 2, -1), (1, 3, -1)], vlabel=[-1, -1, 3, 3])),
    ("square", any_query(4, [(0, 1, -1), (1, 2, -1), (3, 2, -1), (0, 3, -1)])),
])
@pytest.mark.parametrize("path", PATHS)
def test_tiny_large_outputs(name, q, path, tiny_kg, oracle_tiny):
    """Unlabelled queries with thousands of rows: multi-tile joins, radix
    ordering (multi-kernel and in-kernel) and column permutations."""
    say(f"case: tiny large-output {name} path={path}")
    g = P.Graph.from_kg(tiny_kg, path=path)
    want = oracle_tiny.match_query(q)
    try:
        got, st = g.match_query(q, with_stats=True)
    except P.SGMError as e:
        # only a query that outgrows a persistent-kernel slot may be refused
        assert path == P.SGM_PATH_NARROW and e.code == P.SGM_EUNSUPPORTED
        ga = P.Graph.from_kg(tiny_kg)
        got, st = ga.match_query(q, with_stats=True)
        assert st["path"] == P.SGM_PATH_WIDE and st["fallback"] in (1, 2, 4, 8, 16)
        ga.close()
    same(got, want)
    if st["path"] == P.SGM_PATH_NARROW:
        # 0: a regular slot; otherwise the reason it moved to a large slot
        assert st["fallback"] in (0, 1, 2, 8)
    if name == "square" and path != P.SGM_PATH_WIDE:
        # a 0.9M-row level outgrows the tiny graph's 8 MB slot, fits a large one
        assert st["path"] == P.SGM_PATH_NARROW and st["fallback"] == 2
    g.close()


def test_medium_large_output(g_medium, oracle_medium):
    """~8.5M-row 2-path table on the medium graph (hub rows, big-degree
    paths, multi-pass radix ordering)."""
    q = any_query(3, [(1, 0, -1), (2, 1, -1)])
    say("case: medium 2-path any")
    same(g_medium.match_query(q), oracle_medium.match_query(q))


def test_medium_hub_star(medium_kg, g_medium, oracle_medium):
    """Pinned hub centre: candidates pushed from a ~64K-degree row."""
    hub = int(np.argmax(np.diff(medium_kg.row_ptr)))
    for t in (0, 9):
        q = any_query(3, [(0, 1, -1), (0, 2, 0)], vlabel=[-1, t, -1], vpin=[hub, -1, -1])
        say(f"case: medium hub star type={t}")
        same(g_medium.match_query(q), oracle_medium.match_query(q))
    q = any_query(3, [(1, 0, -1), (2, 1, -1)], vlabel=[-1, -1, 4], vpin=[hub, -1, -1])
    same(g_medium.match_query(q), oracle_medium.match_query(q))


@pytest.mark.parametrize("direction", ["out", "in"])
def test_medium_hub_rows_by_type_and_relation(direction, medium_kg, oracle_medium):
    """Hub rows (the medium graph's largest row, 64303 entries) read through
    their per-type index: every mix of typed / untyped neighbour and labelled
    / variable edge, pinned hub and unpinned hub-type centre, on every path,
    in one batch and alone. The in-direction case runs on the reversed graph,
    where that row is an in-row."""
    kg = medium_kg.ensure_in()
    og = oracle_medium
    if direction == "in":
        kg = kggen.KG(kg.V, kg.E, kg.in_ptr.astype(np.int32), kg.in_col, kg.in_rel, kg.vtype)
        og = oracle.graph_from_kg(kg)
    deg = np.diff(medium_kg.row_ptr)
    hub = int(np.argmax(deg))
    say(f"case: {direction} hub {hub} with {int(deg[hub])} entries")
    qs = []
    for t in (-1, 2, 9):
        for r in (-1, 0, 2):
            e1 = (0, 1, r) if direction == "out" else (1, 0, r)
            e2 = (1, 2, -1) if direction == "out" else (2, 1, -1)
            qs.append(any_query(3, [e1, e2], vlabel=[-1, t, 5], vpin=[hub, -1, -1]))
            qs.append(any_query(2, [e1], vlabel=[int(kg.vtype[hub]), t], vpin=[-1, -1]))
    want = [og.match_query(q) for q in qs]
    assert max(len(w) for w in want) > 10000
    for path in PATHS:
        g = P.Graph.from_kg(kg, path=path)
        for q, w in zip(qs, want):
            same(g.match_query(q), w)
        for r, w in zip(g.match_batch(qs), want):
            same(r, w)
        g.close()


@pytest.mark.parametrize("opts", [dict(refine_rounds=0), dict(refine_rounds=-1),
                                  dict(refine_reversed=0), dict(low_conn_degree=0),
                                  dict(low_conn_degree=4, refine_rounds=3)])
def test_filter_options_do_not_change_results(opts, medium_kg, oracle_medium, medium_queries):
    say(f"case: options {opts}")
    g = P.Graph.from_kg(medium_kg, **opts)
    for q in medium_queries[:25]:
        same(g.match_query(q), oracle_medium.match_query(q))
    g.close()


@pytest.mark.parametrize("name,q", [
    ("path3", any_query(3, [(2, 1, -1), (1, 0, -1)])),
    ("square", any_query(4, [(0, 1, -1), (1, 2, -1), (3, 2, -1), (0, 3, -1)])),
])
def test_chunked_join(name, q, tiny_kg, oracle_tiny):
    """A 4 KB join budget splits every level into many pair chunks
    (depth-first); rows and their order are unchanged."""
    say(f"case: chunked {name}")
    g = P.Graph.from_kg(tiny_kg, path=P.SGM_PATH_WIDE, join_budget_bytes=4096)
    rows, st = g.match_query(q, with_stats=True)
    same(rows, oracle_tiny.match_query(q))
    assert st["n_chunks"] > 1
    assert g.match_query(q, count_only=True) == len(rows)
    g.close()


def test_count_only_and_cap(tiny_kg, oracle_tiny):
    q = any_query(3, [(0, 1, -1), (1, 2, -1)])
    want = oracle_tiny.match_query(q, count_only=True)
    g = P.Graph.from_kg(tiny_kg, result_cap_rows=10)
    with pytest.raises(P.SGMError) as e:
        g.match_query(q)
    assert e.value.code == P.SGM_ETOOBIG and e.value.n_rows == want
    g.close()
    g = P.Graph.from_kg(tiny_kg)
    assert g.match_query(q, count_only=True) == want
    g.close()


def test_invalid_queries(g_tiny):
    for q, code in [(any_query(2, [(0, 0, -1)]), P.SGM_EINVAL),
                    (any_query(3, [(0, 1, -1)]), P.SGM_EINVAL),
                    (any_query(2, [(0, 1, 1), (0, 1, 1)]), P.SGM_EINVAL)]:
        with pytest.raises(P.SGMError) as e:
            g_tiny.match_query(q)
        assert e.value.code == code


def test_single_vertex_and_empty(tiny_kg, g_tiny, oracle_tiny):
    for q in [any_query(1, []), any_query(1, [], vlabel=[7]), any_query(1, [], vpin=[5]),
              any_query(2, [(0, 1, 99)]), any_query(2, [(0, 1, -1)], vlabel=[63, 99])]:
        same(g_tiny.match_query(q), oracle_tiny.match_query(q))


def test_batch_equals_alone(g_medium, medium_queries):
    qs = medium_queries[:20] + [any_query(2, [(0, 0, -1)])]
    alone = [g_medium.match_query(q) for q in qs[:-1]]
    batch = g_medium.match_batch(qs)
    for a, b in zip(alone, batch[:-1]):
        same(b, a)
    assert isinstance(batch[-1], P.SGMError) and batch[-1].code == P.SGM_EINVAL


def test_repeat_is_deterministic(g_medium, medium_queries):
    q = medium_queries[3]
    a, sa = g_medium.match_query(q, with_stats=True)
    b, sb = g_medium.match_query(q, with_stats=True)
    same(a, b)
    assert sa["cand"] == sb["cand"] and sa["level_rows"] == sb["level_rows"]


# --------------------------------------------------------------------------
# stage parity: candidate sets and candidate-edge counts
# --------------------------------------------------------------------------

def stage_check(g, og, q, opts):
    lists, ec = g.inspect_query(q)
    cand = og.filter(q, rounds=opts.get("refine_rounds", 1),
                     reversed=opts.get("refine_reversed", 1),
                     low_conn=opts.get("low_conn_degree", 1))
    for u in range(q.n):
        assert np.array_equal(lists[u], np.nonzero(cand[u])[0].astype(np.int32)), (q, u)
    if q.m and all(len(x) for x in lists):
        assert ec.tolist() == og.edge_candidates(q, cand).tolist()
    return cand


STAGE_OPTS = [dict(), dict(refine_rounds=0), dict(refine_rounds=-1), dict(refine_reversed=0),
              dict(low_conn_degree=0)]


@pytest.mark.parametrize("opts", STAGE_OPTS)
@pytest.mark.parametrize("seed", range(6))
def test_stage_parity_micro(seed, opts):
    rng = np.random.default_rng(900 + seed)
    V = int(rng.integers(3, 40))
    mg = random_graph(rng, V, int(rng.integers(V, 4 * V)), n_types=3, n_rels=3)
    rp, col, rel, typ = mg.csr()
    say(f"case: stage micro seed={seed} opts={opts}")
    g = P.Graph(rp, col, rel, typ, **opts)
    og = oracle.Graph(V, mg.src, mg.dst, mg.rel, mg.vtype)
    for _ in range(8):
        q = random_query(rng, int(rng.integers(1, 7)), 3, 3, V, p_pin=0.15, extra=3)
        stage_check(g, og, q, opts)
    g.close()


@pytest.mark.parametrize("opts", STAGE_OPTS)
def test_stage_parity_medium(opts, medium_kg, oracle_medium, medium_queries):
    """Candidate sets of every query vertex after filtering, and candidate
    edge counts, equal the oracle's stage functions; the persistent kernel's
    per-vertex counts and edge counts agree too."""
    say(f"case: stage medium opts={opts}")
    g = P.Graph.from_kg(medium_kg, **opts)
    gn = P.Graph.from_kg(medium_kg, path=P.SGM_PATH_NARROW, **opts)
    for i, q in enumerate(medium_queries[:40]):
        cand = stage_check(g, oracle_medium, q, opts)
        try:
            _, st = gn.match_query(q, with_stats=True)
        except P.SGMError as e:
            assert e.code == P.SGM_EUNSUPPORTED
            continue
        counts = cand.sum(axis=1).tolist()
        if all(counts):
            assert st["cand"] == counts, (i, st["cand"], counts)
            assert st["ec"] == oracle_medium.edge_candidates(q, cand).tolist()
    g.close()
    gn.close()
