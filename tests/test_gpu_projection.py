"""Projection (thesis Ch. 3, Sec. "GpSense": a commonsense query asks only
for the matches of a subset of its nodes): sgm_match_query_proj and
sgm_match_batch_proj return the distinct projected tuples, sorted; they
equal the oracle's projection of its full table (oracle.project_rows) on
the persistent kernel, the multi-kernel path and in batches."""
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


def same(a, b):
    assert a.shape == b.shape, (a.shape, b.shape)
    assert np.array_equal(a, b)


def cols_of(mask, n):
    return [u for u in range(n) if (mask >> u) & 1]


@pytest.fixture(scope="module")
def medium_proj(medium_kg, oracle_medium):
    qs, _ = kggen.medium_queries(medium_kg, 100)
    rng = np.random.default_rng(17)
    masks = [int(rng.integers(1, 1 << q.n)) for q in qs]
    full = [oracle_medium.match_query(q) for q in qs]
    want = [oracle.project_rows(f, cols_of(m, q.n)) for f, m, q in zip(full, masks, qs)]
    return qs, masks, want


@pytest.mark.parametrize("path", [P.SGM_PATH_AUTO, P.SGM_PATH_WIDE])
def test_projection_medium(path, medium_kg, medium_proj):
    qs, masks, want = medium_proj
    say(f"case: projection of 100 medium queries, path {path}")
    g = P.Graph.from_kg(medium_kg, path=path)
    for i, (q, m, w) in enumerate(zip(qs, masks, want)):
        got = g.match_query(q, project=m)
        same(got, w)
        assert g.match_query(q, project=m, count_only=True) == len(w)
    g.close()


def test_projection_batch_medium(medium_kg, medium_proj):
    qs, masks, want = medium_proj
    say("case: projection in one batch")
    g = P.Graph.from_kg(medium_kg)
    got = g.match_batch(qs, projects=masks)
    for r, w in zip(got, want):
        same(r, w)
    counts = g.match_batch(qs, projects=masks, count_only=True)
    assert counts == [len(w) for w in want]
    # the full mask is the plain match
    full = g.match_batch(qs[:20], projects=[(1 << q.n) - 1 for q in qs[:20]])
    for q, r in zip(qs[:20], full):
        same(r, g.match_query(q))
    g.close()


@pytest.mark.parametrize("seed", range(6))
def test_projection_micro_every_mask(seed):
    """Every non-empty projection of micro queries (repeated triples, pins,
    any-labels), both paths."""
    rng = np.random.default_rng(500 + seed)
    mg = random_graph(rng, V=int(rng.integers(5, 12)), E=int(rng.integers(8, 40)), n_types=2,
                      n_rels=2)
    og = oracle.Graph(mg.V, mg.src, mg.dst, mg.rel, mg.vtype)
    rp, col, rel, typ = mg.csr()
    gs = [P.Graph(rp, col, rel, typ, path=p) for p in (P.SGM_PATH_AUTO, P.SGM_PATH_WIDE)]
    for _ in range(4):
        q = random_query(rng, int(rng.integers(2, 5)), 2, 2, mg.V, p_pin=0.1)
        full = og.match_query(q)
        for m in range(1, 1 << q.n):
            w = oracle.project_rows(full, cols_of(m, q.n))
            for g in gs:
                same(g.match_query(q, project=m), w)
    for g in gs:
        g.close()


def test_projection_large_tables(medium_kg, oracle_medium):
    """Projections of tables beyond the in-LDS orderings (radix orderings on
    both paths, millions of rows collapsing to far fewer tuples): an
    unlabelled 2-path onto its middle vertex and onto its ends."""
    q = MicroQuery(3, [4, -1, -1], [-1] * 3, [0, 1], [1, 2], [-1, -1])
    full = oracle_medium.match_query(q)
    say(f"case: projections of a {len(full)}-row 2-path")
    assert len(full) > 100_000
    for path in (P.SGM_PATH_AUTO, P.SGM_PATH_WIDE):
        g = P.Graph.from_kg(medium_kg, path=path)
        for cols in ([1], [0, 2], [1, 2], [0]):
            same(g.match_query(q, project=cols), oracle.project_rows(full, cols))
        g.close()


def test_projection_errors(medium_kg, medium_proj):
    qs, _, _ = medium_proj
    g = P.Graph.from_kg(medium_kg)
    q = qs[0]
    for bad in (0, 1 << q.n, (1 << (q.n + 1)) - 1):
        with pytest.raises(P.SGMError) as e:
            g.match_query(q, project=bad)
        assert e.value.code == P.SGM_EINVAL
    res = g.match_batch(qs[:3], projects=[0, 1, 1 << 20])
    assert isinstance(res[0], P.SGMError) and res[0].code == P.SGM_EINVAL
    assert isinstance(res[1], np.ndarray)
    assert isinstance(res[2], P.SGMError) and res[2].code == P.SGM_EINVAL
    g.close()


def test_projection_large_batch():
    """Projections onto the unpinned vertices of large-graph batch queries
    (the commonsense answer: the variable nodes' bindings) equal the
    oracle's, for the queries it finishes quickly."""
    kg = kggen.named_graph("large")
    og = oracle.graph_from_kg(kg)
    g = P.Graph.from_kg(kg)
    qs, _ = kggen.load_large_batch(96)
    masks = []
    for q in qs:
        m = sum(1 << u for u in range(q.n) if q.vpin[u] < 0)
        masks.append(m if m else 1)
    got = g.match_batch(qs, projects=masks)
    say("case: projection of 96 large batch queries")
    compared = 0
    for q, m, r in zip(qs, masks, got):
        try:
            full = og.match_query(q, max_steps=50_000_000)
        except oracle.OracleError as e:
            assert e.code == oracle.OR_EBUDGET
            continue
        same(r, oracle.project_rows(full, cols_of(m, q.n)))
        compared += 1
    say(f"  {compared} compared")
    assert compared >= 80
    g.close()
