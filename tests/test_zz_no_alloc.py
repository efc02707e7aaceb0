"""The entry point that allocates nothing (sgm_match_query_noalloc): its
tables equal sgm_match_query's, bit for bit, on calls in a row that share
the fixed device area, including a call with a smaller input after a larger
one (the area keeps the last call's contents)."""
import sys

import numpy as np
import pytest

import kggen
import paper_1807_08804_amd as P
from tests.micro import MicroQuery

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    assert a.shape == b.shape, (a.shape, b.shape)
    assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def g_medium_na(medium_kg):
    return P.Graph.from_kg(medium_kg)


@pytest.fixture(scope="module")
def medium_qs(medium_kg):
    return kggen.medium_queries(medium_kg, 100)[0]


def test_no_alloc_larger_then_smaller(g_medium_na, medium_qs):
    """A large query, then a smaller one (fewer vertices and rows): both equal
    sgm_match_query, and the second call's buffer past its rows is untouched."""
    want = [g_medium_na.match_query(q) for q in medium_qs]
    order = sorted(range(len(medium_qs)), key=lambda i: (len(want[i]) * medium_qs[i].n, i))
    big, small = order[-1], order[0]
    assert len(want[big]) * medium_qs[big].n > len(want[small]) * medium_qs[small].n
    say(f"case: no-alloc query {big} ({len(want[big])} rows) then {small} "
        f"({len(want[small])} rows)")
    got = g_medium_na.match_query_noalloc(medium_qs[big], rows_cap=len(want[big]) + 10)
    same(got, want[big])
    buf = np.full((len(want[small]) + 7, medium_qs[small].n), -12345, np.int32)
    got = g_medium_na.match_query_noalloc(medium_qs[small], rows_cap=len(buf), out=buf)
    same(got, want[small])
    assert np.all(buf[len(want[small]):] == -12345)


def test_no_alloc_every_medium_query(g_medium_na, medium_qs):
    """All 100 medium queries in a row through the fixed area, each equal to
    sgm_match_query's table; counts alone too."""
    say("case: no-alloc on 100 medium queries")
    for i, q in enumerate(medium_qs):
        want = g_medium_na.match_query(q)
        same(g_medium_na.match_query_noalloc(q, rows_cap=len(want)), want)
        assert g_medium_na.match_query_noalloc(q, 0, count_only=True) == len(want)


def test_no_alloc_row_cap_and_errors(g_medium_na, medium_qs):
    q = max(medium_qs, key=lambda x: len(g_medium_na.match_query(x)))
    n = len(g_medium_na.match_query(q))
    assert n > 1
    say(f"case: no-alloc row cap {n - 1} of {n}")
    with pytest.raises(P.SGMError) as e:
        g_medium_na.match_query_noalloc(q, rows_cap=n - 1)
    assert e.value.code == P.SGM_ETOOBIG and e.value.n_rows == n
    bad = MicroQuery(2, [-1, -1], [-1, -1], [0], [0], [-1])  # self-loop
    with pytest.raises(P.SGMError) as e:
        g_medium_na.match_query_noalloc(bad, rows_cap=4)
    assert e.value.code == P.SGM_EINVAL
    # and the next call is still right
    same(g_medium_na.match_query_noalloc(medium_qs[0], rows_cap=n + 100),
         g_medium_na.match_query(medium_qs[0]))


def test_no_alloc_large_graph(g_medium_na, medium_qs):
    """Batch queries of the 4M-vertex graph (the fixed area holds its slot),
    alternating with medium-graph queries (the two graphs lay their slot
    bitmaps over different parts of the area): each equals sgm_match_query,
    or is ENOMEM for a query that outgrows the area, after which the next
    query is still right."""
    kg = kggen.named_graph("large")
    g = P.Graph.from_kg(kg)
    qs, _ = kggen.load_large_batch(48)
    say("case: no-alloc on 48 large batch queries, medium queries between them")
    outgrew = 0
    for i, q in enumerate(qs):
        want = g.match_query(q)
        try:
            got = g.match_query_noalloc(q, rows_cap=len(want))
        except P.SGMError as e:
            assert e.code == P.SGM_ENOMEM, (i, e.code)
            outgrew += 1
            continue
        same(got, want)
        if i % 8 == 7:
            mq = medium_qs[i]
            mw = g_medium_na.match_query(mq)
            same(g_medium_na.match_query_noalloc(mq, rows_cap=len(mw)), mw)
    say(f"  {outgrew} outgrew the fixed area")
    assert outgrew < len(qs)
    g.close()
