"""Served form: queries arriving while others run are batched continuously
over several streams; each result must equal the same query matched alone
(bit-exact), whatever the arrival rate, batch window or memory cap."""
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
def g_medium_s(medium_kg):
    return P.Graph.from_kg(medium_kg)


@pytest.fixture(scope="module")
def medium_alone(g_medium_s, medium_kg):
    qs, _ = kggen.medium_queries(medium_kg, 100)
    return qs, [g_medium_s.match_query(q) for q in qs]


@pytest.mark.parametrize("qps", [500, 5000, 50000])
def test_served_equals_alone(qps, g_medium_s, medium_alone):
    qs, alone = medium_alone
    # 300 arrivals cycling over the 100 queries
    stream = [qs[i % len(qs)] for i in range(300)]
    want = [alone[i % len(qs)] for i in range(300)]
    arr = kggen.poisson_arrivals(len(stream), qps, seed=qps)
    say(f"case: served at {qps} qps")
    srv = P.Server(g_medium_s, streams=4, max_batch=64, max_wait_ns=50_000)
    lat, res = srv.replay(stream, arr)
    st = srv.stats()
    srv.close()
    for r, w in zip(res, want):
        same(r, w)
    assert np.all(lat > 0)
    assert st["completed"] == len(stream) and st["batches"] >= 1
    say(f"  batches={st['batches']} max_in_flight={st['max_in_flight']} "
        f"p50={np.percentile(lat, 50) / 1e3:.0f}us p99={np.percentile(lat, 99) / 1e3:.0f}us")


def test_served_tiny_cap_and_errors(g_medium_s, medium_alone):
    """A 1-byte admission cap admits one query at a time (stalls are
    counted); an invalid query fails alone without touching the others."""
    qs, alone = medium_alone
    bad = MicroQuery(2, [-1, -1], [-1, -1], [0], [0], [-1])  # self-loop
    stream = qs[:20] + [bad] + qs[20:40]
    srv = P.Server(g_medium_s, streams=2, max_batch=8, max_wait_ns=0, admission_cap_bytes=1)
    tickets = [srv.submit(q) for q in stream]
    outs = [srv.wait(t, q.n) for t, q in zip(tickets, stream)]
    st = srv.stats()
    srv.close()
    for i, (status, rows, _) in enumerate(outs):
        if i == 20:
            assert status == P.SGM_EINVAL and rows is None
        else:
            assert status == P.SGM_OK
            same(rows, alone[i if i < 20 else i - 1])
    assert st["max_in_flight"] == 1
    assert st["admission_stalls"] >= 1


def test_served_admission_cap_admits_some(g_medium_s, medium_kg, oracle_medium):
    """Admission by per-query estimates (sgm_estimate_query): with a cap
    worth about six typical queries, a burst of 100 queries runs several at
    a time but never all at once (admission stalls occur), and every result
    equals the oracle's."""
    qs, _ = kggen.medium_queries(medium_kg, 100)
    tf = np.bincount(medium_kg.vtype, minlength=64)
    rf = np.bincount(medium_kg.rel, minlength=32)
    est = np.array([P.sgm_estimate_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel,
                                         medium_kg.V, tf, rf) for q in qs])
    cap = int(6 * np.median(est))
    say(f"case: admission cap {cap} bytes (estimates {est.min()}..{est.max()})")
    srv = P.Server(g_medium_s, streams=4, max_batch=16, max_wait_ns=0, admission_cap_bytes=cap)
    tickets = [srv.submit(q) for q in qs]
    outs = [srv.wait(t, q.n) for t, q in zip(tickets, qs)]
    st = srv.stats()
    srv.close()
    for q, (status, rows, _) in zip(qs, outs):
        assert status == P.SGM_OK
        same(rows, oracle_medium.match_query(q))
    say(f"  stalls={st['admission_stalls']} max_in_flight={st['max_in_flight']} "
        f"batches={st['batches']}")
    assert st["admission_stalls"] > 0
    assert 1 < st["max_in_flight"] < len(qs)


def test_served_large_graph(large_kg_serve):
    """Walk queries on the 4M/20M graph at 5000 qps: served == alone."""
    g, qs, alone = large_kg_serve
    arr = kggen.poisson_arrivals(len(qs), 5000)
    srv = P.Server(g)
    lat, res = srv.replay(qs, arr)
    srv.close()
    for r, w in zip(res, alone):
        same(r, w)


@pytest.fixture(scope="module")
def large_kg_serve():
    kg = kggen.named_graph("large")
    kg.ensure_in()
    g = P.Graph.from_kg(kg)
    qs, _ = kggen.load_large_serve(128)
    say("case: large serve set ready")
    return g, qs, [g.match_query(q) for q in qs]
