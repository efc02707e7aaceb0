"""Per-request failure isolation: a query made to fail on the device (the
host-forced hook sgm_inject_fault; every kernel still exits normally)
reports SGM_EDEVICE, and every other query of the same launch, and the
next launch on the same graph, still equal the oracle's tables."""
import sys

import numpy as np
import pytest

import kggen
import paper_1807_08804_amd as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mix(medium_kg, oracle_medium):
    qs, _ = kggen.medium_queries(medium_kg, 40)
    return qs, [oracle_medium.match_query(q) for q in qs]


def test_fault_confined_to_its_batch_member(medium_kg, mix):
    qs, want = mix
    g = P.Graph.from_kg(medium_kg)
    for bad in (0, 7, len(qs) - 1):
        say(f"case: injected fault on member {bad} of a {len(qs)}-query batch")
        g.inject_fault(bad)
        got = g.match_batch(qs)
        for i, (r, w) in enumerate(zip(got, want)):
            if i == bad:
                assert isinstance(r, P.SGMError) and r.code == P.SGM_EDEVICE, (i, r)
            else:
                assert isinstance(r, np.ndarray) and np.array_equal(r, w), i
        # the hook is one-shot: the next launch is whole
        for r, w in zip(g.match_batch(qs), want):
            assert np.array_equal(r, w)
    g.close()


def test_fault_on_a_single_query(medium_kg, mix):
    qs, want = mix
    g = P.Graph.from_kg(medium_kg)
    say("case: injected fault on a single query")
    g.inject_fault(0)
    with pytest.raises(P.SGMError) as e:
        g.match_query(qs[3])
    assert e.value.code == P.SGM_EDEVICE
    assert np.array_equal(g.match_query(qs[3]), want[3])
    # cancelled before any launch: nothing fails
    g.inject_fault(0)
    g.inject_fault(-1)
    assert np.array_equal(g.match_query(qs[4]), want[4])
    with pytest.raises(P.SGMError):
        g.inject_fault(-2)
    g.close()


def test_fault_in_a_served_stream(medium_kg, mix):
    """One query of a served stream fails; the server keeps serving and
    every other result equals the oracle's."""
    qs, want = mix
    g = P.Graph.from_kg(medium_kg)
    say("case: injected fault in a served stream")
    g.inject_fault(0)
    srv = P.Server(g)
    lat, res = srv.replay(qs, kggen.poisson_arrivals(len(qs), 2000))
    st = srv.stats()
    srv.close()
    failed = [i for i, r in enumerate(res) if isinstance(r, P.SGMError)]
    assert len(failed) == 1 and res[failed[0]].code == P.SGM_EDEVICE
    for i, (r, w) in enumerate(zip(res, want)):
        if i not in failed:
            assert np.array_equal(r, w), i
    assert st["completed"] == len(qs)
    g.close()
