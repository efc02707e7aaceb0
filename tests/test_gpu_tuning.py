"""Work division and join schedule of the persistent kernel (sgm_tuning) and
the autotuner: results are identical under every tuning, bit for bit, and
equal to the oracle's."""
import sys

import numpy as np
import pytest

import kggen
import paper_1807_08804_amd as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    assert a.shape == b.shape, (a.shape, b.shape)
    assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def medium_set(medium_kg, oracle_medium):
    qs, _ = kggen.medium_queries(medium_kg, 100)
    return qs[:40], [oracle_medium.match_query(q) for q in qs[:40]]


# the second and fourth share every filter step of 64 or more candidates
# with helper workgroups (many helpers, and only three)
TUNINGS = [
    dict(slots=512, group_lanes=64, wg_rows=8192, join_policy=0, help_items=1024, helpers=64,
         help_wait=0),
    dict(slots=7, group_lanes=1, wg_rows=64, join_policy=1, help_items=64, helpers=512, help_wait=0),
    dict(slots=256, group_lanes=16, wg_rows=32768, join_policy=1, help_items=0, helpers=0,
         help_wait=0),
    dict(slots=1, group_lanes=4, wg_rows=2048, join_policy=0, help_items=64, helpers=3, help_wait=0),
]


@pytest.mark.parametrize("tune", TUNINGS)
def test_results_do_not_depend_on_tuning(tune, medium_kg, medium_set):
    qs, want = medium_set
    say(f"case: tuning {tune}")
    g = P.Graph.from_kg(medium_kg, path=P.SGM_PATH_NARROW)
    g.set_tuning(**tune)
    assert g.tuning() == tune
    for r, w in zip(g.match_batch(qs), want):
        same(r, w)
    for q, w in zip(qs[:10], want[:10]):
        same(g.match_query(q), w)
    g.close()


def test_tuning_validation(medium_kg):
    g = P.Graph.from_kg(medium_kg)
    for bad in (dict(slots=0), dict(slots=513), dict(group_lanes=3), dict(group_lanes=128),
                dict(wg_rows=32), dict(join_policy=2), dict(help_items=63), dict(help_items=-1),
                dict(helpers=-1), dict(helpers=513), dict(help_wait=-1)):
        with pytest.raises(P.SGMError) as e:
            g.set_tuning(**bad)
        assert e.value.code == P.SGM_EINVAL
    assert g.tuning() == TUNINGS[0]
    g.close()


def test_autotune_keeps_results(medium_kg, medium_set):
    qs, want = medium_set
    say("case: autotune")
    g = P.Graph.from_kg(medium_kg)
    best = g.autotune(qs, reps=1)
    assert best["slots"] in (256, 512) and best["group_lanes"] in (16, 64)
    assert best["wg_rows"] in (2048, 8192, 32768) and best["join_policy"] in (0, 1)
    assert best["help_items"] in (0, 1024) and best["helpers"] == 64
    assert g.tuning() == best
    for r, w in zip(g.match_batch(qs), want):
        same(r, w)
    say(f"  picked {best}")
    g.close()


@pytest.fixture(scope="module")
def medium_filter(oracle_medium, medium_set):
    """The oracle's candidate counts per query vertex after filtering, and
    its candidate-edge counts when no set is empty."""
    qs, _ = medium_set
    out = []
    for q in qs:
        cand = oracle_medium.filter(q)
        ec = None
        if len(q.esrc) and cand.any(axis=1).all():
            ec = oracle_medium.edge_candidates(q, cand).tolist()
        out.append((cand.sum(axis=1).tolist(), ec))
    return out


@pytest.mark.parametrize("tune", TUNINGS)
def test_candidates_match_oracle_filter(tune, medium_kg, medium_set, medium_filter):
    """Final candidate sets and candidate-edge counts of the persistent
    kernel equal the oracle's under every tuning, shared filter steps
    included (a step's removals must all reach the compaction)."""
    qs, _ = medium_set
    say(f"case: candidates under tuning {tune}")
    g = P.Graph.from_kg(medium_kg, path=P.SGM_PATH_NARROW)
    g.set_tuning(**tune)
    for i, (q, (cnt, ec)) in enumerate(zip(qs, medium_filter)):
        _, st = g.match_query(q, with_stats=True)
        assert st["cand"] == cnt, (i, st["cand"], cnt)
        if ec is not None:
            assert st["ec"] == ec, (i, st["ec"], ec)
    g.close()


def test_helper_give_up_retires_slot(medium_kg, medium_set):
    """The owner of a shared step may give up waiting for its helpers (an
    error path, forced here from the host with a wait bound of one poll, so
    every kernel still exits normally). Such a query is rerun outside the
    launch's slots, its slot takes no further query in that launch (helpers
    may still be writing it) and the next launch clears the slot before use.
    Every table of this launch and of the following ones, on the same slots,
    equals the oracle's."""
    qs, want = medium_set
    say("case: shared steps given up after one poll")
    g = P.Graph.from_kg(medium_kg)
    g.set_tuning(slots=8, group_lanes=64, wg_rows=8192, join_policy=0, help_items=64,
                 helpers=512, help_wait=1)
    gave_up = 0
    for rep in range(3):
        got, stats = g.match_batch(qs, with_stats=True)
        for i, (r, w) in enumerate(zip(got, want)):
            same(r, w)
        gave_up += sum(st["fallback"] == 32 for st in stats)
        say(f"  launch {rep}: {sum(st['fallback'] == 32 for st in stats)} queries rerun")
    # single queries: one slot and many helper workgroups
    for q, w in zip(qs[:10], want[:10]):
        same(g.match_query(q), w)
    # back to the default wait: the slots left dirty are cleared and reused
    g.set_tuning(help_wait=0)
    for rep in range(2):
        got, stats = g.match_batch(qs, with_stats=True)
        for r, w in zip(got, want):
            same(r, w)
        assert not any(st["fallback"] == 32 for st in stats)
    say(f"  {gave_up} queries given up in all")
    assert gave_up > 0
    g.close()
