"""The refinement and two-graph ablation (thesis Ch. 3, Sec. "Effect of
Optimization Techniques"; Sec. "GpSense Framework", incoming and outgoing
graphs, one-time refinement): the four refinement variants, each with both
graph representations and with the outgoing graph alone, return the oracle's
rows exactly; only the intermediate sizes and the time change."""
import sys

import numpy as np
import pytest

import kggen
import oracle
import paper_1807_08804_amd as P
from tests.micro import random_graph, random_query

pytestmark = pytest.mark.gpu

# (refine_rounds, refine_reversed): to convergence, to convergence reversed,
# one round reversed (the default), none
VARIANTS = [(-1, 0), (-1, 1), (1, 1), (0, 1)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(gpu_rows, want):
    assert gpu_rows.shape == want.shape, (gpu_rows.shape, want.shape)
    assert np.array_equal(gpu_rows, want)


@pytest.mark.parametrize("seed", range(6))
def test_out_only_micro_graphs(seed):
    """Random small graphs (repeated triples, multi-relation pairs, self
    loops) and random queries with edges in both directions, pins, variable
    labels and relations and extra cycle edges: every variant, out-only and
    in+out, in one batch and alone."""
    rng = np.random.default_rng(7100 + seed)
    V = int(rng.integers(8, 60))
    mg = random_graph(rng, V, int(rng.integers(V, 4 * V)), n_types=3, n_rels=3)
    rp, col, rel, typ = mg.csr()
    og = oracle.Graph(V, mg.src, mg.dst, mg.rel, mg.vtype)
    qs = [random_query(rng, int(rng.integers(1, 8)), 3, 3, V, p_pin=0.15, extra=3)
          for _ in range(12)]
    want = [og.match_query(q) for q in qs]
    for rounds, rev in VARIANTS:
        for out_only in (1, 0):
            say(f"case: ablation micro seed={seed} V={V} rounds={rounds} reversed={rev} "
                f"out_only={out_only}")
            g = P.Graph(rp, col, rel, typ, out_only=out_only, refine_rounds=rounds,
                        refine_reversed=rev, path=P.SGM_PATH_WIDE)
            for q, w in zip(qs, want):
                same(g.match_query(q), w)
            for r, w in zip(g.match_batch(qs), want):
                same(r, w)
            g.close()


@pytest.fixture(scope="module")
def medium_mix(medium_kg, oracle_medium):
    qs, _ = kggen.medium_queries(medium_kg, 40)
    return qs, [oracle_medium.match_query(q) for q in qs]


@pytest.mark.parametrize("variant", VARIANTS)
def test_out_only_medium_graph(variant, medium_kg, medium_mix):
    """The medium graph's query mix under every variant, with both graphs
    and with the outgoing graph alone: results equal the oracle's."""
    rounds, rev = variant
    qs, want = medium_mix
    say(f"case: ablation medium rounds={rounds} reversed={rev}")
    go = P.Graph.from_kg(medium_kg, out_only=1, refine_rounds=rounds, refine_reversed=rev)
    gb = P.Graph.from_kg(medium_kg, path=P.SGM_PATH_WIDE, refine_rounds=rounds,
                         refine_reversed=rev)
    assert go.info()["max_in"] == 0
    for q, w in zip(qs, want):
        ro, so = go.match_query(q, with_stats=True)
        same(ro, w)
        same(gb.match_query(q), w)
        assert so["path"] == P.SGM_PATH_WIDE
    go.close()
    gb.close()


def test_out_only_transposed_edge_tables(medium_kg, oracle_medium):
    """Queries whose join binds an edge's destination first (a pinned
    destination with several incoming query edges, a cycle against the edge
    direction): the destination-keyed candidate edges come from transposing
    the source-keyed ones."""
    kg = medium_kg.ensure_in()
    hub = int(np.argmax(np.diff(kg.in_ptr)))
    Q = kggen.Query
    qs = [
        Q(3, np.array([-1, -1, -1], np.int32), np.array([hub, -1, -1], np.int32),
          np.array([1, 2], np.int32), np.array([0, 0], np.int32), np.array([-1, -1], np.int32)),
        Q(3, np.array([-1, -1, -1], np.int32), np.array([hub, -1, -1], np.int32),
          np.array([1, 2, 2], np.int32), np.array([0, 1, 0], np.int32),
          np.array([-1, -1, -1], np.int32)),
        Q(4, np.array([-1, 3, -1, -1], np.int32), np.array([hub, -1, -1, -1], np.int32),
          np.array([1, 2, 3], np.int32), np.array([0, 1, 2], np.int32),
          np.array([-1, -1, -1], np.int32)),
    ]
    go = P.Graph.from_kg(medium_kg, out_only=1)
    for q in qs:
        say(f"case: transposed tables {q.n} vertices, hub {hub}")
        same(go.match_query(q), oracle_medium.match_query(q))
    go.close()


def test_out_only_entry_points_that_need_the_persistent_kernel(tiny_kg):
    g = P.Graph.from_kg(tiny_kg, out_only=1)
    q = kggen.tiny_query(tiny_kg)
    with pytest.raises(P.SGMError) as e:
        g.match_query_noalloc(q, 1000)
    assert e.value.code == P.SGM_EINVAL
    with pytest.raises(P.SGMError) as e:
        g.autotune([q])
    assert e.value.code == P.SGM_EINVAL
    g.close()
