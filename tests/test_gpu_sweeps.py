"""Query-size / degree sweeps and the graph kept in host memory, against the
CPU oracle (thesis Ch. 3, Sec. "Comparison with state-of-the-art CPU
algorithms": 6..14 query vertices, average degree 8..24; Sec. "Scalability
Test": the data graph in device or in main memory). Bit-exact tables."""
import sys

import numpy as np
import pytest

import kggen
import oracle
import paper_1807_08804_amd as P
from tests.micro import random_graph, random_query

pytestmark = pytest.mark.gpu

PATHS = [P.SGM_PATH_AUTO, P.SGM_PATH_WIDE, P.SGM_PATH_NARROW]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(got, want, what):
    assert isinstance(got, np.ndarray), (what, got)
    assert got.shape == want.shape and np.array_equal(got, want), what


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", range(6))
def test_host_graph_micro(seed, path):
    """Micro graphs (repeated triples, self-loops, hub-free and tiny rows)
    kept in host memory: single queries and one batch equal the oracle."""
    rng = np.random.default_rng(900 + seed)
    V = int(rng.integers(2, 40))
    mg = random_graph(rng, V, int(rng.integers(1, 4 * V)), n_types=3, n_rels=3)
    rp, col, rel, typ = mg.csr()
    say(f"case: host-graph micro seed={seed} path={path} V={V} E={len(col)}")
    g = P.Graph(rp, col, rel, typ, path=path, host_graph=1)
    og = oracle.Graph(V, mg.src, mg.dst, mg.rel, mg.vtype)
    qs = [random_query(rng, int(rng.integers(1, 6)), 3, 3, V, p_pin=0.15, extra=3)
          for _ in range(10)]
    want = [og.match_query(q) for q in qs]
    for i, (q, w) in enumerate(zip(qs, want)):
        try:
            same(g.match_query(q), w, i)
        except P.SGMError as e:
            assert path == P.SGM_PATH_NARROW and e.code == P.SGM_EUNSUPPORTED
    for i, (r, w) in enumerate(zip(g.match_batch(qs), want)):
        if isinstance(r, P.SGMError):
            assert path == P.SGM_PATH_NARROW and r.code == P.SGM_EUNSUPPORTED
        else:
            same(r, w, i)
    g.close()


def test_host_graph_medium(medium_kg, oracle_medium):
    """The medium graph in host memory: 40 walk queries one at a time, as
    one batch and with projection, equal the oracle."""
    qs, _ = kggen.medium_queries(medium_kg, 40)
    want = [oracle_medium.match_query(q) for q in qs]
    say("case: host-graph medium, one at a time and batched")
    g = P.Graph.from_kg(medium_kg, host_graph=1)
    for i, (q, w) in enumerate(zip(qs, want)):
        same(g.match_query(q), w, i)
    for i, (r, w) in enumerate(zip(g.match_batch(qs), want)):
        same(r, w, i)
    for i, (q, w) in enumerate(zip(qs[:10], want[:10])):
        keep = [0, q.n - 1]
        proj = np.unique(w[:, keep], axis=0) if len(w) else np.zeros((0, 2), np.int32)
        same(g.match(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel, project=keep), proj, i)
    g.close()


def test_host_graph_hub_rows():
    """Hub rows (the type-sorted copies of long adjacency rows) in host
    memory: a graph with a few 20,000-entry rows and queries that start at
    them, against the oracle."""
    rng = np.random.default_rng(77)
    V, hubs = 60_000, 4
    src = [np.repeat(np.arange(hubs), 20_000)]
    dst = [rng.integers(hubs, V, hubs * 20_000)]
    E2 = 120_000
    src.append(rng.integers(0, V, E2))
    dst.append(rng.integers(0, V, E2))
    src, dst = np.concatenate(src), np.concatenate(dst)
    rel = rng.integers(0, 3, len(src)).astype(np.int32)
    typ = rng.integers(0, 8, V).astype(np.int32)
    order = np.argsort(src, kind="stable")
    rp = np.zeros(V + 1, np.int32)
    np.cumsum(np.bincount(src, minlength=V), out=rp[1:])
    og = oracle.Graph(V, src.astype(np.int32), dst.astype(np.int32), rel, typ)
    g = P.Graph(rp, dst[order].astype(np.int32), rel[order], typ, host_graph=1)
    say("case: host-graph hub rows")
    for h in range(hubs):
        for lab in range(3):
            # typed neighbours of the hub over one relation, then any step
            q = dict(n=3, vlabel=[int(typ[h]), (3 * lab + h) % 8, -1], vpin=[h, -1, -1],
                     esrc=[0, 1], edst=[1, 2], elabel=[lab, -1])
            want = og.match(**q)
            same(g.match(**q), want, (h, lab))
    g.close()


@pytest.fixture(scope="module")
def small_sweep():
    """Sweep graphs at 40,000 vertices (the bench's recipe at a size the
    oracle finishes in seconds): degrees 8 and 24, queries of 6, 10 and 14
    vertices."""
    out = []
    for d in (8, 24):
        kg = kggen.sweep_graph(d, V=40_000)
        og = oracle.graph_from_kg(kg)
        for n in (6, 10, 14):
            qs, _ = kggen.sweep_queries(kg, n, 12, seed=kggen.BASE_SEED + 700 + 10 * d + n)
            out.append((d, n, kg, qs, [og.match_query(q) for q in qs]))
    return out


@pytest.mark.parametrize("host_graph", [0, 1])
def test_sweep_graphs(small_sweep, host_graph):
    """Size / degree sweep workloads: one batch per (degree, size) point and
    the same queries one at a time, graph in device or host memory."""
    for d, n, kg, qs, want in small_sweep:
        say(f"case: sweep degree={d} size={n} host_graph={host_graph}")
        g = P.Graph.from_kg(kg, host_graph=host_graph)
        for i, (r, w) in enumerate(zip(g.match_batch(qs), want)):
            same(r, w, (d, n, i))
        for i, (q, w) in enumerate(zip(qs[:4], want[:4])):
            same(g.match_query(q), w, (d, n, i))
        g.close()


def test_scale_graph_host_equals_device_and_oracle():
    """The smallest scalability graph (100,000 vertices, 500,000 edges) with
    64 six-vertex queries: host-memory and device-memory graphs give the
    oracle's tables."""
    kg = kggen.scale_graph(kggen.SCALE_VERTICES[0])
    qs, _ = kggen.sweep_queries(kg, 6, 64, seed=kggen.BASE_SEED + 800)
    og = oracle.graph_from_kg(kg)
    want = [og.match_query(q) for q in qs]
    for hg in (0, 1):
        say(f"case: scale graph V={kg.V} host_graph={hg}")
        g = P.Graph.from_kg(kg, host_graph=hg)
        for i, (r, w) in enumerate(zip(g.match_batch(qs), want)):
            same(r, w, (hg, i))
        g.close()


@pytest.fixture(scope="module")
def sweep_fixture():
    return kggen.load_sweep()


@pytest.mark.parametrize("degree", kggen.SWEEP_DEGREES)
def test_sweep_fixture_full_size(sweep_fixture, degree):
    """The stored sweep workloads at their full size (1M-vertex graphs):
    every query of the degree point, and on the degree-16 graph every query
    of the size points, as one batch each and the heaviest one alone (the
    one whose edge-candidate tables are built by many workgroups), against
    the oracle."""
    kg = kggen.sweep_graph(degree)
    og = oracle.graph_from_kg(kg)
    g = P.Graph.from_kg(kg)
    keys = [f"degree/{degree}"]
    if degree == kggen.SWEEP_SIZE_DEGREE:
        keys += [f"size/{n}" for n in kggen.SWEEP_SIZES]
    for key in keys:
        qs = sweep_fixture[key]
        want = [og.match_query(q) for q in qs]
        say(f"case: sweep fixture {key} (batch of {len(qs)})")
        for i, (r, w) in enumerate(zip(g.match_batch(qs), want)):
            same(r, w, (key, i))
        big = max(range(len(qs)), key=lambda i: (len(want[i]), -i))
        say(f"case: sweep fixture {key} query {big} alone ({len(want[big])} rows)")
        same(g.match_query(qs[big]), want[big], (key, big))
    g.close()


def test_sweep_shared_steps_forced(sweep_fixture):
    """Every step of at least 64 items shared (filter steps, long rows,
    edge-candidate tables and their long keys, join levels), 512 helper
    workgroups: the degree-16 and size-8 workloads still equal the oracle."""
    kg = kggen.sweep_graph(kggen.SWEEP_SIZE_DEGREE)
    og = oracle.graph_from_kg(kg)
    g = P.Graph.from_kg(kg)
    g.set_tuning(slots=16, group_lanes=64, wg_rows=2048, join_policy=0, help_items=64,
                 helpers=512, help_wait=0)
    for key in ("degree/16", "size/8"):
        qs = sweep_fixture[key]
        want = [og.match_query(q) for q in qs]
        say(f"case: sweep {key} with forced sharing")
        for i, (r, w) in enumerate(zip(g.match_batch(qs), want)):
            same(r, w, (key, i))
        for i in range(0, len(qs), 8):
            same(g.match_query(qs[i]), want[i], (key, i))
    g.close()


def test_host_graph_served_and_allocation_free(medium_kg, oracle_medium):
    """The served form and the allocation-free entry point on a graph kept
    in host memory: a served stream and single queries into a caller's
    buffer, against the oracle."""
    qs, _ = kggen.medium_queries(medium_kg, 30)
    want = [oracle_medium.match_query(q) for q in qs]
    g = P.Graph.from_kg(medium_kg, host_graph=1)
    say("case: host-graph served stream")
    srv = P.Server(g)
    lat, res = srv.replay(qs, kggen.poisson_arrivals(len(qs), 1000))
    srv.close()
    for i, (r, w) in enumerate(zip(res, want)):
        same(r, w, i)
    say("case: host-graph allocation-free entry point")
    for i, (q, w) in enumerate(zip(qs[:10], want[:10])):
        same(g.match_query_noalloc(q, max(len(w), 1)), w, i)
    g.close()
