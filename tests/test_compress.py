"""Multi-level graph compression (thesis Ch. 3, Sec. "Multi-level Graph
Compression"), checked on the CPU against what Def. 3.4-3.5 and Thm.
3.1-3.2 require of its output, on graphs with similar vertices
(kggen.twin_graph) and on random micro graphs. The compression is host code:
no device is touched."""
import ctypes

import numpy as np
import pytest

import kggen
import oracle
import paper_1807_08804_amd as P
from tests.micro import random_graph, random_query


@pytest.fixture(scope="module")
def twin_small():
    return kggen.twin_named("twin-small")


@pytest.fixture(scope="module")
def comp_small(twin_small):
    return P.Compressed.from_kg(twin_small)


def _edges(kg):
    src = np.repeat(np.arange(kg.V, dtype=np.int64), np.diff(kg.row_ptr))
    return src, kg.col.astype(np.int64), kg.rel.astype(np.int64)


def _dedup(src, dst, rel):
    k = np.unique(np.stack([src, dst, rel], 1), axis=0)
    return k[:, 0], k[:, 1], k[:, 2]


def test_mapping_lists_partition_the_vertices(twin_small, comp_small):
    c = comp_small
    assert c.n_original == twin_small.V and c.levels >= 1
    assert np.array_equal(np.sort(c.map_ids), np.arange(c.n_original))
    for x in range(c.n_vertices):
        m = c.map_ids[c.map_off[x]:c.map_off[x + 1]]
        assert len(m) >= 1 and np.all(np.diff(m) > 0)
        assert np.all(c.hyper_of[m] == x)
        assert np.all(twin_small.vtype[m] == c.type[x])  # one label per weighted vertex
    # every level shrinks the graph, and the last level is what is returned
    assert all(b <= a for a, b in zip(c.level_size, c.level_size[1:]))
    assert c.level_size[-1] == c.n_vertices + c.n_edges


def test_weights_bound_every_member(twin_small, comp_small):
    """Def. 3.4's weights as used by Def. 3.5: an entry (X -> Y, l) exists
    for every original l-edge from M(X) to M(Y), with a weight of at least
    the l-edges any one member of M(X) has into M(Y); and the entry weights
    summed bound each member's degree in both directions."""
    c = comp_small
    s, d, r = _dedup(*_edges(twin_small))
    hs, hd = c.hyper_of[s].astype(np.int64), c.hyper_of[d].astype(np.int64)
    wsrc = np.repeat(np.arange(c.n_vertices, dtype=np.int64), np.diff(c.row_ptr))
    R = int(max(r.max(), c.rel.max())) + 1
    W = np.int64(c.n_vertices)
    ent_key = (wsrc * W + c.col) * R + c.rel
    assert np.all(np.diff(ent_key) > 0)  # sorted, unique entries
    # per member: l-edges into each M(Y)
    key = (s * W + hd) * R + r
    uk, cnt = np.unique(key, return_counts=True)
    mem, hy, rl = uk // (W * R), (uk // R) % W, uk % R
    need = (c.hyper_of[mem].astype(np.int64) * W + hy) * R + rl
    pos = np.searchsorted(ent_key, need)
    assert np.all(pos < len(ent_key)) and np.all(ent_key[pos] == need)  # every edge has its entry
    assert np.all(c.weight[pos] >= cnt)
    outdeg = np.bincount(s, minlength=c.n_original)
    indeg = np.bincount(d, minlength=c.n_original)
    assert np.all(outdeg <= c.out_bound[c.hyper_of])
    assert np.all(indeg <= c.in_bound[c.hyper_of])


def _query_degrees(q):
    qout = [len({int(q.edst[e]) for e in range(q.m) if q.esrc[e] == u}) for u in range(q.n)]
    qin = [len({int(q.esrc[e]) for e in range(q.m) if q.edst[e] == u}) for u in range(q.n)]
    return qout, qin


@pytest.fixture(scope="module")
def twin_queries(twin_small):
    rng = np.random.Generator(np.random.PCG64(kggen.BASE_SEED + 900))
    return [kggen.draw_query(twin_small, rng, int(rng.integers(3, 8)),
                             ("path", "tree", "star")[i % 3], int(rng.integers(0, 3)))
            for i in range(30)]


def test_thm31_candidates_keep_their_weighted_vertex(twin_small, comp_small, twin_queries):
    """Thm. 3.1: if v is a candidate of u in G (label and degrees), the
    weighted vertex holding v is a candidate of u in G_w (Def. 3.5)."""
    c = comp_small
    outdeg = np.diff(twin_small.row_ptr)
    s, d, _ = _edges(twin_small)
    indeg = np.bincount(d, minlength=twin_small.V)
    for q in twin_queries:
        qout, qin = _query_degrees(q)
        for u in range(q.n):
            cand = (twin_small.vtype == q.vlabel[u]) & (outdeg >= qout[u]) & (indeg >= qin[u])
            if q.vpin[u] >= 0:
                only = np.zeros_like(cand)
                only[q.vpin[u]] = True
                cand &= only
            x = c.hyper_of[np.nonzero(cand)[0]]
            assert np.all(c.type[x] == q.vlabel[u])
            assert np.all(c.out_bound[x] >= qout[u]) and np.all(c.in_bound[x] >= qin[u])


def test_thm32_matches_map_onto_weighted_matches(twin_small, comp_small, twin_queries):
    """Thm. 3.2: every match of q in G, read through the mapping lists, is
    a match of q in G_w (labels, pins' weighted vertices and every query
    edge, as a homomorphism). So matching G_w and expanding loses none."""
    c = comp_small
    og = oracle.graph_from_kg(twin_small)
    wsrc = np.repeat(np.arange(c.n_vertices, dtype=np.int64), np.diff(c.row_ptr))
    ents = set(zip(wsrc.tolist(), c.col.tolist(), c.rel.tolist()))
    pairs = set(zip(wsrc.tolist(), c.col.tolist()))
    total = 0
    for q in twin_queries:
        rows = og.match_query(q)
        total += len(rows)
        for row in rows[:200]:
            h = c.hyper_of[row]
            for u in range(q.n):
                assert q.vlabel[u] < 0 or c.type[h[u]] == q.vlabel[u]
                assert q.vpin[u] < 0 or h[u] == c.hyper_of[q.vpin[u]]
            for e in range(q.m):
                a, b, lab = int(h[q.esrc[e]]), int(h[q.edst[e]]), int(q.elabel[e])
                assert ((a, b, lab) in ents) if lab >= 0 else ((a, b) in pairs)
    assert total > 0


@pytest.mark.parametrize("seed", range(6))
def test_micro_graph_compression_is_sound(seed):
    """Random micro graphs (repeated triples, self-loops, few types) at
    every threshold: the mapping lists partition the vertices and the
    weights bound every member's degrees."""
    rng = np.random.default_rng(1300 + seed)
    V = int(rng.integers(2, 60))
    mg = random_graph(rng, V, int(rng.integers(1, 5 * V)), n_types=2, n_rels=2)
    rp, col, rel, typ = mg.csr()
    for delta in (1.0, 0.5, 0.2):
        c = P.Compressed(rp, col, rel, typ, max_levels=4, delta=delta)
        assert np.array_equal(np.sort(c.map_ids), np.arange(V))
        s, d, _ = _dedup(mg.src.astype(np.int64), mg.dst.astype(np.int64), mg.rel.astype(np.int64))
        assert np.all(np.bincount(s, minlength=V) <= c.out_bound[c.hyper_of])
        assert np.all(np.bincount(d, minlength=V) <= c.in_bound[c.hyper_of])
        for x in range(c.n_vertices):
            m = c.map_ids[c.map_off[x]:c.map_off[x + 1]]
            assert np.all(typ[m] == c.type[x])
        # every original edge has an entry between the weighted vertices
        wsrc = np.repeat(np.arange(c.n_vertices), np.diff(c.row_ptr))
        ents = set(zip(wsrc.tolist(), c.col.tolist(), c.rel.tolist()))
        for a, b, r in zip(s.tolist(), d.tolist(), _dedup(mg.src.astype(np.int64),
                                                          mg.dst.astype(np.int64),
                                                          mg.rel.astype(np.int64))[2].tolist()):
            assert (int(c.hyper_of[a]), int(c.hyper_of[b]), r) in ents


def test_identical_neighbourhoods_merge_at_delta_one():
    """Two vertices of one type with the same entries (the thesis' v0, v1
    example) merge at delta = 1; a third of another type does not."""
    # 0 and 1: both -> 3 (rel 0) and <- 4 (rel 1); 2 the same but type 1
    src = [0, 1, 2, 4, 4, 4]
    dst = [3, 3, 3, 0, 1, 2]
    rel = [0, 0, 0, 1, 1, 1]
    typ = np.array([0, 0, 1, 2, 3], np.int32)
    order = np.argsort(src, kind="stable")
    rp = np.zeros(6, np.int32)
    np.cumsum(np.bincount(src, minlength=5), out=rp[1:])
    c = P.Compressed(rp, np.array(dst, np.int32)[order], np.array(rel, np.int32)[order], typ,
                     max_levels=1, delta=1.0)
    assert c.n_vertices == 4 and c.hyper_of[0] == c.hyper_of[1] != c.hyper_of[2]
    x = c.hyper_of[0]
    assert list(c.map_ids[c.map_off[x]:c.map_off[x + 1]]) == [0, 1]
    # the weighted vertex 4 -> {0, 1}: one edge per member, weight 1 + 1
    y = c.hyper_of[4]
    sl = slice(c.row_ptr[y], c.row_ptr[y + 1])
    got = dict(zip(zip(c.col[sl].tolist(), c.rel[sl].tolist()), c.weight[sl].tolist()))
    assert got[(int(x), 1)] == 2 and got[(int(c.hyper_of[2]), 1)] == 1
    assert c.in_bound[x] == 1 and c.out_bound[x] == 1


def test_compress_options_checked():
    rp = np.array([0, 1, 1], np.int32)
    col, rel, typ = np.array([1], np.int32), np.array([0], np.int32), np.array([0, 0], np.int32)
    for kw in (dict(delta=0.0), dict(delta=1.5), dict(max_levels=9), dict(max_partners=0),
               dict(target_ratio=-1.0)):
        with pytest.raises(P.SGMError) as e:
            P.Compressed(rp, col, rel, typ, **kw)
        assert e.value.code == P.SGM_EINVAL
    with pytest.raises(P.SGMError):
        P.Compressed(np.array([0, 2, 1], np.int32), col, rel, typ)
    c = P.Compressed(rp, col, rel, typ, max_levels=0)
    assert c.levels == 0 and c.n_vertices == 2
