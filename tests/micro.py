"""Seeded micro graphs and queries for tests (inputs only, no matching logic)
plus a brute-force enumerator written straight from the result definition
(thesis Ch. 3, Def. 3.2 with concept nodes and relation-labelled edges)."""
from __future__ import annotations

import itertools

import numpy as np


class MicroGraph:
    """Raw triples (may repeat, may hold self-loops and multi-relation
    pairs) plus types; ``csr()`` gives an unsorted out-CSR with repeats."""

    def __init__(self, V, src, dst, rel, vtype):
        self.V = V
        self.src = np.asarray(src, np.int32)
        self.dst = np.asarray(dst, np.int32)
        self.rel = np.asarray(rel, np.int32)
        self.vtype = np.asarray(vtype, np.int32)

    def csr(self):
        order = np.argsort(self.src, kind="stable")
        cnt = np.bincount(self.src, minlength=self.V)
        row_ptr = np.zeros(self.V + 1, np.int32)
        np.cumsum(cnt, out=row_ptr[1:])
        return row_ptr, self.dst[order], self.rel[order], self.vtype

    def edge_set(self):
        return set(zip(self.src.tolist(), self.dst.tolist(), self.rel.tolist()))


class MicroQuery:
    def __init__(self, n, vlabel, vpin, esrc, edst, elabel):
        self.n = n
        self.vlabel = np.asarray(vlabel, np.int32)
        self.vpin = np.asarray(vpin, np.int32)
        self.esrc = np.asarray(esrc, np.int32)
        self.edst = np.asarray(edst, np.int32)
        self.elabel = np.asarray(elabel, np.int32)

    @property
    def m(self):
        return len(self.esrc)

    def __repr__(self):
        return (f"MicroQuery(n={self.n}, vlabel={self.vlabel.tolist()}, vpin={self.vpin.tolist()}, "
                f"edges={list(zip(self.esrc.tolist(), self.edst.tolist(), self.elabel.tolist()))})")


def random_graph(rng, V, E, n_types, n_rels, self_loops=True):
    src = rng.integers(0, V, E)
    dst = rng.integers(0, V, E)
    if not self_loops:
        dst = np.where(dst == src, (dst + 1) % V, dst)
    rel = rng.integers(0, n_rels, E)
    # repeat a few triples and add some multi-relation pairs
    k = max(1, E // 8)
    src = np.concatenate([src, src[:k], src[:k]])
    dst = np.concatenate([dst, dst[:k], dst[:k]])
    rel = np.concatenate([rel, rel[:k], (rel[:k] + 1) % n_rels])
    vtype = rng.integers(0, n_types, V)
    return MicroGraph(V, src, dst, rel, vtype)


def random_query(rng, n, n_types, n_rels, V, p_any_label=0.3, p_any_rel=0.3, p_pin=0.15,
                 extra=2):
    edges = []
    seen = set()
    for v in range(1, n):
        u = int(rng.integers(0, v))
        a, b = (u, v) if rng.random() < 0.5 else (v, u)
        r = -1 if rng.random() < p_any_rel else int(rng.integers(0, n_rels))
        edges.append((a, b, r))
        seen.add((a, b, r))
    for _ in range(int(rng.integers(0, extra + 1)) if n > 1 else 0):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        r = -1 if rng.random() < p_any_rel else int(rng.integers(0, n_rels))
        if (a, b, r) not in seen:
            edges.append((a, b, r))
            seen.add((a, b, r))
    vlabel = [-1 if rng.random() < p_any_label else int(rng.integers(0, n_types)) for _ in range(n)]
    vpin = [int(rng.integers(0, V)) if rng.random() < p_pin else -1 for _ in range(n)]
    perm = rng.permutation(len(edges)) if edges else []
    edges = [edges[i] for i in perm]
    return MicroQuery(n, vlabel, vpin, [e[0] for e in edges], [e[1] for e in edges],
                      [e[2] for e in edges])


def brute_force(g: MicroGraph, q: MicroQuery):
    """Every map f: {0..n-1} -> V that is injective, keeps types and pins,
    and sends every query edge onto some data triple (any relation for -1).
    Sorted list of tuples."""
    E = g.edge_set()
    pairs_any = set((s, d) for s, d, _ in E)
    out = []
    for f in itertools.product(range(g.V), repeat=q.n):
        if len(set(f)) != q.n:
            continue
        ok = True
        for u in range(q.n):
            if q.vlabel[u] >= 0 and g.vtype[f[u]] != q.vlabel[u]:
                ok = False
                break
            if q.vpin[u] >= 0 and f[u] != q.vpin[u]:
                ok = False
                break
        if not ok:
            continue
        for a, b, r in zip(q.esrc.tolist(), q.edst.tolist(), q.elabel.tolist()):
            if r < 0:
                if (f[a], f[b]) not in pairs_any:
                    ok = False
                    break
            elif (f[a], f[b], r) not in E:
                ok = False
                break
        if ok:
            out.append(tuple(f))
    return sorted(out)
