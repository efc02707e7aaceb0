"""Seeded synthetic inputs: power-law knowledge graphs and query graphs.

This module only *draws* inputs. It holds none of the matching method's
arithmetic (no candidate filter, no edge collection, no join): the GPU path
and the CPU oracle both receive the arrays produced here and nothing else.

Data graphs stand in for the commonsense knowledge graphs of the thesis
(Ch. 3, Sec. "Commonsense Knowledge as a Graph": triples become directed,
relation-labelled edges; Sec. "Performance Evaluation": SenticNet, Gowalla and
Enron, none of which ship here). Recipe, per graph:

* out-degrees: i.i.d. discrete power law P(d) ~ d^-2.1 on [1, V-1], drawn by
  inverse CDF, then corrected to exactly E edges (proportional scaling, then
  largest-remainder +-1, keeping 1 <= d <= V-1);
* destinations: d distinct uniform vertices other than the source (the graph
  is simple: no parallel (src, dst) pairs, no self-loops);
* vertex types: uniform over 64; edge relations: Zipf(1.2) over 32.

Queries are grown on the data graph itself (random walk, random tree, star,
or a tree plus extra data edges for cycles), keep each data vertex's type as
the query vertex label and each data edge's relation and direction, and pin
some vertices to their data vertex (concept nodes, Ch. 3 Sec. "Commonsense
Graph Transformation"). Because every query is a copy of a piece of the data
graph, it has at least one embedding.

A query may be accepted only when H(q), the number of homomorphisms of its
spanning tree under the label / pin / relation constraints, falls in a band;
H(q) is an upper bound on the embeddings of that tree and is used purely to
keep the sampled workloads enumerable.
"""
from __future__ import annotations

import dataclasses
import numpy as np

N_TYPES = 64
N_RELS = 32
DEG_EXPONENT = 2.1
ZIPF_S = 1.2
BASE_SEED = 180708804

# Graph sizes of the synthetic workloads: name -> (vertices, edges, seed offset)
GRAPHS = {
    "tiny": (2_000, 8_000, 0),
    "medium": (300_000, 1_600_000, 1),
    "large": (4_000_000, 20_000_000, 2),
}


@dataclasses.dataclass
class KG:
    """A directed, edge-labelled, vertex-typed graph in int32 CSR form.

    ``row_ptr[V+1]``, ``col[E]``, ``rel[E]``: out-adjacency, each row sorted by
    (dst, rel). ``vtype[V]``: vertex type. ``in_ptr``/``in_col``/``in_rel``:
    the same edges grouped by destination (used by the query generator only).
    """

    V: int
    E: int
    row_ptr: np.ndarray
    col: np.ndarray
    rel: np.ndarray
    vtype: np.ndarray
    in_ptr: np.ndarray | None = None
    in_col: np.ndarray | None = None
    in_rel: np.ndarray | None = None

    def src(self) -> np.ndarray:
        return np.repeat(np.arange(self.V, dtype=np.int32), np.diff(self.row_ptr))

    def edge_list(self):
        """(src, dst, rel) int32 triples, the form the oracle takes."""
        return self.src(), self.col, self.rel

    def type_members(self, t: int) -> np.ndarray:
        """Vertices of type t (ascending), from a cached index."""
        if getattr(self, "_tidx", None) is None:
            order = np.argsort(self.vtype, kind="stable").astype(np.int64)
            cnt = np.bincount(self.vtype, minlength=int(self.vtype.max()) + 1)
            off = np.zeros(len(cnt) + 1, np.int64)
            np.cumsum(cnt, out=off[1:])
            self._tidx = (order, off)
        order, off = self._tidx
        if t < 0 or t + 1 >= len(off):
            return order[:0]
        return order[off[t]:off[t + 1]]

    def ensure_in(self):
        if self.in_ptr is None:
            src = self.src()
            order = np.lexsort((self.rel, src, self.col))  # by dst, then src, then rel
            self.in_col = np.ascontiguousarray(src[order])
            self.in_rel = np.ascontiguousarray(self.rel[order])
            cnt = np.bincount(self.col, minlength=self.V)
            self.in_ptr = np.zeros(self.V + 1, np.int64)
            np.cumsum(cnt, out=self.in_ptr[1:])
        return self


@dataclasses.dataclass
class Query:
    """A query graph: ``n`` vertices, edges ``(src[i], dst[i], label[i])``.

    ``vlabel[u]`` is a vertex type or -1 (any type); ``vpin[u]`` a data vertex
    id (concept node) or -1 (variable node); ``elabel[i]`` a relation or -1
    (variable edge). ``walk`` is the data vertex each query vertex was grown
    from (a known embedding), kept for tests.
    """

    n: int
    vlabel: np.ndarray
    vpin: np.ndarray
    esrc: np.ndarray
    edst: np.ndarray
    elabel: np.ndarray
    walk: np.ndarray | None = None
    shape: str = ""

    @property
    def m(self) -> int:
        return int(len(self.esrc))

    def as_dict(self):
        return dict(n=self.n, vlabel=self.vlabel.tolist(), vpin=self.vpin.tolist(),
                    esrc=self.esrc.tolist(), edst=self.edst.tolist(),
                    elabel=self.elabel.tolist(), shape=self.shape,
                    walk=None if self.walk is None else self.walk.tolist())

    @staticmethod
    def from_dict(d):
        return Query(n=int(d["n"]), vlabel=np.asarray(d["vlabel"], np.int32),
                     vpin=np.asarray(d["vpin"], np.int32),
                     esrc=np.asarray(d["esrc"], np.int32),
                     edst=np.asarray(d["edst"], np.int32),
                     elabel=np.asarray(d["elabel"], np.int32),
                     walk=None if d.get("walk") is None else np.asarray(d["walk"], np.int64),
                     shape=d.get("shape", ""))


# --------------------------------------------------------------------------
# data graphs
# --------------------------------------------------------------------------

def _powerlaw_outdegrees(rng, V: int, E: int, alpha: float = DEG_EXPONENT,
                         dmax: int = 0) -> np.ndarray:
    d = np.arange(1, V, dtype=np.float64)
    cdf = np.cumsum(d ** -alpha)
    cdf /= cdf[-1]
    deg = np.searchsorted(cdf, rng.random(V), side="right").astype(np.int64) + 1
    dmax = V - 1 if dmax <= 0 else min(dmax, V - 1)
    np.minimum(deg, dmax, out=deg)
    # proportional correction to exactly E, then largest remainder +-1
    scaled = deg * (E / float(deg.sum()))
    base = np.clip(np.floor(scaled).astype(np.int64), 1, dmax)
    frac = scaled - np.floor(scaled)
    tie = rng.random(V)
    for _ in range(64):
        diff = int(E - base.sum())
        if diff == 0:
            break
        if diff > 0:
            elig = np.nonzero(base < dmax)[0]
            order = elig[np.lexsort((tie[elig], -frac[elig]))]
            take = order[:diff]
            base[take] += 1
        else:
            elig = np.nonzero(base > 1)[0]
            order = elig[np.lexsort((tie[elig], frac[elig]))]
            take = order[:-diff]
            base[take] -= 1
    if int(base.sum()) != E:
        raise RuntimeError("degree correction did not converge")
    return base


def _distinct_destinations(rng, V: int, deg: np.ndarray) -> np.ndarray:
    """For each source, deg[src] distinct uniform destinations != src,
    returned grouped by source and ascending within each source."""
    E = int(deg.sum())
    src = np.repeat(np.arange(V, dtype=np.int64), deg)
    dst = rng.integers(0, V - 1, size=E, dtype=np.int64)
    dst += dst >= src
    idx = np.arange(E, dtype=np.int64)  # edges still under duplicate check
    for _ in range(10_000):
        key = src[idx] * V + dst[idx]
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dupm = np.zeros(len(idx), bool)
        dupm[order[1:]] = sk[1:] == sk[:-1]
        nd = int(dupm.sum())
        if nd == 0:
            break
        bad = idx[dupm]
        new = rng.integers(0, V - 1, size=nd, dtype=np.int64)
        new += new >= src[bad]
        dst[bad] = new
        # re-check only the rows that held a duplicate
        rows = np.unique(src[bad])
        rp = np.zeros(V + 1, np.int64)
        np.cumsum(deg, out=rp[1:])
        starts, ends = rp[rows], rp[rows + 1]
        lens = ends - starts
        idx = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens) + np.arange(lens.sum())
    else:
        raise RuntimeError("destination sampling did not converge")
    # sort within rows
    order = np.lexsort((dst, src))
    return dst[order]


def make_graph(V: int, E: int, seed: int, n_types: int = N_TYPES, n_rels: int = N_RELS,
               alpha: float = DEG_EXPONENT, zipf_s: float = ZIPF_S, dmax: int = 0) -> KG:
    """Draw a seeded power-law knowledge graph (recipe in the module doc);
    dmax > 0 caps the out-degree (default V - 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = _powerlaw_outdegrees(rng, V, E, alpha, dmax)
    dst = _distinct_destinations(rng, V, deg)
    k = np.arange(1, n_rels + 1, dtype=np.float64)
    zcdf = np.cumsum(k ** -zipf_s)
    zcdf /= zcdf[-1]
    rel = np.searchsorted(zcdf, rng.random(E), side="right").astype(np.int32)
    np.minimum(rel, n_rels - 1, out=rel)
    vtype = rng.integers(0, n_types, size=V, dtype=np.int32)
    row_ptr = np.zeros(V + 1, np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    return KG(V=V, E=E, row_ptr=row_ptr.astype(np.int32), col=dst.astype(np.int32),
              rel=rel, vtype=vtype)


def named_graph(name: str) -> KG:
    V, E, off = GRAPHS[name]
    return make_graph(V, E, BASE_SEED + off)


# --------------------------------------------------------------------------
# queries
# --------------------------------------------------------------------------

def _out_row(g: KG, v: int):
    a, b = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
    return g.col[a:b], g.rel[a:b]


def _in_row(g: KG, v: int):
    a, b = int(g.in_ptr[v]), int(g.in_ptr[v + 1])
    return g.in_col[a:b], g.in_rel[a:b]


def _has_edge(g: KG, x: int, y: int):
    """Relation of data edge x->y, or None."""
    cols, rels = _out_row(g, x)
    i = int(np.searchsorted(cols, y))
    if i < len(cols) and cols[i] == y:
        return int(rels[i])
    return None


def _random_neighbour(g: KG, rng, x: int, exclude: set, tries: int = 32):
    """A uniformly drawn undirected neighbour of x not in ``exclude``, with the
    data edge joining them as (src, dst, rel); None if none found."""
    oc, orl = _out_row(g, x)
    ic, irl = _in_row(g, x)
    no, ni = len(oc), len(ic)
    tot = no + ni
    if tot == 0:
        return None
    for _ in range(tries):
        j = int(rng.integers(tot))
        if j < no:
            y, e = int(oc[j]), (x, int(oc[j]), int(orl[j]))
        else:
            y, e = int(ic[j - no]), (int(ic[j - no]), x, int(irl[j - no]))
        if y not in exclude:
            return y, e
    if tot <= 4096:  # exhaustive fallback for small rows
        cand = [(int(y), (x, int(y), int(r))) for y, r in zip(oc, orl) if int(y) not in exclude]
        cand += [(int(y), (int(y), x, int(r))) for y, r in zip(ic, irl) if int(y) not in exclude]
        if cand:
            return cand[int(rng.integers(len(cand)))]
    return None


def _grow(g: KG, rng, n: int, shape: str):
    """Grow n distinct data vertices and a spanning set of data edges."""
    for _attempt in range(1000):
        start = int(rng.integers(g.V))
        verts = [start]
        inset = {start}
        edges = []
        ok = True
        if shape == "star":
            oc, _ = _out_row(g, start)
            ic, _ = _in_row(g, start)
            if len(oc) + len(ic) < n - 1:
                continue
        while len(verts) < n:
            if shape == "path":
                x = verts[-1]
            elif shape == "star":
                x = start
            else:
                x = verts[int(rng.integers(len(verts)))]
            r = _random_neighbour(g, rng, x, inset)
            if r is None:
                if shape in ("path", "star"):
                    ok = False
                    break
                continue_tries = False
                for x2 in rng.permutation(verts):
                    r = _random_neighbour(g, rng, int(x2), inset)
                    if r is not None:
                        continue_tries = True
                        break
                if not continue_tries:
                    ok = False
                    break
            y, e = r
            verts.append(y)
            inset.add(y)
            edges.append(e)
        if ok:
            return verts, edges
    raise RuntimeError("could not grow a query")


def _extra_edges(g: KG, verts, edges):
    """All data edges among ``verts`` that are not already in ``edges``."""
    have = set((s, d) for s, d, _ in edges)
    out = []
    vs = set(verts)
    for x in verts:
        cols, rels = _out_row(g, x)
        if len(cols) > 4 * len(verts):
            for y in verts:
                if y != x and (x, y) not in have:
                    r = _has_edge(g, x, y)
                    if r is not None:
                        out.append((x, y, r))
        else:
            for y, r in zip(cols.tolist(), rels.tolist()):
                if y in vs and (x, y) not in have:
                    out.append((x, y, r))
    return out


def _to_query(g: KG, verts, edges, pins, shape) -> Query:
    idx = {v: i for i, v in enumerate(verts)}
    n = len(verts)
    vlabel = g.vtype[np.asarray(verts, np.int64)].astype(np.int32)
    vpin = np.full(n, -1, np.int32)
    for p in pins:
        vpin[p] = verts[p]
    es = np.asarray([idx[s] for s, _, _ in edges], np.int32)
    ed = np.asarray([idx[d] for _, d, _ in edges], np.int32)
    el = np.asarray([r for _, _, r in edges], np.int32)
    return Query(n=n, vlabel=vlabel, vpin=vpin, esrc=es, edst=ed, elabel=el,
                 walk=np.asarray(verts, np.int64), shape=shape)


def draw_query(g: KG, rng, n: int, shape: str, n_pins: int, n_cycles: int = 0) -> Query:
    """One query of ``n`` vertices grown on ``g`` (module doc), with ``n_pins``
    pinned vertices and, for shape "cyclic", ``n_cycles`` extra edges."""
    g.ensure_in()
    base = "tree" if shape == "cyclic" else shape
    for _ in range(10_000):
        verts, edges = _grow(g, rng, n, base)
        if n_cycles > 0:
            extra = _extra_edges(g, verts, edges)
            if len(extra) < n_cycles:
                continue
            pick = rng.choice(len(extra), size=n_cycles, replace=False)
            edges = edges + [extra[int(i)] for i in sorted(pick)]
        pins = sorted(rng.choice(n, size=n_pins, replace=False).tolist()) if n_pins else []
        return _to_query(g, verts, edges, pins, shape)
    raise RuntimeError("could not draw a query")


def draw_cyclic_dense(g: KG, rng, n: int, n_cycles: int, n_pins: int = 0,
                      max_tries: int = 2_000) -> Query:
    """A connected query of n vertices with n-1+n_cycles edges. Grows greedily
    towards vertices with the most data edges into the chosen set so that the
    cycles exist; cycles are sparse in these random graphs otherwise."""
    g.ensure_in()
    for _ in range(max_tries):
        start = int(rng.integers(g.V))
        verts = [start]
        inset = {start}
        edges = []
        fail = False
        while len(verts) < n:
            # sample frontier
            cand = {}
            for x in verts:
                for _k in range(8):
                    r = _random_neighbour(g, rng, x, inset, tries=4)
                    if r is not None:
                        cand.setdefault(r[0], r[1])
            if not cand:
                fail = True
                break
            ys = list(cand.keys())
            score = []
            for y in ys:
                s = 0
                for x in verts:
                    if _has_edge(g, x, y) is not None or _has_edge(g, y, x) is not None:
                        s += 1
                score.append(s)
            best = max(score)
            choices = [y for y, s in zip(ys, score) if s == best]
            y = choices[int(rng.integers(len(choices)))]
            verts.append(y)
            inset.add(y)
            edges.append(cand[y])
        if fail:
            continue
        extra = _extra_edges(g, verts, edges)
        if len(extra) < n_cycles:
            continue
        pick = rng.choice(len(extra), size=n_cycles, replace=False)
        edges = edges + [extra[int(i)] for i in sorted(pick)]
        pins = sorted(rng.choice(n, size=n_pins, replace=False).tolist()) if n_pins else []
        return _to_query(g, verts, edges, pins, "cyclic")
    raise RuntimeError("could not draw a cyclic query")


# --------------------------------------------------------------------------
# acceptance bound H(q)
# --------------------------------------------------------------------------

def _rel_matrix(g: KG, lab: int, fwd: bool):
    """Sparse 0/1 matrix M with (M h)(v) = sum of h(x) over the data edges
    v -> x (fwd) or x -> v (not fwd) with relation lab (-1: any), cached on
    the graph."""
    import scipy.sparse as sp
    cache = g.__dict__.setdefault("_relmat", {})
    key = (lab, fwd)
    if key not in cache:
        ptr, nb, rl = (g.row_ptr, g.col, g.rel) if fwd else (g.in_ptr, g.in_col, g.in_rel)
        ptr = np.asarray(ptr, np.int64)
        if lab >= 0:
            keep = rl == lab
            rows = np.repeat(np.arange(g.V, dtype=np.int64), np.diff(ptr))
            cnt = np.bincount(rows[keep], minlength=g.V)
            nptr = np.zeros(g.V + 1, np.int64)
            np.cumsum(cnt, out=nptr[1:])
            nb = nb[keep]
            ptr = nptr
        cache[key] = sp.csr_matrix((np.ones(len(nb)), np.asarray(nb, np.int64), ptr),
                                   shape=(g.V, g.V))
    return cache[key]


def tree_hom_bound(g: KG, q: Query) -> float:
    """H(q): homomorphisms of a BFS spanning tree of q (rooted at query vertex
    0) into g under the vertex-type, pin and relation constraints, by a sparse
    post-order dynamic program. Float64 (overflow gives inf). Assumes g has no
    parallel (src, dst) pairs, which holds for generated graphs."""
    g.ensure_in()
    n = q.n
    adj = [[] for _ in range(n)]
    for i in range(q.m):
        a, b = int(q.esrc[i]), int(q.edst[i])
        adj[a].append((b, i, True))    # a -> b: from a, follow out-edges
        adj[b].append((a, i, False))   # from b, follow in-edges
    parent = [-1] * n
    pedge = [None] * n
    order = [0]
    seen = {0}
    for u in order:
        for v, i, fwd in adj[u]:
            if v not in seen:
                seen.add(v)
                parent[v] = u
                pedge[v] = (i, fwd)
                order.append(v)
    if len(order) != n:
        raise ValueError("query not connected")

    def base_support(u):
        if q.vpin[u] >= 0:
            p = int(q.vpin[u])
            ok = q.vlabel[u] < 0 or g.vtype[p] == q.vlabel[u]
            return np.asarray([p] if ok else [], np.int64), np.ones(1 if ok else 0)
        if q.vlabel[u] >= 0:
            s = g.type_members(int(q.vlabel[u]))
        else:
            s = np.arange(g.V, dtype=np.int64)
        return s.astype(np.int64), np.ones(len(s))

    h = {}
    for u in reversed(order):
        sup, val = base_support(u)
        for c in range(n):
            if parent[c] != u:
                continue
            csup, cval = h.pop(c)
            i, fwd = pedge[c]
            lab = int(q.elabel[i])
            # edge u->c (fwd) : s(v) = sum over out-edges v->x of h_c(x)
            #   -> push h_c(x) along in-edges of x
            ptr, nb, rl = (g.in_ptr, g.in_col, g.in_rel) if fwd else (g.row_ptr, g.col, g.rel)
            if len(csup) == 0:
                sup, val = sup[:0], val[:0]
                break
            st = ptr[csup].astype(np.int64)
            ln = (ptr[csup + 1] - ptr[csup]).astype(np.int64)
            tot = int(ln.sum())
            if tot == 0:
                sup, val = sup[:0], val[:0]
                break
            if tot > g.V:
                # large push: one sparse matrix-vector product over the
                # relation's adjacency (integer sums below 2^53 are exact in
                # float64, so the result equals the gather path's)
                hc = np.zeros(g.V)
                hc[csup] = cval
                val = val * (_rel_matrix(g, lab, fwd) @ hc)[sup]
                keep = val > 0
                sup, val = sup[keep], val[keep]
                continue
            eidx = np.repeat(st - np.concatenate(([0], np.cumsum(ln)[:-1])), ln) + np.arange(tot)
            w = np.repeat(cval, ln)
            tgt = nb[eidx].astype(np.int64)
            if lab >= 0:
                keep = rl[eidx] == lab
                tgt, w = tgt[keep], w[keep]
            if len(tgt) == 0:
                sup, val = sup[:0], val[:0]
                break
            if len(tgt) * 8 > g.V:
                dense = np.bincount(tgt, weights=w, minlength=g.V)
                val = val * dense[sup]
            else:
                ut, inv = np.unique(tgt, return_inverse=True)
                sv = np.bincount(inv, weights=w)
                pos = np.searchsorted(ut, sup)
                pos[pos >= len(ut)] = 0
                hitm = ut[pos] == sup
                val = np.where(hitm, val * sv[pos], 0.0)
            keep = val > 0
            sup, val = sup[keep], val[keep]
        h[u] = (sup, val)
    return float(h[0][1].sum()) if len(h[0][1]) else 0.0


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def tiny_query(g: KG, seed: int = BASE_SEED + 100) -> Query:
    """One 4-vertex, 4-edge query (one cycle) with one pinned vertex."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return draw_cyclic_dense(g, rng, 4, 1, n_pins=1)


def medium_queries(g: KG, count: int = 100, seed: int = BASE_SEED + 1 + 100,
                   hmax: float = 1e7):
    """Random-walk queries of 6..10 vertices, half paths and half trees, 0..2
    pinned vertices, accepted when H(q) <= hmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    rejected = 0
    while len(out) < count:
        n = int(rng.integers(6, 11))
        shape = "path" if len(out) % 2 == 0 else "tree"
        pins = int(rng.integers(0, 3))
        q = draw_query(g, rng, n, shape, pins)
        if tree_hom_bound(g, q) <= hmax:
            out.append(q)
        else:
            rejected += 1
    return out, rejected


def batch_queries(g: KG, count: int = 1024, seed: int = BASE_SEED + 3 + 100,
                  hmax: float = 1e6):
    """Mixed batch on the large graph: sizes uniform in 3..16, shapes in equal
    shares (path, star, tree, cyclic with 1-3 extra edges), pinned fraction per
    query uniform in [0, 0.5]; accepted when H(q) <= hmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = ("path", "star", "tree", "cyclic")
    out, rejected = [], 0
    while len(out) < count:
        shape = shapes[len(out) % 4]
        n = int(rng.integers(3, 17))
        pins = int(round(rng.random() * 0.5 * n))
        try:
            if shape == "cyclic":
                cyc = min(int(rng.integers(1, 4)), max(1, n - 2))
                q = draw_cyclic_dense(g, rng, n, cyc, n_pins=pins)
            else:
                q = draw_query(g, rng, n, shape, pins)
        except RuntimeError:
            rejected += 1
            continue
        if tree_hom_bound(g, q) <= hmax:
            out.append(q)
        else:
            rejected += 1
    return out, rejected


def serve_queries(g: KG, count: int, seed: int = BASE_SEED + 4 + 100, hmax: float = 1e6):
    """Served stream: 3..12-vertex walk queries (a tree plus 0 or 1 extra
    edge), 0..2 pinned vertices; accepted when H(q) <= hmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, rejected = [], 0
    while len(out) < count:
        n = int(rng.integers(3, 13))
        pins = min(n, int(rng.integers(0, 3)))
        try:
            if rng.random() < 0.5:
                q = draw_cyclic_dense(g, rng, n, 1, n_pins=pins)
            else:
                q = draw_query(g, rng, n, "tree", pins)
        except RuntimeError:
            rejected += 1
            continue
        if tree_hom_bound(g, q) <= hmax:
            out.append(q)
        else:
            rejected += 1
    return out, rejected


# Size / degree sweeps and graph-size scaling (thesis Ch. 3, Sec.
# "Comparison with state-of-the-art CPU algorithms": query graphs of 6..14
# vertices, and average degrees 8..24 at 10 query vertices; Sec. "Scalability
# Test": data graphs of growing vertex count, 6-vertex queries, kept in device
# or in host memory). Same generator as the named graphs; only V and E vary.
SWEEP_V = 1_000_000
SWEEP_DEGREES = (8, 12, 16, 20, 24)
SWEEP_SIZES = (6, 8, 10, 12, 14)
SWEEP_SIZE_DEGREE = 16
SCALE_VERTICES = (100_000, 1_000_000, 4_000_000, 16_000_000)
SCALE_DEGREE = 5


SWEEP_DMAX_DIV = 32  # out-degree cap V / 32: keeps the densest sweep graphs simple to draw


def sweep_graph(avg_degree: int, V: int = SWEEP_V) -> KG:
    """Power-law graph of V vertices and avg_degree * V edges."""
    return make_graph(V, avg_degree * V, BASE_SEED + 10 + avg_degree, dmax=V // SWEEP_DMAX_DIV)


def scale_graph(V: int) -> KG:
    """Power-law graph of V vertices and SCALE_DEGREE * V edges."""
    return make_graph(V, SCALE_DEGREE * V, BASE_SEED + 40 + V % 997, dmax=V // SWEEP_DMAX_DIV)


def sweep_queries(g: KG, n: int, count: int, seed: int, hmax: float = 1e6,
                  p_any_vertex: float = 0.5, p_any_edge: float = 0.25):
    """``count`` queries of exactly ``n`` vertices: trees and trees with one
    extra data edge (a cycle) alternately, one pinned vertex (a concept
    node); every other vertex label is dropped to "any" with probability
    p_any_vertex and every edge label with probability p_any_edge, so that
    candidate sets and intermediate tables grow with the degree; accepted
    when H(q) <= hmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, rejected = [], 0
    while len(out) < count:
        try:
            if len(out) % 2:
                q = draw_cyclic_dense(g, rng, n, 1, n_pins=1)
            else:
                q = draw_query(g, rng, n, "tree", 1)
        except RuntimeError:
            rejected += 1
            continue
        anyv = (rng.random(q.n) < p_any_vertex) & (q.vpin < 0)
        q.vlabel = np.where(anyv, -1, q.vlabel).astype(np.int32)
        q.elabel = np.where(rng.random(q.m) < p_any_edge, -1, q.elabel).astype(np.int32)
        if tree_hom_bound(g, q) <= hmax:
            out.append(q)
        else:
            rejected += 1
    return out, rejected


# Graphs with similar vertices, for multi-level compression (thesis Ch. 3,
# Sec. "Multi-level Graph Compression": a commonsense knowledge graph has
# many concepts that share the same neighbours). Each round gives every
# vertex, with probability p_twin, a twin of its type that keeps each of its
# out-edges and each of its in-edges with probability p_keep; twins of twins
# come from later rounds.
def twin_graph(V: int, E: int, seed: int, rounds: int = 2, p_twin: float = 0.5,
               p_keep: float = 0.9) -> KG:
    base = make_graph(V, E, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    src = np.repeat(np.arange(base.V, dtype=np.int64), np.diff(base.row_ptr))
    dst = base.col.astype(np.int64)
    rel = base.rel.astype(np.int64)
    vtype = base.vtype.astype(np.int32)
    n = base.V
    for _ in range(rounds):
        tw = np.nonzero(rng.random(n) < p_twin)[0]
        new_id = np.full(n, -1, np.int64)
        new_id[tw] = n + np.arange(len(tw))
        # out-edges of the twinned vertices, then their in-edges
        mo = (new_id[src] >= 0) & (rng.random(len(src)) < p_keep)
        mi = (new_id[dst] >= 0) & (rng.random(len(src)) < p_keep)
        src, dst, rel = (np.concatenate((src, new_id[src[mo]], src[mi])),
                         np.concatenate((dst, dst[mo], new_id[dst[mi]])),
                         np.concatenate((rel, rel[mo], rel[mi])))
        vtype = np.concatenate((vtype, vtype[tw]))
        n += len(tw)
    order = np.lexsort((rel, dst, src))
    src, dst, rel = src[order], dst[order], rel[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return KG(V=n, E=len(dst), row_ptr=row_ptr.astype(np.int32), col=dst.astype(np.int32),
              rel=rel.astype(np.int32), vtype=vtype)


TWIN_GRAPHS = {"twin-small": (20_000, 80_000, 60), "twin-medium": (300_000, 1_600_000, 61),
               "twin-large": (2_000_000, 10_000_000, 62)}


def twin_named(name: str) -> KG:
    V, E, off = TWIN_GRAPHS[name]
    return twin_graph(V, E, BASE_SEED + off)


def twin_queries(kg: KG, count: int, seed: int, hmax: float = 2e5):
    """Queries of 2..8 vertices on a twin graph: paths, trees and stars with
    0..2 pins, and every fourth a cycle with one pin; every fifth has
    vertex labels dropped to "any" with probability 0.4 and edge labels with
    probability 0.3; accepted when H(q) <= hmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < count:
        i = len(out)
        n = int(rng.integers(2, 9))
        try:
            if i % 4 == 3:
                q = draw_cyclic_dense(kg, rng, max(n, 4), 1, n_pins=1)
            else:
                q = draw_query(kg, rng, n, ("path", "tree", "star")[i % 3], int(rng.integers(0, 3)))
        except RuntimeError:
            continue
        if i % 5 == 4:
            q.vlabel = np.where(rng.random(q.n) < 0.4, -1, q.vlabel).astype(np.int32)
            q.elabel = np.where(rng.random(q.m) < 0.3, -1, q.elabel).astype(np.int32)
        if tree_hom_bound(kg, q) <= hmax:
            out.append(q)
    return out


SWEEP_COUNT = 64  # queries per sweep point
SWEEP_RECIPE = ("sweep_queries(g, n, 64, seed=BASE_SEED+600+k) per sweep_points() entry k; "
                "p_any_vertex=0.5, p_any_edge=0.25, H <= 1e6")


def sweep_points():
    """The sweep workloads as (key, graph kind, graph parameter, query size):
    average degree 8..24 at 10 query vertices and 6..14 query vertices at
    degree 16 (each on a SWEEP_V-vertex graph), and 6-vertex queries on the
    SCALE_VERTICES graphs."""
    pts = [(f"degree/{d}", "sweep", d, 10) for d in SWEEP_DEGREES]
    pts += [(f"size/{n}", "sweep", SWEEP_SIZE_DEGREE, n) for n in SWEEP_SIZES]
    pts += [(f"scale/{v}", "scale", v, 6) for v in SCALE_VERTICES]
    return pts


def sweep_point_graph(kind: str, param: int) -> KG:
    return sweep_graph(param) if kind == "sweep" else scale_graph(param)


def load_sweep():
    """The stored sweep workloads (written by kggen/make_fixtures.py from
    ``sweep_points`` and ``sweep_queries``): key -> list of queries."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fixtures", "sweep.json")
    with open(path) as f:
        doc = json.load(f)
    if doc["recipe"] != SWEEP_RECIPE:
        raise RuntimeError("sweep.json was drawn from another recipe; rerun make_fixtures")
    return {k: [Query.from_dict(d) for d in v] for k, v in doc["points"].items()}


def poisson_arrivals(count: int, qps: float, seed: int = BASE_SEED + 4 + 200) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream of rate qps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


LARGE_CYCLIC_RECIPE = ("large_queries(named_graph('large'), 50, seed=BASE_SEED+102, "
                       "hmin=1e7, hmax=2e9, p_any=0.5)")


LARGE_BATCH_RECIPE = ("batch_queries(named_graph('large'), 1024, seed=BASE_SEED+103, "
                      "hmax=1e6)")
LARGE_SERVE_RECIPE = ("serve_queries(named_graph('large'), 512, seed=BASE_SEED+104, "
                      "hmax=1e6)")


def _load_fixture(name, recipe):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fixtures", name)
    with open(path) as f:
        doc = json.load(f)
    if doc["recipe"] != recipe:
        raise RuntimeError(f"{name} was drawn from another recipe; rerun make_fixtures")
    return [Query.from_dict(d) for d in doc["queries"]], int(doc.get("rejected", 0))


def load_large_cyclic():
    """The stored 50-query large-graph cyclic workload (written by
    kggen/make_fixtures.py from ``large_queries``)."""
    return _load_fixture("large_cyclic.json", LARGE_CYCLIC_RECIPE)[0]


TWIN_LARGE_RECIPE = "twin_queries(twin_named('twin-large'), 64, seed=BASE_SEED+930)"


def load_twin_large():
    """The stored 64 queries of the large graph with similar vertices
    (written by kggen/make_fixtures.py from ``twin_queries``)."""
    return _load_fixture("twin_large.json", TWIN_LARGE_RECIPE)[0]


def load_large_batch(count: int = 1024):
    """The stored 1,024-query mixed batch of the large graph (written by
    kggen/make_fixtures.py from ``batch_queries``; the first ``count``, which
    are what ``batch_queries(g, count)`` draws) and the rejection count."""
    qs, rej = _load_fixture("large_batch.json", LARGE_BATCH_RECIPE)
    if count > len(qs):
        raise ValueError(f"the stored batch holds {len(qs)} queries")
    return qs[:count], rej


def load_large_serve(count: int = 512):
    """The stored 512 served-stream queries of the large graph (written by
    kggen/make_fixtures.py from ``serve_queries``; the first ``count``)."""
    qs, rej = _load_fixture("large_serve.json", LARGE_SERVE_RECIPE)
    if count > len(qs):
        raise ValueError(f"the stored serve set holds {len(qs)} queries")
    return qs[:count], rej


def large_queries(g: KG, count: int = 50, seed: int = BASE_SEED + 2 + 100,
                  hmin: float = 1e7, hmax: float = 2e9, p_any: float = 0.5):
    """Large-graph queries: 8..16 vertices with 1..3 cycles and no pins; each
    vertex label and edge label is dropped to "any" with probability p_any so
    that intermediate tables grow; accepted when hmin <= H(q) <= hmax."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, rejected = [], 0
    while len(out) < count:
        n = int(rng.integers(8, 17))
        try:
            q = draw_cyclic_dense(g, rng, n, int(rng.integers(1, 4)))
        except RuntimeError:
            rejected += 1
            continue
        q.vlabel = np.where(rng.random(q.n) < p_any, -1, q.vlabel).astype(np.int32)
        q.elabel = np.where(rng.random(q.m) < p_any, -1, q.elabel).astype(np.int32)
        h = tree_hom_bound(g, q)
        if hmin <= h <= hmax:
            out.append(q)
        else:
            rejected += 1
    return out, rejected
