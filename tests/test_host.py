"""CPU-only checks of the library: it loads, exports every declared symbol,
and its host logic (query checks, query plan, CSR checks) behaves as the
thesis describes. No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1807_08804_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "sgm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sgm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = declared_functions()
    assert "sgm_load_graph" in names and "sgm_match_batch" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P.EXPORTS)


def plan(n, vlabel, vpin, edges, V=1000, type_freq=None):
    tf = np.full(64, 10) if type_freq is None else type_freq
    return P.sgm_plan_query(n, vlabel, vpin, [e[0] for e in edges], [e[1] for e in edges],
                            [e[2] for e in edges], V, tf)


def err(n, vlabel, vpin, edges, V=1000):
    with pytest.raises(P.SGMError) as e:
        plan(n, vlabel, vpin, edges, V)
    return e.value.code


def test_query_checks():
    assert err(2, [-1, -1], [-1, -1], [(0, 0, -1)]) == P.SGM_EINVAL          # self-loop
    assert err(3, [-1] * 3, [-1] * 3, [(0, 1, -1)]) == P.SGM_EINVAL           # disconnected
    assert err(2, [-1, -1], [-1, -1], [(0, 1, 2), (0, 1, 2)]) == P.SGM_EINVAL  # duplicate
    assert err(2, [-1, -1], [5000, -1], [(0, 1, -1)]) == P.SGM_EINVAL         # pin out of range
    assert err(2, [-1, -1], [-1, -1], [(0, 2, -1)]) == P.SGM_EINVAL           # bad index
    assert err(2, [-2, -1], [-1, -1], [(0, 1, -1)]) == P.SGM_EINVAL           # bad label
    assert err(17, [-1] * 17, [-1] * 17, [(i, i + 1, -1) for i in range(16)]) == P.SGM_EUNSUPPORTED
    # same pair, two relations, both directions: allowed
    plan(2, [-1, -1], [-1, -1], [(0, 1, 2), (0, 1, 3), (1, 0, -1)])


def check_tree(p, n, edges):
    # parents form a spanning tree rooted at visit_order[0] whose parent edges
    # join each vertex to its parent
    root = p["visit_order"][0]
    assert p["parent"][root] == -1
    assert sorted(p["init_order"]) == list(range(n))
    assert p["init_order"][0] == root
    for u in range(n):
        if u == root:
            continue
        par, e = p["parent"][u], p["parent_edge"][u]
        assert {edges[e][0], edges[e][1]} == {u, par}
        assert par in p["visit_order"]
        # the parent entered the tree before u
        assert p["init_order"].index(par) < p["init_order"].index(u)
    # the expanded vertices are exactly the tree's internal vertices
    internal = {p["parent"][u] for u in range(n) if p["parent"][u] >= 0}
    assert internal == set(p["visit_order"]) or n == 1


def test_plan_prefers_pinned_vertex_of_max_degree():
    # star centre 0 (degree 3) pinned, leaf 3 pinned: centre first
    edges = [(0, 1, -1), (0, 2, -1), (3, 0, -1), (1, 2, -1)]
    p = plan(4, [1, 1, 1, 1], [7, -1, -1, 9], edges)
    assert p["visit_order"][0] == 0
    check_tree(p, 4, edges)


def test_plan_starts_at_concept_node_of_max_degree():
    # concept nodes 0 and 1 (degree 2 each) are adjacent, concept node 4 has
    # degree 3: the edge rule would start at edge (0, 1) (f sum 4 > 3), the
    # commonsense rule starts at the concept node of maximum degree, 4
    edges = [(0, 1, -1), (0, 2, -1), (1, 3, -1), (4, 2, -1), (4, 3, -1), (4, 5, -1)]
    p = plan(6, [-1] * 6, [10, 11, -1, -1, 12, -1], edges)
    assert p["visit_order"][0] == 4
    check_tree(p, 6, edges)
    # ties: the lower index
    p = plan(6, [-1] * 6, [10, 11, -1, -1, -1, -1], edges)
    assert p["visit_order"][0] == 0


def test_plan_rank_by_degree_over_frequency():
    # unpinned: f(u) = deg(u) / freq(label); rare label wins
    tf = np.full(64, 100)
    tf[5] = 2
    edges = [(0, 1, -1), (1, 2, -1), (2, 3, -1)]
    p = plan(4, [1, 1, 1, 5], [-1] * 4, edges, type_freq=tf)
    # edge (2,3): f(2)=2/100, f(3)=1/2 -> largest sum; u = 3 (larger f)
    assert p["visit_order"][0] == 3
    check_tree(p, 4, edges)


def test_plan_next_vertex_reaches_most_new_vertices():
    # path 0-1-2 with a fan at 2 (2 -> 3,4,5); root pinned at 0
    edges = [(0, 1, -1), (1, 2, -1), (2, 3, -1), (2, 4, -1), (2, 5, -1)]
    p = plan(6, [-1] * 6, [4, -1, -1, -1, -1, -1], edges)
    assert p["visit_order"] == [0, 1, 2]
    check_tree(p, 6, edges)


@pytest.mark.parametrize("seed", range(30))
def test_plan_random_queries_give_spanning_trees(seed):
    from tests.micro import random_query
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 17))
    q = random_query(rng, n, 4, 3, 1000, extra=4)
    edges = list(zip(q.esrc.tolist(), q.edst.tolist(), q.elabel.tolist()))
    p = plan(n, q.vlabel, q.vpin, edges, type_freq=rng.integers(1, 500, 64))
    check_tree(p, n, edges)


def test_load_graph_rejects_malformed_csr_before_touching_device():
    for row_ptr, col, rel, typ in [
        ([0, 1, 5], [1, 0], [0, 0], [0, 0]),       # row_ptr[V] != E
        ([0, 2, 1], [1, 0], [0, 0], [0, 0]),       # decreasing
        ([0, 1, 2], [1, 2], [0, 0], [0, 0]),       # col out of range
        ([0, 1, 2], [1, 0], [0, -1], [0, 0]),      # negative relation
        ([0, 1, 2], [1, 0], [0, 0], [0, -3]),      # negative type
    ]:
        with pytest.raises(P.SGMError) as e:
            P.sgm_load_graph(len(row_ptr) - 1, row_ptr[-1] if row_ptr[-1] <= 2 else 2, row_ptr,
                             col, rel, typ)
        assert e.value.code == P.SGM_EINVAL


def test_out_only_graph_options_checked_before_touching_device():
    """The outgoing-graph-only option runs on the multi-kernel path alone:
    asking for the persistent kernel with it, or a value other than 0/1, is
    refused before any device call."""
    for out_only, path in [(1, P.SGM_PATH_NARROW), (2, P.SGM_PATH_AUTO), (-1, P.SGM_PATH_WIDE)]:
        o = P.sgm_options()
        P.lib().sgm_default_options(ctypes.byref(o))
        o.out_only, o.path = out_only, path
        with pytest.raises(P.SGMError) as e:
            P.sgm_load_graph(2, 2, [0, 1, 2], [1, 0], [0, 0], [0, 0], o)
        assert e.value.code == P.SGM_EINVAL


def test_host_graph_option_checked_before_touching_device():
    """The host-memory graph option takes 0 or 1; other values are refused
    before any device call."""
    for hg in (2, -1):
        o = P.sgm_options()
        P.lib().sgm_default_options(ctypes.byref(o))
        o.host_graph = hg
        with pytest.raises(P.SGMError) as e:
            P.sgm_load_graph(2, 2, [0, 1, 2], [1, 0], [0, 0], [0, 0], o)
        assert e.value.code == P.SGM_EINVAL


def test_batch_packing_points_at_each_querys_arrays():
    """_pack_queries (one int32 block and one array of C query structs for a
    whole batch) gives every struct the counts and the five arrays of its
    query, read back through the struct's own addresses."""
    from tests.micro import random_query
    rng = np.random.default_rng(11)
    qs = [random_query(rng, int(rng.integers(1, 17)), 4, 3, 1000, extra=4) for _ in range(50)]
    arr, keep = P._pack_queries(qs)
    structs = ctypes.cast(arr.ctypes.data, ctypes.POINTER(P.sgm_query))
    for i, q in enumerate(qs):
        sq = structs[i]
        assert sq.n_vertices == q.n and sq.n_edges == len(q.esrc)
        for name, want in (("vertex_label", q.vlabel), ("vertex_pin", q.vpin),
                           ("edge_src", q.esrc), ("edge_dst", q.edst), ("edge_label", q.elabel)):
            if len(want) == 0:
                continue
            got = np.ctypeslib.as_array(ctypes.cast(getattr(sq, name), ctypes.POINTER(ctypes.c_int32)),
                                        (len(want),))
            assert np.array_equal(got, want), (i, name)
    with pytest.raises(ValueError):
        bad = random_query(rng, 3, 4, 3, 1000)
        bad.vpin = bad.vpin[:1]
        P._pack_queries([bad])


def test_strerror():
    assert P.sgm_strerror(P.SGM_ETOOBIG)
    assert P.sgm_strerror(12345) == "unknown error"


def test_query_marshalling_points_at_the_arrays():
    """The binding packs a query's five arrays into one int32 block; every
    pointer of the C struct must address its own array."""

    def read(addr, k):
        return list((ctypes.c_int32 * k).from_address(addr)) if k else []

    cases = [(3, [1, -1, 7], [-1, 5, -1], [0, 1], [1, 2], [4, -1]),
             (1, [2], [-1], [], [], []),
             (4, np.array([0, 1, 2, 3], np.int64), [9, -1, -1, -1], [0, 1, 2, 3, 0],
              [1, 2, 3, 0, 2], [0, 1, 2, 3, -1])]
    for n, vl, vp, es, ed, el in cases:
        q, keep = P._make_query(n, vl, vp, es, ed, el)
        assert q.n_vertices == n and q.n_edges == len(es)
        assert read(q.vertex_label, n) == [int(x) for x in vl]
        assert read(q.vertex_pin, n) == [int(x) for x in vp]
        assert read(q.edge_src, len(es)) == list(es)
        assert read(q.edge_dst, len(es)) == list(ed)
        assert read(q.edge_label, len(es)) == list(el)
    with pytest.raises(ValueError):
        P._make_query(2, [0, 0], [-1], [0], [1], [0])
    with pytest.raises(ValueError):
        P._make_query(2, [0, 0], [-1, -1], [0], [1, 0], [0])


def test_default_tuning_matches_the_header():
    """sgm_default_tuning fills the defaults sgm.h documents (no device)."""
    t = P.sgm_tuning()
    P.lib().sgm_default_tuning(ctypes.byref(t))
    assert {k: getattr(t, k) for k in P.TUNING_FIELDS} == dict(
        slots=512, group_lanes=64, wg_rows=8192, join_policy=0, help_items=1024, helpers=64,
        help_wait=0)
    header = open(os.path.join(os.path.dirname(__file__), "..", "include", "sgm.h")).read()
    assert "help_items 1024, helpers 64,\n * help_wait 0." in header


def test_traffic_record_hash_follows_code_only():
    """The kernel-source hash that guards recorded counter traffic ignores
    comments and blank lines but not code."""
    from paper_1807_08804_amd import prof_summary as ps
    base = {rel: "int f(int x) {\n    return x + 1;\n}\n" for rel in ps.KERNEL_SOURCES}
    h0 = ps.kernel_source_hash(lambda rel: base[rel])
    noted = dict(base)
    first = ps.KERNEL_SOURCES[0]
    noted[first] = "// a note\n/* a block\n   comment */\n" + base[first].replace(
        "return x + 1;", "return x + 1;  // trailing note") + "\n\n"
    assert ps.kernel_source_hash(lambda rel: noted[rel]) == h0
    changed = dict(base)
    changed[first] = base[first].replace("x + 1", "x + 2")
    assert ps.kernel_source_hash(lambda rel: changed[rel]) != h0
    assert ps.kernel_source_hash() == ps.kernel_source_hash(
        lambda rel: open(os.path.join(os.path.dirname(ps.__file__), rel)).read())


def _est(n, vl, vp, es, ed, el, V, tf, rf):
    return P.sgm_estimate_query(n, vl, vp, es, ed, el, V, tf, rf)


def test_admission_estimate_closed_forms():
    """The served form's admission estimate (host only) on cases with a
    closed form: one typed vertex holds its type's count of rows; an
    unlabelled one-edge query holds V rows, then E (two columns); a pinned
    root starts from one row."""
    V, tf, rf = 1000, [600, 400], [3000, 1000]
    E = sum(rf)
    bitmap = 8 * ((V + 63) // 64)
    assert _est(1, [1], [-1], [], [], [], V, tf, rf) == bitmap + 4 * 400
    assert _est(2, [-1, -1], [-1, -1], [0], [1], [-1], V, tf, rf) == 2 * bitmap + 4 * V + 8 * E
    # relation 1 from a pinned vertex: 1 row, then 1000 / V per vertex, all types
    assert _est(2, [-1, -1], [5, -1], [0], [1], [1], V, tf, rf) == 2 * bitmap + 4 + 8
    # the typed vertex (rank 1/600 > 1/V) is the plan's root: 600 rows, then
    # 600 * (E / V) * (V / V) over the variable edge
    got = _est(2, [-1, 0], [-1, -1], [0], [1], [-1], V, tf, rf)
    assert got == 2 * bitmap + 4 * 600 + 8 * 600 * E // V


@pytest.mark.parametrize("seed", range(5))
def test_admission_estimate_monotone_in_edge_labels(seed):
    """Edge labels do not change the plan (ranks use degrees and type
    frequencies), so giving a variable edge the rarest relation never raises
    the estimate, and the estimate never falls below the bitmaps."""
    from tests.micro import random_query
    rng = np.random.default_rng(seed)
    V, tf, rf = 5000, [1000, 1500, 2500], [8000, 3000, 1000]
    for _ in range(20):
        q = random_query(rng, int(rng.integers(1, 9)), 3, 3, V)
        base = _est(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel, V, tf, rf)
        assert base >= q.n * 8 * ((V + 63) // 64)
        for i in range(len(q.esrc)):
            dup = any(q.esrc[j] == q.esrc[i] and q.edst[j] == q.edst[i] and q.elabel[j] == 2
                      for j in range(len(q.esrc)))
            if q.elabel[i] < 0 and not dup:
                el = list(q.elabel)
                el[i] = 2
                assert _est(q.n, q.vlabel, q.vpin, q.esrc, q.edst, el, V, tf, rf) <= base


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the public structs have the C layout of
    include/sgm.h (size and every field offset, from a C compiler)."""
    import subprocess
    structs = {"sgm_options": P.sgm_options, "sgm_query": P.sgm_query, "sgm_stats": P.sgm_stats,
               "sgm_result": P.sgm_result, "sgm_kstat": P.sgm_kstat, "sgm_tuning": P.sgm_tuning,
               "sgm_serve_options": P.sgm_serve_options, "sgm_serve_stats": P.sgm_serve_stats,
               "sgm_compress_options": P.sgm_compress_options,
               "sgm_compressed": P.sgm_compressed}
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sgm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", inc, "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        name, field, val = line.split()
        cls = structs[name]
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(val) == want, (name, field, int(val), want)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())
