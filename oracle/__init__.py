"""CPU oracle for exact subgraph matching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never imports, links
or calls it, and the two share no code.

The C file ``sgm_oracle.c`` holds the enumerator (definition of the result:
thesis Ch. 3, Def. 3.1 / Def. 3.2, see the file header). This module only
marshals numpy arrays through ctypes and compiles the C file on demand.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK, OR_EINVAL, OR_ENOMEM, OR_ETOOBIG, OR_EBUDGET = 0, -1, -2, -4, -6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O3)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-shared", "-fPIC",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_graph_build.restype = ctypes.c_void_p
        lib.oracle_graph_build.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, i32p]
        lib.oracle_graph_free.argtypes = [ctypes.c_void_p]
        lib.oracle_graph_num_edges.restype = ctypes.c_int64
        lib.oracle_graph_num_edges.argtypes = [ctypes.c_void_p]
        lib.oracle_match.restype = ctypes.c_int
        lib.oracle_match.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, i32p, i32p,
                                     i32p, i32p, i32p, ctypes.c_int64, ctypes.c_int,
                                     ctypes.POINTER(i32p), ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_match_budget.restype = ctypes.c_int
        lib.oracle_match_budget.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, i32p,
                                            i32p, i32p, i32p, i32p, ctypes.c_int64,
                                            ctypes.c_int64, ctypes.c_int,
                                            ctypes.POINTER(i32p), ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_plan.restype = ctypes.c_int
        lib.oracle_plan.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, i32p, i32p,
                                    i32p, i32p, i32p, i32p, i32p, i32p, i32p]
        lib.oracle_filter.restype = ctypes.c_int
        lib.oracle_filter.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, i32p, i32p,
                                      i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, u8p]
        lib.oracle_edge_candidates.restype = ctypes.c_int
        lib.oracle_edge_candidates.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                               i32p, i32p, i32p, u8p, i64p]
        _lib = lib
    return _lib


def _i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class OracleError(RuntimeError):
    def __init__(self, code, n_rows=0):
        super().__init__(f"oracle error {code}")
        self.code = code
        self.n_rows = n_rows


class Graph:
    """The oracle's own adjacency, built from a raw (src, dst, rel) triple
    list; duplicate triples collapse into one edge."""

    def __init__(self, V: int, src, dst, rel, vtype):
        lib = _load()
        self._keep = [_i32(src), _i32(dst), _i32(rel), _i32(vtype)]
        (s, sp), (d, dp), (r, rp), (t, tp) = self._keep
        if not (len(s) == len(d) == len(r)) or len(t) != V:
            raise ValueError("array lengths")
        self.V = int(V)
        self._h = lib.oracle_graph_build(int(V), int(len(s)), sp, dp, rp, tp)
        if not self._h:
            raise ValueError("invalid graph")
        self._keep = None
        self.E = int(lib.oracle_graph_num_edges(self._h))

    def __del__(self):
        if getattr(self, "_h", None):
            _load().oracle_graph_free(self._h)
            self._h = None

    def match(self, n, vlabel, vpin, esrc, edst, elabel, max_rows: int = -1,
              nthreads: int = 0, count_only: bool = False, max_steps: int = -1):
        """All matches as an [rows, n] int32 array in ascending lexicographic
        order (or the count if ``count_only``). ``max_steps`` bounds the
        candidate tests (OracleError with code OR_EBUDGET beyond it)."""
        lib = _load()
        (vl, vlp), (vp, vpp) = _i32(vlabel), _i32(vpin)
        (es, esp), (ed, edp), (el, elp) = _i32(esrc), _i32(edst), _i32(elabel)
        if len(vl) != n or len(vp) != n or not (len(es) == len(ed) == len(el)):
            raise ValueError("query array lengths")
        rows = ctypes.POINTER(ctypes.c_int32)()
        nrows = ctypes.c_int64(0)
        rc = lib.oracle_match_budget(self._h, int(n), int(len(es)), vlp, vpp, esp, edp, elp,
                                     int(max_rows), int(max_steps), int(nthreads),
                                     None if count_only else ctypes.byref(rows),
                                     ctypes.byref(nrows))
        if rc != OR_OK:
            raise OracleError(rc, nrows.value)
        if count_only:
            return int(nrows.value)
        k = int(nrows.value)
        out = np.empty((k, n), np.int32)
        if k:
            ctypes.memmove(out.ctypes.data, rows, k * n * 4)
        lib.oracle_free(rows)
        return out

    def match_query(self, q, **kw):
        """Same as :meth:`match` for a ``kggen.Query``-like object."""
        return self.match(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel, **kw)

    def _qargs(self, q):
        arrs = [_i32(q.vlabel), _i32(q.vpin), _i32(q.esrc), _i32(q.edst), _i32(q.elabel)]
        return arrs, [a[1] for a in arrs]

    def plan(self, q):
        """The query plan: dict of visit_order, parent, parent_edge,
        init_order."""
        arrs, ptrs = self._qargs(q)
        outs = [np.full(max(q.n, 1), -7, np.int32) for _ in range(4)]
        rc = _load().oracle_plan(self._h, int(q.n), int(len(q.esrc)), *ptrs,
                                 *[o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for o in outs])
        if rc != OR_OK:
            raise OracleError(rc)
        vo, par, pe, io = outs
        return dict(visit_order=[int(x) for x in vo[:q.n] if x >= 0], parent=par[:q.n].tolist(),
                    parent_edge=pe[:q.n].tolist(), init_order=[int(x) for x in io[:q.n] if x >= 0])

    def filter(self, q, rounds=1, reversed=1, low_conn=1):
        """Candidate sets after the filtering phase: [n][V] bool."""
        arrs, ptrs = self._qargs(q)
        out = np.zeros((q.n, self.V), np.uint8)
        rc = _load().oracle_filter(self._h, int(q.n), int(len(q.esrc)), *ptrs, int(rounds),
                                   int(reversed), int(low_conn),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        if rc != OR_OK:
            raise OracleError(rc)
        return out.astype(bool)

    def edge_candidates(self, q, cand):
        """Candidate-edge count of every query edge for candidate sets cand."""
        arrs, ptrs = self._qargs(q)
        c = np.ascontiguousarray(np.asarray(cand, np.uint8))
        ec = np.zeros(max(len(q.esrc), 1), np.int64)
        rc = _load().oracle_edge_candidates(self._h, int(q.n), int(len(q.esrc)), ptrs[2], ptrs[3],
                                            ptrs[4], c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                            ec.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        if rc != OR_OK:
            raise OracleError(rc)
        return ec[:len(q.esrc)]


def project_rows(rows: np.ndarray, cols) -> np.ndarray:
    """Projection of a full match table (thesis Ch. 3, Sec. "GpSense": only
    the matches of a subset of the query's nodes are wanted): the distinct
    tuples (f(u) for u in cols, cols in ascending order) over the rows,
    ascending lexicographic, as an [k, len(cols)] int32 array. Plain
    definition: the set of projected tuples, sorted."""
    cols = sorted(int(c) for c in cols)
    if len(rows) == 0:
        return np.empty((0, len(cols)), np.int32)
    sub = np.ascontiguousarray(np.asarray(rows, np.int32)[:, cols])
    return np.unique(sub, axis=0).astype(np.int32)


def graph_from_kg(kg) -> Graph:
    s, d, r = kg.edge_list()
    return Graph(kg.V, s, d, r, kg.vtype)
