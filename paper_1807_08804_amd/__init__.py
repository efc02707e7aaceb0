"""Python binding of the MI355X subgraph-matching library (``libsgm.so``).

Argument marshalling only: every step of a match runs in the library's HIP
kernels. The entry points keep the C names of ``include/sgm.h``
(``sgm_load_graph``, ``sgm_match_query``, ``sgm_match_batch``,
``sgm_free_result``, ...); :class:`Graph` wraps them for numpy callers.

Importing this package never compiles anything; ``build()`` does. If the
shared library is missing, every entry point raises ``RuntimeError``: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgm.so")

SGM_OK, SGM_EINVAL, SGM_ENOMEM, SGM_EDEVICE, SGM_ETOOBIG, SGM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SGM_MAX_QV, SGM_MAX_QE = 16, 64
SGM_SORTED, SGM_COUNT_ONLY = 0, 1
SGM_PATH_AUTO, SGM_PATH_WIDE, SGM_PATH_NARROW = 0, 1, 2
SGM_TRACE_CAP = 256
EVENT_NAMES = {1: "start", 2: "root", 3: "explore", 4: "refine", 5: "lists", 6: "edges",
               7: "order", 8: "level", 9: "sort", 10: "output", 11: "shared",
               12: "longrows"}
(SGM_K_CHECK, SGM_K_COLLECT, SGM_K_EXPLORE, SGM_K_REFINE, SGM_K_EC_COUNT, SGM_K_EC_WRITE,
 SGM_K_JOIN, SGM_K_SORT, SGM_K_OTHER, SGM_K_PERSIST, SGM_K_COUNT) = range(11)
KERNEL_NAMES = ["check", "collect", "explore", "refine", "ec_count", "ec_write", "join",
                "sort", "other", "persist"]

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class sgm_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("refine_rounds", ctypes.c_int32),
                ("refine_reversed", ctypes.c_int32), ("low_conn_degree", ctypes.c_int32),
                ("result_cap_rows", ctypes.c_int64), ("join_budget_bytes", ctypes.c_int64),
                ("profile", ctypes.c_int32), ("path", ctypes.c_int32),
                ("graphs", ctypes.c_int32), ("out_only", ctypes.c_int32),
                ("host_graph", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class sgm_query(ctypes.Structure):
    # the five int32 array pointers of the C struct, held as addresses
    _fields_ = [("n_vertices", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("vertex_label", ctypes.c_void_p), ("vertex_pin", ctypes.c_void_p),
                ("edge_src", ctypes.c_void_p), ("edge_dst", ctypes.c_void_p),
                ("edge_label", ctypes.c_void_p)]


class sgm_stats(ctypes.Structure):
    _fields_ = [("cand", ctypes.c_int64 * SGM_MAX_QV), ("ec", ctypes.c_int64 * SGM_MAX_QE),
                ("level_rows", ctypes.c_int64 * SGM_MAX_QV),
                ("join_order", ctypes.c_int32 * SGM_MAX_QV),
                ("visit_order", ctypes.c_int32 * SGM_MAX_QV),
                ("peak_rows", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("n_chunks", ctypes.c_int32), ("n_launches", ctypes.c_int32),
                ("ns_total", ctypes.c_int64), ("ns_filter", ctypes.c_int64),
                ("ns_collect", ctypes.c_int64), ("ns_join", ctypes.c_int64),
                ("ns_finish", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("phase_bytes", ctypes.c_int64 * 4),
                ("path", ctypes.c_int32), ("fallback", ctypes.c_int32)]


class sgm_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("n_rows", ctypes.c_int64), ("rows", _i32p), ("stats", sgm_stats)]


class sgm_serve_options(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("max_wait_ns", ctypes.c_int64), ("admission_cap_bytes", ctypes.c_int64),
                ("reserved", ctypes.c_int32 * 8)]


class sgm_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("admission_stalls", ctypes.c_int64),
                ("max_in_flight", ctypes.c_int64), ("wide_fallbacks", ctypes.c_int64)]


class sgm_tuning(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("group_lanes", ctypes.c_int32),
                ("wg_rows", ctypes.c_int32), ("join_policy", ctypes.c_int32),
                ("help_items", ctypes.c_int32), ("helpers", ctypes.c_int32),
                ("help_wait", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]

TUNING_FIELDS = ("slots", "group_lanes", "wg_rows", "join_policy", "help_items", "helpers",
                 "help_wait")


class sgm_compress_options(ctypes.Structure):
    _fields_ = [("max_levels", ctypes.c_int32), ("delta", ctypes.c_float * 8),
                ("target_ratio", ctypes.c_double), ("max_partners", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class sgm_compressed(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("n_original", ctypes.c_int32),
                ("n_edges", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("rel", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("type", ctypes.c_void_p),
                ("out_bound", ctypes.c_void_p), ("in_bound", ctypes.c_void_p),
                ("map_off", ctypes.c_void_p), ("map_ids", ctypes.c_void_p),
                ("hyper_of", ctypes.c_void_p), ("level_size", ctypes.c_int64 * 9)]


class sgm_kstat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("bytes_total", ctypes.c_double)]


EXPORTS = {
    "sgm_default_options": (None, [ctypes.POINTER(sgm_options)]),
    "sgm_load_graph": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p,
                                      ctypes.POINTER(sgm_options), ctypes.POINTER(ctypes.c_void_p)]),
    "sgm_match_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query), ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.POINTER(sgm_result))]),
    "sgm_match_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query), ctypes.c_int32,
                                       ctypes.c_uint32, ctypes.POINTER(ctypes.POINTER(sgm_result))]),
    "sgm_match_query_proj": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query),
                                            ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.POINTER(ctypes.POINTER(sgm_result))]),
    "sgm_match_batch_proj": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query),
                                            ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32,
                                            ctypes.c_uint32,
                                            ctypes.POINTER(ctypes.POINTER(sgm_result))]),
    "sgm_free_result": (None, [ctypes.POINTER(sgm_result)]),
    "sgm_free_graph": (None, [ctypes.c_void_p]),
    "sgm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sgm_last_error": (ctypes.c_char_p, []),
    "sgm_graph_info": (ctypes.c_int, [ctypes.c_void_p, _i32p, _i64p, _i32p, _i32p]),
    "sgm_trace_events": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i64p, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double)]),
    "sgm_kernel_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(sgm_kstat)]),
    "sgm_default_tuning": (None, [ctypes.POINTER(sgm_tuning)]),
    "sgm_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_tuning)]),
    "sgm_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_tuning)]),
    "sgm_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query), ctypes.c_int32,
                                    ctypes.c_int32, ctypes.POINTER(sgm_tuning)]),
    "sgm_reset_kernel_stats": (ctypes.c_int, [ctypes.c_void_p]),
    "sgm_plan_query": (ctypes.c_int, [ctypes.POINTER(sgm_query), ctypes.c_int32, _i64p,
                                      ctypes.c_int32, _i32p, _i32p, _i32p, _i32p]),
    "sgm_match_query_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query),
                                               ctypes.c_uint32, _i32p, ctypes.c_int64, _i64p]),
    "sgm_inject_fault": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "sgm_results_summary": (None, [ctypes.POINTER(ctypes.POINTER(sgm_result)), ctypes.c_int32,
                                   _i64p]),
    "sgm_estimate_query": (ctypes.c_int, [ctypes.POINTER(sgm_query), ctypes.c_int32, ctypes.c_int64,
                                          _i64p, ctypes.c_int32, _i64p, ctypes.c_int32, _i64p]),
    "sgm_inspect_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query), _i64p,
                                         ctypes.POINTER(_i32p), _i64p]),
    "sgm_free_ids": (None, [_i32p]),
    "sgm_default_serve_options": (None, [ctypes.POINTER(sgm_serve_options)]),
    "sgm_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_serve_options),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "sgm_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query), ctypes.c_uint32,
                                  ctypes.POINTER(ctypes.c_uint64)]),
    "sgm_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                ctypes.POINTER(ctypes.POINTER(sgm_result))]),
    "sgm_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_serve_stats)]),
    "sgm_server_destroy": (None, [ctypes.c_void_p]),
    "sgm_serve_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_query), _i64p,
                                        ctypes.c_int32, ctypes.c_uint32, _i64p,
                                        ctypes.POINTER(ctypes.POINTER(sgm_result))]),
    "sgm_default_compress_options": (None, [ctypes.POINTER(sgm_compress_options)]),
    "sgm_compress": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p,
                                    ctypes.POINTER(sgm_compress_options),
                                    ctypes.POINTER(ctypes.POINTER(sgm_compressed))]),
    "sgm_free_compressed": (None, [ctypes.POINTER(sgm_compressed)]),
    "sgm_load_compressed": (ctypes.c_int, [ctypes.POINTER(sgm_compressed),
                                           ctypes.POINTER(sgm_options),
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "sgm_attach_mapping": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(sgm_compressed)]),
    "sgm_match_compressed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(sgm_query), ctypes.c_uint32,
                                            ctypes.POINTER(ctypes.POINTER(sgm_result))]),
}

_lib = None


def build() -> str:
    """Compile libsgm.so (hipcc, gfx950)."""
    from . import builder
    return builder.build()


def lib():
    """The loaded ``libsgm.so`` (RuntimeError if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


class SGMError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        l = lib()
        msg = l.sgm_strerror(code).decode()
        detail = (l.sgm_last_error() or b"").decode()
        super().__init__(f"{where}: {msg} ({code}) {detail}".strip())
        self.code = code


def _arr(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(_i32p)


# --- C-named entry points -------------------------------------------------------------

def sgm_default_options() -> sgm_options:
    o = sgm_options()
    lib().sgm_default_options(ctypes.byref(o))
    return o


def sgm_load_graph(n_vertices, n_edges, row_ptr, col, rel, vtype, opts=None):
    """Returns an opaque graph handle (raises SGMError on failure)."""
    (rp, rpp), (c, cp), (r, rlp), (t, tp) = _arr(row_ptr), _arr(col), _arr(rel), _arr(vtype)
    h = ctypes.c_void_p()
    rc = lib().sgm_load_graph(int(n_vertices), int(n_edges), rpp, cp, rlp, tp,
                              ctypes.byref(opts) if opts is not None else None, ctypes.byref(h))
    if rc != SGM_OK:
        raise SGMError(rc, "sgm_load_graph")
    return h


def _make_query(n, vlabel, vpin, esrc, edst, elabel):
    """The C query struct and the buffer its pointers refer to (keep it alive
    as long as the struct is used): all five arrays in one int32 block."""
    nv, m = len(vlabel), len(esrc)
    if len(vpin) != nv or len(edst) != m or len(elabel) != m:
        raise ValueError("vertex arrays and edge arrays must have matching lengths")
    buf = np.concatenate((vlabel, vpin, esrc, edst, elabel)).astype(np.int32, copy=False)
    base = buf.__array_interface__["data"][0]
    q = sgm_query(int(n), m, base, base + 4 * nv, base + 8 * nv, base + 8 * nv + 4 * m,
                  base + 8 * nv + 8 * m)
    return q, buf


# numpy view of an array of sgm_query structs (two int32, five addresses)
_QUERY_DTYPE = np.dtype({"names": ["n", "m", "p0", "p1", "p2", "p3", "p4"],
                         "formats": [np.int32, np.int32] + [np.uint64] * 5,
                         "offsets": [sgm_query.n_vertices.offset, sgm_query.n_edges.offset,
                                     sgm_query.vertex_label.offset, sgm_query.vertex_pin.offset,
                                     sgm_query.edge_src.offset, sgm_query.edge_dst.offset,
                                     sgm_query.edge_label.offset],
                         "itemsize": ctypes.sizeof(sgm_query)})


def _pack_queries(queries):
    """The C query structs of a list of queries in one array, and the one
    int32 block their pointers refer to (keep both alive while in use):
    the same layout _make_query gives each query, built with whole-array
    operations."""
    nq = len(queries)
    arrs = []
    ext = arrs.extend
    for q in queries:
        ext((q.vlabel, q.vpin, q.esrc, q.edst, q.elabel))
    lens = np.fromiter(map(len, arrs), np.int64, count=5 * nq).reshape(nq, 5)
    if nq and ((lens[:, 1] != lens[:, 0]).any() or (lens[:, 3] != lens[:, 2]).any()
               or (lens[:, 4] != lens[:, 2]).any()):
        raise ValueError("vertex arrays and edge arrays must have matching lengths")
    buf = np.concatenate(arrs).astype(np.int32, copy=False) if nq else np.zeros(1, np.int32)
    starts = np.zeros((nq, 5), np.int64)
    flat = np.cumsum(lens.reshape(-1))
    starts.reshape(-1)[1:] = flat[:-1]
    base = buf.__array_interface__["data"][0]
    arr = np.zeros(max(nq, 1), _QUERY_DTYPE)
    arr["n"][:nq] = np.fromiter((q.n for q in queries), np.int32, count=nq)
    arr["m"][:nq] = lens[:, 2]
    for f in range(5):
        arr[f"p{f}"][:nq] = base + 4 * starts[:, f]
    return arr, buf


def sgm_match_query(g, q: sgm_query, flags: int = SGM_SORTED):
    out = ctypes.POINTER(sgm_result)()
    rc = lib().sgm_match_query(g, ctypes.byref(q), int(flags), ctypes.byref(out))
    return rc, out


def sgm_match_batch(g, qs, flags: int = SGM_SORTED, raw: bool = False):
    """qs: a list of sgm_query, or a packed array from _pack_queries. The
    results as a list of pointers, or (raw) the ctypes array itself."""
    n = len(qs)
    if isinstance(qs, np.ndarray):
        arr = qs.ctypes.data_as(ctypes.POINTER(sgm_query))
    else:
        arr = (sgm_query * max(n, 1))(*qs)
    outs = (ctypes.POINTER(sgm_result) * max(n, 1))()
    rc = lib().sgm_match_batch(g, arr, n, int(flags), outs)
    return rc, outs if raw else [outs[i] for i in range(n)]


def sgm_match_query_proj(g, q: sgm_query, project: int, flags: int = SGM_SORTED):
    out = ctypes.POINTER(sgm_result)()
    rc = lib().sgm_match_query_proj(g, ctypes.byref(q), int(project), int(flags), ctypes.byref(out))
    return rc, out


def sgm_match_batch_proj(g, qs, projects, flags: int = SGM_SORTED, raw: bool = False):
    n = len(qs)
    if isinstance(qs, np.ndarray):
        arr = qs.ctypes.data_as(ctypes.POINTER(sgm_query))
    else:
        arr = (sgm_query * max(n, 1))(*qs)
    pm = (ctypes.c_uint32 * max(n, 1))(*[int(x) for x in projects])
    outs = (ctypes.POINTER(sgm_result) * max(n, 1))()
    rc = lib().sgm_match_batch_proj(g, arr, pm, n, int(flags), outs)
    return rc, outs if raw else [outs[i] for i in range(n)]


def project_mask(project) -> int:
    """A projection as a bit mask: an int mask, or an iterable of query
    vertex indices."""
    if isinstance(project, (int, np.integer)):
        return int(project)
    m = 0
    for u in project:
        m |= 1 << int(u)
    return m


def sgm_free_result(r):
    lib().sgm_free_result(r)


def sgm_free_graph(g):
    lib().sgm_free_graph(g)


def sgm_strerror(code: int) -> str:
    return lib().sgm_strerror(code).decode()


def sgm_plan_query(n, vlabel, vpin, esrc, edst, elabel, n_vertices, type_freq):
    """Host-only query plan: dict with visit_order, parent, parent_edge,
    init_order (each trimmed of -1 padding where it is an order)."""
    q, keep = _make_query(n, vlabel, vpin, esrc, edst, elabel)
    tf = np.ascontiguousarray(np.asarray(type_freq, np.int64))
    outs = [np.full(SGM_MAX_QV, -7, np.int32) for _ in range(4)]
    rc = lib().sgm_plan_query(ctypes.byref(q), int(n_vertices), tf.ctypes.data_as(_i64p),
                              int(len(tf)), *[o.ctypes.data_as(_i32p) for o in outs])
    if rc != SGM_OK:
        raise SGMError(rc, "sgm_plan_query")
    vo, par, pe, io = outs
    return dict(visit_order=[int(x) for x in vo if x >= 0], parent=par[:n].tolist(),
                parent_edge=pe[:n].tolist(), init_order=[int(x) for x in io if x >= 0])


def sgm_estimate_query(n, vlabel, vpin, esrc, edst, elabel, n_vertices, type_freq, rel_freq):
    """Host-only admission estimate of the served form (bytes)."""
    q, keep = _make_query(n, vlabel, vpin, esrc, edst, elabel)
    tf = np.ascontiguousarray(np.asarray(type_freq, np.int64))
    rf = np.ascontiguousarray(np.asarray(rel_freq, np.int64))
    est = ctypes.c_int64(0)
    rc = lib().sgm_estimate_query(ctypes.byref(q), int(n_vertices), int(rf.sum()),
                                  tf.ctypes.data_as(_i64p), int(len(tf)), rf.ctypes.data_as(_i64p),
                                  int(len(rf)), ctypes.byref(est))
    if rc != SGM_OK:
        raise SGMError(rc, "sgm_estimate_query")
    return int(est.value)


# --- numpy convenience ----------------------------------------------------------------

class _ResultOwner:
    """Keeps one library result alive while numpy arrays view its rows."""

    __slots__ = ("r",)

    def __init__(self, r):
        self.r = r

    def __del__(self):
        r, self.r = self.r, None
        if r is not None:
            try:
                sgm_free_result(r)
            except Exception:  # interpreter shutdown
                pass


def _take_rows(r, n):
    """(row count, rows) of a result, taking ownership of r: rows is an
    (n_rows, n) int32 array viewing the library's buffer without a copy (the
    result is freed when the last view of it goes), or None for count-only
    results."""
    res = r.contents
    k = int(res.n_rows)
    if not res.rows or k == 0:
        out = np.empty((k, n), np.int32) if res.rows else None
        sgm_free_result(r)
        return k, out
    addr = ctypes.cast(res.rows, ctypes.c_void_p).value
    return k, np.asarray(_RowsView(addr, k, n, _ResultOwner(r)))


class _BatchOwner:
    """Keeps the results of one sgm_match_batch call alive while numpy
    arrays view any of their rows; frees them all after the last."""

    __slots__ = ("outs", "n")

    def __init__(self, outs, n):
        self.outs, self.n = outs, n

    def __del__(self):
        outs, self.outs = self.outs, None
        if outs is not None:
            try:
                for i in range(self.n):
                    sgm_free_result(outs[i])
            except Exception:
                pass


class _RowsView:
    """The array interface of a result's row table: numpy arrays made from
    it keep it (and so the library's result) alive."""
    __slots__ = ("__array_interface__", "_owner")

    def __init__(self, addr, k, n, owner):
        self.__array_interface__ = {"data": (addr, False), "shape": (k, n), "typestr": "<i4",
                                    "version": 3}
        self._owner = owner


def stats_dict(st: sgm_stats, n: int, m: int) -> dict:
    return dict(cand=list(st.cand[:n]), ec=list(st.ec[:m]), level_rows=list(st.level_rows[:n]),
                join_order=list(st.join_order[:n]),
                visit_order=[x for x in st.visit_order if x >= 0],
                peak_rows=st.peak_rows, peak_bytes=st.peak_bytes, n_chunks=st.n_chunks,
                n_launches=st.n_launches, ns_total=st.ns_total, ns_filter=st.ns_filter,
                ns_collect=st.ns_collect, ns_join=st.ns_join, ns_finish=st.ns_finish,
                device_bytes=st.device_bytes, phase_bytes=list(st.phase_bytes),
                path=st.path, fallback=st.fallback)


class Graph:
    """A data graph resident on the GPU."""

    def __init__(self, row_ptr, col, rel, vtype, **options):
        opts = sgm_default_options()
        for k, v in options.items():
            setattr(opts, k, v)
        row_ptr = np.asarray(row_ptr)
        self.V = int(len(row_ptr) - 1)
        self._h = sgm_load_graph(self.V, int(row_ptr[-1]), row_ptr, col, rel, vtype, opts)

    @classmethod
    def from_kg(cls, kg, **options):
        return cls(kg.row_ptr, kg.col, kg.rel, kg.vtype, **options)

    def close(self):
        if getattr(self, "_h", None):
            sgm_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        nv, ne, mo, mi = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        lib().sgm_graph_info(self._h, ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(mo),
                             ctypes.byref(mi))
        return dict(n_vertices=nv.value, n_edges=ne.value, max_out=mo.value, max_in=mi.value)

    def match(self, n, vlabel, vpin, esrc, edst, elabel, count_only=False, with_stats=False,
              project=None):
        """All matches as an [rows, n] int32 array (ascending lexicographic),
        or the count when ``count_only``; with ``project`` (vertex indices or
        a bit mask) the distinct projected tuples (sgm_match_query_proj).
        Raises SGMError on failure."""
        q, keep = _make_query(n, vlabel, vpin, esrc, edst, elabel)
        fl = SGM_COUNT_ONLY if count_only else SGM_SORTED
        if project is None:
            rc, r = sgm_match_query(self._h, q, fl)
        else:
            rc, r = sgm_match_query_proj(self._h, q, project_mask(project), fl)
        if rc != SGM_OK:
            err = SGMError(rc, "sgm_match_query")
            if r:
                err.n_rows = int(r.contents.n_rows)
                sgm_free_result(r)
            raise err
        st = None
        if with_stats:
            try:
                st = stats_dict(r.contents.stats, n, q.n_edges)
            except Exception:
                sgm_free_result(r)
                raise
        k, rows = _take_rows(r, int(r.contents.n_cols) if project is not None else n)
        out = k if count_only else rows
        return (out, st) if with_stats else out

    def match_query(self, q, **kw):
        return self.match(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel, **kw)

    def match_query_noalloc(self, q, rows_cap: int, count_only=False, out=None):
        """sgm_match_query_noalloc: the table in a caller-owned int32 buffer
        of rows_cap rows (``out``, allocated here when not given): returns
        the view of its first n_rows rows, or the count when count_only.
        Raises SGMError (with the exact n_rows on ETOOBIG)."""
        sq, keep = _make_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel)
        if out is None and not count_only:
            out = np.empty((max(int(rows_cap), 0), q.n), np.int32)
        ptr = None if count_only else out.ctypes.data_as(_i32p)
        n = ctypes.c_int64(0)
        rc = lib().sgm_match_query_noalloc(self._h, ctypes.byref(sq),
                                           SGM_COUNT_ONLY if count_only else SGM_SORTED, ptr,
                                           int(rows_cap), ctypes.byref(n))
        if rc != SGM_OK:
            err = SGMError(rc, "sgm_match_query_noalloc")
            err.n_rows = int(n.value)
            raise err
        k = int(n.value)
        return k if count_only else out.reshape(-1, q.n)[:k]

    def match_batch(self, queries, count_only=False, with_stats=False, projects=None):
        """Results (arrays, counts, or SGMError instances) for a list of
        kggen-style queries, through sgm_match_batch (sgm_match_batch_proj
        with ``projects``, one projection per query); with_stats=True also
        returns each member's statistics as a dict."""
        arr, keep = _pack_queries(queries)
        fl = SGM_COUNT_ONLY if count_only else SGM_SORTED
        if projects is None:
            rc, outs = sgm_match_batch(self._h, arr[:len(queries)], fl, raw=True)
        else:
            rc, outs = sgm_match_batch_proj(self._h, arr[:len(queries)],
                                            [project_mask(p) for p in projects], fl, raw=True)
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_match_batch")
        n = len(queries)
        # every member's (status, columns, rows, row address) in one call; the
        # batch's results are freed together once no table of it is in use
        info = np.zeros((max(n, 1), 4), np.int64)
        lib().sgm_results_summary(outs, n, info.ctypes.data_as(_i64p))
        owner = _BatchOwner(outs, n)
        stats = [stats_dict(outs[i].contents.stats, q.n, len(q.esrc))
                 for i, q in enumerate(queries)] if with_stats else []
        rows = info[:n].tolist()
        # tables that sit close together (one launch's row block) are sliced
        # from one view over their span instead of one view each
        flat, lo = None, 0
        if not count_only and n > 8:
            spans = [(a, a + 4 * k * c) for st, c, k, a in rows if st == SGM_OK and k and a]
            if spans:
                lo = min(a for a, _ in spans)
                hi = max(b for _, b in spans)
                used = sum(b - a for a, b in spans)
                if hi - lo <= 2 * used + (1 << 20):
                    flat = np.asarray(_RowsView(lo, (hi - lo) // 4, 1, owner)).reshape(-1)
        res = []
        for st, ncol, k, addr in rows:
            if st != SGM_OK:
                res.append(SGMError(st, "batch member"))
            elif count_only:
                res.append(k)
            elif k == 0 or not addr:
                res.append(np.empty((k, ncol), np.int32))
            elif flat is not None:
                o = (addr - lo) >> 2
                res.append(flat[o:o + k * ncol].reshape(k, ncol))
            else:
                res.append(np.asarray(_RowsView(addr, k, ncol, owner)))
        return (res, stats) if with_stats else res

    def inspect_query(self, q):
        """(candidate lists per query vertex, candidate-edge counts) after the
        filtering phase, through sgm_inspect_query."""
        sq, keep = _make_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel)
        counts = np.zeros(SGM_MAX_QV, np.int64)
        ec = np.zeros(SGM_MAX_QE, np.int64)
        ids = _i32p()
        rc = lib().sgm_inspect_query(self._h, ctypes.byref(sq), counts.ctypes.data_as(_i64p),
                                     ctypes.byref(ids), ec.ctypes.data_as(_i64p))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_inspect_query")
        total = int(counts.sum())
        flat = np.empty(total, np.int32)
        if total:
            ctypes.memmove(flat.ctypes.data, ids, total * 4)
        lib().sgm_free_ids(ids)
        lists, off = [], 0
        for u in range(q.n):
            lists.append(flat[off:off + counts[u]])
            off += counts[u]
        return lists, ec[:sq.n_edges]

    def trace(self, i=0):
        """Step events of query i of the last match call (profile=2): a list
        of (event name, microseconds since the query's start)."""
        buf = np.zeros(SGM_TRACE_CAP, np.int64)
        tick = ctypes.c_double()
        n = lib().sgm_trace_events(self._h, i, buf.ctypes.data_as(_i64p), SGM_TRACE_CAP,
                                   ctypes.byref(tick))
        if n < 0:
            raise SGMError(n, "sgm_trace_events")
        ev = buf[:min(n, SGM_TRACE_CAP)]
        if len(ev) == 0:
            return []
        t = (ev >> 8) - (ev[0] >> 8)
        return [(EVENT_NAMES.get(int(c), str(int(c))), float(x) * tick.value / 1e3)
                for c, x in zip(ev & 255, t)]

    def tuning(self) -> dict:
        """The persistent kernel's tuning (sgm_get_tuning)."""
        t = sgm_tuning()
        rc = lib().sgm_get_tuning(self._h, ctypes.byref(t))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_get_tuning")
        return {k: getattr(t, k) for k in TUNING_FIELDS}

    def set_tuning(self, **kw):
        """Change tuning fields (sgm_set_tuning); results do not depend on them."""
        t = sgm_tuning()
        lib().sgm_get_tuning(self._h, ctypes.byref(t))
        for k, v in kw.items():
            if k not in TUNING_FIELDS:
                raise TypeError(f"unknown tuning field {k!r}")
            setattr(t, k, int(v))
        rc = lib().sgm_set_tuning(self._h, ctypes.byref(t))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_set_tuning")

    def autotune(self, queries, reps: int = 3) -> dict:
        """Pick the fastest tuning for a sample batch (sgm_autotune)."""
        built = [_make_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel) for q in queries]
        arr = (sgm_query * len(built))(*[b[0] for b in built])
        t = sgm_tuning()
        rc = lib().sgm_autotune(self._h, arr, len(built), int(reps), ctypes.byref(t))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_autotune")
        return {k: getattr(t, k) for k in TUNING_FIELDS}

    def kernel_stats(self):
        out = {}
        for kid, name in enumerate(KERNEL_NAMES):
            s = sgm_kstat()
            lib().sgm_kernel_stats(self._h, kid, ctypes.byref(s))
            out[name] = dict(launches=s.launches, ms=s.ms_total, bytes=s.bytes_total)
        return out

    def inject_fault(self, query_index: int):
        """sgm_inject_fault: member query_index of the next persistent-kernel
        launch fails with SGM_EDEVICE (a failure-isolation test hook)."""
        rc = lib().sgm_inject_fault(self._h, int(query_index))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_inject_fault")

    def reset_kernel_stats(self):
        lib().sgm_reset_kernel_stats(self._h)


class Compressed:
    """A multi-level compression of a graph (sgm_compress; thesis Ch. 3, Sec.
    "Multi-level Graph Compression"): the weighted graph G_w and the mapping
    lists, as numpy copies of the library's host arrays."""

    def __init__(self, row_ptr, col, rel, vtype, max_levels=3, delta=None, target_ratio=0.0,
                 max_partners=64):
        o = sgm_compress_options()
        lib().sgm_default_compress_options(ctypes.byref(o))
        o.max_levels = int(max_levels)
        if delta is not None:
            ds = [float(delta)] * 8 if np.isscalar(delta) else list(delta)
            for i, d in enumerate(ds[:8]):
                o.delta[i] = d
        o.target_ratio = float(target_ratio)
        o.max_partners = int(max_partners)
        row_ptr = np.asarray(row_ptr)
        (rp, rpp), (c, cp), (r, rlp), (t, tp) = _arr(row_ptr), _arr(col), _arr(rel), _arr(vtype)
        ptr = ctypes.POINTER(sgm_compressed)()
        rc = lib().sgm_compress(int(len(row_ptr) - 1), int(row_ptr[-1]), rpp, cp, rlp, tp,
                                ctypes.byref(o), ctypes.byref(ptr))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_compress")
        self._p = ptr
        cc = ptr.contents
        self.n_vertices, self.n_original = int(cc.n_vertices), int(cc.n_original)
        self.n_edges, self.levels = int(cc.n_edges), int(cc.levels)
        self.level_size = [int(x) for x in cc.level_size[:self.levels + 1]]

        def grab(addr, n):
            out = np.empty(n, np.int32)
            if n:
                ctypes.memmove(out.ctypes.data, addr, 4 * n)
            return out
        nw, V, E = self.n_vertices, self.n_original, self.n_edges
        self.row_ptr = grab(cc.row_ptr, nw + 1)
        self.col, self.rel, self.weight = grab(cc.col, E), grab(cc.rel, E), grab(cc.weight, E)
        self.type = grab(cc.type, nw)
        self.out_bound, self.in_bound = grab(cc.out_bound, nw), grab(cc.in_bound, nw)
        self.map_off, self.map_ids = grab(cc.map_off, nw + 1), grab(cc.map_ids, V)
        self.hyper_of = grab(cc.hyper_of, V)

    @classmethod
    def from_kg(cls, kg, **kw):
        return cls(kg.row_ptr, kg.col, kg.rel, kg.vtype, **kw)

    def close(self):
        if getattr(self, "_p", None):
            lib().sgm_free_compressed(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CompressedGraph:
    """GpSense over a compressed graph (thesis Ch. 3, Sec. "GpSense
    Framework"): the weighted graph resident for matching, and the original
    graph (possibly kept in host memory) given the mapping lists; a query's
    matches are found on the weighted graph and expanded on the device."""

    def __init__(self, graph: Graph, comp: Compressed, **options):
        if comp._p is None:
            raise ValueError("compression already freed")
        opts = sgm_default_options()
        for k, v in options.items():
            setattr(opts, k, v)
        h = ctypes.c_void_p()
        rc = lib().sgm_load_compressed(comp._p, ctypes.byref(opts), ctypes.byref(h))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_load_compressed")
        rc = lib().sgm_attach_mapping(graph._h, comp._p)
        if rc != SGM_OK:
            sgm_free_graph(h)
            raise SGMError(rc, "sgm_attach_mapping")
        self._hw = h
        self.graph = graph
        self.hyper_of = comp.hyper_of

    def close(self):
        if getattr(self, "_hw", None):
            sgm_free_graph(self._hw)
            self._hw = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def match(self, n, vlabel, vpin, esrc, edst, elabel, count_only=False):
        """Matches of the query in the original graph, as Graph.match."""
        q, keep = _make_query(n, vlabel, vpin, esrc, edst, elabel)
        out = ctypes.POINTER(sgm_result)()
        fl = SGM_COUNT_ONLY if count_only else SGM_SORTED
        rc = lib().sgm_match_compressed(self.graph._h, self._hw, ctypes.byref(q), fl,
                                        ctypes.byref(out))
        if rc != SGM_OK:
            err = SGMError(rc, "sgm_match_compressed")
            if out:
                err.n_rows = int(out.contents.n_rows)
                sgm_free_result(out)
            raise err
        k, rows = _take_rows(out, n)
        return k if count_only else rows

    def match_query(self, q, **kw):
        return self.match(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel, **kw)

    def match_weighted(self, q, count_only=False):
        """Matches of the query on the weighted graph alone (homomorphisms,
        pins moved to their weighted vertices)."""
        vpin = np.where(q.vpin >= 0, self.hyper_of[np.maximum(q.vpin, 0)], -1).astype(np.int32)
        qq, keep = _make_query(q.n, q.vlabel, vpin, q.esrc, q.edst, q.elabel)
        rc, r = sgm_match_query(self._hw, qq, SGM_COUNT_ONLY if count_only else SGM_SORTED)
        if rc != SGM_OK:
            if r:
                sgm_free_result(r)
            raise SGMError(rc, "sgm_match_query")
        k, rows = _take_rows(r, q.n)
        return k if count_only else rows


class Server:
    """The served form on a resident Graph (continuous batching over
    streams; see sgm_server_create)."""

    def __init__(self, graph: Graph, **options):
        o = sgm_serve_options()
        lib().sgm_default_serve_options(ctypes.byref(o))
        for k, v in options.items():
            setattr(o, k, v)
        self.graph = graph
        h = ctypes.c_void_p()
        rc = lib().sgm_server_create(graph._h, ctypes.byref(o), ctypes.byref(h))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_server_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().sgm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, q, count_only=False) -> int:
        sq, keep = _make_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel)
        t = ctypes.c_uint64()
        rc = lib().sgm_submit(self._h, ctypes.byref(sq), SGM_COUNT_ONLY if count_only else 0,
                              ctypes.byref(t))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_submit")
        return t.value

    def wait(self, ticket: int, n_cols: int, timeout_ns: int = -1):
        """(status, rows or None, stats dict) of a ticket."""
        out = ctypes.POINTER(sgm_result)()
        rc = lib().sgm_wait(self._h, ticket, timeout_ns, ctypes.byref(out))
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_wait")
        st = out.contents.status
        stats = stats_dict(out.contents.stats, n_cols, 0)
        if st != SGM_OK:
            sgm_free_result(out)
            return st, None, stats
        k, rows = _take_rows(out, n_cols)
        return st, rows, stats

    def stats(self) -> dict:
        s = sgm_serve_stats()
        lib().sgm_server_stats(self._h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def replay(self, queries, arrival_s, count_only=False, keep_results=True):
        """Submit queries at their arrival times (seconds, from now), wait
        for all; returns (latencies in ns, results list or None)."""
        n = len(queries)
        built = [_make_query(q.n, q.vlabel, q.vpin, q.esrc, q.edst, q.elabel) for q in queries]
        arr = (sgm_query * max(n, 1))(*[b[0] for b in built])
        at = np.ascontiguousarray(np.round(np.asarray(arrival_s) * 1e9).astype(np.int64))
        lat = np.zeros(n, np.int64)
        outs = (ctypes.POINTER(sgm_result) * max(n, 1))() if keep_results else None
        rc = lib().sgm_serve_replay(self._h, arr, at.ctypes.data_as(_i64p), n,
                                    SGM_COUNT_ONLY if count_only else 0,
                                    lat.ctypes.data_as(_i64p), outs)
        res = None
        if keep_results:
            res = []
            for q, r in zip(queries, outs):
                if not r:
                    res.append(None)
                    continue
                st = r.contents.status
                if st == SGM_OK:
                    k, rows = _take_rows(r, q.n)
                    res.append(k if count_only else rows)
                else:
                    res.append(SGMError(st, "served query"))
                    sgm_free_result(r)
        if rc != SGM_OK:
            raise SGMError(rc, "sgm_serve_replay")
        return lat, res
