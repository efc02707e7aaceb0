/*
 * sgm.h -- C ABI of the MI355X (gfx950) subgraph-matching library.
 *
 * The library finds every embedding of a small labelled query graph in a
 * large directed, relation-labelled, vertex-typed data graph with the
 * filtering-and-joining method of the thesis (Ch. 3, Sec. "Subgraph
 * Similarity Search", Alg. 3.1): plan on the host, initialise and refine
 * per-query-vertex candidate sets on the GPU (Alg. 3.2 and Sec. "Candidate
 * Nodes Refinement"), collect candidate edges per query edge (Sec. "Joining
 * Phase", two-step output), and join them into full matches.
 *
 * Conventions for every entry point:
 *  - ids, labels and CSR offsets are int32; counts that can pass 2^31 are
 *    int64;
 *  - pointer arguments are HOST pointers; the library copies what it needs
 *    during the call, so the caller may free its arrays on return;
 *  - objects the library returns (graphs, results) are library-owned and
 *    freed only with the matching sgm_free_* call (NULL is accepted);
 *  - the return value is SGM_OK (0) or a negative SGM_E* code; on error
 *    every output pointer is set to NULL; no C++ exception crosses the ABI;
 *  - a graph is immutable after load; calls on one graph are serialised
 *    internally, so several threads may share it.
 */
#ifndef SGM_H
#define SGM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGM_OK 0
#define SGM_EINVAL (-1)       /* malformed CSR or query (see each call) */
#define SGM_ENOMEM (-2)       /* host or device allocation failed / admission refused */
#define SGM_EDEVICE (-3)      /* a HIP call failed; sgm_last_error() has the text */
#define SGM_ETOOBIG (-4)      /* result rows exceed options.result_cap_rows */
#define SGM_EUNSUPPORTED (-5) /* query beyond the library's limits */

#define SGM_MAX_QV 16 /* query vertices */
#define SGM_MAX_QE 64 /* query edges */

/* sgm_match_* flags */
#define SGM_SORTED 0u     /* default: rows unique, ascending lexicographic */
#define SGM_COUNT_ONLY 1u /* only n_rows (rows == NULL) */

typedef struct sgm_graph sgm_graph;

/* Tuning knobs; sgm_default_options() fills the defaults. */
typedef struct {
    int32_t device;            /* HIP device ordinal (default 0) */
    int32_t refine_rounds;     /* refinement rounds after initialisation (default 1;
                                  -1 = repeat until no candidate is removed) */
    int32_t refine_reversed;   /* 1 (default): refine in reversed visit order */
    int32_t low_conn_degree;   /* query vertices of at most this many distinct
                                  neighbours are skipped by refinement (default 1) */
    int64_t result_cap_rows;   /* > 0: fail with SGM_ETOOBIG above this many rows */
    int64_t join_budget_bytes; /* > 0: bound on one join level's output table;
                                  larger levels are processed in chunks */
    int32_t profile;           /* 1: time every kernel launch with HIP events
                                  (sgm_kernel_stats); 2: in addition record the
                                  persistent kernel's per-step event trace
                                  (sgm_trace_events) */
    int32_t path;              /* SGM_PATH_AUTO (default), SGM_PATH_WIDE or
                                  SGM_PATH_NARROW (see below) */
    int32_t graphs;            /* 1 (default): a persistent-kernel batch (upload,
                                  root sweep, kernel, readback) is one HIP graph
                                  launch; 0: separate launches. Not used while
                                  profile != 0 (kernels are timed one by one) */
    int32_t out_only;          /* 1: keep only the outgoing graph (thesis Ch. 3,
                                  Sec. "GpSense Framework": the incoming graph is
                                  the second of the two representations). A query
                                  vertex reached only over an edge into a filtered
                                  vertex then starts from every vertex of its label
                                  and is pruned over its own outgoing edges; edge
                                  candidates keyed by a destination are built by
                                  transposing the source-keyed ones. Results are
                                  unchanged; it exists to measure what the
                                  incoming graph saves. Runs on SGM_PATH_WIDE only
                                  (AUTO means WIDE; NARROW, servers, autotuning
                                  and sgm_match_query_noalloc: SGM_EINVAL) */
    int32_t host_graph;        /* 1: keep the graph's adjacency arrays (every
                                  O(edges) array) in pinned host memory, mapped
                                  into the device's address space; kernels read
                                  them in place over the host link, and only the
                                  O(vertices) arrays (row offsets, types, degrees)
                                  and the per-query buffers use device memory.
                                  For graphs larger than device memory (thesis
                                  Ch. 3, Sec. "Scalability Test": the data graph
                                  kept in main memory). Results are unchanged;
                                  0 (default): everything in device memory. Other
                                  values: SGM_EINVAL */
    int32_t reserved[3];
} sgm_options;

/* Execution paths. NARROW: one persistent kernel in which each workgroup
 * runs whole queries (used for batches and for single queries that fit a
 * workgroup's slot); a query that outgrows its slot (candidate lists, slot
 * memory, output arena) runs again in one of a few large slots. WIDE: one
 * multi-kernel pipeline per query using the whole GPU for each phase. AUTO
 * runs NARROW first and reruns on WIDE every query that fits no slot;
 * NARROW alone fails such a query with SGM_EUNSUPPORTED. Results are
 * identical on every path. */
#define SGM_PATH_AUTO 0
#define SGM_PATH_WIDE 1
#define SGM_PATH_NARROW 2

/* A query graph (thesis Ch. 3, Sec. "Commonsense Graph Transformation" and
 * Def. 3.2): 1..SGM_MAX_QV vertices, 0..SGM_MAX_QE directed edges.
 *   vertex_label[u]: vertex type >= 0, or -1 for any type;
 *   vertex_pin[u]:   data vertex id (a concept node), or -1 (variable node);
 *   edge_src/dst[i]: query vertex indices, src != dst;
 *   edge_label[i]:   relation >= 0, or -1 (variable edge: any relation).
 * The query must be connected as an undirected graph and may not repeat an
 * identical (src, dst, label) edge. */
typedef struct {
    int32_t n_vertices;
    int32_t n_edges;
    const int32_t *vertex_label;
    const int32_t *vertex_pin;
    const int32_t *edge_src;
    const int32_t *edge_dst;
    const int32_t *edge_label;
} sgm_query;

/* Per-query statistics (filled for every successful or ETOOBIG result). */
typedef struct {
    int64_t cand[SGM_MAX_QV];      /* final candidate-set size per query vertex */
    int64_t ec[SGM_MAX_QE];        /* candidate-edge count per query edge */
    int64_t level_rows[SGM_MAX_QV];/* rows after each join level (level 0 = seed keys) */
    int32_t join_order[SGM_MAX_QV];/* query vertex bound at each join level */
    int32_t visit_order[SGM_MAX_QV];/* filtering visit order O; -1 padded */
    int64_t peak_rows;             /* largest intermediate table, rows */
    int64_t peak_bytes;            /* largest intermediate table, bytes */
    int32_t n_chunks;              /* join chunks (1 = no chunking) */
    int32_t n_launches;            /* kernel launches for this query */
    int64_t ns_total;              /* host wall time of the call (of the whole batch
                                      for sgm_match_batch) */
    int64_t ns_filter, ns_collect, ns_join, ns_finish; /* phase times: host-measured on
                                      the multi-kernel path, device clock on the
                                      persistent kernel */
    int64_t device_bytes;          /* persistent kernel: algorithmic bytes moved */
    int64_t phase_bytes[4];        /* persistent kernel: the same bytes by phase
                                      (filter, collect, join, finish; the device
                                      times are ns_filter .. ns_finish) */
    int32_t path;                  /* SGM_PATH_WIDE or SGM_PATH_NARROW: where it ran */
    int32_t fallback;              /* why a query outgrew a regular persistent-kernel
                                      slot: 1 candidate list capacity, 2 slot
                                      memory, 4 ordering key > 64 bits, 8 output
                                      arena full, 16 plan descriptor size, 32 a
                                      shared filter step not finished by its
                                      helpers in time (an internal error; the
                                      query is rerun). With path NARROW it then
                                      ran in a large slot; with path WIDE on the
                                      multi-kernel path */
} sgm_stats;

typedef struct {
    int32_t status;   /* SGM_OK or an SGM_E* code (batch members) */
    int32_t n_cols;   /* = query n_vertices; column u holds f(u) */
    int64_t n_rows;   /* number of matches (exact, also for ETOOBIG) */
    int32_t *rows;    /* host, row-major [n_rows][n_cols], unique, ascending
                         lexicographic; non-NULL (also for 0 rows) on SGM_OK
                         without SGM_COUNT_ONLY, NULL otherwise */
    sgm_stats stats;
} sgm_result;

/* Per-kernel timing, accumulated while options.profile = 1. */
typedef struct {
    int64_t launches;
    double ms_total;      /* sum of HIP-event durations on the library stream */
    double bytes_total;   /* algorithmic bytes (what the step must move) */
} sgm_kstat;

#define SGM_K_CHECK 0     /* candidate initialisation sweep (label/degree) */
#define SGM_K_COLLECT 1   /* bitmap -> sorted candidate list + rank table */
#define SGM_K_EXPLORE 2   /* prune + push along spanning-tree edges */
#define SGM_K_REFINE 3    /* prune over all query edges */
#define SGM_K_EC_COUNT 4  /* candidate edges, count pass */
#define SGM_K_EC_WRITE 5  /* candidate edges, write pass */
#define SGM_K_JOIN 6      /* join levels (fan, count, write) */
#define SGM_K_SORT 7      /* final ordering */
#define SGM_K_OTHER 8     /* scans, clears, gathers */
#define SGM_K_PERSIST 9   /* persistent per-query kernel (whole queries) */
#define SGM_K_COUNT 10

/* Fill *o with the defaults documented above. */
void sgm_default_options(sgm_options *o);

/*
 * Load a data graph onto the device (thesis Ch. 3: nodes array + edges array
 * + node-label and edge-label arrays; Sec. "GpSense" optimisations: both an
 * outgoing and an incoming graph).
 *   row_ptr[n_vertices+1]: out-CSR offsets, row_ptr[0] = 0, non-decreasing,
 *                          row_ptr[n_vertices] = n_edges;
 *   col[n_edges]:  destination of each edge, 0 <= col < n_vertices;
 *   rel[n_edges]:  relation label >= 0;
 *   type[n_vertices]: vertex type >= 0.
 * Rows may be unsorted and may repeat a (dst, rel) pair: the library sorts
 * each row by (dst, rel), drops exact duplicate triples (the edge set of
 * Def. 3.1) and builds the incoming CSR. Self-loops are kept (they never
 * match, since matches are injective).
 * opts may be NULL (defaults). Errors: SGM_EINVAL for malformed CSR,
 * SGM_ENOMEM, SGM_EDEVICE. On success *out owns all device memory.
 */
int sgm_load_graph(int32_t n_vertices, int32_t n_edges, const int32_t *row_ptr,
                   const int32_t *col, const int32_t *rel, const int32_t *type,
                   const sgm_options *opts, sgm_graph **out);

/*
 * All matches of q in g (thesis Alg. 3.1; result contract of Def. 3.2: f
 * injective, type labels and pins respected, every query edge present in
 * the data graph with its relation or any relation for -1).
 * flags: SGM_SORTED (0) or SGM_COUNT_ONLY.
 * Errors: SGM_EINVAL (disconnected query, self-loop, index out of range,
 * duplicate edge, pin out of range), SGM_EUNSUPPORTED (more than
 * SGM_MAX_QV vertices or SGM_MAX_QE edges), SGM_ETOOBIG (then *out still
 * holds the exact n_rows and stats, rows = NULL), SGM_ENOMEM, SGM_EDEVICE.
 * On SGM_OK or SGM_ETOOBIG, *out is a library-owned result.
 */
int sgm_match_query(sgm_graph *g, const sgm_query *q, uint32_t flags, sgm_result **out);

/*
 * n queries at once; out[i] receives one result per query (free each with
 * sgm_free_result). A failure of one query is reported in out[i]->status
 * and does not affect the others; the call itself returns SGM_OK unless
 * the arguments are invalid (SGM_EINVAL) or a global failure occurs.
 */
int sgm_match_batch(sgm_graph *g, const sgm_query *qs, int32_t n, uint32_t flags,
                    sgm_result **out);

/*
 * Projection (thesis Ch. 3, Sec. "Joining Phase", closing remarks on
 * commonsense reasoning, and Sec. "GpSense": a commonsense query asks only
 * for the matches of a subset of its nodes): the distinct tuples
 * (f(u) for u in the projected set) over all matches f of q, as rows of
 * popcount(project) columns (the projected vertices in index order), unique
 * and ascending lexicographic; n_rows counts those distinct tuples (with
 * SGM_COUNT_ONLY too). Equal tuples are collapsed on the device after the
 * projected columns are ordered.
 *   project: bit u set = query vertex u is returned; non-zero and within
 *            the query's vertices (SGM_EINVAL otherwise); all vertices set
 *            = sgm_match_query.
 * Other arguments, errors and ownership as sgm_match_query /
 * sgm_match_batch (project[i] for qs[i]); options.result_cap_rows bounds the
 * distinct tuples on the persistent kernel and the full matches on the
 * multi-kernel path.
 */
int sgm_match_query_proj(sgm_graph *g, const sgm_query *q, uint32_t project, uint32_t flags,
                         sgm_result **out);
int sgm_match_batch_proj(sgm_graph *g, const sgm_query *qs, const uint32_t *project, int32_t n,
                         uint32_t flags, sgm_result **out);

void sgm_free_result(sgm_result *r);
void sgm_free_graph(sgm_graph *g);

/* Static text for an SGM_E* code. */
const char *sgm_strerror(int code);
/* Text of the last SGM_EDEVICE / SGM_EINVAL detail on this thread. */
const char *sgm_last_error(void);

/*
 * Step trace of the persistent kernel (options.profile = 2). Events of query
 * i (its index in the last sgm_match_query / sgm_match_batch call on this
 * graph), oldest first; each is (device wall-clock tick << 8) | SGM_EV_*
 * code, written by the workgroup that ran the query when the step ended.
 * Copies at most cap events to out and returns the number recorded (0 for a
 * query that did not run on the persistent kernel), or a negative SGM_E*
 * code. *ns_per_tick (may be NULL) receives the clock period. Not for
 * queries of a server; not thread-safe against concurrent match calls on the
 * same graph.
 */
#define SGM_TRACE_CAP 256
#define SGM_EV_START 1     /* query taken from the work queue */
#define SGM_EV_ROOT 2      /* root candidates ready (Alg. 3.2 initialisation) */
#define SGM_EV_EXPLORE 3   /* one kernel_explore step along the spanning tree */
#define SGM_EV_REFINE 4    /* one refinement step */
#define SGM_EV_LISTS 5     /* candidate lists sorted */
#define SGM_EV_EDGES 6     /* one candidate-edge table built */
#define SGM_EV_ORDER 7     /* join order chosen */
#define SGM_EV_LEVEL 8     /* one join level written */
#define SGM_EV_SORT 9      /* final rows ordered */
#define SGM_EV_OUTPUT 10   /* rows copied to the output arena */
#define SGM_EV_SHARED 11   /* a shared join level: no chunk left for its owner to claim */
#define SGM_EV_LONGROWS 12 /* a filter step's regular candidates done; its long rows follow */
int sgm_trace_events(sgm_graph *g, int32_t i, int64_t *out, int32_t cap, double *ns_per_tick);

/*
 * Work division and join schedule of the persistent kernel (the batched
 * form). Results never depend on these; speed does. Defaults: slots 512,
 * group_lanes 64, wg_rows 8192, join_policy 0, help_items 1024, helpers 64,
 * help_wait 0.
 *   slots        workgroups of one persistent launch that take queries
 *                (1..512; two per CU fit)
 *   group_lanes  most lanes working on one candidate's rows (1, 2, 4, ..., 64)
 *   wg_rows      rows longer than this are scanned by the whole workgroup
 *                (>= 64; shorter long rows get one wave)
 *   join_policy  0: bind the vertex of the cheapest candidate-edge table
 *                next (thesis Sec. "Joining Phase"); 1: bind the vertex with
 *                the most edges to bound vertices first, cheapest on ties
 *   help_items   work sharing inside a launch (0: none; else >= 64): a
 *                filter step over at least this many candidates is shared
 *                with the launch's idle workgroups, which claim chunks of
 *                its candidate list, and the pushes of candidates with long
 *                rows are shared as row segments in any filter step
 *   helpers      a launch with fewer queries than this adds workgroups that
 *                only help, up to this many workgroups in all (0..512; used
 *                only with help_items > 0; the served form adds none)
 *   help_wait    polls of a shared step's completion count before its owner
 *                gives up (0: the default, 4,194,304; >= 0). Giving up is an
 *                error path (claimed chunks always finish in bounded time):
 *                the query is rerun outside the launch's regular slots, and
 *                the slot takes no further query in that launch, since
 *                chunks its helpers claimed may still write it; the next
 *                launch clears the whole slot first. Small values exercise
 *                that path in tests.
 * The multi-kernel path keeps the thesis order.
 */
typedef struct {
    int32_t slots;
    int32_t group_lanes;
    int32_t wg_rows;
    int32_t join_policy;
    int32_t help_items;
    int32_t helpers;
    int32_t help_wait;
    int32_t reserved[1];
} sgm_tuning;

void sgm_default_tuning(sgm_tuning *t);
/* Current tuning of a graph. */
int sgm_get_tuning(const sgm_graph *g, sgm_tuning *t);
/* Set a graph's tuning (SGM_EINVAL for values out of range). Not while a
 * server of the graph runs or another match call is in flight. */
int sgm_set_tuning(sgm_graph *g, const sgm_tuning *t);
/*
 * Autotuner: runs the n sample queries as persistent-kernel batches (count
 * only, reps times each) under every tuning of a small grid (slots 256/512,
 * group_lanes 16/64, wg_rows 2048/8192/32768, join_policy 0/1, help_items
 * 0/1024; helpers as set), keeps the
 * one with the lowest median batch time, sets it on the graph and returns it
 * in *best (may be NULL). Every tuning must give the same per-query row
 * counts; otherwise the previous tuning is restored and SGM_EDEVICE
 * returned. Same threading rule as sgm_set_tuning.
 */
int sgm_autotune(sgm_graph *g, const sgm_query *qs, int32_t n, int32_t reps, sgm_tuning *best);

/* Graph properties after load (deduplicated edge count etc.). */
int sgm_graph_info(const sgm_graph *g, int32_t *n_vertices, int64_t *n_edges,
                   int32_t *max_out_degree, int32_t *max_in_degree);

/* Per-kernel timing accumulated since load or the last reset
 * (options.profile = 1). kernel is one of SGM_K_*. */
int sgm_kernel_stats(sgm_graph *g, int32_t kernel, sgm_kstat *out);
int sgm_reset_kernel_stats(sgm_graph *g);

/*
 * Query plan on the host only (no device needed), thesis Ch. 3 Sec. "Query
 * Plan Generation" with the commonsense variant of Sec. "GpSense":
 * rank f(u) = deg(u) / freq(u), freq = 1 for a pinned vertex, else the number
 * of data vertices of u's type (type_freq[label], or n_vertices for -1).
 *   type_freq[n_types]: data vertex count per type;
 *   visit_order[SGM_MAX_QV]: out, the expanded vertices O, -1 padded;
 *   parent[SGM_MAX_QV]: out, spanning-tree parent (-1 for the root);
 *   parent_edge[SGM_MAX_QV]: out, query edge joining u to its parent (-1);
 *   init_order[SGM_MAX_QV]: out, the order in which vertices obtain
 *                           candidate sets.
 * Errors as for sgm_match_query's query checks.
 */
int sgm_plan_query(const sgm_query *q, int32_t n_vertices, const int64_t *type_freq,
                   int32_t n_types, int32_t *visit_order, int32_t *parent,
                   int32_t *parent_edge, int32_t *init_order);

/*
 * Admission estimate of the served form, on the host only (no device
 * needed): estimated device bytes of a query's intermediate tables. The
 * thesis ties the join's running time and partial-solution memory to
 * candidate counts (Ch. 3, Sec. "Joining Phase"); this estimate takes that
 * dependence from graph statistics alone. Along the spanning tree of the
 * query plan (as sgm_plan_query), in the order vertices enter it: the root
 * starts with the number of data vertices its label admits (1 if pinned, V
 * for any type); a vertex reached over a tree edge of relation r multiplies
 * the rows by rel_freq[r] / V (E / V for a variable edge) and by the
 * fraction of data vertices its label admits (1 / V if pinned); each further
 * query edge between placed vertices multiplies by min(1, that per-vertex
 * edge count / V). Level k's table has k + 1 int32 columns, and a level's
 * input and output tables count together; the estimate is the largest such
 * pair plus one V-bit candidate bitmap per query vertex.
 *   type_freq[n_types]: data vertices per type;
 *   rel_freq[n_rels]:   data edges per relation (after dropping duplicate
 *                       triples); n_edges = their sum.
 * Errors as for sgm_match_query's query checks; SGM_EINVAL for bad sizes.
 */
int sgm_estimate_query(const sgm_query *q, int32_t n_vertices, int64_t n_edges,
                       const int64_t *type_freq, int32_t n_types, const int64_t *rel_freq,
                       int32_t n_rels, int64_t *est_bytes);

/*
 * Verification entry point: the candidate set of every query vertex after
 * the filtering phase (thesis Alg. 3.2 initialisation along the plan's
 * spanning tree, then the configured refinement, Sec. "Candidate Nodes
 * Refinement") and the candidate-edge count of every query edge (Sec.
 * "Joining Phase"), computed by the multi-kernel path's kernels (the
 * persistent kernel runs the same filter program).
 *   counts[SGM_MAX_QV]: out, number of candidates of each query vertex;
 *   *ids: out, library-owned ascending candidate lists concatenated in
 *         query-vertex order (free with sgm_free_ids);
 *   ec[SGM_MAX_QE]: out, candidate edges of each query edge (all 0 when a
 *         candidate set is empty).
 * Errors as for sgm_match_query's query checks, SGM_ENOMEM, SGM_EDEVICE.
 */
int sgm_inspect_query(sgm_graph *g, const sgm_query *q, int64_t *counts, int32_t **ids,
                      int64_t *ec);
void sgm_free_ids(int32_t *ids);

/*
 * sgm_match_query for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid allocation; the call synchronises
 * with its stream, so it cannot be captured into a HIP graph): the same
 * match on the persistent kernel,
 * with every device buffer taken from one fixed 64 MB area of device memory
 * that the library holds on each GPU until the process ends (its address
 * is taken once per device when a graph is loaded). No hipMalloc, hipFree,
 * pinned-host allocation or other allocating routine is called.
 *   rows:     caller-owned host buffer of rows_cap * n_vertices int32 (may
 *             be NULL with SGM_COUNT_ONLY or rows_cap = 0); receives the
 *             sorted table as sgm_match_query's result rows;
 *   rows_cap: capacity of rows in rows (>= 0);
 *   *n_rows:  the exact number of matches (also on SGM_ETOOBIG).
 * Limits and errors: SGM_EUNSUPPORTED if the graph is too large for the
 * area (one slot needs 17 V-bit bitmaps, 16 candidate lists of min(V, 65536)
 * ints and a 16 MB slab, and at least 1 MB must remain for the output
 * table: about 19M vertices at most) or the query needs a 128-bit ordering
 * key; SGM_ENOMEM if the query outgrows the area's slot or output table
 * (sgm_match_query then still answers it); SGM_ETOOBIG if more than rows_cap
 * rows match (rows untouched); SGM_EINVAL / SGM_EUNSUPPORTED for queries as
 * sgm_match_query; SGM_EDEVICE. The area keeps each call's contents; calls
 * on one device are serialised inside the library (one area per device).
 * No statistics are returned.
 */
int sgm_match_query_noalloc(sgm_graph *g, const sgm_query *q, uint32_t flags, int32_t *rows,
                            int64_t rows_cap, int64_t *n_rows);

/* ------------------------------------------------------------------------
 * Served form: a request loop that keeps the graph resident, admits arriving
 * queries against an intermediate-memory cap, batches them as they come and
 * runs several batches on the device at once (continuous batching over
 * streams). Results are identical to sgm_match_query's.
 * ------------------------------------------------------------------------ */
typedef struct sgm_server sgm_server;

typedef struct {
    int32_t streams;              /* batches on the device at once (default 4) */
    int32_t max_batch;            /* queries per batch (default 256) */
    int64_t max_wait_ns;          /* a batch closes this long after its first
                                     query arrived (default 100 us) */
    int64_t admission_cap_bytes;  /* cap on the summed admission estimates
                                     (sgm_estimate_query) of admitted,
                                     unfinished queries (default 64 GiB); one
                                     query is always admitted when none runs */
    int32_t reserved[8];
} sgm_serve_options;

typedef struct {
    int64_t submitted, completed, batches;
    int64_t admission_stalls;     /* batches held back by the memory cap */
    int64_t max_in_flight;        /* most queries admitted at once */
    int64_t wide_fallbacks;       /* queries rerun on the multi-kernel path */
} sgm_serve_stats;

void sgm_default_serve_options(sgm_serve_options *o);

/* The results of a batch at a glance, for bindings: for each of rs[0 .. n)
 * four int64 values at out[4 i]: status, n_cols, n_rows and the address of
 * rows (0 when NULL). A NULL entry reads as (SGM_EINVAL, 0, 0, 0). Takes no
 * ownership; out holds 4 n values (caller-owned). */
void sgm_results_summary(sgm_result *const *rs, int32_t n, int64_t *out);

/* Failure isolation test hook (not for production use): the member with
 * index query_index (its position in the sgm_match_batch call, 0 for
 * sgm_match_query) of the next persistent-kernel launch on g ends, on the
 * device, as a fault confined to it would: its result carries SGM_EDEVICE,
 * every other member of the launch completes normally. One-shot; -1
 * cancels. Queries on the multi-kernel path are not affected. Errors:
 * SGM_EINVAL for a NULL graph or an index below -1. */
int sgm_inject_fault(sgm_graph *g, int64_t query_index);

/* Start a server on g (g must outlive it). Errors: SGM_EINVAL, SGM_ENOMEM,
 * SGM_EDEVICE. The server owns its streams and its host threads: a
 * dispatcher (batching and admission), one completer per stream (each
 * completes the batch of its stream as soon as that batch ends, whatever
 * runs on the others) and a rerun thread (queries that outgrew their slot
 * run again in a large slot or on the multi-kernel path without holding up
 * the completers). */
int sgm_server_create(sgm_graph *g, const sgm_serve_options *opts, sgm_server **out);

/* Queue one query (copied; the caller may free it on return); *ticket
 * identifies it for sgm_wait. Invalid queries are accepted and complete
 * with their error status. Thread-safe. */
int sgm_submit(sgm_server *s, const sgm_query *q, uint32_t flags, uint64_t *ticket);

/* Wait for a ticket (timeout_ns < 0: forever). SGM_OK: *out receives the
 * library-owned result (its status may be an error code of that query;
 * stats.ns_total = completion - submission). SGM_ETOOBIG is not returned
 * here: it appears in (*out)->status. SGM_EINVAL: unknown ticket;
 * SGM_EDEVICE on timeout (then the ticket stays valid). */
int sgm_wait(sgm_server *s, uint64_t ticket, int64_t timeout_ns, sgm_result **out);

int sgm_server_stats(sgm_server *s, sgm_serve_stats *out);

/* Stop accepting, finish everything queued, join the threads, free. */
void sgm_server_destroy(sgm_server *s);

/* Load generator: submit qs[i] at arrival_ns[i] after the call starts
 * (non-decreasing), wait for all, and write latency_ns[i] = completion time -
 * scheduled arrival. out (NULL allowed) receives the results. */
int sgm_serve_replay(sgm_server *s, const sgm_query *qs, const int64_t *arrival_ns, int32_t n,
                     uint32_t flags, int64_t *latency_ns, sgm_result **out);

/* ---- Multi-level graph compression (thesis Ch. 3, Sec. "Multi-level Graph
 * Compression", Def. 3.4-3.5, Thm. 3.1-3.2; Sec. "GpSense Framework") ----
 *
 * For graphs beyond device memory the thesis compresses the graph offline
 * into a smaller weighted graph G_w whose vertices stand for groups of
 * similar original vertices (mapping lists M(x)), matches queries on G_w
 * and expands each weighted match through the mapping lists into the
 * original graph's matches. */
typedef struct {
    int32_t max_levels;   /* levels of merging, 0..8 (default 3) */
    float delta[8];       /* similarity threshold of each level, in (0, 1]:
                             two vertices of one type merge when common
                             edges make up at least this share of either's
                             entries (default 0.8, then 0.7) */
    double target_ratio;  /* > 0: stop once (|V_i| + |E_i|) / (|V| + |E|)
                             is at most this (default 0: every level) */
    int32_t max_partners; /* partners looked at per shared entry (default 64) */
    int32_t reserved[3];
} sgm_compress_options;

/* A compressed graph (library-owned, host memory; sgm_free_compressed). */
typedef struct {
    int32_t n_vertices;       /* |V_w| */
    int32_t n_original;       /* |V| of the input */
    int64_t n_edges;          /* entries of the out-CSR below */
    int32_t levels;           /* levels applied */
    int32_t *row_ptr;         /* [n_vertices + 1] out-CSR of G_w */
    int32_t *col, *rel;       /* [n_edges], rows ascending by (neighbour, relation);
                                 an edge inside one group is a self-loop */
    int32_t *weight;          /* [n_edges] w(x -> y, rel): at most this many
                                 rel-edges from any vertex of M(x) into M(y) */
    int32_t *type;            /* [n_vertices] the type of every member */
    int32_t *out_bound;       /* [n_vertices] sum of x's out-entry weights:
                                 bounds the out-degree of every member (Def. 3.5) */
    int32_t *in_bound;        /* [n_vertices] the same for in-degrees */
    int32_t *map_off;         /* [n_vertices + 1] mapping lists M(x) ... */
    int32_t *map_ids;         /* [n_original] ... as ascending original ids */
    int32_t *hyper_of;        /* [n_original] the weighted vertex of each vertex */
    int64_t level_size[9];    /* |V_i| + |E_i| after level i (0: the input,
                                 repeated triples removed) */
} sgm_compressed;

void sgm_default_compress_options(sgm_compress_options *o);

/* Compress a graph given as sgm_load_graph takes it (host arrays, not
 * kept). SGM_EINVAL for malformed input or options, SGM_ENOMEM. Host-only:
 * no device is touched. */
int sgm_compress(int32_t n_vertices, int32_t n_edges, const int32_t *row_ptr, const int32_t *col,
                 const int32_t *rel, const int32_t *type, const sgm_compress_options *opts,
                 sgm_compressed **out);
void sgm_free_compressed(sgm_compressed *c);

/* Make G_w resident for matching (like sgm_load_graph on c's CSR). A
 * vertex's degree bounds are c's out/in bounds (Def. 3.5: a weighted vertex
 * is a candidate when the query vertex's degree is at most its weight), and
 * matches are homomorphisms: several query vertices may take one weighted
 * vertex, and a query edge may take a self-loop, since the original match
 * may use several members of one group. Both execution paths serve it;
 * servers, autotuning and sgm_match_query_noalloc refuse it (SGM_EINVAL),
 * and so does options.out_only. c is not kept. */
int sgm_load_compressed(const sgm_compressed *c, const sgm_options *opts, sgm_graph **out);

/* Give the original graph g (resident, possibly with options.host_graph)
 * the mapping lists of c, in device memory, for sgm_match_compressed.
 * Replaces an earlier mapping. SGM_EINVAL when c was not made from a graph
 * of g's vertex count. */
int sgm_attach_mapping(sgm_graph *g, const sgm_compressed *c);

/* Every match of q in the original graph g through the compressed graph gw
 * (GpSense, Sec. "GpSense Framework"): q's pinned vertices take their
 * weighted vertices, q is matched on gw, and each weighted match is
 * expanded on the device: every choice of members of its groups that is
 * injective, keeps the pins and holds every query edge in g is a match
 * (Thm. 3.2: no match of g is lost). The result is that of
 * sgm_match_query(g, q, flags): unique rows in ascending order. g needs
 * sgm_attach_mapping of the compression gw was loaded from. */
int sgm_match_compressed(sgm_graph *g, sgm_graph *gw, const sgm_query *q, uint32_t flags,
                         sgm_result **out);

#ifdef __cplusplus
}
#endif
#endif /* SGM_H */
