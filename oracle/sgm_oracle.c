/*
 * CPU oracle for exact subgraph matching -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package smoke check and the benchmark's
 * CPU-baseline leg may load this library. The GPU product path never calls
 * it, never links it and shares no code, header or table with it.
 *
 * What it computes (thesis Ch. 3, Def. 3.1 and Def. 3.2, with the readings
 * listed below): given a data graph -- vertices 0..V-1 with a type each and a
 * SET of directed, relation-labelled edges (s, d, r) -- and a query graph --
 * vertices 0..n-1 with a type label or -1 (any type), a pin (concept node,
 * Ch. 3 "Commonsense Graph Transformation") or -1 (variable node), and
 * directed edges (a, b, rho) with a relation or -1 (variable edge) -- the
 * result is the set of all maps f: {0..n-1} -> V such that
 *   1. f is injective                                      (Def. 3.2);
 *   2. label(u) = -1 or type(f(u)) = label(u)              (Def. 3.2);
 *   3. pin(u)   = -1 or f(u) = pin(u)                      (concept nodes);
 *   4. for every query edge (a, b, rho) some data edge (f(a), f(b), r)
 *      exists with rho = -1 or r = rho (directed, non-induced).
 * Each f is one row (f(0), ..., f(n-1)); rows are unique and returned in
 * ascending lexicographic order. Several data relations between the same
 * pair still give one row, because a match is the vertex map.
 *
 * How: plain depth-first backtracking over the query vertices, testing each
 * condition above directly; the next vertex placed is a pinned one, else the
 * one whose candidates (the entries of a placed neighbour's row) are fewest. It performs no
 * candidate filtering of any kind: every check is one clause of the
 * definition. A vertex's candidates are read from the adjacency row of an
 * already-placed neighbour, indexed by relation and by the neighbour's type
 * so that only entries that can satisfy clauses 2 and 4 for that edge are
 * read. OpenMP splits the work over the candidates of the first vertex and
 * pieces of the second vertex's rows.
 *
 * Parity pins (tests): brute-force enumeration of all V^n maps on micro
 * graphs, closed-form counts (complete digraphs, directed cycles, stars,
 * trace(A^3) and friends via scipy.sparse), and networkx's monomorphism
 * matcher on small simple graphs.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2
#define OR_ETOOBIG -4
#define OR_EBUDGET -6
#define OR_MAXQ 32

typedef struct {
    int32_t dst;
    int32_t rel;
} or_pair;

typedef struct oracle_graph {
    int32_t V;
    int64_t E;          /* distinct triples */
    int64_t *out_off;   /* [V+1] */
    or_pair *out;       /* sorted by (dst, rel) within each source */
    int64_t *in_off;    /* [V+1] */
    or_pair *in;        /* (src, rel) sorted within each destination */
    or_pair *out_r;     /* the rows of out, each sorted by (rel, type(dst), dst) */
    or_pair *in_r;      /* the rows of in, each sorted by (rel, type(src), src) */
    or_pair *out_t;     /* the rows of out, each sorted by (type(dst), dst, rel) */
    or_pair *in_t;      /* the rows of in, each sorted by (type(src), src, rel) */
    int32_t *vtype;     /* [V] */
    int32_t n_types, n_rels;
    int64_t *type_count;  /* [n_types] vertices per type */
    int64_t *rel_count;   /* [n_rels] distinct triples per relation */
} oracle_graph;

static int pair_cmp(const void *a, const void *b) {
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    if (x->dst != y->dst) return x->dst < y->dst ? -1 : 1;
    if (x->rel != y->rel) return x->rel < y->rel ? -1 : 1;
    return 0;
}

/* Group (key, other, rel) triples by key with a counting pass, sort each
 * group by (other, rel) and drop exact duplicates. Returns the number of
 * distinct triples, fills off[V+1] and arr. */
static int64_t group_edges(int32_t V, int64_t E, const int32_t *key, const int32_t *other,
                           const int32_t *rel, int64_t *off, or_pair *arr) {
    memset(off, 0, sizeof(int64_t) * ((size_t)V + 1));
    for (int64_t i = 0; i < E; i++) off[key[i] + 1]++;
    for (int32_t v = 0; v < V; v++) off[v + 1] += off[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
    if (!fill) return -1;
    memcpy(fill, off, sizeof(int64_t) * ((size_t)V + 1));
    for (int64_t i = 0; i < E; i++) {
        or_pair p;
        p.dst = other[i];
        p.rel = rel[i];
        arr[fill[key[i]]++] = p;
    }
    free(fill);
    /* sort + dedupe each group, compacting in place */
    int64_t w = 0;
    int64_t start = 0;
    for (int32_t v = 0; v < V; v++) {
        int64_t end = off[v + 1];
        int64_t len = end - start;
        if (len > 1) qsort(arr + start, (size_t)len, sizeof(or_pair), pair_cmp);
        int64_t row_begin = w;
        for (int64_t i = start; i < end; i++) {
            if (w > row_begin && arr[w - 1].dst == arr[i].dst && arr[w - 1].rel == arr[i].rel) continue;
            arr[w++] = arr[i];
        }
        off[v] = row_begin;
        start = end;
    }
    off[V] = w;
    return w;
}

/* Sort keys of the indexed row copies (qsort_r with the vertex types). */
static int pair_cmp_rel_type(const void *a, const void *b, void *t) {
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    const int32_t *vt = (const int32_t *)t;
    if (x->rel != y->rel) return x->rel < y->rel ? -1 : 1;
    if (vt[x->dst] != vt[y->dst]) return vt[x->dst] < vt[y->dst] ? -1 : 1;
    if (x->dst != y->dst) return x->dst < y->dst ? -1 : 1;
    return 0;
}

static int pair_cmp_type(const void *a, const void *b, void *t) {
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    const int32_t *vt = (const int32_t *)t;
    if (vt[x->dst] != vt[y->dst]) return vt[x->dst] < vt[y->dst] ? -1 : 1;
    if (x->dst != y->dst) return x->dst < y->dst ? -1 : 1;
    if (x->rel != y->rel) return x->rel < y->rel ? -1 : 1;
    return 0;
}

/* A copy of the rows of arr (extents off) with each row sorted by cmp: the
 * entries of one relation (and type), or of one type, are then contiguous. */
static or_pair *indexed_rows(int32_t V, const int64_t *off, const or_pair *arr,
                             const int32_t *vtype,
                             int (*cmp)(const void *, const void *, void *)) {
    or_pair *r = (or_pair *)malloc(sizeof(or_pair) * (size_t)(off[V] > 0 ? off[V] : 1));
    if (!r) return NULL;
    memcpy(r, arr, sizeof(or_pair) * (size_t)off[V]);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t v = 0; v < V; v++)
        if (off[v + 1] - off[v] > 1)
            qsort_r(r + off[v], (size_t)(off[v + 1] - off[v]), sizeof(or_pair), cmp,
                    (void *)vtype);
    return r;
}

void oracle_graph_free(oracle_graph *g) {
    if (!g) return;
    free(g->out_off);
    free(g->out);
    free(g->in_off);
    free(g->in);
    free(g->out_r);
    free(g->in_r);
    free(g->out_t);
    free(g->in_t);
    free(g->type_count);
    free(g->rel_count);
    free(g->vtype);
    free(g);
}

/* Build the oracle's own adjacency from a raw triple list. Duplicate triples
 * collapse (the edge set of Def. 3.1). Returns NULL on bad input. */
oracle_graph *oracle_graph_build(int32_t V, int64_t E, const int32_t *src, const int32_t *dst,
                                 const int32_t *rel, const int32_t *vtype) {
    if (V <= 0 || E < 0) return NULL;
    for (int64_t i = 0; i < E; i++)
        if (src[i] < 0 || src[i] >= V || dst[i] < 0 || dst[i] >= V || rel[i] < 0) return NULL;
    for (int32_t v = 0; v < V; v++)
        if (vtype[v] < 0) return NULL;
    oracle_graph *g = (oracle_graph *)calloc(1, sizeof(oracle_graph));
    if (!g) return NULL;
    g->V = V;
    g->out_off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
    g->in_off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
    g->out = (or_pair *)malloc(sizeof(or_pair) * (size_t)(E > 0 ? E : 1));
    g->in = (or_pair *)malloc(sizeof(or_pair) * (size_t)(E > 0 ? E : 1));
    g->vtype = (int32_t *)malloc(sizeof(int32_t) * (size_t)V);
    if (!g->out_off || !g->in_off || !g->out || !g->in || !g->vtype) {
        oracle_graph_free(g);
        return NULL;
    }
    memcpy(g->vtype, vtype, sizeof(int32_t) * (size_t)V);
    int64_t e1 = group_edges(V, E, src, dst, rel, g->out_off, g->out);
    int64_t e2 = group_edges(V, E, dst, src, rel, g->in_off, g->in);
    if (e1 < 0 || e2 < 0 || e1 != e2) {
        oracle_graph_free(g);
        return NULL;
    }
    g->E = e1;
    g->out_r = indexed_rows(V, g->out_off, g->out, g->vtype, pair_cmp_rel_type);
    g->in_r = indexed_rows(V, g->in_off, g->in, g->vtype, pair_cmp_rel_type);
    g->out_t = indexed_rows(V, g->out_off, g->out, g->vtype, pair_cmp_type);
    g->in_t = indexed_rows(V, g->in_off, g->in, g->vtype, pair_cmp_type);
    int32_t mt = 0, mr = 0;
    for (int32_t v = 0; v < V; v++) mt = vtype[v] > mt ? vtype[v] : mt;
    for (int64_t i = 0; i < g->E; i++) mr = g->out[i].rel > mr ? g->out[i].rel : mr;
    g->n_types = mt + 1;
    g->n_rels = mr + 1;
    g->type_count = (int64_t *)calloc((size_t)g->n_types, sizeof(int64_t));
    g->rel_count = (int64_t *)calloc((size_t)g->n_rels, sizeof(int64_t));
    if (!g->out_r || !g->in_r || !g->out_t || !g->in_t || !g->type_count || !g->rel_count) {
        oracle_graph_free(g);
        return NULL;
    }
    for (int32_t v = 0; v < V; v++) g->type_count[vtype[v]]++;
    for (int64_t i = 0; i < g->E; i++) g->rel_count[g->out[i].rel]++;
    return g;
}

int64_t oracle_graph_num_edges(const oracle_graph *g) { return g ? g->E : -1; }

/* Does the data edge x -> y exist with relation rho (rho = -1: any)? */
static int has_edge(const oracle_graph *g, int32_t x, int32_t y, int32_t rho) {
    int64_t lo = g->out_off[x], hi = g->out_off[x + 1];
    /* first entry with (dst, rel) >= (y, rho or -inf) */
    int32_t r0 = rho < 0 ? INT32_MIN : rho;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        const or_pair *p = &g->out[mid];
        if (p->dst < y || (p->dst == y && p->rel < r0)) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= g->out_off[x + 1]) return 0;
    const or_pair *p = &g->out[lo];
    if (p->dst != y) return 0;
    return rho < 0 || p->rel == rho;
}

typedef struct {
    int32_t n, m;
    const int32_t *vlabel, *vpin, *esrc, *edst, *elabel;
} or_query;

typedef struct {
    int32_t *rows;
    int64_t n_rows, cap;
    int failed;
} or_buf;

static int buf_push(or_buf *b, const int32_t *row, int32_t n) {
    if (b->n_rows == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        int32_t *nr = (int32_t *)realloc(b->rows, sizeof(int32_t) * (size_t)nc * (size_t)n);
        if (!nr) return -1;
        b->rows = nr;
        b->cap = nc;
    }
    memcpy(b->rows + (size_t)b->n_rows * (size_t)n, row, sizeof(int32_t) * (size_t)n);
    b->n_rows++;
    return 0;
}


/* Clauses 1-4 of the definition for query vertex u mapped to data vertex x,
 * against every query vertex already placed (bit v of placed). */
static int consistent(const oracle_graph *g, const or_query *q, const int32_t *f, uint32_t placed,
                      int32_t u, int32_t x) {
    if (q->vlabel[u] >= 0 && g->vtype[x] != q->vlabel[u]) return 0;
    if (q->vpin[u] >= 0 && x != q->vpin[u]) return 0;
    for (int v = 0; v < q->n; v++)
        if (((placed >> v) & 1u) && f[v] == x) return 0;
    for (int i = 0; i < q->m; i++) {
        int32_t a = q->esrc[i], b = q->edst[i];
        if (a == u && ((placed >> b) & 1u)) {
            if (!has_edge(g, x, f[b], q->elabel[i])) return 0;
        } else if (b == u && ((placed >> a) & 1u)) {
            if (!has_edge(g, f[a], x, q->elabel[i])) return 0;
        }
    }
    return 1;
}

/* Narrow [lo, hi) of a row sorted with key(entry) ascending to the entries
 * whose key equals k: key 0 = relation, 1 = type of the other endpoint. */
static void key_slice(const oracle_graph *g, const or_pair *arr, int64_t *lo, int64_t *hi,
                      int key, int32_t k) {
#define OR_KEY(e) (key == 0 ? (e).rel : g->vtype[(e).dst])
    int64_t a = *lo, b = *hi;
    while (a < b) { /* first entry with key >= k */
        int64_t mid = a + (b - a) / 2;
        if (OR_KEY(arr[mid]) < k) a = mid + 1;
        else b = mid;
    }
    int64_t c = a, d = *hi;
    while (c < d) { /* first entry with key > k */
        int64_t mid = c + (d - c) / 2;
        if (OR_KEY(arr[mid]) <= k) c = mid + 1;
        else d = mid;
    }
#undef OR_KEY
    *lo = a;
    *hi = c;
}

/* The data entries that generate the candidates of an unpinned vertex u,
 * from the placed neighbour whose entries are fewest: for a query edge
 * a -> u the out-row of f(a), for u -> b the in-row of f(b); of that row
 * only the entries of the edge's relation (a labelled edge) and of u's type
 * (a typed u), read from a copy of the row sorted by those keys, since any
 * other entry fails clause 2 or clause 4 for this edge. 0 if u has no
 * placed neighbour. */
static int gen_range(const oracle_graph *g, const or_query *q, const int32_t *f, uint32_t placed,
                     int32_t u, int64_t *lo_out, int64_t *hi_out, const or_pair **arr_out) {
    int best_len_set = 0;
    int64_t best_lo = 0, best_hi = 0;
    const or_pair *best_arr = NULL;
    for (int i = 0; i < q->m; i++) {
        int32_t a = q->esrc[i], b = q->edst[i], rho = q->elabel[i], t = q->vlabel[u];
        int64_t lo, hi;
        const or_pair *arr;
        if (b == u && ((placed >> a) & 1u)) { /* f(a) -> x : x among out-neighbours of f(a) */
            lo = g->out_off[f[a]];
            hi = g->out_off[f[a] + 1];
            arr = rho >= 0 ? g->out_r : t >= 0 ? g->out_t : g->out;
        } else if (a == u && ((placed >> b) & 1u)) { /* x -> f(b) : x among in-neighbours */
            lo = g->in_off[f[b]];
            hi = g->in_off[f[b] + 1];
            arr = rho >= 0 ? g->in_r : t >= 0 ? g->in_t : g->in;
        } else {
            continue;
        }
        if (rho >= 0) key_slice(g, arr, &lo, &hi, 0, rho);
        if (t >= 0) key_slice(g, arr, &lo, &hi, 1, t);
        if (!best_len_set || hi - lo < best_hi - best_lo) {
            best_len_set = 1;
            best_lo = lo;
            best_hi = hi;
            best_arr = arr;
        }
    }
    *lo_out = best_lo;
    *hi_out = best_hi;
    *arr_out = best_arr;
    return best_len_set;
}

/* The next vertex to place (fail first): an unplaced pinned vertex (one
 * candidate), else the unplaced vertex with a placed neighbour whose
 * generating entries are fewest (lowest index on ties). Every order places
 * each vertex once and checks every clause against all placed vertices, so
 * the order decides only how fast the search runs. Returns the vertex; its
 * entries in *lo..*hi of *arr (hi < 0 for a pinned vertex). */
static int32_t pick_next(const oracle_graph *g, const or_query *q, const int32_t *f,
                         uint32_t placed, int64_t *lo_out, int64_t *hi_out,
                         const or_pair **arr_out) {
    int32_t best = -1;
    int64_t best_len = 0;
    for (int32_t v = 0; v < q->n; v++) {
        if ((placed >> v) & 1u) continue;
        if (q->vpin[v] >= 0) {
            *lo_out = 0;
            *hi_out = -1;
            *arr_out = NULL;
            return v;
        }
        int64_t lo, hi;
        const or_pair *arr;
        if (!gen_range(g, q, f, placed, v, &lo, &hi, &arr)) continue;
        if (best < 0 || hi - lo < best_len) {
            best = v;
            best_len = hi - lo;
            *lo_out = lo;
            *hi_out = hi;
            *arr_out = arr;
        }
    }
    return best;
}

typedef struct {
    const oracle_graph *g;
    const or_query *q;
    or_buf *buf;
    int count_only;
    int64_t max_rows;
    int64_t *total;   /* shared running count */
    int *abort_flag;  /* 1: row cap exceeded, 2: work budget exceeded */
    int64_t max_steps; /* candidate tests allowed in total (-1: no limit) */
    int64_t *steps;    /* shared running count of candidate tests */
    int64_t local_steps;
} or_ctx;

/* Count one candidate test; past the budget, stop the whole search. */
static int over_budget(or_ctx *c) {
    if (c->max_steps < 0) return 0;
    if (++c->local_steps < 4096) return 0;
    int64_t t = __atomic_add_fetch(c->steps, c->local_steps, __ATOMIC_RELAXED);
    c->local_steps = 0;
    if (t > c->max_steps) {
        __atomic_store_n(c->abort_flag, 2, __ATOMIC_RELAXED);
        return 1;
    }
    return 0;
}

static void dfs_range(or_ctx *c, int32_t *f, uint32_t placed, int depth, int32_t u, int64_t lo,
                      int64_t hi, const or_pair *arr);

/* Extend the partial map f (vertices in placed, depth of them) by one more
 * vertex; a full map is one row. */
static void dfs(or_ctx *c, int32_t *f, uint32_t placed, int depth) {
    const or_query *q = c->q;
    const oracle_graph *g = c->g;
    if (__atomic_load_n(c->abort_flag, __ATOMIC_RELAXED)) return;
    if (depth == q->n) {
        int64_t t = __atomic_add_fetch(c->total, 1, __ATOMIC_RELAXED);
        if (c->max_rows >= 0 && t > c->max_rows) {
            __atomic_store_n(c->abort_flag, 1, __ATOMIC_RELAXED);
            return;
        }
        if (!c->count_only && buf_push(c->buf, f, q->n) != 0) {
            c->buf->failed = 1;
            __atomic_store_n(c->abort_flag, 1, __ATOMIC_RELAXED);
        }
        return;
    }
    int64_t lo, hi;
    const or_pair *arr;
    int32_t u = pick_next(g, q, f, placed, &lo, &hi, &arr);
    if (u < 0) return; /* unreachable for connected queries */
    if (hi < 0) {
        int32_t x = q->vpin[u];
        if (consistent(g, q, f, placed, u, x)) {
            f[u] = x;
            dfs(c, f, placed | (1u << u), depth + 1);
        }
        return;
    }
    dfs_range(c, f, placed, depth, u, lo, hi, arr);
}

/* Candidates of vertex u from entries [lo, hi) of the data row gen_range
 * chose (a full row is sorted by destination, and a repeated destination,
 * i.e. another relation, is one candidate; a relation's slice holds each
 * destination once; pieces of a row never split a run of equal
 * destinations). */
static void dfs_range(or_ctx *c, int32_t *f, uint32_t placed, int depth, int32_t u, int64_t lo,
                      int64_t hi, const or_pair *arr) {
    const or_query *q = c->q;
    const oracle_graph *g = c->g;
    int32_t prev = -1;
    for (int64_t k = lo; k < hi; k++) {
        int32_t x = arr[k].dst;
        if (x == prev) continue; /* same neighbour, other relation */
        prev = x;
        if (over_budget(c)) return;
        if (consistent(g, q, f, placed, u, x)) {
            f[u] = x;
            dfs(c, f, placed | (1u << u), depth + 1);
            if (__atomic_load_n(c->abort_flag, __ATOMIC_RELAXED)) return;
        }
    }
}

/* A unit of the parallel search: root candidate x, and either the whole
 * search below it (hi < 0) or the second vertex's candidates from entries
 * [lo, hi) of row array arr. */
typedef struct {
    int32_t x, u2;
    int64_t lo, hi;
    const or_pair *arr;
} or_item;

/* Row entries per work item of a split root. */
#define OR_PIECE 4096

static int row_cmp(const void *a, const void *b, void *arg) {
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    int n = *(const int *)arg;
    for (int i = 0; i < n; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

/* Validate a query: 1..32 vertices, edge endpoints in range, no self-loop,
 * connected as an undirected graph. */
static int query_ok(int32_t V, int32_t n, int32_t m, const int32_t *vpin, const int32_t *esrc,
                    const int32_t *edst) {
    if (n < 1 || n > OR_MAXQ || m < 0) return 0;
    for (int u = 0; u < n; u++)
        if (vpin[u] >= V) return 0;
    for (int i = 0; i < m; i++) {
        if (esrc[i] < 0 || esrc[i] >= n || edst[i] < 0 || edst[i] >= n) return 0;
        if (esrc[i] == edst[i]) return 0;
    }
    int seen[OR_MAXQ] = {0}, stack[OR_MAXQ], sp = 0, cnt = 1;
    seen[0] = 1;
    stack[sp++] = 0;
    while (sp) {
        int u = stack[--sp];
        for (int i = 0; i < m; i++) {
            int v = -1;
            if (esrc[i] == u) v = edst[i];
            else if (edst[i] == u) v = esrc[i];
            if (v >= 0 && !seen[v]) {
                seen[v] = 1;
                cnt++;
                stack[sp++] = v;
            }
        }
    }
    return cnt == n;
}

/*
 * All matches of the query in g (definition in the file header).
 * rows_out: if non-NULL receives a malloc'd row-major [n_rows][n] int32
 *           table, unique rows in ascending lexicographic order (free with
 *           oracle_free); if NULL only the count is produced.
 * max_rows: stop with OR_ETOOBIG once more rows than this exist (-1: no cap).
 * nthreads: OpenMP threads (<= 0: runtime default).
 * Returns OR_OK, OR_EINVAL (malformed query), OR_ENOMEM or OR_ETOOBIG.
 */
int oracle_match_budget(const oracle_graph *g, int32_t n, int32_t m, const int32_t *vlabel,
                        const int32_t *vpin, const int32_t *esrc, const int32_t *edst,
                        const int32_t *elabel, int64_t max_rows, int64_t max_steps,
                        int nthreads, int32_t **rows_out, int64_t *nrows_out);

int oracle_match(const oracle_graph *g, int32_t n, int32_t m, const int32_t *vlabel,
                 const int32_t *vpin, const int32_t *esrc, const int32_t *edst,
                 const int32_t *elabel, int64_t max_rows, int nthreads, int32_t **rows_out,
                 int64_t *nrows_out) {
    return oracle_match_budget(g, n, m, vlabel, vpin, esrc, edst, elabel, max_rows, -1, nthreads,
                               rows_out, nrows_out);
}

/* As oracle_match; also stops with OR_EBUDGET after max_steps candidate
 * tests (max_steps < 0: no limit). */
int oracle_match_budget(const oracle_graph *g, int32_t n, int32_t m, const int32_t *vlabel,
                        const int32_t *vpin, const int32_t *esrc, const int32_t *edst,
                        const int32_t *elabel, int64_t max_rows, int64_t max_steps,
                        int nthreads, int32_t **rows_out, int64_t *nrows_out) {
    if (!g || !nrows_out) return OR_EINVAL;
    *nrows_out = 0;
    if (rows_out) *rows_out = NULL;
    if (!query_ok(g->V, n, m, vpin, esrc, edst)) return OR_EINVAL;
    or_query q;
    q.n = n;
    q.m = m;
    q.vlabel = vlabel;
    q.vpin = vpin;
    q.esrc = esrc;
    q.edst = edst;
    q.elabel = elabel;
    /* root: the lowest-index pinned vertex, else the vertex whose type
     * matches the fewest data vertices (lowest index on ties) */
    int32_t root = -1;
    for (int u = 0; u < n && root < 0; u++)
        if (vpin[u] >= 0) root = u;
    if (root < 0) {
        int64_t best = -1;
        for (int u = 0; u < n; u++) {
            int64_t c = 0;
            if (vlabel[u] < 0) c = g->V;
            else
                for (int32_t v = 0; v < g->V; v++) c += g->vtype[v] == vlabel[u];
            if (best < 0 || c < best) {
                best = c;
                root = u;
            }
        }
    }
    /* first-level candidates */
    int32_t *roots = NULL;
    int64_t n_roots = 0;
    if (vpin[root] >= 0) {
        roots = (int32_t *)malloc(sizeof(int32_t));
        if (!roots) return OR_ENOMEM;
        roots[0] = vpin[root];
        n_roots = 1;
    } else {
        roots = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->V);
        if (!roots) return OR_ENOMEM;
        for (int32_t v = 0; v < g->V; v++)
            if (vlabel[root] < 0 || g->vtype[v] == vlabel[root]) roots[n_roots++] = v;
    }

    /* Work items for the threads: a root candidate with the whole search
     * below it, or, when the second vertex placed (chosen as in dfs) is
     * generated from a data row, a root candidate with a piece of that row
     * (so that a hub root's search is spread over threads). Pieces never
     * split a run of equal destinations. Every item is an independent part
     * of the same depth-first search; rows are sorted at the end, so the
     * split does not change the result. */
    or_item *items = NULL;
    int64_t n_items = 0, cap_items = 0;
    {
        int32_t f0[OR_MAXQ];
        const uint32_t p0 = 1u << root;
        for (int64_t i = 0; i < n_roots; i++) {
            int32_t x = roots[i];
            if (!consistent(g, &q, f0, 0u, root, x)) continue;
            f0[root] = x;
            int64_t lo = 0, hi = -1;
            const or_pair *arr = NULL;
            const int32_t u2 = n > 1 ? pick_next(g, &q, f0, p0, &lo, &hi, &arr) : -1;
            int split = u2 >= 0 && hi >= 0;
            int64_t a = split ? lo : 0, end = split ? hi : 0;
            do {
                int64_t b = split ? (end - a > OR_PIECE ? a + OR_PIECE : end) : 0;
                while (split && b < end && arr[b].dst == arr[b - 1].dst) b++;
                if (n_items == cap_items) {
                    cap_items = cap_items ? 2 * cap_items : 1024;
                    or_item *t = (or_item *)realloc(items, sizeof(or_item) * (size_t)cap_items);
                    if (!t) {
                        free(items);
                        free(roots);
                        return OR_ENOMEM;
                    }
                    items = t;
                }
                items[n_items].x = x;
                items[n_items].u2 = u2;
                items[n_items].lo = split ? a : 0;
                items[n_items].hi = split ? b : -1;
                items[n_items].arr = arr;
                n_items++;
                a = b;
            } while (split && a < end);
        }
    }
    free(roots);

    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
    or_buf *bufs = (or_buf *)calloc((size_t)nt, sizeof(or_buf));
    if (!bufs) {
        free(items);
        return OR_ENOMEM;
    }
    int64_t total = 0;
    int abort_flag = 0;
    int64_t steps = 0;
#pragma omp parallel num_threads(nt)
    {
        int tid = omp_get_thread_num();
        or_ctx c;
        c.g = g;
        c.q = &q;
        c.buf = &bufs[tid];
        c.count_only = rows_out == NULL;
        c.max_rows = max_rows;
        c.total = &total;
        c.abort_flag = &abort_flag;
        c.max_steps = max_steps;
        c.steps = &steps;
        c.local_steps = 0;
        int32_t f[OR_MAXQ];
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n_items; i++) {
            if (__atomic_load_n(&abort_flag, __ATOMIC_RELAXED)) continue;
            if (over_budget(&c)) continue;
            f[root] = items[i].x;
            if (items[i].hi < 0) dfs(&c, f, 1u << root, 1);
            else dfs_range(&c, f, 1u << root, 1, items[i].u2, items[i].lo, items[i].hi, items[i].arr);
        }
    }
    free(items);
    int failed = 0;
    for (int t = 0; t < nt; t++) failed |= bufs[t].failed;
    if (failed) {
        for (int t = 0; t < nt; t++) free(bufs[t].rows);
        free(bufs);
        return OR_ENOMEM;
    }
    if (abort_flag) {
        for (int t = 0; t < nt; t++) free(bufs[t].rows);
        free(bufs);
        *nrows_out = total;
        return abort_flag == 2 ? OR_EBUDGET : OR_ETOOBIG;
    }
    *nrows_out = total;
    if (rows_out) {
        int32_t *all = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1) * (size_t)n);
        if (!all) {
            for (int t = 0; t < nt; t++) free(bufs[t].rows);
            free(bufs);
            return OR_ENOMEM;
        }
        int64_t off = 0;
        for (int t = 0; t < nt; t++) {
            if (bufs[t].n_rows)
                memcpy(all + (size_t)off * (size_t)n, bufs[t].rows,
                       sizeof(int32_t) * (size_t)bufs[t].n_rows * (size_t)n);
            off += bufs[t].n_rows;
        }
        int nn = n;
        if (total > 1) qsort_r(all, (size_t)total, sizeof(int32_t) * (size_t)n, row_cmp, &nn);
        *rows_out = all;
    }
    for (int t = 0; t < nt; t++) free(bufs[t].rows);
    free(bufs);
    return OR_OK;
}

void oracle_free(void *p) { free(p); }

/* ========================================================================
 * Stage oracles: the query plan, the filtering phase and the candidate-edge
 * counts of the thesis' method, written from its text (Ch. 3) in plain
 * sequential C, for stage-by-stage checks of the GPU path. They share no
 * code with the library.
 * ===================================================================== */

typedef struct {
    int32_t n, m;
    const int32_t *vlabel, *vpin, *esrc, *edst, *elabel;
    uint32_t nbr[OR_MAXQ];  /* undirected neighbour masks */
    int32_t deg[OR_MAXQ], qout[OR_MAXQ], qin[OR_MAXQ];
} st_query;

static void st_query_init(st_query *q, int32_t n, int32_t m, const int32_t *vlabel,
                          const int32_t *vpin, const int32_t *esrc, const int32_t *edst,
                          const int32_t *elabel) {
    memset(q, 0, sizeof(*q));
    q->n = n;
    q->m = m;
    q->vlabel = vlabel;
    q->vpin = vpin;
    q->esrc = esrc;
    q->edst = edst;
    q->elabel = elabel;
    uint32_t outm[OR_MAXQ] = {0}, inm[OR_MAXQ] = {0};
    for (int i = 0; i < m; i++) {
        outm[esrc[i]] |= 1u << edst[i];
        inm[edst[i]] |= 1u << esrc[i];
    }
    for (int u = 0; u < n; u++) {
        q->nbr[u] = outm[u] | inm[u];
        q->deg[u] = __builtin_popcount(q->nbr[u]);
        q->qout[u] = __builtin_popcount(outm[u]);
        q->qin[u] = __builtin_popcount(inm[u]);
    }
}

/* f(u) = deg(u) / freq(u): a concept (pinned) node has frequency 1, a
 * variable node the number of data vertices of its type (all V for -1). */
static int64_t st_freq(const oracle_graph *g, const st_query *q, int u) {
    if (q->vpin[u] >= 0) return 1;
    if (q->vlabel[u] < 0) return g->V;
    int64_t c = 0;
    for (int32_t v = 0; v < g->V; v++) c += g->vtype[v] == q->vlabel[u];
    return c > 0 ? c : 1;
}

/*
 * Query plan (Ch. 3 Sec. "Query Plan Generation", commonsense variant of
 * Sec. "GpSense"): a query with concept (pinned) nodes starts at the concept
 * node of maximum degree (lowest id on ties), the commonsense rule; a query
 * without any starts at the first query edge maximising f(a) + f(b) (lowest
 * edge index on ties), at its endpoint of larger f (lower id on ties), the
 * general rule; expanding a vertex adds its unreached neighbours to the spanning
 * tree (parent edge = lowest-index edge between them); the next vertex to
 * expand is the reached, unexpanded one with the most unreached neighbours
 * (then larger f, then lower id), until every vertex is reached.
 * visit[], init_order[]: -1 padded to OR_MAXQ... sized n by the caller.
 */
int oracle_plan(const oracle_graph *g, int32_t n, int32_t m, const int32_t *vlabel,
                const int32_t *vpin, const int32_t *esrc, const int32_t *edst,
                const int32_t *elabel, int32_t *visit, int32_t *parent, int32_t *parent_edge,
                int32_t *init_order) {
    if (!g || !query_ok(g->V, n, m, vpin, esrc, edst)) return OR_EINVAL;
    st_query q;
    st_query_init(&q, n, m, vlabel, vpin, esrc, edst, elabel);
    int64_t fnum[OR_MAXQ], fden[OR_MAXQ];
    for (int u = 0; u < n; u++) {
        fnum[u] = q.deg[u];
        fden[u] = st_freq(g, &q, u);
        visit[u] = -1;
        parent[u] = -1;
        parent_edge[u] = -1;
        init_order[u] = -1;
    }
    int nv = 0, ni = 0;
    if (m == 0) {
        visit[0] = 0;
        init_order[0] = 0;
        return OR_OK;
    }
    int root = -1;
    for (int v = 0; v < n; v++)
        if (vpin[v] >= 0 && (root < 0 || q.deg[v] > q.deg[root])) root = v;
    if (root < 0) {
        int best = 0;
        for (int i = 1; i < m; i++) {
            int a = esrc[best], b = edst[best], c = esrc[i], d = edst[i];
            __int128 lhs = ((__int128)fnum[a] * fden[b] + (__int128)fnum[b] * fden[a]) *
                           ((__int128)fden[c] * fden[d]);
            __int128 rhs = ((__int128)fnum[c] * fden[d] + (__int128)fnum[d] * fden[c]) *
                           ((__int128)fden[a] * fden[b]);
            if (rhs > lhs) best = i;
        }
        int a = esrc[best], b = edst[best];
        __int128 fa = (__int128)fnum[a] * fden[b], fb = (__int128)fnum[b] * fden[a];
        root = fa > fb ? a : fb > fa ? b : (a < b ? a : b);
    }
    uint32_t reached = 1u << root, expanded = 0;
    init_order[ni++] = root;
    int u = root;
    for (;;) {
        expanded |= 1u << u;
        visit[nv++] = u;
        for (int x = 0; x < n; x++) {
            if (!((q.nbr[u] >> x) & 1u) || ((reached >> x) & 1u)) continue;
            reached |= 1u << x;
            parent[x] = u;
            for (int i = 0; i < m; i++)
                if ((esrc[i] == u && edst[i] == x) || (esrc[i] == x && edst[i] == u)) {
                    parent_edge[x] = i;
                    break;
                }
            init_order[ni++] = x;
        }
        if (__builtin_popcount(reached) == n) break;
        int nxt = -1, nn_best = 0;
        for (int v = 0; v < n; v++) {
            if (!((reached >> v) & 1u) || ((expanded >> v) & 1u)) continue;
            int nn = __builtin_popcount(q.nbr[v] & ~reached);
            if (nn == 0) continue;
            int better = nxt < 0 || nn > nn_best;
            if (!better && nn == nn_best) {
                __int128 fv = (__int128)fnum[v] * fden[nxt], fx = (__int128)fnum[nxt] * fden[v];
                better = fv > fx;
            }
            if (better) {
                nxt = v;
                nn_best = nn;
            }
        }
        if (nxt < 0) return OR_EINVAL;
        u = nxt;
    }
    return OR_OK;
}

/* Candidate predicate (Def. 3.3): type and pin, and at least as many data
 * out-edges (in-edges) as the query vertex has distinct out-neighbours
 * (in-neighbours). */
static int st_pred(const oracle_graph *g, const st_query *q, int u, int32_t v) {
    if (q->vpin[u] >= 0 && v != q->vpin[u]) return 0;
    if (q->vlabel[u] >= 0 && g->vtype[v] != q->vlabel[u]) return 0;
    if (g->out_off[v + 1] - g->out_off[v] < q->qout[u]) return 0;
    if (g->in_off[v + 1] - g->in_off[v] < q->qin[u]) return 0;
    return 1;
}

/* Does x have a neighbour y (out-neighbour for dir 0, in-neighbour for dir
 * 1) joined by relation rho (-1: any) with ok[y]? ok == NULL: the predicate
 * of query vertex w. When push != NULL, mark every such y instead and return
 * whether any exists. */
static int st_scan(const oracle_graph *g, const st_query *q, int32_t x, int dir, int32_t rho,
                   const uint8_t *ok, int w, uint8_t *push) {
    const int64_t *off = dir ? g->in_off : g->out_off;
    const or_pair *arr = dir ? g->in : g->out;
    int any = 0;
    for (int64_t k = off[x]; k < off[x + 1]; k++) {
        if (rho >= 0 && arr[k].rel != rho) continue;
        int32_t y = arr[k].dst;
        int good = ok ? ok[y] : st_pred(g, q, w, y);
        if (!good) continue;
        any = 1;
        if (!push) return 1;
        push[y] = 1;
    }
    return any;
}

/*
 * Candidate sets after the filtering phase: the initialisation of Alg. 3.2
 * along the plan's spanning tree (kernel_check for the first vertex of the
 * visit order, then for each visited vertex u: prune the candidates u' of u
 * lacking, for some tree neighbour w, a neighbour that is a candidate of w --
 * w's set if already initialised, w's predicate otherwise -- and push the
 * matching neighbours: an uninitialised w receives them as its set, an
 * initialised one is intersected with them), followed by `rounds` rounds
 * of refinement (Sec. "Candidate Nodes Refinement"; -1: until nothing is
 * removed): every vertex of more than low_conn distinct neighbours, in
 * reversed (or forward) order of initialisation, is pruned against every
 * query edge to such a vertex.
 * cand: out, [n][V] bytes (1 = candidate).
 */
int oracle_filter(const oracle_graph *g, int32_t n, int32_t m, const int32_t *vlabel,
                  const int32_t *vpin, const int32_t *esrc, const int32_t *edst,
                  const int32_t *elabel, int32_t rounds, int32_t reversed, int32_t low_conn,
                  uint8_t *cand) {
    int32_t visit[OR_MAXQ], parent[OR_MAXQ], pedge[OR_MAXQ], init[OR_MAXQ];
    int rc = oracle_plan(g, n, m, vlabel, vpin, esrc, edst, elabel, visit, parent, pedge, init);
    if (rc != OR_OK) return rc;
    st_query q;
    st_query_init(&q, n, m, vlabel, vpin, esrc, edst, elabel);
    const int32_t V = g->V;
    memset(cand, 0, (size_t)n * (size_t)V);
    uint8_t *push = (uint8_t *)malloc((size_t)V);
    uint8_t *alive = (uint8_t *)malloc((size_t)V);
    if (!push || !alive) {
        free(push);
        free(alive);
        return OR_ENOMEM;
    }
    int initialized[OR_MAXQ] = {0};
    for (int oi = 0; oi < n && visit[oi] >= 0; oi++) {
        const int u = visit[oi];
        uint8_t *cu = cand + (size_t)u * V;
        if (!initialized[u]) {
            for (int32_t v = 0; v < V; v++) cu[v] = (uint8_t)st_pred(g, &q, u, v);
            initialized[u] = 1;
        }
        /* tree neighbours: parent first, then children */
        int tw[OR_MAXQ], te[OR_MAXQ], nt = 0;
        if (parent[u] >= 0) {
            tw[nt] = parent[u];
            te[nt++] = pedge[u];
        }
        for (int x = 0; x < n; x++)
            if (parent[x] == u) {
                tw[nt] = x;
                te[nt++] = pedge[x];
            }
        if (nt == 0) continue;
        /* prune against the state at the start of the step */
        for (int32_t v = 0; v < V; v++) {
            alive[v] = cu[v];
            if (!cu[v]) continue;
            for (int t = 0; t < nt && alive[v]; t++) {
                const int w = tw[t], e = te[t];
                const int dir = esrc[e] == u ? 0 : 1;
                alive[v] = (uint8_t)st_scan(g, &q, v, dir, elabel[e],
                                            initialized[w] ? cand + (size_t)w * V : NULL, w, NULL);
            }
        }
        for (int t = 0; t < nt; t++) {
            const int w = tw[t], e = te[t];
            const int dir = esrc[e] == u ? 0 : 1;
            uint8_t *cw = cand + (size_t)w * V;
            memset(push, 0, (size_t)V);
            for (int32_t v = 0; v < V; v++)
                if (alive[v])
                    st_scan(g, &q, v, dir, elabel[e], initialized[w] ? cw : NULL, w, push);
            if (initialized[w])
                for (int32_t y = 0; y < V; y++) cw[y] &= push[y];
            else
                memcpy(cw, push, (size_t)V);
        }
        memcpy(cu, alive, (size_t)V);
        for (int t = 0; t < nt; t++) initialized[tw[t]] = 1;
    }
    /* refinement */
    int order[OR_MAXQ], no = 0;
    for (int i = 0; i < n; i++) {
        const int u = init[reversed ? n - 1 - i : i];
        if (q.deg[u] > low_conn) order[no++] = u;
    }
    const int max_rounds = rounds < 0 ? 32 : rounds;
    for (int r = 0; r < max_rounds; r++) {
        int64_t removed = 0;
        for (int oi = 0; oi < no; oi++) {
            const int u = order[oi];
            uint8_t *cu = cand + (size_t)u * V;
            int ne = 0;
            for (int e = 0; e < m; e++) {
                const int w = esrc[e] == u ? edst[e] : edst[e] == u ? esrc[e] : -1;
                if (w >= 0 && q.deg[w] > low_conn) ne++;
            }
            if (ne == 0) continue;
            for (int32_t v = 0; v < V; v++) {
                if (!cu[v]) continue;
                int ok = 1;
                for (int e = 0; e < m && ok; e++) {
                    int w, dir;
                    if (esrc[e] == u) {
                        w = edst[e];
                        dir = 0;
                    } else if (edst[e] == u) {
                        w = esrc[e];
                        dir = 1;
                    } else {
                        continue;
                    }
                    if (q.deg[w] <= low_conn) continue;
                    ok = st_scan(g, &q, v, dir, elabel[e], cand + (size_t)w * V, w, NULL);
                }
                if (!ok) {
                    cu[v] = 0;
                    removed++;
                }
            }
        }
        if (rounds < 0 && removed == 0) break;
    }
    free(push);
    free(alive);
    return OR_OK;
}

/* Candidate edges of every query edge (a, b, rho) given candidate sets:
 * #{(x, y) : cand[a][x], cand[b][y], x != y, some data edge (x, y, r) with
 * rho = -1 or r = rho} (Sec. "Joining Phase"). ec: out, [m]. */
int oracle_edge_candidates(const oracle_graph *g, int32_t n, int32_t m, const int32_t *esrc,
                           const int32_t *edst, const int32_t *elabel, const uint8_t *cand,
                           int64_t *ec) {
    if (!g) return OR_EINVAL;
    const int32_t V = g->V;
    for (int e = 0; e < m; e++) {
        const int a = esrc[e], b = edst[e];
        if (a < 0 || a >= n || b < 0 || b >= n) return OR_EINVAL;
        int64_t c = 0;
        for (int32_t x = 0; x < V; x++) {
            if (!cand[(size_t)a * V + x]) continue;
            int32_t prev = -1;
            for (int64_t k = g->out_off[x]; k < g->out_off[x + 1]; k++) {
                const int32_t y = g->out[k].dst;
                if (elabel[e] >= 0 && g->out[k].rel != elabel[e]) continue;
                if (y == prev) continue;
                prev = y;
                if (y != x && cand[(size_t)b * V + y]) c++;
            }
        }
        ec[e] = c;
    }
    return OR_OK;
}
