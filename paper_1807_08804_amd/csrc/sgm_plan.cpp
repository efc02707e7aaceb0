// Host-side query checks and query plan (no device code).
//
// Plan: thesis Ch. 3, Sec. "Query Plan Generation" (rank f(u) = deg(u) /
// freq(u.label); first edge maximising f(u) + f(v); spanning tree T and
// visit order O of expanded vertices) and the commonsense variant of Sec.
// "GpSense" (a query with concept nodes starts at the concept node of
// maximum degree; the next vertex is the one whose adjacency holds the most
// vertices not yet reached; stop once the tree covers the query).
#include "sgm_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace sgm {

int check_query(const sgm_query *q, int32_t V, QInfo *qi) {
    if (!q) return SGM_EINVAL;
    const int n = q->n_vertices, m = q->n_edges;
    if (n < 1 || m < 0) return SGM_EINVAL;
    if (n > SGM_MAX_QV || m > SGM_MAX_QE) return SGM_EUNSUPPORTED;
    if (!q->vertex_label || !q->vertex_pin || (m > 0 && (!q->edge_src || !q->edge_dst || !q->edge_label)))
        return SGM_EINVAL;
    std::memset(qi, 0, sizeof(*qi));
    qi->n = n;
    qi->m = m;
    for (int u = 0; u < n; ++u) {
        qi->label[u] = q->vertex_label[u];
        qi->pin[u] = q->vertex_pin[u];
        if (qi->label[u] < -1 || qi->pin[u] < -1 || qi->pin[u] >= V) return SGM_EINVAL;
    }
    for (int i = 0; i < m; ++i) {
        const int a = q->edge_src[i], b = q->edge_dst[i], r = q->edge_label[i];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b || r < -1) return SGM_EINVAL;
        for (int j = 0; j < i; ++j)
            if (qi->esrc[j] == a && qi->edst[j] == b && qi->elabel[j] == r) return SGM_EINVAL;
        qi->esrc[i] = a;
        qi->edst[i] = b;
        qi->elabel[i] = r;
        qi->out_mask[a] |= 1u << b;
        qi->in_mask[b] |= 1u << a;
    }
    for (int u = 0; u < n; ++u) {
        qi->qout[u] = __builtin_popcount(qi->out_mask[u]);
        qi->qin[u] = __builtin_popcount(qi->in_mask[u]);
        qi->deg[u] = __builtin_popcount(qi->out_mask[u] | qi->in_mask[u]);
    }
    // connected (undirected)
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t next = 0;
        for (int u = 0; u < n; ++u)
            if (frontier & (1u << u)) next |= qi->out_mask[u] | qi->in_mask[u];
        next &= ~seen;
        seen |= next;
        frontier = next;
    }
    if (seen != ((n == 32) ? 0xffffffffu : ((1u << n) - 1u))) return SGM_EINVAL;
    qi->proj = 0;
    qi->n_out = n;
    return SGM_OK;
}

int set_projection(QInfo *qi, uint32_t mask) {
    const uint32_t all = (1u << qi->n) - 1u;
    if (mask == 0 || (mask & ~all)) return SGM_EINVAL;
    qi->proj = mask == all ? 0u : mask;
    qi->n_out = __builtin_popcount(mask);
    return SGM_OK;
}

namespace {

// f(u) = deg(u) / freq(u) as an exact fraction
struct Frac {
    int64_t num, den;
};

Frac rank_f(const QInfo &qi, int u, int32_t V, const int64_t *type_freq, int32_t n_types) {
    int64_t freq;
    if (qi.pin[u] >= 0) freq = 1;
    else if (qi.label[u] < 0) freq = V;
    else freq = (qi.label[u] < n_types) ? type_freq[qi.label[u]] : 0;
    if (freq < 1) freq = 1;  // no data vertex of this type: no match either way
    return Frac{qi.deg[u], freq};
}

// a < b for non-negative fractions
bool frac_less(Frac a, Frac b) {
    return (__int128)a.num * b.den < (__int128)b.num * a.den;
}

bool sum_less(Frac a1, Frac a2, Frac b1, Frac b2) {
    // (a1 + a2) < (b1 + b2) with 128-bit intermediates
    const __int128 an = (__int128)a1.num * a2.den + (__int128)a2.num * a1.den;
    const __int128 ad = (__int128)a1.den * a2.den;
    const __int128 bn = (__int128)b1.num * b2.den + (__int128)b2.num * b1.den;
    const __int128 bd = (__int128)b1.den * b2.den;
    // an/ad < bn/bd  <=>  an*bd < bn*ad ; magnitudes: an <= 2^36, bd <= 2^62
    // -> products <= 2^98 fit in 128 bits
    return an * bd < bn * ad;
}

}  // namespace

int make_plan(const QInfo &qi, int32_t V, const int64_t *type_freq, int32_t n_types, Plan *p) {
    const int n = qi.n, m = qi.m;
    std::memset(p, 0, sizeof(*p));
    for (int u = 0; u < SGM_MAX_QV; ++u) {
        p->parent[u] = -1;
        p->parent_edge[u] = -1;
        p->visit[u] = -1;
        p->init[u] = -1;
    }
    Frac f[SGM_MAX_QV];
    for (int u = 0; u < n; ++u) f[u] = rank_f(qi, u, V, type_freq, n_types);
    if (m == 0) {
        p->n_visit = 1;
        p->visit[0] = 0;
        p->n_init = 1;
        p->init[0] = 0;
        return SGM_OK;
    }
    // commonsense rule: the concept (pinned) node of maximum degree, lowest
    // id on ties
    int root = -1;
    for (int v = 0; v < n; ++v)
        if (qi.pin[v] >= 0 && (root < 0 || qi.deg[v] > qi.deg[root])) root = v;
    if (root < 0) {
        // general rule: first edge of maximum f(a) + f(b), lowest edge index
        // on ties; its endpoint with f(u) >= f(v), lower vertex id if equal
        int best = 0;
        for (int i = 1; i < m; ++i)
            if (sum_less(f[qi.esrc[best]], f[qi.edst[best]], f[qi.esrc[i]], f[qi.edst[i]]))
                best = i;
        const int a = qi.esrc[best], b = qi.edst[best];
        if (frac_less(f[a], f[b])) root = b;
        else if (frac_less(f[b], f[a])) root = a;
        else root = std::min(a, b);
    }

    uint32_t in_tree = 0, expanded = 0;
    auto nbr_mask = [&](int u) { return qi.out_mask[u] | qi.in_mask[u]; };
    auto lowest_edge = [&](int u, int v) {
        for (int i = 0; i < m; ++i)
            if ((qi.esrc[i] == u && qi.edst[i] == v) || (qi.esrc[i] == v && qi.edst[i] == u))
                return i;
        return -1;
    };
    auto expand = [&](int u) {
        expanded |= 1u << u;
        p->visit[p->n_visit++] = u;
        const uint32_t nb = nbr_mask(u) & ~in_tree;
        for (int x = 0; x < n; ++x) {
            if (!(nb & (1u << x))) continue;
            in_tree |= 1u << x;
            p->parent[x] = u;
            p->parent_edge[x] = lowest_edge(u, x);
            p->init[p->n_init++] = x;
        }
    };
    in_tree |= 1u << root;
    p->init[p->n_init++] = root;
    expand(root);
    const uint32_t all = (1u << n) - 1u;
    while (in_tree != all) {
        // next: reached but unexpanded vertex whose adjacency holds the most
        // unreached vertices; then larger f; then lower id
        int nxt = -1, nxt_new = 0;
        for (int v = 0; v < n; ++v) {
            if (!(in_tree & (1u << v)) || (expanded & (1u << v))) continue;
            const int nn = __builtin_popcount(nbr_mask(v) & ~in_tree);
            if (nn == 0) continue;
            if (nxt < 0 || nn > nxt_new || (nn == nxt_new && frac_less(f[nxt], f[v]))) {
                nxt = v;
                nxt_new = nn;
            }
        }
        if (nxt < 0) return SGM_EINVAL;  // disconnected (checked earlier)
        expand(nxt);
    }
    return SGM_OK;
}

void build_program(const QInfo &qi, const Plan &pl, int low_conn_degree, int refine_reversed,
                   Program *pr) {
    pr->init.clear();
    pr->refine.clear();
    pr->nbr.clear();
    const int n = qi.n;
    bool initialized[SGM_MAX_QV] = {};
    for (int oi = 0; oi < pl.n_visit; ++oi) {
        const int u = pl.visit[oi];
        initialized[u] = true;
        PStep s{u, (int)pr->nbr.size(), 0, 1, -1, 0};
        auto add = [&](int v, int e) {
            PNbr d{};
            d.v = v;
            d.dir = qi.esrc[e] == u ? 0 : 1;
            d.rel = qi.elabel[e];
            d.mode = initialized[v] ? 0 : 1;
            if (initialized[v]) s.parent = v;
            pr->nbr.push_back(d);
        };
        if (pl.parent[u] >= 0) add(pl.parent[u], pl.parent_edge[u]);
        for (int x = 0; x < n; ++x)
            if (pl.parent[x] == u) add(x, pl.parent_edge[x]);
        s.count = (int)pr->nbr.size() - s.first;
        if (s.count) pr->init.push_back(s);
        for (int x = 0; x < n; ++x)
            if (pl.parent[x] == u) initialized[x] = true;
    }
    for (int i = 0; i < pl.n_init; ++i) {
        const int u = pl.init[refine_reversed ? pl.n_init - 1 - i : i];
        if (qi.deg[u] <= low_conn_degree) continue;
        PStep s{u, (int)pr->nbr.size(), 0, 0, -1, 0};
        for (int e = 0; e < qi.m; ++e) {
            PNbr d{};
            if (qi.esrc[e] == u) {
                d.v = qi.edst[e];
                d.dir = 0;
            } else if (qi.edst[e] == u) {
                d.v = qi.esrc[e];
                d.dir = 1;
            } else {
                continue;
            }
            if (qi.deg[d.v] <= low_conn_degree) continue;
            d.rel = qi.elabel[e];
            d.mode = 0;
            pr->nbr.push_back(d);
        }
        s.count = (int)pr->nbr.size() - s.first;
        if (s.count) pr->refine.push_back(s);
    }
}

void build_program_out_only(const QInfo &qi, const Plan &pl, int low_conn_degree,
                            int refine_reversed, Program *pr) {
    pr->init.clear();
    pr->refine.clear();
    pr->nbr.clear();
    const int n = qi.n;
    bool swept[SGM_MAX_QV] = {};
    auto nbr = [&](int v, int32_t rel, int mode) {
        PNbr d{};
        d.v = v;
        d.dir = 0;
        d.rel = rel;
        d.mode = mode;
        pr->nbr.push_back(d);
    };
    for (int oi = 0; oi < pl.n_visit; ++oi) {
        const int u = pl.visit[oi];
        PStep s{u, (int)pr->nbr.size(), 0, 1, -1, 0};
        // the tree edge u -> parent, unless u's sweep step has tested it
        const int pe = pl.parent_edge[u];
        if (pl.parent[u] >= 0 && qi.esrc[pe] == u && !swept[u]) {
            nbr(pl.parent[u], qi.elabel[pe], 0);
            s.parent = pl.parent[u];
        }
        for (int x = 0; x < n; ++x)
            if (pl.parent[x] == u && qi.esrc[pl.parent_edge[x]] == u)
                nbr(x, qi.elabel[pl.parent_edge[x]], 1);
        s.count = (int)pr->nbr.size() - s.first;
        if (s.count) pr->init.push_back(s);
        // children with an edge into u: swept, then tested against u
        for (int x = 0; x < n; ++x) {
            if (pl.parent[x] != u || qi.esrc[pl.parent_edge[x]] != x) continue;
            PStep t{x, (int)pr->nbr.size(), 1, 1, u, 1};
            nbr(u, qi.elabel[pl.parent_edge[x]], 0);
            pr->init.push_back(t);
            swept[x] = true;
        }
    }
    for (int i = 0; i < pl.n_init; ++i) {
        const int u = pl.init[refine_reversed ? pl.n_init - 1 - i : i];
        if (qi.deg[u] <= low_conn_degree) continue;
        // out-edges of u: tested on u's candidates
        PStep s{u, (int)pr->nbr.size(), 0, 0, -1, 0};
        for (int e = 0; e < qi.m; ++e)
            if (qi.esrc[e] == u && qi.deg[qi.edst[e]] > low_conn_degree)
                nbr(qi.edst[e], qi.elabel[e], 0);
        s.count = (int)pr->nbr.size() - s.first;
        if (s.count) pr->refine.push_back(s);
        // edges v -> u: a step on v pushing into u
        for (int e = 0; e < qi.m; ++e) {
            const int v = qi.esrc[e];
            if (qi.edst[e] != u || qi.deg[v] <= low_conn_degree) continue;
            PStep t{v, (int)pr->nbr.size(), 1, 1, u, 0};
            nbr(u, qi.elabel[e], 0);
            pr->refine.push_back(t);
        }
    }
}

}  // namespace sgm

namespace sgm {

// Rows of the join levels estimated along the spanning tree of the plan, in
// the order its vertices enter the tree: the root starts with as many rows
// as it has candidates by label (1 if pinned); a vertex reached over a tree
// edge of relation r multiplies the rows by the average number of r-edges
// per data vertex and by the fraction of data vertices its label admits (1/V
// if pinned); every further query edge between vertices already placed
// multiplies them by the chance that a given ordered pair carries such an
// edge. Level k's table holds k + 1 int32 columns; a level's input and
// output tables are live together. The thesis ties the join's running time
// and partial-solution memory to candidate counts (Sec. "Joining Phase");
// this is the cheap, graph-statistics form of that dependence.
int64_t estimate_bytes(const QInfo &qi, const Plan &pl, int32_t V, int64_t E,
                       const int64_t *type_freq, int32_t n_types, const int64_t *rel_freq,
                       int32_t n_rels) {
    const double dV = std::max<double>(V, 1);
    auto admitted = [&](int u) -> double {
        if (qi.pin[u] >= 0) return 1.0;
        if (qi.label[u] < 0) return dV;
        return qi.label[u] < n_types ? (double)type_freq[qi.label[u]] : 0.0;
    };
    auto per_vertex = [&](int32_t r) -> double {
        const double cnt = r < 0 ? (double)E : (r < n_rels ? (double)rel_freq[r] : 0.0);
        return cnt / dV;
    };
    bool placed[SGM_MAX_QV] = {};
    double rows = 0, prev_bytes = 0, peak = 0;
    for (int k = 0; k < pl.n_init; ++k) {
        const int u = pl.init[k];
        if (k == 0) {
            rows = admitted(u);
        } else {
            const int e = pl.parent_edge[u];
            rows *= per_vertex(qi.elabel[e]) * admitted(u) / dV;
        }
        placed[u] = true;
        for (int i = 0; i < qi.m; ++i) {
            if (k > 0 && i == pl.parent_edge[u]) continue;
            const int a = qi.esrc[i], b = qi.edst[i];
            if ((a == u && placed[b]) || (b == u && placed[a]))
                rows *= std::min(1.0, per_vertex(qi.elabel[i]) / dV);
        }
        const double bytes = rows * 4.0 * (k + 1);
        peak = std::max(peak, prev_bytes + bytes);
        prev_bytes = bytes;
    }
    const double bitmaps = (double)qi.n * 8.0 * std::ceil(dV / 64.0);
    const double est = bitmaps + peak;
    return est >= 9.0e18 ? INT64_MAX : (int64_t)std::ceil(est);
}

}  // namespace sgm

extern "C" int sgm_estimate_query(const sgm_query *q, int32_t n_vertices, int64_t n_edges,
                                  const int64_t *type_freq, int32_t n_types,
                                  const int64_t *rel_freq, int32_t n_rels, int64_t *est_bytes) {
    if (!est_bytes || n_vertices < 1 || n_edges < 0 || n_types < 0 || n_rels < 0 ||
        (n_types > 0 && !type_freq) || (n_rels > 0 && !rel_freq))
        return SGM_EINVAL;
    *est_bytes = 0;
    sgm::QInfo qi;
    int rc = sgm::check_query(q, n_vertices, &qi);
    if (rc != SGM_OK) return rc;
    sgm::Plan p;
    rc = sgm::make_plan(qi, n_vertices, type_freq, n_types, &p);
    if (rc != SGM_OK) return rc;
    *est_bytes = sgm::estimate_bytes(qi, p, n_vertices, n_edges, type_freq, n_types, rel_freq,
                                     n_rels);
    return SGM_OK;
}

extern "C" int sgm_plan_query(const sgm_query *q, int32_t n_vertices, const int64_t *type_freq,
                              int32_t n_types, int32_t *visit_order, int32_t *parent,
                              int32_t *parent_edge, int32_t *init_order) {
    if (n_vertices < 1 || (n_types > 0 && !type_freq) || n_types < 0) return SGM_EINVAL;
    sgm::QInfo qi;
    int rc = sgm::check_query(q, n_vertices, &qi);
    if (rc != SGM_OK) return rc;
    sgm::Plan p;
    rc = sgm::make_plan(qi, n_vertices, type_freq, n_types, &p);
    if (rc != SGM_OK) return rc;
    for (int u = 0; u < SGM_MAX_QV; ++u) {
        if (visit_order) visit_order[u] = p.visit[u];
        if (parent) parent[u] = p.parent[u];
        if (parent_edge) parent_edge[u] = p.parent_edge[u];
        if (init_order) init_order[u] = p.init[u];
    }
    return SGM_OK;
}
