// Multi-level graph compression (thesis Ch. 3, Sec. "Multi-level Graph
// Compression"): an offline host step that merges similar vertices into
// weighted vertices, level by level, and keeps the mapping lists M(x).
//
// Per level, on the current weighted graph:
// * Two vertices of one type are similar when they share enough "common
//   edges" e(l, z): the same relation l to, or from, the same vertex z. The
//   thesis prints the test as a ratio of adjacency size to common edges
//   compared with a threshold 0 < delta <= 1, which no pair could fail;
//   read as the share of a vertex's entries that are common,
//   max(|common| / |adj(u)|, |common| / |adj(v)|) >= delta.
// * Pairs are formed greedily in ascending vertex order: each unpaired
//   vertex takes, among unpaired vertices of its type that share one of its
//   first 8 entries (at most max_partners looked at per entry, found among
//   at most 8 max_partners entries of the shared neighbour), the most
//   similar one that passes the test (ties: the lowest id). The thesis does
//   not fix the pairing.
// * A pair {p, q} becomes one weighted vertex X with M(X) = M(p) u M(q).
//   Every entry keeps its relation and direction. Its weight follows
//   Def. 3.4: w(X -> Y, l) = sum over the parts y of Y of the max over the
//   parts x of X of w(x -> y, l), with weight 1 for every original edge; an
//   edge between the two parts becomes a self-loop, whose weight plays the
//   part of the vertex weight w(X). So w(X -> Y, l) bounds, for any original
//   vertex of M(X), its l-edges into M(Y), and the sum of a vertex's entry
//   weights bounds the degree of each of its original vertices (Def. 3.5,
//   used by Thm. 3.1); incoming entries are weighted the same way.
// * Levels stop at max_levels, when a level merges nothing, or once
//   (|V_i| + |E_i|) / (|V| + |E|) falls to target_ratio.
#include <stdint.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/sgm.h"

namespace {

struct Ent {
    int32_t nb, rel, w;
};

// One level's graph: per vertex its out- and in-entries sorted by
// (neighbour, relation), its type and its mapping list.
struct WGraph {
    int32_t n = 0;
    std::vector<int64_t> ooff, ioff;
    std::vector<Ent> oe, ie;
    std::vector<int32_t> type;
    std::vector<int64_t> moff;
    std::vector<int32_t> mids;
    int64_t entries() const { return (int64_t)oe.size(); }
};

bool ent_less(const Ent &a, const Ent &b) { return a.nb != b.nb ? a.nb < b.nb : a.rel < b.rel; }

// entries (neighbour, relation) that both sorted lists hold
int64_t common_count(const Ent *a, int64_t na, const Ent *b, int64_t nb) {
    int64_t i = 0, j = 0, c = 0;
    while (i < na && j < nb) {
        if (ent_less(a[i], b[j])) ++i;
        else if (ent_less(b[j], a[i])) ++j;
        else {
            ++c;
            ++i;
            ++j;
        }
    }
    return c;
}

int64_t common_edges(const WGraph &g, int32_t u, int32_t v) {
    return common_count(&g.oe[g.ooff[u]], g.ooff[u + 1] - g.ooff[u], &g.oe[g.ooff[v]],
                        g.ooff[v + 1] - g.ooff[v]) +
           common_count(&g.ie[g.ioff[u]], g.ioff[u + 1] - g.ioff[u], &g.ie[g.ioff[v]],
                        g.ioff[v + 1] - g.ioff[v]);
}

int64_t adj_size(const WGraph &g, int32_t u) {
    return (g.ooff[u + 1] - g.ooff[u]) + (g.ioff[u + 1] - g.ioff[u]);
}

// Greedy pairing of one level; part[u] = the new vertex of u.
int32_t pair_up(const WGraph &g, double delta, int32_t max_partners, std::vector<int32_t> &part) {
    const int32_t n = g.n;
    std::vector<int32_t> mate((size_t)n, -1);
    const int kEntriesTried = 8;   // first entries of u whose sharers are looked at
    const int64_t kScanCap = 8;    // entries read per sharer found, at most
    for (int32_t u = 0; u < n; ++u) {
        if (mate[u] >= 0) continue;
        const int64_t au = adj_size(g, u);
        if (au == 0) continue;
        int32_t best = -1;
        double best_s = -1.0;
        auto consider = [&](int32_t v) {
            if (v == u || mate[v] >= 0 || g.type[v] != g.type[u] || (best >= 0 && v >= best && best_s >= 1.0))
                return;
            const int64_t av = adj_size(g, v);
            if (av == 0) return;
            const int64_t c = common_edges(g, u, v);
            if (c == 0) return;
            const double s = std::max((double)c / (double)au, (double)c / (double)av);
            if (s >= delta && (s > best_s || (s == best_s && v < best))) {
                best = v;
                best_s = s;
            }
        };
        // vertices sharing an out-entry (l, z) of u: the l-sources among z's
        // in-entries; sharing an in-entry (l, y): the l-targets of y
        int tried = 0;
        for (int64_t i = g.ooff[u]; i < g.ooff[u + 1] && tried < kEntriesTried; ++i, ++tried) {
            const Ent &e = g.oe[i];
            int32_t seen = 0;
            const int64_t k1 = std::min(g.ioff[e.nb + 1], g.ioff[e.nb] + kScanCap * max_partners);
            for (int64_t k = g.ioff[e.nb]; k < k1 && seen < max_partners; ++k)
                if (g.ie[k].rel == e.rel) {
                    consider(g.ie[k].nb);
                    ++seen;
                }
        }
        tried = 0;
        for (int64_t i = g.ioff[u]; i < g.ioff[u + 1] && tried < kEntriesTried; ++i, ++tried) {
            const Ent &e = g.ie[i];
            int32_t seen = 0;
            const int64_t k1 = std::min(g.ooff[e.nb + 1], g.ooff[e.nb] + kScanCap * max_partners);
            for (int64_t k = g.ooff[e.nb]; k < k1 && seen < max_partners; ++k)
                if (g.oe[k].rel == e.rel) {
                    consider(g.oe[k].nb);
                    ++seen;
                }
        }
        if (best >= 0) {
            mate[u] = best;
            mate[best] = u;
        }
    }
    part.assign((size_t)n, -1);
    int32_t nn = 0, merged = 0;
    for (int32_t u = 0; u < n; ++u) {
        if (part[u] >= 0) continue;
        part[u] = nn;
        if (mate[u] >= 0) {
            part[mate[u]] = nn;
            ++merged;
        }
        ++nn;
    }
    return merged;
}

// Entries of the merged vertices in one direction: for each new vertex X,
// sum over the parts y of each neighbour Y of the max over X's parts.
void merge_entries(const WGraph &g, const std::vector<int64_t> &off, const std::vector<Ent> &ents,
                   const std::vector<int32_t> &part, const std::vector<int64_t> &poff,
                   const std::vector<int32_t> &pmem, int32_t nn, std::vector<int64_t> &noff,
                   std::vector<Ent> &nents) {
    noff.assign((size_t)nn + 1, 0);
    nents.clear();
    struct T {
        int32_t Y, rel, y, w;
    };
    std::vector<T> t;
    for (int32_t X = 0; X < nn; ++X) {
        t.clear();
        for (int64_t m = poff[X]; m < poff[X + 1]; ++m) {
            const int32_t x = pmem[m];
            for (int64_t i = off[x]; i < off[x + 1]; ++i)
                t.push_back(T{part[ents[i].nb], ents[i].rel, ents[i].nb, ents[i].w});
        }
        std::sort(t.begin(), t.end(), [](const T &a, const T &b) {
            if (a.Y != b.Y) return a.Y < b.Y;
            if (a.rel != b.rel) return a.rel < b.rel;
            if (a.y != b.y) return a.y < b.y;
            return a.w > b.w;
        });
        size_t i = 0;
        while (i < t.size()) {
            size_t j = i;
            int32_t sum = 0;
            while (j < t.size() && t[j].Y == t[i].Y && t[j].rel == t[i].rel) {
                // first of each (Y, rel, y) run holds the max over X's parts
                if (j == i || t[j].y != t[j - 1].y) sum += t[j].w;
                ++j;
            }
            nents.push_back(Ent{t[i].Y, t[i].rel, sum});
            i = j;
        }
        noff[X + 1] = (int64_t)nents.size();
    }
    (void)g;
}

void next_level(const WGraph &g, const std::vector<int32_t> &part, int32_t nn, WGraph &h) {
    // parts of every new vertex, in ascending old id
    std::vector<int64_t> poff((size_t)nn + 1, 0);
    for (int32_t u = 0; u < g.n; ++u) ++poff[part[u] + 1];
    for (int32_t X = 0; X < nn; ++X) poff[X + 1] += poff[X];
    std::vector<int32_t> pmem((size_t)g.n);
    {
        std::vector<int64_t> fill(poff.begin(), poff.end() - 1);
        for (int32_t u = 0; u < g.n; ++u) pmem[fill[part[u]]++] = u;
    }
    h.n = nn;
    merge_entries(g, g.ooff, g.oe, part, poff, pmem, nn, h.ooff, h.oe);
    merge_entries(g, g.ioff, g.ie, part, poff, pmem, nn, h.ioff, h.ie);
    h.type.assign((size_t)nn, 0);
    h.moff.assign((size_t)nn + 1, 0);
    h.mids.clear();
    h.mids.reserve(g.mids.size());
    for (int32_t X = 0; X < nn; ++X) {
        h.type[X] = g.type[pmem[poff[X]]];
        const size_t first = h.mids.size();
        for (int64_t m = poff[X]; m < poff[X + 1]; ++m) {
            const int32_t x = pmem[m];
            h.mids.insert(h.mids.end(), g.mids.begin() + g.moff[x], g.mids.begin() + g.moff[x + 1]);
        }
        std::sort(h.mids.begin() + first, h.mids.end());
        h.moff[X + 1] = (int64_t)h.mids.size();
    }
}

template <class T>
T *copy_out(const std::vector<T> &v) {
    T *p = (T *)std::malloc(sizeof(T) * std::max<size_t>(v.size(), 1));
    if (p && !v.empty()) std::memcpy(p, v.data(), sizeof(T) * v.size());
    return p;
}

}  // namespace

extern "C" {

void sgm_default_compress_options(sgm_compress_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_levels = 3;
    o->delta[0] = 0.8f;  // the thesis' SenticNet levels: 0.8, 0.7, 0.7
    for (int i = 1; i < 8; ++i) o->delta[i] = 0.7f;
    o->target_ratio = 0.0;
    o->max_partners = 64;
}

int sgm_compress(int32_t n_vertices, int32_t n_edges, const int32_t *row_ptr, const int32_t *col,
                 const int32_t *rel, const int32_t *type, const sgm_compress_options *opts,
                 sgm_compressed **out) {
    if (!out) return SGM_EINVAL;
    *out = nullptr;
    sgm_compress_options o;
    if (opts) o = *opts;
    else sgm_default_compress_options(&o);
    if (n_vertices < 1 || n_edges < 0 || !row_ptr || !type || (n_edges > 0 && (!col || !rel)) ||
        o.max_levels < 0 || o.max_levels > 8 || o.max_partners < 1 || o.target_ratio < 0.0)
        return SGM_EINVAL;
    for (int i = 0; i < o.max_levels; ++i)
        if (!(o.delta[i] > 0.0f && o.delta[i] <= 1.0f)) return SGM_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[n_vertices] != n_edges) return SGM_EINVAL;
    for (int32_t v = 0; v < n_vertices; ++v)
        if (row_ptr[v + 1] < row_ptr[v] || type[v] < 0) return SGM_EINVAL;
    for (int32_t i = 0; i < n_edges; ++i)
        if (col[i] < 0 || col[i] >= n_vertices || rel[i] < 0) return SGM_EINVAL;
    sgm_compressed *c = nullptr;
    try {
        // level 0: the input with repeated (neighbour, relation) entries
        // removed, every edge of weight 1
        WGraph g;
        const int32_t V = n_vertices;
        g.n = V;
        g.ooff.assign((size_t)V + 1, 0);
        g.oe.reserve((size_t)n_edges);
        for (int32_t v = 0; v < V; ++v) {
            const size_t first = g.oe.size();
            for (int32_t i = row_ptr[v]; i < row_ptr[v + 1]; ++i) g.oe.push_back(Ent{col[i], rel[i], 1});
            std::sort(g.oe.begin() + first, g.oe.end(), ent_less);
            g.oe.erase(std::unique(g.oe.begin() + first, g.oe.end(),
                                   [](const Ent &a, const Ent &b) { return a.nb == b.nb && a.rel == b.rel; }),
                       g.oe.end());
            g.ooff[v + 1] = (int64_t)g.oe.size();
        }
        g.ioff.assign((size_t)V + 1, 0);
        for (const Ent &e : g.oe) ++g.ioff[e.nb + 1];
        for (int32_t v = 0; v < V; ++v) g.ioff[v + 1] += g.ioff[v];
        g.ie.resize(g.oe.size());
        {
            std::vector<int64_t> fill(g.ioff.begin(), g.ioff.end() - 1);
            for (int32_t v = 0; v < V; ++v)
                for (int64_t i = g.ooff[v]; i < g.ooff[v + 1]; ++i)
                    g.ie[fill[g.oe[i].nb]++] = Ent{v, g.oe[i].rel, 1};  // ascending sources
        }
        g.type.assign(type, type + V);
        g.moff.resize((size_t)V + 1);
        g.mids.resize((size_t)V);
        for (int32_t v = 0; v <= V; ++v) g.moff[v] = v;
        for (int32_t v = 0; v < V; ++v) g.mids[v] = v;

        c = (sgm_compressed *)std::calloc(1, sizeof(sgm_compressed));
        if (!c) return SGM_ENOMEM;
        const double size0 = (double)V + (double)g.entries();
        c->level_size[0] = (int64_t)size0;
        int levels = 0;
        for (int lv = 0; lv < o.max_levels; ++lv) {
            if (o.target_ratio > 0.0 && ((double)g.n + (double)g.entries()) / size0 <= o.target_ratio)
                break;
            std::vector<int32_t> part;
            const int32_t merged = pair_up(g, o.delta[lv], o.max_partners, part);
            if (merged == 0) break;
            WGraph h;
            next_level(g, part, g.n - merged, h);
            g = std::move(h);
            ++levels;
            c->level_size[levels] = (int64_t)g.n + g.entries();
        }
        c->levels = levels;
        c->n_vertices = g.n;
        c->n_edges = g.entries();
        std::vector<int32_t> rp((size_t)g.n + 1), cl(g.oe.size()), rl(g.oe.size()), wt(g.oe.size());
        std::vector<int32_t> ob((size_t)g.n), ib((size_t)g.n), mo((size_t)g.n + 1), hy((size_t)V);
        for (int32_t X = 0; X <= g.n; ++X) {
            rp[X] = (int32_t)g.ooff[X];
            mo[X] = (int32_t)g.moff[X];
        }
        for (size_t i = 0; i < g.oe.size(); ++i) {
            cl[i] = g.oe[i].nb;
            rl[i] = g.oe[i].rel;
            wt[i] = g.oe[i].w;
        }
        for (int32_t X = 0; X < g.n; ++X) {
            int64_t so = 0, si = 0;
            for (int64_t i = g.ooff[X]; i < g.ooff[X + 1]; ++i) so += g.oe[i].w;
            for (int64_t i = g.ioff[X]; i < g.ioff[X + 1]; ++i) si += g.ie[i].w;
            ob[X] = (int32_t)std::min<int64_t>(so, INT32_MAX);
            ib[X] = (int32_t)std::min<int64_t>(si, INT32_MAX);
            for (int64_t m = g.moff[X]; m < g.moff[X + 1]; ++m) hy[g.mids[m]] = X;
        }
        c->row_ptr = copy_out(rp);
        c->col = copy_out(cl);
        c->rel = copy_out(rl);
        c->weight = copy_out(wt);
        c->type = copy_out(g.type);
        c->out_bound = copy_out(ob);
        c->in_bound = copy_out(ib);
        c->map_off = copy_out(mo);
        c->map_ids = copy_out(g.mids);
        c->hyper_of = copy_out(hy);
        c->n_original = V;
        if (!c->row_ptr || !c->col || !c->rel || !c->weight || !c->type || !c->out_bound ||
            !c->in_bound || !c->map_off || !c->map_ids || !c->hyper_of) {
            sgm_free_compressed(c);
            return SGM_ENOMEM;
        }
    } catch (const std::bad_alloc &) {
        if (c) sgm_free_compressed(c);
        return SGM_ENOMEM;
    }
    *out = c;
    return SGM_OK;
}

void sgm_free_compressed(sgm_compressed *c) {
    if (!c) return;
    void *ps[] = {c->row_ptr, c->col,      c->rel,     c->weight,  c->type,
                  c->out_bound, c->in_bound, c->map_off, c->map_ids, c->hyper_of};
    for (void *p : ps) std::free(p);
    std::free(c);
}

}  // extern "C"
