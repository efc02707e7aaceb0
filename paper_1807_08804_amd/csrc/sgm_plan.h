// Host-side query checks and query plan of the sgm library (internal).
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/sgm.h"

namespace sgm {

// A validated query with its per-vertex neighbour masks.
struct QInfo {
    int n, m;
    int32_t label[SGM_MAX_QV], pin[SGM_MAX_QV];
    int32_t esrc[SGM_MAX_QE], edst[SGM_MAX_QE], elabel[SGM_MAX_QE];
    uint32_t out_mask[SGM_MAX_QV];  // bit v: some edge u -> v
    uint32_t in_mask[SGM_MAX_QV];   // bit v: some edge v -> u
    int32_t qout[SGM_MAX_QV];       // distinct out-neighbours
    int32_t qin[SGM_MAX_QV];        // distinct in-neighbours
    int32_t deg[SGM_MAX_QV];        // distinct neighbours, either direction
    // projection (thesis Ch. 3, Sec. "GpSense": only the matches of a subset
    // of the query's nodes are wanted): bit u set = column u is returned;
    // 0 = every column (no projection). n_out = columns returned.
    uint32_t proj;
    int32_t n_out;
};

// Set a projection on a checked query: SGM_EINVAL for an empty mask or bits
// beyond its vertices; a mask naming every vertex means no projection.
int set_projection(QInfo *qi, uint32_t mask);

// Spanning tree T and orders of the filtering phase.
struct Plan {
    int n_visit;
    int32_t visit[SGM_MAX_QV];        // O: expanded vertices in order
    int32_t parent[SGM_MAX_QV];       // tree parent, -1 for the root
    int32_t parent_edge[SGM_MAX_QV];  // query edge to the parent, -1 for the root
    int n_init;
    int32_t init[SGM_MAX_QV];         // order in which vertices enter T
};

// The filtering phase as a fixed sequence of steps. Explore steps follow the
// visit order (Alg. 3.2): each tests and pushes along its spanning-tree
// edges; the parent (already initialised) is tested against its bitmap and
// intersected with what the step pushes (parent >= 0), the children are
// tested against their candidate predicate and receive the pushes. Refine
// steps (one round) prune a vertex against all query edges to vertices above
// the low-connectivity threshold.
struct PStep {
    int u, first, count, push, parent;
    int sweep;  // 1: u starts from every vertex its predicate admits (out-only graph)
};
struct PNbr {
    int v, dir, rel, mode;  // dir 0: out-edges of the candidate; mode 0: bitmap test
};
// A vector of at most N elements stored in place (planning allocates no
// memory, so the entry point that allocates nothing can plan too).
template <class T, int N>
struct FixedVec {
    T v[N];
    int n = 0;
    void clear() { n = 0; }
    void push_back(const T &x) { v[n++] = x; }
    int size() const { return n; }
    bool empty() const { return n == 0; }
    const T &operator[](int i) const { return v[i]; }
    const T *begin() const { return v; }
    const T *end() const { return v + n; }
};
// Explore steps hold each tree edge twice at most (2 (n - 1) entries),
// refine steps each query edge twice at most (2 m); with the outgoing graph
// only there are up to two explore steps per vertex and one refine step per
// vertex and per edge.
struct Program {
    FixedVec<PStep, 2 * SGM_MAX_QV> init;
    FixedVec<PStep, SGM_MAX_QV + SGM_MAX_QE> refine;
    FixedVec<PNbr, 2 * SGM_MAX_QV + 2 * SGM_MAX_QE> nbr;
};
void build_program(const QInfo &qi, const Plan &pl, int low_conn_degree, int refine_reversed,
                   Program *pr);
// The same phase with the outgoing graph only: every descriptor scans out-
// edges (dir 0). A tree child reached over an edge into its parent starts
// from a sweep of its predicate and is tested against the parent's bitmap,
// pushing back into the parent; refinement over an edge v -> u runs as such
// a step on v. Steps with parent >= 0 push into a scratch bitmap that is
// then intersected into the parent.
void build_program_out_only(const QInfo &qi, const Plan &pl, int low_conn_degree,
                            int refine_reversed, Program *pr);

// Estimated device bytes of a query's intermediate tables (the served
// form's admission unit): candidate bitmaps of its vertices plus the largest
// pair of consecutive join tables, with the rows of each level estimated
// along the plan's spanning tree under independence (see the definition).
int64_t estimate_bytes(const QInfo &qi, const Plan &pl, int32_t V, int64_t E,
                       const int64_t *type_freq, int32_t n_types, const int64_t *rel_freq,
                       int32_t n_rels);

// SGM_OK, SGM_EINVAL or SGM_EUNSUPPORTED (see sgm_match_query).
int check_query(const sgm_query *q, int32_t V, QInfo *qi);
int make_plan(const QInfo &qi, int32_t V, const int64_t *type_freq, int32_t n_types, Plan *p);

}  // namespace sgm
