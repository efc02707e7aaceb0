// Persistent per-query kernel of the sgm library (internal): one workgroup
// runs a whole query -- filtering, candidate edges, join, ordering -- out of
// its own slot of device memory, then takes the next query from a queue;
// idle workgroups of the launch help with large filter steps.
#pragma once

#include <stdint.h>

#include "sgm_internal.h"

namespace sgm {

constexpr int kNarrowThreads = 512;  // threads per workgroup (8 wave64)

// One filter launch of the plan: explore (push = 1) or refine (push = 0) of
// vertex u against nbr[first .. first+count).
struct NStep {
    int8_t u, push, parent;  // parent: vertex intersected with the push scratch, or -1
    int8_t pad;
    int16_t first, count;
};

struct NNbr {
    int8_t v;     // the other query vertex
    int8_t dir;   // 0: out-edges of the candidate, 1: in-edges
    int8_t mode;  // 0: test v's bitmap; 1: test v's predicate
    int8_t pad;
    int32_t rel;  // -1: any
};

constexpr int kNMaxSteps = 2 * SGM_MAX_QV;
constexpr int kNMaxNbr = 2 * SGM_MAX_QE + 2 * SGM_MAX_QV;

// Packed query + plan, built on the host.
struct NQuery {
    int32_t n, m;
    VPred pred[SGM_MAX_QV];
    int32_t esrc[SGM_MAX_QE], edst[SGM_MAX_QE], elabel[SGM_MAX_QE];
    int32_t root;           // first vertex of the visit order
    int32_t root_slot;      // row of the root sweep output, -1 if the root is pinned
    int32_t n_init, n_ref;  // explore steps, then refine steps (one round)
    int32_t refine_rounds;  // -1: until nothing is removed
    uint32_t proj;          // projected columns (bit u = query vertex u kept; 0: all)
    int32_t fault;          // 1: fail as a device fault would (sgm_inject_fault)
    int32_t homo;           // 1: matches are homomorphisms (a compressed graph)
    NStep steps[kNMaxSteps];
    NNbr nbr[kNMaxNbr];
};

// Per-query outcome.
struct NResult {
    int32_t status;        // SGM_OK, or kNeedWide / kOutFull (rerun on the multi-kernel path)
    int32_t reason;        // kWhy* for kNeedWide
    int32_t n_cols;
    int32_t pad;
    int64_t n_rows;
    int64_t offset;        // first int32 of the rows in the output arena
    int64_t cand[SGM_MAX_QV];
    int64_t ec[SGM_MAX_QE];
    int64_t level_rows[SGM_MAX_QV];
    int32_t join_order[SGM_MAX_QV];
    int64_t bytes;         // algorithmic bytes the query's phases moved
    int64_t ticks[4];      // device wall-clock ticks: filter, edges, join, ordering
    int64_t pbytes[4];     // algorithmic bytes of the same four phases
    int64_t need;          // kWhySlab at a join level: slab bytes its pairs could take
    // a large final table left unordered in the slot's slab for the host to
    // order with whole-GPU kernels after the launch: device addresses of the
    // table ([n_rows][n] in join-level column order, see join_order) and of
    // the sorted candidate lists of its key columns (those of more than one
    // candidate that the result keeps, concatenated in query-vertex order;
    // cand[u] entries each); the key has key_bits bits
    int32_t host_order, key_bits;
    int64_t table_ptr, list_ptr;
};

constexpr int32_t kNeedWide = 1;  // a capacity of the per-query slot was exceeded
constexpr int32_t kOutFull = 2;   // the shared output arena was full
constexpr int32_t kFault = 3;     // an injected device fault (no rerun: SGM_EDEVICE)
// why a query left the persistent kernel
constexpr int32_t kWhyList = 1;   // a candidate list outgrew its slot capacity
constexpr int32_t kWhySlab = 2;   // edge tables / join tables / sort buffers outgrew the slab
constexpr int32_t kWhyKey = 4;    // the ordering key would need more than 64 bits
constexpr int32_t kWhyHelp = 8;   // shared filter step not finished by its helpers in time
// A join level whose pairs (an upper bound on its rows) would need more than
// this many times the slab left stops at once instead of filling the slab.
constexpr int64_t kPairSlack = 8;
// Polls of a shared step's completion count before its owner gives up
// (sgm_tuning.help_wait = 0).
constexpr int64_t kHelpWaitDefault = 1ll << 22;

// One filter step shared by several workgroups: the owner of a query posts
// the step here, and idle workgroups of the same launch claim chunks of its
// candidate list. During the step its counters live here instead of in the
// owner's LDS. One entry per slot workgroup; entries are zeroed when
// allocated and every posted step is retired before its owner moves on.
// claim packs (sequence:24 | chunks:20 | next chunk:20): one atomic add
// claims a chunk and returns which step it belongs to and whether it exists.
// One join level as every workgroup that works on it sees it: the parent
// table, the extension edge's candidate-edge table (keyed by the parent
// vertex's sorted candidates pk), the check edges' tables (each keyed by the
// sorted candidates kl of the vertex at row column col) and the output.
struct JChk {
    const int32_t *kl, *offs, *cnt, *vals;
    int32_t nkl, col;
};
struct JLevel {
    const int32_t *table;
    int64_t rows;
    int32_t k, cp;  // columns of the parent table; column of the parent vertex
    const int32_t *pk;
    int32_t npk, nchk;
    const int32_t *eoffs, *ecnt, *evals;
    int32_t *out;
    int64_t cap;   // output rows that fit
    int32_t nsub;  // shared: chunks per block of NT parent rows
    int32_t homo;  // 1: a value may repeat one of the row (a compressed graph)
    JChk chk[SGM_MAX_QE];
};

// One edge-candidate table build shared with helpers: the key vertex's
// sorted candidates, the table's per-key space (degoff), counts and values,
// the list of keys whose rows go to a later tier (ovl), the other
// endpoint's candidate bitmap and sorted list, the edge's relation and the
// direction of the rows scanned (0: out-rows of sources). tier 0: chunks of
// key positions, G lanes per key; tier 1: chunks of items (positions of
// long keys), one wave per key; tier 2: one item per chunk, the whole
// workgroup per key.
struct EcJob {
    const int32_t *keys, *degoff;
    int32_t *num, *vals, *ovl;
    const uint64_t *ob;
    const int32_t *ol, *items;
    int32_t nk, rel, dir, no, tier;
    int32_t homo;  // 1: a key may pair with itself (a compressed graph)
};

struct HelpJob {
    unsigned long long claim;
    unsigned long long bytes;  // algorithmic bytes of the helpers' chunks
    const int4 *seg;           // kind 1: the row segments, one per chunk
    const int32_t *ul;         // kind 0: the items (a candidate list, or long rows)
    int32_t chunk, done, q, kind;  // kind 0: chunks of the candidate list; 1: row segments;
                                   // 2: parent rows of a join level; 3: keys of an
                                   // edge-candidate table; 4: rows above wg_rows of a
                                   // prune-only step, one per chunk
    int32_t n_items, G, ncount, revd;
    NStep st;
    int32_t nbig, removed, nmarks, abort_;
    // 1 after the owner gave up on a step whose claimed chunks had not all
    // been reported: helpers may still write the slot's bitmaps, so its
    // workgroup takes no more queries in that launch and the next launch
    // clears the whole slot before using it
    int32_t dirty;
    // kind 0: 1 when the chunks' items are long rows, which one wave takes
    // up to wg_rows entries (longer ones go on to the workgroup tier)
    int32_t nodefer;
    int32_t cnt[SGM_MAX_QV];
    NNbr nbl[SGM_MAX_QE];
    // kind 2: chunks of a join level's parent rows; jrows counts the output
    // rows placed so far (kind 3: the table entries written so far)
    unsigned long long jrows;
    JLevel jl;
    EcJob ecj;  // kind 3
};

struct NArgs {
    DevGraph g;
    const NQuery *qs;
    int32_t nq;
    NResult *res;
    int32_t *queue;           // [1] next query index
    uint64_t *bits;           // [slots][(SGM_MAX_QV + 1) * nwords], zero between queries
    int32_t *lists;           // [slots][SGM_MAX_QV * lcap]
    int32_t lcap;
    char *slab;               // [slots][slab_bytes]
    int64_t slab_bytes;
    const uint64_t *rootbits; // [n_root_slots][nwords] root sweep output
    int32_t *out;             // output arena (int32 rows)
    int64_t out_cap;          // in int32 elements
    unsigned long long *out_used;
    int64_t *trace;           // [nq][SGM_TRACE_CAP] step events, or null
    // work-division and schedule knobs (sgm_tuning); results do not depend
    // on them
    int32_t group_lanes;      // most lanes per candidate group (power of two, 1..64)
    int32_t wg_rows;          // rows longer than this get the whole workgroup
    int32_t join_policy;      // 0: cheapest edge first; 1: most-constrained vertex first
    // shared filter steps: workgroups [0, nslot) own slots and take queries;
    // the others, and slot workgroups whose queue ran dry, help. A step of
    // at least help_items candidates is shared (0: never).
    int32_t nslot;
    int32_t ngrid;            // workgroups of the launch (>= nslot)
    int32_t help_items;
    HelpJob *board;           // [nslot]
    int32_t *hctr;            // [0] posted steps, [1] slot workgroups done
    int64_t help_wait;        // polls of a shared step's completion before its owner gives up
    // final tables of at least this many rows are left in the slab for the
    // host to order (0: never); the slab below such a table serves the
    // slot's later queries of the launch
    int64_t host_order_rows;
};

// Root sweep: rootbits[j][w] = vertices satisfying predicate j, for the
// distinct predicates of a batch's unpinned roots. It also zeroes ctr[0..2]
// (the persistent kernel's work queue, output-arena use and helper
// counters), so it runs
// before every persistent launch, with n_pred = 0 when no root needs it.
struct SweepArgs {
    DevGraph g;
    const VPred *preds;   // untyped first, then by type
    int32_t n_pred;
    int32_t n_any;        // predicates without a type
    uint64_t *rootbits;
    unsigned long long *ctr;
    // type_off[t] = first predicate with type >= t, for t in [0, n_types];
    // n_types = 0: no table (types found by binary search)
    const int32_t *type_off;
    int32_t n_types;
};
void launch_root_sweep(hipStream_t s, const SweepArgs &a);
void launch_narrow(hipStream_t s, const NArgs &a, int grid);
// Kernel-node parameters of the sweep and of the persistent kernel for a
// HIP graph. The argument pointers refer to *sa, *na and args[0..8], which
// must stay valid until the parameters have been handed to HIP.
void narrow_node_params(SweepArgs *sa, NArgs *na, int narrow_grid, void **args,
                        hipKernelNodeParams *sweep, hipKernelNodeParams *narrow);
size_t narrow_lds_bytes();

}  // namespace sgm
