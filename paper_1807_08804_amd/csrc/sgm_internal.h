// Internal declarations of the sgm library: device graph view, kernel
// argument blocks and the launchers implemented in sgm_kernels.hip.
// Nothing here is part of the public ABI (include/sgm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sgm.h"

namespace sgm {

// Block size used by every kernel (4 wave64 wavefronts).
constexpr int kBlock = 256;
// Candidate items with more adjacency entries than this are handled by a
// whole workgroup instead of a 16-lane group.
constexpr int kBigDegree = 256;
constexpr int kMaxNbr = SGM_MAX_QE;

// Read-only view of the device-resident data graph. Each adjacency entry is
// {neighbour id, relation}; out-rows are sorted by (dst, rel), in-rows by
// (src, rel), exact duplicate triples removed.
struct DevGraph {
    int32_t V;
    int32_t nwords;  // ceil(V / 64): words of one candidate bitmap
    const int32_t *out_off;  // [V+1]
    const int32_t *in_off;   // [V+1]
    const int2 *out_adj;     // [E]
    const int2 *in_adj;      // [E]
    // [V] per-vertex predicate inputs in one 8-byte word: x = type,
    // y = min(out-degree, 255) | min(in-degree, 255) << 8 (a query vertex has
    // at most 15 distinct neighbours per direction, so the clamp is exact)
    const int2 *vinfo;
    // Hub rows (at least kHubRow entries) are also kept in two re-sorted
    // copies of the adjacency arrays (same row extents; other rows keep the
    // original order there): ta by (type of the other end, relation, other
    // end) and tb by (type of the other end, other end, relation). For a
    // vertex with a hub row, hub_of[v] = h >= 0 and
    // hub_toff[((h * 2 + dir) * 2 + order) * hub_types + t] is the offset,
    // from the row start, of the first entry whose other end has type >= t
    // (t in [0, hub_types), order 0: ta, 1: tb). hub_types = 0: no index.
    const int2 *out_ta, *out_tb, *in_ta, *in_tb;
    const int32_t *hub_of;
    const int32_t *hub_toff;
    int32_t hub_types;
};

// rows this long get the per-type index above
constexpr int32_t kHubRow = 16384;

// Candidate predicate of one query vertex (thesis Def. 3.3 with pins and the
// incoming-graph degree): type, pin, out-degree and in-degree bounds.
struct VPred {
    int32_t label;  // -1: any
    int32_t pin;    // -1: none
    int32_t qout;   // distinct out-neighbours in the query
    int32_t qin;    // distinct in-neighbours in the query
};

// One query edge seen from the vertex being explored/refined.
struct NbrDesc {
    int32_t dir;        // 0: data out-edges of the candidate; 1: in-edges
    int32_t rel;        // required relation, -1 any
    int32_t mode;       // 0: neighbour tested against test_bits; 1: against pred
    int32_t push;       // 1: push matching neighbours into push_bits
    VPred pred;
    const uint64_t *test_bits;
    uint64_t *push_bits;
};

// Filter step (explore or refine) over the candidate list of one query
// vertex.
struct FilterArgs {
    DevGraph g;
    const int32_t *items;     // candidate list of the vertex
    const int32_t *count;     // device-resident length of items
    uint64_t *self_bits;      // candidate bitmap of the vertex (pruned in place)
    const NbrDesc *nbr;       // [n_nbr] in device memory
    int32_t n_nbr;
    int32_t do_push;          // explore (1) or refine (0)
    int32_t *big_items;       // overflow list of high-degree items
    int32_t *big_count;
    unsigned long long *removed;  // count of pruned candidates
};

// Candidate-edge collection for one query edge in one orientation.
struct ECDesc {
    int32_t key_vertex;       // query vertex whose candidates are the keys
    int32_t dir;              // 0: scan out-edges of keys; 1: in-edges
    int32_t rel;              // -1: any relation (distinct pairs)
    const int32_t *keys;      // candidate list of key_vertex
    const int32_t *key_count; // device count
    const uint64_t *other_bits;  // candidate bitmap of the other endpoint
    int32_t *cnt;             // [|keys|] per-key counts (count pass)
    const int32_t *offs;      // [|keys|+1] exclusive scan (write pass)
    int32_t *vals;            // [|EC|] (write pass)
    unsigned long long *total;  // total pairs (count pass)
    int32_t *big_items;       // overflow list (key indices)
    int32_t *big_count;
    int32_t homomorphic;      // 1: a key may pair with itself (compressed graphs)
};

// Rank structure of one candidate bitmap: rank(x) = prefix[x>>6] +
// popcount(bits[x>>6] & below(x)).
struct RankRef {
    const uint64_t *bits;
    const int32_t *prefix;
};

struct JoinEdge {
    int32_t col;              // table column of the already-bound endpoint
    RankRef rank;             // rank structure of that endpoint's candidates
    const int32_t *offs;      // EC keyed by that endpoint
    const int32_t *vals;
};

// One join level: extend every row by the new vertex through `ext`, keep
// the value if it is absent from the row and present in every `chk` list.
struct JoinArgs {
    const int32_t *table;     // [R][k]
    int64_t R;
    int32_t k;
    JoinEdge ext;
    int32_t n_chk;
    JoinEdge chk[SGM_MAX_QV];
    const int64_t *pair_off;  // [R+1] exclusive scan of per-row fan-out
    int64_t p0;               // first pair of this launch (chunking)
    int64_t P;                // one past the last pair of this launch
    int32_t *out;             // [..][k+1] (write pass)
    int64_t *block_cnt;       // per-tile valid counts (count pass) / offsets (write pass)
    int64_t out_base;         // first output row (chunking)
    int32_t homomorphic;      // 1: the new value may repeat one of the row (compressed graphs)
};

// ---- launchers (sgm_kernels.hip) ----
void launch_check_sweep(hipStream_t s, const DevGraph &g, VPred p, uint64_t *bits);
void launch_check_pin(hipStream_t s, const DevGraph &g, VPred p, uint64_t *bits);
// one workgroup per listed bitmap slot (slots: device array of nslots ids,
// or NULL for slots 0..nslots-1)
void launch_collect_multi(hipStream_t s, const DevGraph &g, const uint64_t *bits_base,
                          int64_t bits_stride, int32_t *list_base, int64_t list_stride,
                          int32_t *count_base, int32_t *prefix_base, int64_t prefix_stride,
                          const int32_t *slots, int nslots);
void launch_filter(hipStream_t s, const FilterArgs &a, int grid_small, int grid_big);
// dst &= src over nwords; removed (optional, device) counts the bits cleared
void launch_and(hipStream_t s, uint64_t *dst, const uint64_t *src, int32_t nwords,
                unsigned long long *removed = nullptr);
// transposition input of a source-keyed candidate-edge table: per pair, the
// destination's rank and the source; cnt (zeroed) counts pairs per rank
void launch_ec_pairs(hipStream_t s, const int32_t *keys, const int32_t *key_count, int64_t n_keys,
                     const int32_t *offs, const int32_t *vals, RankRef rk, int32_t *rank,
                     int32_t *src, int32_t *cnt);
void launch_ec_count(hipStream_t s, const DevGraph &g, const ECDesc &d, int grid_small,
                     int grid_big);
void launch_ec_write(hipStream_t s, const DevGraph &g, const ECDesc &d, int grid_small,
                     int grid_big);
void launch_scan_i32(hipStream_t s, const int32_t *in, const int32_t *n, int32_t *out);
// exclusive scan of n int64 values into out[0..n], out[n] = total;
// tmp holds scan_tmp_words(n) int64
int64_t scan_tmp_words(int64_t n);
void launch_scan_i64(hipStream_t s, const int64_t *in, int64_t n, int64_t *out, int64_t *tmp);
void launch_join_fan(hipStream_t s, const JoinArgs &a, int64_t *fan);
int64_t join_tiles(int64_t P);
void launch_join_count(hipStream_t s, const JoinArgs &a);
void launch_join_write(hipStream_t s, const JoinArgs &a);
void launch_keys_to_table(hipStream_t s, const int32_t *keys, const int32_t *key_cnt_dev,
                          int64_t n, int32_t *table);
// final ordering
void launch_iota(hipStream_t s, int32_t *idx, int64_t n);
int64_t small_sort_limit();
// order of the n rows of a k-wide table by columns colpos[0 .. ncols)
void launch_sort_small(hipStream_t s, const int32_t *table, int32_t k, const int32_t *colpos,
                       int32_t ncols, int32_t n, int32_t *idx);
int64_t radix_tiles(int64_t n);
void launch_gather_key(hipStream_t s, const int32_t *table, int32_t k, int32_t col,
                       const int32_t *idx, int64_t n, int32_t *key);
void launch_radix_hist(hipStream_t s, const int32_t *key, int64_t n, int shift, int64_t *hist);
void launch_radix_scatter(hipStream_t s, const int32_t *key_in, const int32_t *idx_in, int64_t n,
                          int shift, const int64_t *off, int32_t *key_out, int32_t *idx_out);
// out[i] = columns colpos[0 .. ncols) of row idx[i] of a k-wide table
void launch_gather_rows(hipStream_t s, const int32_t *table, int32_t k, const int32_t *idx,
                        int64_t n, const int32_t *colpos, int32_t ncols, int32_t *out);
// Distinct rows of a sorted n x k table, in order, to out; pos[n] (device)
// receives their number. head: n int64, pos: n + 1 int64, tmp:
// scan_tmp_words(n) int64.
void launch_unique_rows(hipStream_t s, const int32_t *rows, int32_t k, int64_t n, int64_t *head,
                        int64_t *pos, int64_t *tmp, int32_t *out);

// Ordering key of a row: the ranks of its values among the candidates of
// their query vertices, concatenated in query-vertex order (nbits[u] bits
// each, 64 in total at most). A rank comes from the vertex's candidate
// bitmap and its per-word prefix counts.
struct KeyCols {
    const uint64_t *bits[SGM_MAX_QV];
    const int32_t *prefix[SGM_MAX_QV];
    int32_t col[SGM_MAX_QV];    // table column of query vertex u
    int32_t nbits[SGM_MAX_QV];
    int32_t n;
};
void launch_row_keys(hipStream_t s, const int32_t *table, int32_t k, const KeyCols &kc, int64_t n,
                     uint64_t *keys);
// Key columns given by their sorted candidate lists (one device array, the
// lists at off[c]): rank = position of the value in its list.
struct ListKeys {
    const int32_t *list;
    int64_t off[SGM_MAX_QV];
    int32_t cnt[SGM_MAX_QV];
    int32_t nbits[SGM_MAX_QV];
    int32_t col[SGM_MAX_QV];
    int32_t n;
};
void launch_row_keys_lists(hipStream_t s, const int32_t *table, int32_t k, const ListKeys &lk,
                           int64_t n, uint64_t *keys);
// key[i] = 32-bit half (hi = 0: low, 1: high) of keys[idx[i]]
void launch_key_half(hipStream_t s, const uint64_t *keys, const int32_t *idx, int64_t n, int hi,
                     int32_t *key);

// Expansion of matches on a compressed graph (thesis Ch. 3, Sec. "GpSense
// Framework"): each weighted match (a row of weighted vertices, one per
// query vertex) stands for the choices of one member of each vertex's
// mapping list; the choices that are injective, keep the pins and hold every
// query edge in the original graph g are matches of g. Query vertices are
// chosen in order[0 .. n); the query edges (es, ed, el) with index in
// [eb[i], eb[i+1]) are checked when order[i] is chosen (both ends chosen).
struct ExpandArgs {
    DevGraph g;
    const int32_t *wrows;  // [nw][n]
    int64_t nw;
    int32_t n;
    const int32_t *map_off, *map_ids;
    int32_t order[SGM_MAX_QV];
    int32_t pin[SGM_MAX_QV];  // per query vertex: its original vertex, or -1
    int32_t eb[SGM_MAX_QV + 1];
    int32_t es[SGM_MAX_QE], ed[SGM_MAX_QE], el[SGM_MAX_QE];
    int64_t *cnt;          // [nw] matches per weighted match (count pass)
    const int64_t *offs;   // [nw + 1] their exclusive scan (write pass)
    int32_t *out;          // [total][n] (write pass)
};
void launch_expand_count(hipStream_t s, const ExpandArgs &a);
void launch_expand_write(hipStream_t s, const ExpandArgs &a);

}  // namespace sgm
