// Persistent per-query kernel (gfx950): each slot workgroup takes queries
// from a queue and runs the whole filtering-and-joining pipeline of one query
// (thesis Alg. 3.1) with barrier-separated phases, in its own slot of device
// memory, then leaves the slot's bitmaps zeroed for the next query. Filter
// steps over many candidates or long rows are shared: the owner posts them on
// a board and the launch's idle workgroups (extra ones, and slot workgroups
// whose queue ran dry) claim chunks of them.
//
// Phases (thesis Ch. 3):
//   root candidates  -- kernel_check / kernel_collect of Alg. 3.2 (the sweep
//                       itself runs once for a whole batch in k_root_sweep);
//   explore          -- kernel_explore of Alg. 3.2 along the spanning tree;
//   refine           -- Sec. "Candidate Nodes Refinement" (prune only);
//   candidate edges  -- Sec. "Joining Phase", two-step output per key;
//   join             -- edge order of Sec. "Joining Phase", one query vertex
//                       per level, rows staged through LDS offsets;
//   ordering         -- rows sorted by a packed key of candidate ranks.
// Candidate lists are kept alongside the bitmaps (a push that sets a new bit
// appends to the list), so no phase scans all V vertices. When a query
// outgrows the slot (list, slab or LDS capacities), the workgroup clears its
// slot and reports kNeedWide; the host then runs the multi-kernel path.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sgm_device.h"
#include "sgm_narrow.h"

namespace sgm {
namespace {

constexpr int NT = kNarrowThreads;
constexpr int NW = NT / 64;
constexpr int kBigCap = 256;         // LDS list of items for the whole workgroup
// A shared step with at least kLongShare long rows (over 64 strides of its
// lanes) shares them too, kLongChunk rows per chunk, one wave per row.
constexpr int32_t kLongShare = 32;
constexpr int32_t kLongChunk = 16;
constexpr int32_t kRevMin = 256;      // candidates of u before a reverse check can pay
constexpr int32_t kRevMaxCand = 4096; // neighbours with at most this many candidates
constexpr int kListSortCap = 8192;    // int32 entries sorted in LDS
constexpr int kRowSortCap = 2048;     // final rows sorted in LDS (u64 key + int32 index);
                                      // more rows use radix passes in the slab

struct Smem {
    int64_t sh[NW + 1];
    int64_t slab_used;
    int64_t ectot[SGM_MAX_QE];
    int32_t *ec_cnt[SGM_MAX_QE];
    int32_t *ec_offs[SGM_MAX_QE];
    int32_t *ec_vals[SGM_MAX_QE];
    int32_t cnt[SGM_MAX_QV];
    int32_t eckey[SGM_MAX_QE];      // key vertex the join needs for each edge
    int32_t ecbuilt[SGM_MAX_QE];    // key vertex of the table built first
    int32_t jorder[SGM_MAX_QV], jpos[SGM_MAX_QV];
    int32_t lv_ext[SGM_MAX_QV], lv_first[SGM_MAX_QV], lv_nchk[SGM_MAX_QV];
    int32_t chk[SGM_MAX_QE];
    int32_t big[kBigCap];
    int32_t pairoff[NT];
    int32_t rowlo[NT];
    JLevel jl;                 // the join level being built
    int32_t wnok[2][NW];       // shared join levels: rows per wave of a block of pairs
    int64_t wbase[2];          // and the block's first output row
    int32_t abort_;
    int32_t q;
    int32_t nev;
    int32_t nbig;
    int32_t ngiant;
    int32_t nnbl;
    int32_t nmarks;
    int32_t ndef;  // candidates whose pushes go to row segments
    int32_t retired;  // this slot gave up on a shared step (see HelpJob::dirty)
    int32_t unsorted; // ordering: some key is above the next one
    int32_t hostord;  // the final table is left in the slab for the host to order
    int32_t keybits;
    int64_t pin_off;  // byte offset of that table in the slab
    const int32_t *tableptr;
    const int32_t *listptr;  // the key columns' sorted candidate lists beside it
    unsigned long long rowhit;  // item_wg: listed rows with a matching entry
    unsigned long long hseq;    // sequence number of the step this workgroup posted
    int32_t hq, hch;            // helper: board entry and chunk claimed (-1: none)
    int8_t qsrc[SGM_MAX_QE], qdst[SGM_MAX_QE];  // the query's edges, staged for join_order
    uint64_t revmask;
    NNbr nbl[SGM_MAX_QE];  // neighbours a step still tests per candidate
    int32_t removed;
    int32_t ctr;
    int32_t empty;
    // per-query outcome, written to global memory by thread 0 at the end
    int32_t status;
    int32_t reason;
    int32_t cand[SGM_MAX_QV];
    int32_t bitsn[SGM_MAX_QV];
    int32_t kdepth;  // steps of the key columns' binary searches
    int32_t ocol[SGM_MAX_QV];  // table position of each output column
    int32_t nout;              // output columns (the projected ones)
    const int32_t *rkl[SGM_MAX_QV];  // list each key column ranks into (LDS copy if it fits)
    int64_t level_rows[SGM_MAX_QV];
    int64_t nrows;
    int64_t offset;
    int64_t need;
    unsigned long long bytes;  // algorithmic bytes moved (see add_bytes)
    int64_t t[5];              // wall clock at the phase boundaries
    unsigned long long pb[5];  // bytes at the phase boundaries
};

// Dynamic LDS, 51 KB: with the static part a workgroup stays within 64 KB,
// and two workgroups per CU remain resident (registers allow no more). List
// sorting uses [0, 32 KB); the final ordering keeps keys and indices
// (bitonic) or digit counts (radix) in [0, 24 KB) and stages the candidate
// lists its keys rank into at [24 KB, 51 KB).
constexpr size_t kDynLds = 51 << 10;
constexpr size_t kStageOff = 24 << 10;
constexpr int32_t kStageInts = (int32_t)((kDynLds - kStageOff) / sizeof(int32_t));
static_assert(sizeof(int32_t) * kListSortCap <= kDynLds, "list sort space");
static_assert((sizeof(uint64_t) + sizeof(int32_t)) * kRowSortCap <= kStageOff, "row sort space");
static_assert(kDynLds + sizeof(Smem) <= (64 << 10), "LDS per workgroup");
static_assert(8 * 256 * sizeof(int32_t) <= kStageOff, "radix counts");

struct Ctx {
    // the launch's graph, read in place from the kernel arguments (a copy in
    // the context would live in scratch memory: its adjacency pointers are
    // chosen by direction at run time)
    const DevGraph &g;
    int32_t lcap;
    int64_t slab_bytes;
    int32_t *out;
    int64_t out_cap;
    unsigned long long *out_used;
    const uint64_t *rootbits;
    const NQuery *Q;
    Smem *s;
    uint64_t *bits;     // slot bitmaps [(SGM_MAX_QV + 1) * nwords]
    uint64_t *scratch;  // the extra bitmap of the slot
    int32_t *lists;     // slot lists [SGM_MAX_QV * lcap]
    char *slab;
    unsigned char *dyn;
    int64_t *trace;     // this query's step events, or null
    int32_t gmax;       // most lanes per candidate group
    int32_t wg_rows;    // rows longer than this get the whole workgroup
    int32_t join_policy;
    int32_t *marks;     // pushes into the scratch bitmap, while filtering (slab)
    HelpJob *job;       // this slot's entry on the helper board
    int32_t *hctr;      // posted shared steps, slot workgroups done
    int32_t help_items; // share filter steps of at least this many candidates (0: never)
    int32_t q;          // index of the query in the batch
    int32_t nslot, ngrid;  // slot workgroups, all workgroups of the launch
    int64_t help_wait;  // polls of a shared step's completion before giving up
    int64_t host_order_rows;  // final tables of this many rows go to the host (0: none)
    int64_t below_top;  // a last join level placed at the slab's top: the slab used below it
    __device__ uint64_t *B(int u) const { return bits + (int64_t)u * g.nwords; }
    __device__ int32_t *L(int u) const { return lists + (int64_t)u * lcap; }
};

__device__ __forceinline__ bool aborted(const Ctx &c) { return c.s->abort_ != 0; }

// Algorithmic byte accounting: every phase adds the global-memory words its
// algorithm must read or write (adjacency entries 8 B, neighbour tests 4 B,
// list / table / edge-table ints 4 B, bitmap words 8 B), not what caches
// happen to serve.
__device__ __forceinline__ void add_bytes(Ctx &c, uint64_t b) {
    if (b) atomicAdd(&c.s->bytes, (unsigned long long)b);
}

// wave-reduced variant: every lane of the wave must call it
__device__ __forceinline__ void add_bytes_wave(Ctx &c, uint64_t b) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b += __shfl_xor(b, o, 64);
    if ((threadIdx.x & 63) == 0) add_bytes(c, b);
}

// step event (uniform call; thread 0 records)
__device__ __forceinline__ void ev(Ctx &c, int code) {
    if (c.trace && threadIdx.x == 0) {
        const int k = c.s->nev++;
        if (k < SGM_TRACE_CAP) c.trace[k] = (int64_t)(wall_clock64() << 8) | code;
    }
}

// Phase boundary i (0 start, 1 filtered, 2 edge tables built, 3 joined,
// 4 ordered and written): its clock and the bytes counted so far. Callers
// have passed a barrier since the phase's last byte count.
__device__ __forceinline__ void mark(Ctx &c, int i) {
    if (threadIdx.x == 0) {
        c.s->t[i] = wall_clock64();
        c.s->pb[i] = c.s->bytes;
    }
}

// Lowest slab offset of a table left for the host: the slot's later
// queries keep the filter's overflow list, marks, deferred list and row
// segments ([0, 12 lcap) and beyond) plus 4 MB below it.
__device__ __forceinline__ int64_t kPinFloor(const Ctx &c) {
    return 16ll * c.lcap + (4ll << 20);
}

// All threads call; returns the same pointer everywhere (nullptr + abort on
// overflow).
__device__ __forceinline__ char *slab_alloc(Ctx &c, int64_t bytes) {
    __syncthreads();
    const int64_t off = (c.s->slab_used + 255) & ~(int64_t)255;
    char *p = (off + bytes <= c.slab_bytes) ? c.slab + off : nullptr;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (p) c.s->slab_used = off + bytes;
        else c.s->abort_ = kWhySlab;
    }
    __syncthreads();
    return p;
}

// Counters a filter step updates: in the workgroup's LDS, or on the helper
// board while several workgroups share the step.
struct LdsCtr {
    Smem *s;
    __device__ int32_t *cnt(int v) const { return &s->cnt[v]; }
    __device__ int32_t *nbig() const { return &s->nbig; }
    __device__ int32_t *removed() const { return &s->removed; }
    __device__ int32_t *nmarks() const { return &s->nmarks; }
    __device__ int32_t *abort_() const { return &s->abort_; }
};
struct BoardCtr {
    HelpJob *j;
    __device__ int32_t *cnt(int v) const { return &j->cnt[v]; }
    __device__ int32_t *nbig() const { return &j->nbig; }
    __device__ int32_t *removed() const { return &j->removed; }
    __device__ int32_t *nmarks() const { return &j->nmarks; }
    __device__ int32_t *abort_() const { return &j->abort_; }
};

// Set bit x; on a newly set bit append x to list tl, or, for a push into
// the scratch bitmap (tl == nullptr: the parent's marks), to the marks list.
template <class K>
__device__ __forceinline__ void push_bit(Ctx &c, const K &k, uint64_t *tb, int32_t *tl, int v,
                                         int32_t x) {
    const uint64_t m = 1ull << (x & 63);
    uint64_t *w = tb + (x >> 6);
    if (__atomic_load_n(w, __ATOMIC_RELAXED) & m) return;
    const uint64_t old = atomicOr((unsigned long long *)w, m);
    if (old & m) return;
    if (tl) {
        const int32_t p = atomicAdd(k.cnt(v), 1);
        if (p < c.lcap) tl[p] = x;
        else *k.abort_() = kWhyList;
    } else {
        // marks are parent candidates, so at most lcap of them
        c.marks[atomicAdd(k.nmarks(), 1)] = x;
    }
}

__device__ __forceinline__ void push_bit(Ctx &c, uint64_t *tb, int32_t *tl, int v, int32_t x) {
    push_bit(c, LdsCtr{c.s}, tb, tl, v, x);
}

// Set bit x in tb; true if it was clear. With `look`, a plain read first
// skips the atomic for a bit already set (pushes from many candidates that
// share neighbours); without, the atomic alone saves a round trip.
template <bool look>
__device__ __forceinline__ bool set_new(uint64_t *tb, int32_t x) {
    const uint64_t m = 1ull << (x & 63);
    uint64_t *w = tb + (x >> 6);
    if (look && (__atomic_load_n(w, __ATOMIC_RELAXED) & m)) return false;
    return (atomicOr((unsigned long long *)w, m) & m) == 0;
}

// push_bit for up to four entries per lane (hk: push xk), appending the
// newly set ones with one counter update per wave: the lanes that reach
// this call take consecutive places in the order of their lane index.
template <class K, bool look = true>
__device__ __forceinline__ void push4(Ctx &c, const K &k, uint64_t *tb, int32_t *tl, int v,
                                      bool h0, int32_t x0, bool h1, int32_t x1, bool h2,
                                      int32_t x2, bool h3, int32_t x3) {
    const bool n0 = h0 && set_new<look>(tb, x0), n1 = h1 && set_new<look>(tb, x1);
    const bool n2 = h2 && set_new<look>(tb, x2), n3 = h3 && set_new<look>(tb, x3);
    const int cnt = (int)n0 + (int)n1 + (int)n2 + (int)n3;
    const uint64_t b0 = __ballot(cnt & 1), b1 = __ballot(cnt & 2), b2 = __ballot(cnt & 4);
    const int tot = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
    if (tot == 0) return;
    const uint64_t lt = lanemask_lt(threadIdx.x & 63);
    const int pre = __popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt);
    const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;
    int32_t base = 0;
    if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(tl ? k.cnt(v) : k.nmarks(), tot);
    base = __builtin_amdgcn_readlane(base, leader);
    int32_t p = base + pre;
    if (tl) {
        // a list may outgrow its capacity: the query then leaves the slot
        if (n0) { if (p < c.lcap) tl[p] = x0; else *k.abort_() = kWhyList; ++p; }
        if (n1) { if (p < c.lcap) tl[p] = x1; else *k.abort_() = kWhyList; ++p; }
        if (n2) { if (p < c.lcap) tl[p] = x2; else *k.abort_() = kWhyList; ++p; }
        if (n3) { if (p < c.lcap) tl[p] = x3; else *k.abort_() = kWhyList; }
    } else {
        // marks are parent candidates, so at most lcap of them
        if (n0) c.marks[p++] = x0;
        if (n1) c.marks[p++] = x1;
        if (n2) c.marks[p++] = x2;
        if (n3) c.marks[p] = x3;
    }
}

// entry i of a row ending at end, or an in-range dummy (vertex 0, no
// relation) past the end
__device__ __forceinline__ int2 adj_at(const int2 *adj, int32_t i, int32_t end) {
    return i < end ? adj[i] : make_int2(0, -1);
}

__device__ __forceinline__ bool nbr_hit(const Ctx &c, const NNbr &d, int2 e) {
    if (d.rel >= 0 && e.y != d.rel) return false;
    return d.mode == 0 ? bit_test(c.B(d.v), e.x) : vpred(c.g, c.Q->pred[d.v], e.x);
}

// Keep only the list entries whose bit is still set, preserving order.
__device__ __forceinline__ void compact_list(Ctx &c, int u) {
    int32_t *l = c.L(u);
    const uint64_t *b = c.B(u);
    __syncthreads();
    const int32_t n = c.s->cnt[u];
    int64_t out = 0;
    // eight consecutive entries per thread, their reads and bit tests all in
    // flight before the block scan; entries keep their order
    constexpr int kI = 8;
    for (int32_t base = 0; base < n; base += kI * NT) {
        const int32_t i0 = base + threadIdx.x * kI;
        int32_t x[kI];
#pragma unroll
        for (int k = 0; k < kI; ++k) x[k] = i0 + k < n ? l[i0 + k] : 0;
        bool keep[kI];
        int32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            keep[k] = i0 + k < n && bit_test(b, x[k]);
            cnt += keep[k] ? 1 : 0;
        }
        int64_t tot;
        int64_t p = out + block_excl_scan(cnt, c.s->sh, &tot);
        // the block scan's barriers ordered every read of this round before
        // these writes, which stay at or below the entries just read
#pragma unroll
        for (int k = 0; k < kI; ++k)
            if (keep[k]) l[p++] = x[k];
        out += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c.s->cnt[u] = (int32_t)out;
        add_bytes(c, 12ull * n + 4ull * out);
    }
    __syncthreads();
}

// Rebuild list u from its bitmap in ascending order (O(V/64) words).
__device__ __forceinline__ void list_from_bits(Ctx &c, int u, const uint64_t *src, bool copy_bits) {
    const int32_t nwords = c.g.nwords;
    uint64_t *b = c.B(u);
    int32_t *l = c.L(u);
    int64_t out = 0;
    // eight consecutive words per thread, all read before any is used (a
    // dependent read per block scan would leave the workgroup waiting)
    constexpr int kW = 8;
    for (int32_t base = 0; base < nwords; base += kW * NT) {
        const int32_t w0 = base + threadIdx.x * kW;
        uint64_t wd[kW];
#pragma unroll
        for (int k = 0; k < kW; ++k) wd[k] = w0 + k < nwords ? src[w0 + k] : 0ull;
        int32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            if (copy_bits && w0 + k < nwords) b[w0 + k] = wd[k];
            cnt += __popcll(wd[k]);
        }
        int64_t tot;
        const int64_t ex = block_excl_scan(cnt, c.s->sh, &tot);
        if (out + tot > c.lcap) {
            if (threadIdx.x == 0) c.s->abort_ = kWhyList;
            break;  // uniform: tot and out are block-uniform
        }
        int64_t p = out + ex;
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            uint64_t word = wd[k];
            while (word) {
                l[p++] = (w0 + k) * 64 + __builtin_ctzll(word);
                word &= word - 1ull;
            }
        }
        out += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0 && !c.s->abort_) {
        c.s->cnt[u] = (int32_t)out;
        add_bytes(c, (copy_bits ? 16ull : 8ull) * nwords + 4ull * out);
    }
    __syncthreads();
}

// Sort list u ascending (LDS bitonic, or a rebuild from the bitmap).
__device__ __forceinline__ void sort_list(Ctx &c, int u) {
    __syncthreads();
    const int32_t n = c.s->cnt[u];
    if (n <= 1) return;
    int32_t N = 1, lg = 0;
    while (N < n) {
        N <<= 1;
        ++lg;
    }
    // barrier rounds of a bitonic network vs. an ordered rebuild from the
    // bitmap (two barriers per NT words)
    const int64_t cost_bitonic = (int64_t)lg * (lg + 1) / 2 * ((N / 2 + NT - 1) / NT);
    const int64_t cost_bits = 2 * ((c.g.nwords + 8 * NT - 1) / (8 * NT));
    if (n > kListSortCap || cost_bits < cost_bitonic) {
        list_from_bits(c, u, c.B(u), false);
        return;
    }
    int32_t *l = c.L(u);
    int32_t *t = (int32_t *)c.dyn;
    for (int32_t i = threadIdx.x; i < N; i += NT) t[i] = i < n ? l[i] : INT32_MAX;
    __syncthreads();
    for (int32_t size = 2; size <= N; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t i = threadIdx.x; i < N / 2; i += NT) {
                const int32_t lo = 2 * i - (i & (stride - 1));
                const int32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t x = t[lo], y = t[hi];
                if ((x > y) == up) {
                    t[lo] = y;
                    t[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int32_t i = threadIdx.x; i < n; i += NT) l[i] = t[i];
    if (threadIdx.x == 0) add_bytes(c, 8ull * n);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// filtering: one explore / refine step (Alg. 3.2 kernel_explore; refinement)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void row_of(const DevGraph &g, int32_t up, int dir, int32_t *beg,
                                       int32_t *end) {
    const int32_t *off = dir ? g.in_off : g.out_off;
    *beg = off[up];
    *end = off[up + 1];
}

// Entries of candidate up's row that can pass test d: a hub row (at least
// kHubRow entries) tested against a typed query vertex is read from its
// copy sorted by the other end's type (then by relation for a labelled
// test), restricted to that type (and relation); any other row in full.
// Every entry left out fails the test (wrong type or relation), so the
// outcome is the full row's; the slice keeps the other ends ascending.
__device__ __forceinline__ const int2 *test_row(const Ctx &c, int32_t up, const NNbr &d,
                                                int32_t *beg, int32_t *end) {
    const DevGraph &g = c.g;
    row_of(g, up, d.dir, beg, end);
    const int2 *adj = d.dir ? g.in_adj : g.out_adj;
    if (g.hub_types == 0 || *end - *beg < kHubRow) return adj;
    const int32_t t = c.Q->pred[d.v].label;
    if (t < 0 || t + 1 >= g.hub_types) return adj;
    const int32_t h = g.hub_of[up];
    const int order = d.rel >= 0 ? 0 : 1;
    const int32_t *toff = g.hub_toff + ((int64_t)(h * 2 + d.dir) * 2 + order) * g.hub_types;
    int32_t b = *beg + toff[t], e = *beg + toff[t + 1];
    const int2 *arr = d.dir ? (order ? g.in_tb : g.in_ta) : (order ? g.out_tb : g.out_ta);
    if (d.rel >= 0) {
        // the type's entries are sorted by relation: its relation's range
        int32_t lo = b, hi = e;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (arr[mid].y < d.rel) lo = mid + 1;
            else hi = mid;
        }
        int32_t lo2 = lo, hi2 = e;
        while (lo2 < hi2) {
            const int32_t mid = (lo2 + hi2) >> 1;
            if (arr[mid].y <= d.rel) lo2 = mid + 1;
            else hi2 = mid;
        }
        b = lo;
        e = lo2;
    }
    *beg = b;
    *end = e;
    return arr;
}

// Whole workgroup on one candidate (uniform call). Prune: the candidate
// survives if every listed query edge has a matching neighbour; explore
// then pushes every matching neighbour.
__device__ __forceinline__ int32_t max_row(const DevGraph &g, const NNbr *nb, int ncount, int32_t up);

template <class K>
__device__ __forceinline__ void item_wg_k(Ctx &c, const K &k, const NStep &st, const NNbr *nb,
                                          int ncount, int32_t up, uint64_t *ub, uint64_t &fb,
                                          int32_t *defer = nullptr) {
    const DevGraph &g = c.g;
    if (ncount <= 16 && max_row(g, nb, ncount, up) <= 4 * NT) {
        // Every listed row fits one pass: all rows are read and tested at
        // once (bit 4j + k of `hits`: entry threadIdx.x + k NT of row j
        // matches), one barrier decides whether the candidate lives, and
        // pushes replay the recorded hits.
        if (threadIdx.x == 0) c.s->rowhit = 0ull;
        __syncthreads();
        uint64_t hits = 0, seen = 0;
        for (int j = 0; j < ncount; ++j) {
            const NNbr d = nb[j];
            const int2 *adj = d.dir ? g.in_adj : g.out_adj;
            int32_t beg, end;
            row_of(g, up, d.dir, &beg, &end);
            const int32_t i = beg + threadIdx.x;
            const int2 e0 = adj_at(adj, i, end), e1 = adj_at(adj, i + NT, end);
            const int2 e2 = adj_at(adj, i + 2 * NT, end), e3 = adj_at(adj, i + 3 * NT, end);
            const uint64_t h = (uint64_t)((i < end) & nbr_hit(c, d, e0)) |
                               (uint64_t)((i + NT < end) & nbr_hit(c, d, e1)) << 1 |
                               (uint64_t)((i + 2 * NT < end) & nbr_hit(c, d, e2)) << 2 |
                               (uint64_t)((i + 3 * NT < end) & nbr_hit(c, d, e3)) << 3;
            if (h) atomicOr(&c.s->rowhit, 1ull << j);
            hits |= h << (4 * j);
            seen += end - beg;
        }
        __syncthreads();
        const bool alive = __popcll(c.s->rowhit) == ncount;
        __syncthreads();  // rowhit is read by all before the next candidate clears it
        if (!alive) {
            if (threadIdx.x == 0) {
                atomicAnd((unsigned long long *)&ub[up >> 6], ~(1ull << (up & 63)));
                atomicAdd(k.removed(), 1);
                fb += 20ull + 12ull * seen;
            }
            return;
        }
        if (st.push)
            for (int j = 0; j < ncount; ++j) {
                const uint32_t hj = (uint32_t)(hits >> (4 * j)) & 15u;
                if (!hj) continue;
                const NNbr d = nb[j];
                const int2 *adj = d.dir ? g.in_adj : g.out_adj;
                int32_t beg, end;
                row_of(g, up, d.dir, &beg, &end);
                uint64_t *tb = d.mode == 0 ? c.scratch : c.B(d.v);
                int32_t *tl = d.mode == 0 ? nullptr : c.L(d.v);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if ((hj >> q) & 1u) push_bit(c, k, tb, tl, d.v, adj[beg + threadIdx.x + q * NT].x);
            }
        if (threadIdx.x == 0) fb += 20ull + 12ull * seen;
        return;
    }
    bool alive = true;
    uint64_t seen = 0;
    for (int j = 0; j < ncount && alive; ++j) {
        const NNbr d = nb[j];
        int32_t beg, end;
        const int2 *adj = test_row(c, up, d, &beg, &end);
        bool found = false;
        for (int32_t base = beg; base < end; base += 4 * NT) {
            bool hit = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t i = base + q * NT + threadIdx.x;
                if (i < end) hit |= nbr_hit(c, d, adj[i]);
            }
            seen += min(4 * NT, end - base);
            if (__syncthreads_or(hit)) {
                found = true;
                break;
            }
        }
        alive = found;
    }
    if (!alive) {
        if (threadIdx.x == 0) {
            atomicAnd((unsigned long long *)&ub[up >> 6], ~(1ull << (up & 63)));
            atomicAdd(k.removed(), 1);
            fb += 20ull + 12ull * seen;
        }
        return;
    }
    if (st.push && defer) {
        if (threadIdx.x == 0) {
            defer[c.s->ndef++] = up;
            fb += 20ull + 12ull * seen;
        }
        return;
    }
    if (st.push) {
        for (int j = 0; j < ncount; ++j) {
            const NNbr d = nb[j];
            int32_t beg, end;
            const int2 *adj = test_row(c, up, d, &beg, &end);
            uint64_t *tb = d.mode == 0 ? c.scratch : c.B(d.v);
            int32_t *tl = d.mode == 0 ? nullptr : c.L(d.v);
            seen += end - beg;
            for (int32_t base = beg; base < end; base += 8 * NT) {
                // eight independent loads in flight per thread; a row's
                // neighbours are distinct, so their bits are set without a
                // look first
                const int32_t i = base + threadIdx.x;
                int2 e[8];
                bool h[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) e[q] = adj_at(adj, i + q * NT, end);
#pragma unroll
                for (int q = 0; q < 8; ++q) h[q] = (i + q * NT < end) && nbr_hit(c, d, e[q]);
                push4<K, false>(c, k, tb, tl, d.v, h[0], e[0].x, h[1], e[1].x,
                                     h[2], e[2].x, h[3], e[3].x);
                push4<K, false>(c, k, tb, tl, d.v, h[4], e[4].x, h[5], e[5].x,
                                     h[6], e[6].x, h[7], e[7].x);
            }
        }
    }
    if (threadIdx.x == 0) fb += 20ull + 12ull * seen;
}

__device__ __forceinline__ void item_wg(Ctx &c, const NStep &st, const NNbr *nb, int ncount, int32_t up,
                                        uint64_t *ub, uint64_t &fb, int32_t *defer = nullptr) {
    item_wg_k(c, LdsCtr{c.s}, st, nb, ncount, up, ub, fb, defer);
}

// One wave on one candidate (wave-uniform call, no workgroup barrier), four
// loads in flight per lane; same outcome as item_wg.
__device__ __forceinline__ void item_wave(Ctx &c, const NStep &st, const NNbr *nb, int ncount,
                                          int32_t up, uint64_t *ub, uint64_t &fb,
                                          int32_t *defer = nullptr) {
    const DevGraph &g = c.g;
    const int lane = threadIdx.x & 63;
    bool alive = true;
    uint64_t seen = 0;
    for (int j = 0; j < ncount && alive; ++j) {
        const NNbr d = nb[j];
        int32_t beg, end;
        const int2 *adj = test_row(c, up, d, &beg, &end);
        bool found = false;
        for (int32_t base = beg; base < end; base += 256) {
            const int32_t i = base + lane;
            const int2 e0 = i < end ? adj[i] : make_int2(-1, -1);
            const int2 e1 = i + 64 < end ? adj[i + 64] : make_int2(-1, -1);
            const int2 e2 = i + 128 < end ? adj[i + 128] : make_int2(-1, -1);
            const int2 e3 = i + 192 < end ? adj[i + 192] : make_int2(-1, -1);
            const bool hit = (e0.x >= 0 && nbr_hit(c, d, e0)) || (e1.x >= 0 && nbr_hit(c, d, e1)) ||
                             (e2.x >= 0 && nbr_hit(c, d, e2)) || (e3.x >= 0 && nbr_hit(c, d, e3));
            seen += min(256, end - base);
            if (__ballot(hit)) {
                found = true;
                break;
            }
        }
        alive = found;
    }
    if (!alive) {
        if (lane == 0) {
            atomicAnd((unsigned long long *)&ub[up >> 6], ~(1ull << (up & 63)));
            atomicAdd(&c.s->removed, 1);
            fb += 20ull + 12ull * seen;
        }
        return;
    }
    if (st.push && defer) {
        // the pushes go to row segments that several workgroups share
        if (lane == 0) {
            defer[atomicAdd(&c.s->ndef, 1)] = up;
            fb += 20ull + 12ull * seen;
        }
        return;
    }
    if (st.push)
        for (int j = 0; j < ncount; ++j) {
            const NNbr d = nb[j];
            int32_t beg, end;
            const int2 *adj = test_row(c, up, d, &beg, &end);
            uint64_t *tb = d.mode == 0 ? c.scratch : c.B(d.v);
            int32_t *tl = d.mode == 0 ? nullptr : c.L(d.v);
            seen += end - beg;
            for (int32_t base = beg; base < end; base += 256) {
                const int32_t i = base + lane;
                const int2 e0 = i < end ? adj[i] : make_int2(-1, -1);
                const int2 e1 = i + 64 < end ? adj[i + 64] : make_int2(-1, -1);
                const int2 e2 = i + 128 < end ? adj[i + 128] : make_int2(-1, -1);
                const int2 e3 = i + 192 < end ? adj[i + 192] : make_int2(-1, -1);
                if (e0.x >= 0 && nbr_hit(c, d, e0)) push_bit(c, tb, tl, d.v, e0.x);
                if (e1.x >= 0 && nbr_hit(c, d, e1)) push_bit(c, tb, tl, d.v, e1.x);
                if (e2.x >= 0 && nbr_hit(c, d, e2)) push_bit(c, tb, tl, d.v, e2.x);
                if (e3.x >= 0 && nbr_hit(c, d, e3)) push_bit(c, tb, tl, d.v, e3.x);
            }
        }
    if (lane == 0) fb += 20ull + 12ull * seen;
}

// longest adjacency row a candidate scans for the listed query edges
__device__ __forceinline__ int32_t max_row(const DevGraph &g, const NNbr *nb, int ncount, int32_t up) {
    int32_t m = 0;
    for (int j = 0; j < ncount; ++j) {
        const int32_t *off = nb[j].dir ? g.in_off : g.out_off;
        m = max(m, off[up + 1] - off[up]);
    }
    return m;
}

// lanes per candidate for n items: the whole workgroup for a handful,
// otherwise a power of two in [1, 64] so that all lanes hold an item
__device__ __forceinline__ int lanes_for(int32_t n, int gmax) {
    int G = gmax;
    while (G > 1 && (int64_t)G * n > NT) G >>= 1;
    return G;
}

// Reverse form of the prune test against one initialised neighbour v with
// few candidates (prune-only steps): mark the candidates of u that have a
// matching edge to some candidate of v, found in the rows of v's candidates
// in the other direction, then drop the unmarked ones. The survivors are the
// same as when each candidate of u scans its own row for a member of v's
// bitmap. Marks go to the slot's scratch bitmap, which a prune-only step
// does not otherwise use; they fall inside u's candidates, so clearing the
// words of u's list leaves it zero again.
__device__ __forceinline__ void prune_reverse(Ctx &c, int u, int v, int dir, int32_t rel,
                                              uint64_t &fb) {
    const DevGraph &g = c.g;
    uint64_t *ub = c.B(u);
    const int32_t *ul = c.L(u);
    const int32_t n = c.s->cnt[u];
    const int32_t *vl = c.L(v);
    const int32_t nv = c.s->cnt[v];
    // a candidate's out-edge (dir 0) is an in-edge of the neighbour, and so on
    const int32_t *off = dir ? g.out_off : g.in_off;
    const int2 *adj = dir ? g.out_adj : g.in_adj;
    const int lane = threadIdx.x & 63;
    uint64_t seen = 0;
    for (int32_t i = threadIdx.x >> 6; i < nv; i += NW) {
        const int32_t y = vl[i];
        const int32_t beg = off[y], end = off[y + 1];
        for (int32_t k = beg + lane; k < end; k += 64) {
            const int2 e = adj[k];
            if ((rel < 0 || e.y == rel) && bit_test(ub, e.x))
                atomicOr((unsigned long long *)&c.scratch[e.x >> 6], 1ull << (e.x & 63));
        }
        if (lane == 0) seen += 12ull + 16ull * (end - beg);
    }
    fb += seen;
    __syncthreads();
    int32_t removed = 0;
    for (int32_t i = threadIdx.x; i < n; i += NT) {
        const int32_t x = ul[i];
        if (bit_test(ub, x) && !bit_test(c.scratch, x)) {
            atomicAnd((unsigned long long *)&ub[x >> 6], ~(1ull << (x & 63)));
            ++removed;
        }
    }
    if (removed) atomicAdd(&c.s->removed, removed);
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += NT) c.scratch[ul[i] >> 6] = 0ull;
    if (threadIdx.x == 0) fb += 28ull * n;
    __syncthreads();
}

// Candidates [it0, it1) of u's list (ul, bitmap ub), G lanes each: a
// candidate lacking a matching neighbour for one of the ncount tests is
// dropped; with push, the neighbours of the others that pass a test are
// pushed. Candidates with a row longer than 64 G entries go to the overflow
// list at the start of the slab for a wider tier. Counters go to k.
template <class K>
__device__ __forceinline__ void filter_items(Ctx &c, const K &k, bool push, const NNbr *nb,
                                             int ncount, const int32_t *ul, uint64_t *ub,
                                             bool revd, int G, int32_t it0, int32_t it1,
                                             uint64_t &fb, bool nodefer = false) {
    const DevGraph &g = c.g;
    const int NGr = NT / G;
    const int lane = threadIdx.x & 63, gl = lane & (G - 1), gb = lane & ~(G - 1);
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << gb;
    // more than 64 strides: a wider tier (a shared pass over long rows
    // keeps the rows up to wg_rows, which the whole workgroup would take
    // next; longer ones stay with the owner, whose pushes become shared
    // row segments)
    const int32_t bigdeg = nodefer ? max(64 * G, c.wg_rows) : 64 * G;
    // The overflow list sits at the start of the slot's slab, which no phase
    // uses while filtering (at most lcap entries, far below its size).
    int32_t *ov = (int32_t *)c.slab;
    // the next item's vertex is read while this one is tested, and its row
    // offsets as soon as it has arrived (one dependent read less per item)
    int32_t it = it0 + threadIdx.x / G;
    int32_t upn = it < it1 ? ul[it] : 0;
    for (; it < it1; it += NGr) {
        const int32_t up = upn;
        const int32_t ob = g.out_off[up], oe = g.out_off[up + 1];
        const int32_t ib = g.in_off[up], ie = g.in_off[up + 1];
        upn = it + NGr < it1 ? ul[it + NGr] : 0;
        if (revd && !bit_test(ub, up)) continue;  // already dropped
        int32_t maxd = 0;
        for (int j = 0; j < ncount; ++j) maxd = max(maxd, nb[j].dir ? ie - ib : oe - ob);
        if (maxd > bigdeg) {
            // long rows: a wider tier after this loop. The overflow list
            // sits at the start of the slot's slab, which no phase uses
            // while filtering (at most lcap entries, far below its size).
            if (gl == 0) ov[atomicAdd(k.nbig(), 1)] = up;
            continue;
        }
        if (push && ncount == 1) {
            // a single neighbour test: one scan pushes the hits it finds,
            // and a candidate with none is dropped (it pushed nothing)
            const NNbr d = nb[0];
            const int2 *adj = d.dir ? g.in_adj : g.out_adj;
            const int32_t beg = d.dir ? ib : ob, end = d.dir ? ie : oe;
            uint64_t *tb = d.mode == 0 ? c.scratch : c.B(d.v);
            int32_t *tl = d.mode == 0 ? nullptr : c.L(d.v);
            bool any = false;
            for (int32_t i = beg + gl; i < end; i += 4 * G) {
                const int2 e0 = adj_at(adj, i, end), e1 = adj_at(adj, i + G, end);
                const int2 e2 = adj_at(adj, i + 2 * G, end), e3 = adj_at(adj, i + 3 * G, end);
                const bool h0 = (i < end) & nbr_hit(c, d, e0);
                const bool h1 = (i + G < end) & nbr_hit(c, d, e1);
                const bool h2 = (i + 2 * G < end) & nbr_hit(c, d, e2);
                const bool h3 = (i + 3 * G < end) & nbr_hit(c, d, e3);
                push4(c, k, tb, tl, d.v, h0, e0.x, h1, e1.x, h2, e2.x, h3, e3.x);
                any |= h0 | h1 | h2 | h3;
            }
            if (!(__ballot(any) & gmask)) {
                if (gl == 0) {
                    atomicAnd((unsigned long long *)&ub[up >> 6], ~(1ull << (up & 63)));
                    atomicAdd(k.removed(), 1);
                }
            }
            if (gl == 0) fb += 20ull + 12ull * (uint64_t)(end - beg);
            continue;
        }
        bool alive = true;
        uint64_t seen = 0;
        for (int j = 0; j < ncount && alive; ++j) {
            const NNbr d = nb[j];
            const int2 *adj = d.dir ? g.in_adj : g.out_adj;
            const int32_t beg = d.dir ? ib : ob, end = d.dir ? ie : oe;
            bool found = false;
            // four entries per lane in flight; lanes past the row test an
            // in-range dummy entry and discard the answer
            for (int32_t base = beg; base < end; base += 4 * G) {
                const int32_t i = base + gl;
                const int2 e0 = adj_at(adj, i, end), e1 = adj_at(adj, i + G, end);
                const int2 e2 = adj_at(adj, i + 2 * G, end), e3 = adj_at(adj, i + 3 * G, end);
                const bool hit = ((i < end) & nbr_hit(c, d, e0)) |
                                 ((i + G < end) & nbr_hit(c, d, e1)) |
                                 ((i + 2 * G < end) & nbr_hit(c, d, e2)) |
                                 ((i + 3 * G < end) & nbr_hit(c, d, e3));
                seen += min(4 * G, end - base);
                if (__ballot(hit) & gmask) {
                    found = true;
                    break;
                }
            }
            alive = found;
        }
        if (!alive) {
            if (gl == 0) {
                atomicAnd((unsigned long long *)&ub[up >> 6], ~(1ull << (up & 63)));
                atomicAdd(k.removed(), 1);
                fb += 20ull + 12ull * seen;
            }
            continue;
        }
        if (push)
            for (int j = 0; j < ncount; ++j) {
                const NNbr d = nb[j];
                const int2 *adj = d.dir ? g.in_adj : g.out_adj;
                const int32_t beg = d.dir ? ib : ob, end = d.dir ? ie : oe;
                uint64_t *tb = d.mode == 0 ? c.scratch : c.B(d.v);
                int32_t *tl = d.mode == 0 ? nullptr : c.L(d.v);
                seen += end - beg;
                for (int32_t i = beg + gl; i < end; i += 4 * G) {
                    const int2 e0 = adj_at(adj, i, end), e1 = adj_at(adj, i + G, end);
                    const int2 e2 = adj_at(adj, i + 2 * G, end), e3 = adj_at(adj, i + 3 * G, end);
                    const bool h0 = (i < end) & nbr_hit(c, d, e0);
                    const bool h1 = (i + G < end) & nbr_hit(c, d, e1);
                    const bool h2 = (i + 2 * G < end) & nbr_hit(c, d, e2);
                    const bool h3 = (i + 3 * G < end) & nbr_hit(c, d, e3);
                    push4(c, k, tb, tl, d.v, h0, e0.x, h1, e1.x, h2, e2.x, h3, e3.x);
                }
            }
        if (gl == 0) fb += 20ull + 12ull * seen;
    }
}

// Empty polls in a row before a helper leaves (helping is optional, so
// leaving early only costs speed; about a second of polling). The owner of
// a shared step polls its completion count at most NArgs::help_wait times
// (default 4M) before it gives up: an error, since every claimed chunk
// finishes in bounded time.
constexpr int64_t kHelpIdle = 1ll << 20;

// Claim word of a posted step, and a claim's outcome.
__device__ __forceinline__ unsigned long long claim_word(uint32_t seq, int32_t nch) {
    return ((unsigned long long)(seq & 0xffffffu) << 40) | ((unsigned long long)nch << 20);
}
__device__ __forceinline__ uint32_t claim_seq(unsigned long long w) { return (uint32_t)(w >> 40); }
__device__ __forceinline__ int32_t claim_nch(unsigned long long w) {
    return (int32_t)((w >> 20) & 0xfffffull);
}
__device__ __forceinline__ int32_t claim_next(unsigned long long w) {
    return (int32_t)(w & 0xfffffull);
}
// A step has at most this many chunks; unsuccessful claims raise the next
// field past the chunk count by at most one per workgroup of the launch, so
// it never reaches the chunk field.
constexpr int32_t kMaxChunks = 1 << 19;

// Take one chunk of board entry j (thread 0): the returned claim word's next
// field is the chunk, which exists if it is below the chunk field. The step
// named by the word stays posted, with fixed parameters, until every chunk
// taken from it is reported done.
__device__ __forceinline__ unsigned long long take_chunk(HelpJob *j) {
    return atomicAdd(&j->claim, 1ull);
}

// Row segments: pushes of long rows of surviving candidates, kSegEntries
// entries of one row and one neighbour test per segment, one pass of a
// whole workgroup each.
constexpr int32_t kSegEntries = 8 * NT;

// The pushes of segment sg = (candidate, test index, first entry, end) of a
// row (whole workgroup). A row's neighbours are distinct, so bits are set
// without a look first.
template <class K>
__device__ __forceinline__ void push_segment(Ctx &c, const K &k, const NNbr *nb, int4 sg,
                                             uint64_t &fb) {
    const NNbr d = nb[sg.y];
    int32_t rb, re;  // the segment indexes the array test_row picks for its row
    const int2 *adj = test_row(c, sg.x, d, &rb, &re);
    uint64_t *tb = d.mode == 0 ? c.scratch : c.B(d.v);
    int32_t *tl = d.mode == 0 ? nullptr : c.L(d.v);
    for (int32_t base = sg.z; base < sg.w; base += kSegEntries) {
        const int32_t i = base + threadIdx.x;
        int2 e[8];
        bool h[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = adj_at(adj, i + q * NT, sg.w);
#pragma unroll
        for (int q = 0; q < 8; ++q) h[q] = (i + q * NT < sg.w) && nbr_hit(c, d, e[q]);
        push4<K, false>(c, k, tb, tl, d.v, h[0], e[0].x, h[1], e[1].x, h[2], e[2].x, h[3], e[3].x);
        push4<K, false>(c, k, tb, tl, d.v, h[4], e[4].x, h[5], e[5].x, h[6], e[6].x, h[7], e[7].x);
    }
    if (threadIdx.x == 0) fb += 12ull * (uint64_t)(sg.w - sg.z);
}

// Segments of the rows of the nd deferred candidates into seg (at most cap);
// the count, or -1 if they do not fit (uniform).
__device__ __forceinline__ int32_t build_segments(Ctx &c, const NNbr *nb, int ncount,
                                                  const int32_t *def, int32_t nd, int4 *seg,
                                                  int64_t cap) {
    int64_t carry = 0;
    for (int32_t base = 0; base < nd; base += NT) {
        const int32_t i = base + threadIdx.x;
        int32_t cnt = 0;
        if (i < nd)
            for (int j = 0; j < ncount; ++j) {
                int32_t b, e;
                test_row(c, def[i], nb[j], &b, &e);
                cnt += (e - b + kSegEntries - 1) / kSegEntries;
            }
        int64_t tot;
        const int64_t ex = block_excl_scan(cnt, c.s->sh, &tot);
        if (i < nd && carry + tot <= cap) {
            int64_t p = carry + ex;
            for (int j = 0; j < ncount; ++j) {
                int32_t b, e;
                test_row(c, def[i], nb[j], &b, &e);
                for (int32_t x = b; x < e; x += kSegEntries)
                    seg[p++] = make_int4(def[i], j, x, min(e, x + kSegEntries));
            }
        }
        carry += tot;
    }
    __syncthreads();
    return carry <= cap ? (int32_t)carry : -1;
}

__device__ __forceinline__ void ec_chunk(Ctx &c, const EcJob &E, HelpJob *j, int32_t i0, int32_t i1,
                                         int G, uint64_t &fb);

// A filter step shared with the launch's idle workgroups through this
// slot's board entry: the counters move to the entry, the work is cut into
// nch chunks that the owner and its helpers claim (kind 0: K candidates of
// u's list, G lanes each; kind 1: one row segment each), and the owner waits
// for the chunks its helpers claimed before taking the counters back.
__device__ __forceinline__ void shared_job(Ctx &c, int kind, const NStep &st, const NNbr *nb,
                                           int ncount, const int32_t *ul, uint64_t *ub, bool revd,
                                           int32_t n_items, int32_t K, int G, int32_t nch,
                                           const int4 *seg, uint64_t &fb,
                                           const EcJob *ecj = nullptr, bool nodefer = false) {
    HelpJob *j = c.job;
    if (threadIdx.x == 0) {
        for (int v = 0; v < SGM_MAX_QV; ++v) j->cnt[v] = c.s->cnt[v];
        j->nbig = 0;
        j->removed = 0;
        j->nmarks = c.s->nmarks;
        j->abort_ = 0;
        j->bytes = 0ull;
        j->done = 0;
        j->kind = kind;
        j->nodefer = nodefer;
        j->seg = seg;
        j->ul = ul;
        j->chunk = K;
        j->q = c.q;
        j->n_items = n_items;
        j->G = G;
        j->ncount = ncount;
        j->revd = revd;
        j->st = st;
        for (int i = 0; i < ncount; ++i) {
            j->nbl[i].v = nb[i].v;
            j->nbl[i].dir = nb[i].dir;
            j->nbl[i].mode = nb[i].mode;
            j->nbl[i].rel = nb[i].rel;
        }
        if (ecj) {
            j->ecj = *ecj;
            j->jrows = 0ull;
        }
        const uint32_t seq =
            claim_seq(__hip_atomic_load(&j->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) + 1u;
        // parameters, and the slot's lists and bitmaps, before the claim word
        __threadfence();
        atomicExch(&j->claim, claim_word(seq, nch));
        atomicAdd(&c.hctr[0], 1);
    }
    __syncthreads();
    int32_t own = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned long long w = take_chunk(j);
            c.s->hch = claim_next(w) < claim_nch(w) ? claim_next(w) : -1;
        }
        __syncthreads();
        const int32_t ch = c.s->hch;
        __syncthreads();
        if (ch < 0) break;
        if (kind == 0)
            filter_items(c, BoardCtr{j}, st.push != 0, nb, ncount, ul, ub, revd, G, ch * K,
                         min(n_items, ch * K + K), fb, nodefer);
        else if (kind == 3)
            ec_chunk(c, *ecj, j, ch * K, min(n_items, ch * K + K), G, fb);
        else if (kind == 4)
            item_wg_k(c, BoardCtr{j}, st, nb, ncount, ul[ch], ub, fb);
        else
            push_segment(c, BoardCtr{j}, nb, seg[ch], fb);
        ++own;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the owner's own chunks need no fence: it reads them itself
        int32_t got = atomicAdd(&j->done, own) + own;
        int64_t n = 0;
        while (got < nch && n < c.help_wait) {
            __builtin_amdgcn_s_sleep(1);
            got = __hip_atomic_load(&j->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ++n;
        }
        if (got < nch) {
            // give up: no further claims on the step (a claim against zero
            // chunks fails), and the slot stays out of use until the next
            // launch clears it, since chunks claimed earlier may still write
            // its bitmaps and lists
            const uint32_t seq = claim_seq(
                __hip_atomic_load(&j->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            atomicExch(&j->claim, claim_word(seq, 0));
            atomicExch(&j->dirty, 1);
            c.s->retired = 1;
        }
        __threadfence();
        atomicSub(&c.hctr[0], 1);
        for (int v = 0; v < SGM_MAX_QV; ++v)
            c.s->cnt[v] = __hip_atomic_load(&j->cnt[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        c.s->nbig += __hip_atomic_load(&j->nbig, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        c.s->removed += __hip_atomic_load(&j->removed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        c.s->nmarks = __hip_atomic_load(&j->nmarks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t ab = __hip_atomic_load(&j->abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ab) c.s->abort_ = ab;
        if (got < nch) c.s->abort_ = kWhyHelp;
        add_bytes(c, __hip_atomic_load(&j->bytes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    __syncthreads();
}

// Chunks of u's candidate list shared as above.
__device__ __forceinline__ void shared_items(Ctx &c, const NStep &st, const NNbr *nb, int ncount,
                                             const int32_t *ul, uint64_t *ub, bool revd,
                                             int32_t n_items, int32_t helpers, uint64_t &fb) {
    const int32_t K = min(512, max(64, max((n_items + helpers) / (helpers + 1),
                                           (n_items + kMaxChunks - 1) / kMaxChunks)));
    const int G = lanes_for(K, c.gmax);
    const int32_t nch = (n_items + K - 1) / K;
    shared_job(c, 0, st, nb, ncount, ul, ub, revd, n_items, K, G, nch, nullptr, fb);
}

// Workgroups that can help this slot now: the launch's extra ones and the
// slot workgroups whose queue ran dry (uniform).
__device__ __forceinline__ int32_t helpers_now(Ctx &c) {
    if (c.help_items <= 0) return 0;
    if (c.ngrid > c.nslot) return c.ngrid - c.nslot;
    __syncthreads();
    if (threadIdx.x == 0)
        c.s->hch = c.ngrid - c.nslot +
                   __hip_atomic_load(&c.hctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int32_t h = c.s->hch;
    __syncthreads();
    return h;
}

// The pushes deferred by the wave and workgroup tiers, as shared row
// segments (or by this workgroup alone when they do not fit the slab).
__device__ __forceinline__ void push_deferred(Ctx &c, const NStep &st, const NNbr *nb, int ncount,
                                              const int32_t *def, uint64_t &fb) {
    __syncthreads();
    const int32_t nd = c.s->ndef;
    if (nd == 0) return;
    int4 *seg = (int4 *)(c.slab + 12 * (int64_t)c.lcap);
    // room in the slab, and no more chunks than a claim word can count
    const int64_t cap = min((c.slab_bytes - 12 * (int64_t)c.lcap) / (int64_t)sizeof(int4),
                            (int64_t)kMaxChunks);
    const int32_t nseg = build_segments(c, nb, ncount, def, nd, seg, cap);
    if (nseg > 0) {
        shared_job(c, 1, st, nb, ncount, nullptr, nullptr, false, 0, 1, NT, nseg, seg, fb);
    } else {
        for (int32_t i = 0; i < nd; ++i)
            for (int j = 0; j < ncount; ++j) {
                int32_t b, e;
                test_row(c, def[i], nb[j], &b, &e);
                push_segment(c, LdsCtr{c.s}, nb, make_int4(def[i], j, b, e), fb);
            }
        __syncthreads();
    }
}

// Where the wave and workgroup tiers of a pushing step list the candidates
// whose pushes become shared row segments, when helpers exist and the slab
// has room beyond the overflow list and the marks; else nullptr (uniform).
__device__ __forceinline__ int32_t *defer_list(Ctx &c, const NStep &st) {
    if (!st.push || c.help_items <= 0) return nullptr;
    if (c.slab_bytes < 12 * (int64_t)c.lcap + 64 * (int64_t)sizeof(int4)) return nullptr;
    if (helpers_now(c) <= 0) return nullptr;
    return (int32_t *)(c.slab + 8 * (int64_t)c.lcap);
}

__device__ __forceinline__ void filter_step(Ctx &c, const NStep &st) {
    const DevGraph &g = c.g;
    const int u = st.u;
    uint64_t *ub = c.B(u);
    int32_t *ul = c.L(u);
    __syncthreads();
    if (threadIdx.x == 0) {
        c.s->nbig = 0;
        c.s->ngiant = 0;
        c.s->removed = 0;
        c.s->nmarks = 0;
        c.s->ndef = 0;
    }
    __syncthreads();
    const int32_t n_items = c.s->cnt[u];
    uint64_t fb = 0;  // algorithmic bytes of this thread's work
    // The step's neighbour tests go to LDS. In prune-only steps over many
    // candidates, a neighbour with few candidates whose rows together are
    // shorter than u's list is instead checked from its side (prune_reverse).
    const bool try_rev = !st.push && n_items >= kRevMin;
    if (threadIdx.x < 64) {
        const NNbr *src = c.Q->nbr + st.first;
        int k = 0;
        uint64_t rm = 0;
        for (int j = 0; j < st.count; ++j) {
            const int v = src[j].v, dir = src[j].dir, mode = src[j].mode;
            const int32_t rel = src[j].rel;
            bool rev = false;
            const int32_t nv = c.s->cnt[v];
            if (try_rev && mode == 0 && nv <= kRevMaxCand && nv < n_items) {
                // reverse cost: v's list plus its rows, against at least one
                // read per candidate of u forward
                const int32_t *off = dir ? g.out_off : g.in_off;
                const int32_t *vl = c.L(v);
                int64_t sum = nv;
                for (int32_t b = 0; b < nv && sum <= n_items; b += 64) {
                    int32_t len = 0;
                    if (b + (int32_t)threadIdx.x < nv) {
                        const int32_t y = vl[b + threadIdx.x];
                        len = off[y + 1] - off[y];
                    }
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) len += __shfl_xor(len, o, 64);
                    sum += len;
                }
                rev = sum <= n_items;
            }
            if (rev) {
                rm |= 1ull << j;
            } else {
                if (threadIdx.x == 0) {
                    NNbr &t = c.s->nbl[k];
                    t.v = (int8_t)v;
                    t.dir = (int8_t)dir;
                    t.mode = (int8_t)mode;
                    t.rel = rel;
                }
                ++k;
            }
        }
        if (threadIdx.x == 0) {
            c.s->revmask = rm;
            c.s->nnbl = k;
        }
    }
    __syncthreads();
    const NNbr *nb = c.s->nbl;
    const int ncount = c.s->nnbl;
    const uint64_t rm = c.s->revmask;
    const bool revd = rm != 0;
    for (int j = 0; j < st.count && revd; ++j)
        if ((rm >> j) & 1ull) {
            const NNbr *d = c.Q->nbr + st.first + j;
            prune_reverse(c, u, d->v, d->dir, d->rel, fb);
        }
    if (ncount == 0) {
        // every test was done from the other side
    } else if (n_items <= NW) {
        int32_t *def = defer_list(c, st);
        for (int32_t it = 0; it < n_items; ++it) item_wg(c, st, nb, ncount, ul[it], ub, fb, def);
        if (def) push_deferred(c, st, nb, ncount, def, fb);
    } else {
        // a step of many candidates is shared whether or not workgroups are
        // idle yet (in a batch they become idle while it runs)
        const bool share = c.help_items > 0 && c.job && n_items >= c.help_items;
        const int32_t helpers = share ? helpers_now(c) : 0;
        if (share)
            shared_items(c, st, nb, ncount, ul, ub, revd, n_items, helpers, fb);
        else
            filter_items(c, LdsCtr{c.s}, st.push != 0, nb, ncount, ul, ub, revd,
                         lanes_for(n_items, c.gmax), 0, n_items, fb);
        const int lane = threadIdx.x & 63;
        int32_t *ov = (int32_t *)c.slab;
        __syncthreads();
        if (c.help_items > 0 && c.job && c.s->nbig >= kLongShare &&
            c.slab_bytes >= 16 * (int64_t)c.lcap) {
            // many long rows: one wave per row up to wg_rows entries,
            // shared like a step of many candidates (the rows move to a
            // list of their own; longer ones come back to the overflow list)
            ev(c, SGM_EV_LONGROWS);
            const int32_t nl = c.s->nbig;
            int32_t *rows = (int32_t *)(c.slab + 12 * (int64_t)c.lcap);
            for (int32_t i = threadIdx.x; i < nl; i += NT) rows[i] = ov[i];
            __syncthreads();
            if (threadIdx.x == 0) c.s->nbig = 0;
            const int32_t nch = (nl + kLongChunk - 1) / kLongChunk;
            shared_job(c, 0, st, nb, ncount, rows, ub, revd, nl, kLongChunk, 64, nch, nullptr,
                       fb, nullptr, true);
            __syncthreads();
        }
        // one wave per long row; rows above wg_rows get the whole workgroup
        const int32_t nbig = c.s->nbig;
        if (nbig > 0) ev(c, SGM_EV_LONGROWS);
        int32_t *def = nbig > 0 ? defer_list(c, st) : nullptr;
        for (int32_t b = threadIdx.x >> 6; b < nbig; b += NW) {
            const int32_t up = ov[b];
            if (max_row(g, nb, ncount, up) > c.wg_rows) {
                int32_t p = 0;
                if (lane == 0) p = atomicAdd(&c.s->ngiant, 1);
                p = __shfl(p, 0, 64);
                if (p < kBigCap) {
                    if (lane == 0) c.s->big[p] = up;
                    continue;
                }
                // LDS list full: this wave handles the row itself
            }
            item_wave(c, st, nb, ncount, up, ub, fb, def);
        }
        __syncthreads();
        const int32_t ngiant = min(c.s->ngiant, kBigCap);
        if (!st.push && ngiant >= 2 && c.help_items > 0 && c.job &&
            c.slab_bytes >= 16 * (int64_t)c.lcap) {
            // rows above wg_rows in a prune-only step: one workgroup each,
            // shared (a pushing step's rows go out as shared row segments)
            int32_t *rows = (int32_t *)(c.slab + 12 * (int64_t)c.lcap);
            for (int32_t i = threadIdx.x; i < ngiant; i += NT) rows[i] = c.s->big[i];
            __syncthreads();
            shared_job(c, 4, st, nb, ncount, rows, ub, revd, ngiant, 1, NT, ngiant, nullptr, fb);
        } else {
            for (int32_t b = 0; b < ngiant; ++b) item_wg(c, st, nb, ncount, c.s->big[b], ub, fb, def);
        }
        if (def) push_deferred(c, st, nb, ncount, def, fb);
    }
    add_bytes_wave(c, fb);
    __syncthreads();
    if (c.s->removed) compact_list(c, u);
    if (st.parent >= 0 && 4 * c.s->nmarks < c.s->cnt[st.parent]) {
        // Intersect the parent's candidates with the pushed marks. The marks
        // are parent candidates, so the intersection is the marks
        // themselves: with few of them, clear the parent's old words and
        // rebuild its bitmap and list from the marks.
        const int p = st.parent;
        uint64_t *pb = c.B(p);
        int32_t *pl = c.L(p);
        const int32_t n = c.s->cnt[p], nm = c.s->nmarks;
        for (int32_t i = threadIdx.x; i < n; i += NT) pb[pl[i] >> 6] = 0ull;
        __syncthreads();
        for (int32_t i = threadIdx.x; i < nm; i += NT) {
            const int32_t x = c.marks[i];
            atomicOr((unsigned long long *)&pb[x >> 6], 1ull << (x & 63));
            pl[i] = x;
        }
        __syncthreads();
        for (int32_t i = threadIdx.x; i < nm; i += NT) c.scratch[pl[i] >> 6] = 0ull;
        if (threadIdx.x == 0) {
            c.s->cnt[p] = nm;
            add_bytes(c, 12ull * n + 24ull * nm);
        }
        __syncthreads();
    } else if (st.parent >= 0) {
        // intersect the parent's candidates with the pushed scratch bitmap
        const int p = st.parent;
        uint64_t *pb = c.B(p);
        const int32_t *pl = c.L(p);
        const int32_t n = c.s->cnt[p];
        for (int32_t i = threadIdx.x; i < n; i += NT) {
            const int32_t x = pl[i];
            if (!bit_test(c.scratch, x))
                atomicAnd((unsigned long long *)&pb[x >> 6], ~(1ull << (x & 63)));
        }
        __syncthreads();
        // scratch only holds parent candidates: zero their words
        for (int32_t i = threadIdx.x; i < n; i += NT) c.scratch[pl[i] >> 6] = 0ull;
        if (threadIdx.x == 0) add_bytes(c, 28ull * n);
        __syncthreads();
        compact_list(c, p);
    }
}

// ---------------------------------------------------------------------------
// candidate edges (Sec. "Joining Phase"): for each key (a candidate of the
// key vertex, sorted), the sorted candidates of the other endpoint joined to
// it by a matching data edge. Space per key comes from the data degrees, so
// one pass writes the table: vals[off[i] .. off[i] + num[i]).
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool ec_hit(int32_t rel, const uint64_t *other, const int2 *adj,
                                       int32_t beg, int32_t i, int32_t key) {
    const int2 e = adj[i];
    if (rel >= 0) {
        if (e.y != rel) return false;
    } else if (i > beg && adj[i - 1].x == e.x) {
        return false;  // same neighbour under another relation: one pair
    }
    return e.x != key && bit_test(other, e.x);
}

// first position in row adj[beg, end) (sorted by neighbour id, then
// relation) whose neighbour id is >= x
__device__ __forceinline__ int32_t row_lower_bound(const int2 *adj, int32_t beg, int32_t end,
                                                   int32_t x) {
    while (beg < end) {
        const int32_t mid = beg + ((end - beg) >> 1);
        if (adj[mid].x < x) beg = mid + 1;
        else end = mid;
    }
    return beg;
}

// does the row hold neighbour x under relation rel (-1: any relation)?
__device__ __forceinline__ bool row_has(const int2 *adj, int32_t beg, int32_t end, int32_t x,
                                        int32_t rel) {
    for (int32_t i = row_lower_bound(adj, beg, end, x); i < end && adj[i].x == x; ++i)
        if (rel < 0 || adj[i].y == rel) return true;
    return false;
}

// Looking each of `no` candidates up in a row of `len` entries costs about
// no * log2(len) reads against len for a scan of the row.
__device__ __forceinline__ bool probe_cheaper(int32_t no, int32_t len) {
    return (int64_t)no * (33 - __clz(len | 1)) < (int64_t)len;
}

__device__ __forceinline__ uint64_t probe_bytes(int32_t no, int32_t len) {
    return (uint64_t)no * (4ull + 8ull * (uint64_t)(33 - __clz(len | 1)));
}

// one key, whole workgroup: the other endpoint's sorted candidates that the
// key's row holds, in order (the lookup form of ec_key_wg)
__device__ __forceinline__ int64_t ec_probe_wg(Ctx &c, int32_t rel, const int32_t *ol, int32_t no,
                                               const int2 *adj, int32_t beg, int32_t end, int32_t k,
                                               int32_t *dst) {
    int64_t n = 0;
    for (int32_t base = 0; base < no; base += NT) {
        const int32_t i = base + threadIdx.x;
        const int32_t x = i < no ? ol[i] : -1;
        const bool hit = x >= 0 && x != k && row_has(adj, beg, end, x, rel);
        int64_t tot;
        const int64_t p = n + block_excl_scan(hit ? 1 : 0, c.s->sh, &tot);
        if (hit) dst[p] = x;
        n += tot;
    }
    return n;
}

// one key, one wave (wave-uniform call): lookup form of ec_key_wave
__device__ __forceinline__ int64_t ec_probe_wave(int32_t rel, const int32_t *ol, int32_t no,
                                                 const int2 *adj, int32_t beg, int32_t end,
                                                 int32_t k, int32_t *dst) {
    const int lane = threadIdx.x & 63;
    int64_t n = 0;
    for (int32_t base = 0; base < no; base += 64) {
        const int32_t i = base + lane;
        const int32_t x = i < no ? ol[i] : -1;
        const bool hit = x >= 0 && x != k && row_has(adj, beg, end, x, rel);
        const uint64_t bm = __ballot(hit);
        if (hit) dst[n + __popcll(bm & lanemask_lt(lane))] = x;
        n += __popcll(bm);
    }
    return n;
}

// one key, whole workgroup, ordered compaction in chunks of 4*NT entries
__device__ __forceinline__ int64_t ec_key_wg(Ctx &c, int32_t rel, const uint64_t *ob, const int2 *adj,
                             int32_t beg, int32_t end, int32_t k, int32_t *dst) {
    int64_t n = 0;
    for (int32_t base = beg; base < end; base += 4 * NT) {
        const int32_t i0 = base + 4 * threadIdx.x;
        uint32_t h = 0;  // bit t: entry i0 + t matches
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (i0 + t < end && ec_hit(rel, ob, adj, beg, i0 + t, k)) h |= 1u << t;
        int64_t tot;
        int64_t p = n + block_excl_scan(__popc(h), c.s->sh, &tot);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if ((h >> t) & 1u) dst[p++] = adj[i0 + t].x;
        n += tot;
    }
    return n;
}

// one key, one wave (wave-uniform call), same ordered output as ec_key_wg
__device__ __forceinline__ int64_t ec_key_wave(int32_t rel, const uint64_t *ob, const int2 *adj,
                                               int32_t beg, int32_t end, int32_t k, int32_t *dst) {
    const int lane = threadIdx.x & 63;
    int64_t n = 0;
    for (int32_t base = beg; base < end; base += 256) {
        const int32_t i0 = base + 4 * lane;
        uint32_t h = 0;  // bit t: entry i0 + t matches
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (i0 + t < end && ec_hit(rel, ob, adj, beg, i0 + t, k)) h |= 1u << t;
        const int32_t inc = wave_incl_scan32(__popc(h), lane);
        int64_t p = n + inc - __popc(h);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if ((h >> t) & 1u) dst[p++] = adj[i0 + t].x;
        n += __shfl(inc, 63, 64);
    }
    return n;
}

// Keys [i0, i1) of a table build, G lanes per key; keys whose rows are
// longer than 64 * G entries go to E.ovl (counted by *nbig) for the wave
// tier. Returns the entries this thread's groups wrote (on their first lane).
__device__ __forceinline__ int64_t ec_keys(const Ctx &c, const EcJob &Ej, int32_t i0, int32_t i1,
                                           int G, int32_t *nbig, uint64_t &fb) {
    const EcJob E = Ej;  // once, before the stores below
    const int32_t *off = E.dir ? c.g.in_off : c.g.out_off;
    const int2 *adj = E.dir ? c.g.in_adj : c.g.out_adj;
    const int NGr = NT / G;
    const int lane = threadIdx.x & 63, gl = lane & (G - 1), gb = lane & ~(G - 1);
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << gb;
    const int32_t bigdeg = 64 * G;
    int64_t mytot = 0;
    for (int32_t it = i0 + (int32_t)threadIdx.x / G; it < i1; it += NGr) {
        const int32_t k = E.keys[it];
        const int32_t beg = off[k], end = off[k + 1];
        if (end - beg > bigdeg) {
            if (gl == 0) E.ovl[atomicAdd(nbig, 1)] = it;
            continue;
        }
        int32_t *dst = E.vals + E.degoff[it];
        int32_t n = 0;
        for (int32_t base = beg; base < end; base += G) {
            const int32_t i = base + gl;
            const bool hit = i < end && ec_hit(E.rel, E.ob, adj, beg, i, E.homo ? -1 : k);
            const uint64_t bm = __ballot(hit) & gmask;
            if (hit) dst[n + __popcll(bm & lanemask_lt(lane))] = adj[i].x;
            n += __popcll(bm);
        }
        if (gl == 0) {
            E.num[it] = n;
            mytot += n;
            fb += 16ull + 12ull * (end - beg) + 4ull * n;
        }
    }
    return mytot;
}

// Long keys E.items[i0, i1), one wave each (scan or lookup, whichever
// reads less); keys with rows above wg_rows go to E.ovl for the owner's
// workgroup tier. Returns the entries written (on lane 0 of each wave).
__device__ __forceinline__ int64_t ec_long_keys(const Ctx &c, const EcJob &Ej, int32_t i0,
                                                int32_t i1, int32_t *ngiant, uint64_t &fb) {
    const EcJob E = Ej;
    const int32_t *off = E.dir ? c.g.in_off : c.g.out_off;
    const int2 *adj = E.dir ? c.g.in_adj : c.g.out_adj;
    const int lane = threadIdx.x & 63;
    int64_t mytot = 0;
    for (int32_t b = i0 + (int32_t)(threadIdx.x >> 6); b < i1; b += NW) {
        const int32_t it = E.items[b];
        const int32_t k = E.keys[it];
        const int32_t beg = off[k], end = off[k + 1];
        if (end - beg > c.wg_rows) {
            if (lane == 0) E.ovl[atomicAdd(ngiant, 1)] = it;
            continue;
        }
        const bool probe = probe_cheaper(E.no, end - beg);
        int32_t *dst = E.vals + E.degoff[it];
        const int32_t ks = E.homo ? -1 : k;  // -1: the key may pair with itself
        const int64_t n = probe ? ec_probe_wave(E.rel, E.ol, E.no, adj, beg, end, ks, dst)
                                : ec_key_wave(E.rel, E.ob, adj, beg, end, ks, dst);
        if (lane == 0) {
            E.num[it] = (int32_t)n;
            mytot += n;
            fb += 16ull + 4ull * n + (probe ? probe_bytes(E.no, end - beg) : 12ull * (end - beg));
        }
    }
    return mytot;
}

// Keys with rows above wg_rows, E.items[i0, i1), the whole workgroup each.
// Returns the entries written (on thread 0).
__device__ __forceinline__ int64_t ec_giant_keys(Ctx &c, const EcJob &Ej, int32_t i0, int32_t i1,
                                                 uint64_t &fb) {
    const EcJob E = Ej;
    const int32_t *off = E.dir ? c.g.in_off : c.g.out_off;
    const int2 *adj = E.dir ? c.g.in_adj : c.g.out_adj;
    int64_t mytot = 0;
    for (int32_t b = i0; b < i1; ++b) {
        const int32_t it = E.items[b];
        const int32_t k = E.keys[it];
        const int32_t beg = off[k], end = off[k + 1];
        const bool probe = probe_cheaper(E.no, end - beg);
        int32_t *dst = E.vals + E.degoff[it];
        const int32_t ks = E.homo ? -1 : k;
        const int64_t n = probe ? ec_probe_wg(c, E.rel, E.ol, E.no, adj, beg, end, ks, dst)
                                : ec_key_wg(c, E.rel, E.ob, adj, beg, end, ks, dst);
        if (threadIdx.x == 0) {
            E.num[it] = (int32_t)n;
            mytot += n;
            fb += 16ull + 4ull * n + (probe ? probe_bytes(E.no, end - beg) : 12ull * (end - beg));
        }
    }
    return mytot;
}

// One chunk of a shared table build (owner or helper): the keys, and the
// chunk's entry count added to the board.
__device__ __forceinline__ void ec_chunk(Ctx &c, const EcJob &E, HelpJob *j, int32_t i0, int32_t i1,
                                         int G, uint64_t &fb) {
    int64_t t = E.tier == 2   ? ec_giant_keys(c, E, i0, i1, fb)
                : E.tier == 1 ? ec_long_keys(c, E, i0, i1, &j->nbig, fb)
                              : ec_keys(c, E, i0, i1, G, &j->nbig, fb);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(&j->jrows, (unsigned long long)t);
}

// One shared pass of a table build (nch chunks of K items); adds the
// entries written to mytot (thread 0). False when the owner gave up on its
// helpers: the query is aborted (and rerun) and the build stops, since key
// lists of unreported chunks may be incomplete.
__device__ __forceinline__ bool ec_shared(Ctx &c, int e, const EcJob &E, int32_t n_items,
                                          int32_t K, int G, const int32_t *ovl, uint64_t &fb,
                                          int64_t &mytot) {
    shared_job(c, 3, NStep{}, nullptr, 0, nullptr, nullptr, false, n_items, K, G,
               (n_items + K - 1) / K, nullptr, fb, &E);
    if (aborted(c)) {
        if (threadIdx.x == 0) {
            c.s->ectot[e] = 0;
            c.s->slab_used = (int64_t)((const char *)ovl - c.slab);
        }
        __syncthreads();
        return false;
    }
    if (threadIdx.x == 0)
        mytot += (int64_t)__hip_atomic_load(&c.job->jrows, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return true;
}

// Build the table of query edge e keyed by `key` (dir 0: keys are sources).
// Sets s.ec_offs/ec_cnt/ec_vals[e], s.eckey[e] and s.ectot[e]. Tiers: G
// lanes per key; one wave per key for rows above 64 G entries; the whole
// workgroup per key above wg_rows. With a helper board, each tier with
// enough keys is shared like a filter step (its chunks write disjoint keys
// of the one-pass layout).
__device__ __forceinline__ void ec_build(Ctx &c, int e, int key, int other, int dir) {
    const DevGraph &g = c.g;
    const int32_t *keys = c.L(key);
    const int32_t nk = c.s->cnt[key];
    const uint64_t *ob = c.B(other);
    const int32_t *ol = c.L(other);  // sorted
    const int32_t no = c.s->cnt[other];
    const int32_t rel = c.Q->elabel[e];
    const int32_t *off = dir ? g.in_off : g.out_off;
    const int2 *adj = dir ? g.in_adj : g.out_adj;
    int32_t *degoff = (int32_t *)slab_alloc(c, 4ll * nk + 4);
    int32_t *num = (int32_t *)slab_alloc(c, 4ll * nk + 4);
    if (!degoff || !num) return;
    // exclusive scan of the keys' degrees: space per key
    int64_t carry = 0;
    for (int32_t base = 0; base < nk; base += NT) {
        const int32_t i = base + threadIdx.x;
        const int32_t d = i < nk ? off[keys[i] + 1] - off[keys[i]] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(d, c.s->sh, &tot);
        if (i < nk) degoff[i] = (int32_t)(carry + ex);
        carry += tot;
    }
    int32_t *vals = (int32_t *)slab_alloc(c, 4 * carry + 4);
    if (!vals) return;
    // keys with long rows, for the wave and workgroup tiers; given back
    // to the slab at the end
    int32_t *ovl = (int32_t *)slab_alloc(c, 4ll * nk + 4);
    if (!ovl) return;
    if (threadIdx.x == 0) {
        degoff[nk] = (int32_t)carry;
        c.s->ec_offs[e] = degoff;
        c.s->ec_cnt[e] = num;
        c.s->ec_vals[e] = vals;
        c.s->eckey[e] = key;
        c.s->nbig = 0;
        c.s->ngiant = 0;
    }
    __syncthreads();
    int64_t mytot = 0;
    uint64_t fb = 0;
    const bool can_share = c.help_items > 0 && c.job;
    const int32_t homo = c.Q->homo;
    const EcJob E{keys, degoff, num, vals, ovl, ob, ol, nullptr, nk, rel, dir, no, 0, homo};
    if (nk <= NW) {
        // a handful of keys: one wave each, rows above wg_rows get the
        // whole workgroup
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (wave < nk) {
            const int32_t k = keys[wave];
            const int32_t beg = off[k], end = off[k + 1];
            if (end - beg > c.wg_rows) {
                if (lane == 0) c.s->big[atomicAdd(&c.s->ngiant, 1)] = wave;  // at most NW
            } else {
                const bool probe = probe_cheaper(no, end - beg);
                const int32_t ks = homo ? -1 : k;
                const int64_t n = probe ? ec_probe_wave(rel, ol, no, adj, beg, end, ks, vals + degoff[wave])
                                        : ec_key_wave(rel, ob, adj, beg, end, ks, vals + degoff[wave]);
                if (lane == 0) {
                    num[wave] = (int32_t)n;
                    mytot += n;
                    fb += 16ull + 4ull * n + (probe ? probe_bytes(no, end - beg) : 12ull * (end - beg));
                }
            }
        }
    } else {
        const int lane = threadIdx.x & 63;
        if (can_share && nk >= c.help_items) {
            const int32_t helpers = helpers_now(c);
            const int32_t K = min(512, max(64, max((nk + helpers) / (helpers + 1),
                                                   (nk + kMaxChunks - 1) / kMaxChunks)));
            if (!ec_shared(c, e, E, nk, K, lanes_for(K, c.gmax), ovl, fb, mytot)) return;
        } else {
            mytot += ec_keys(c, E, 0, nk, lanes_for(nk, c.gmax), &c.s->nbig, fb);
        }
        __syncthreads();
        const int32_t nl = c.s->nbig;
        if (can_share && nl >= kLongShare) {
            // many long keys: one wave per key, shared the same way (the
            // keys move to a list of their own; rows longer than wg_rows
            // come back to ovl)
            int32_t *items = (int32_t *)slab_alloc(c, 4ll * nl + 4);
            if (!items) return;
            for (int32_t i = threadIdx.x; i < nl; i += NT) items[i] = ovl[i];
            __syncthreads();
            if (threadIdx.x == 0) c.s->nbig = 0;
            EcJob E1 = E;
            E1.items = items;
            E1.tier = 1;
            if (!ec_shared(c, e, E1, nl, kLongChunk, 64, ovl, fb, mytot)) return;
        }
        __syncthreads();
        const int32_t nbig = c.s->nbig;
        for (int32_t b = threadIdx.x >> 6; b < nbig; b += NW) {
            const int32_t it = ovl[b];
            const int32_t k = keys[it];
            const int32_t beg = off[k], end = off[k + 1];
            if (end - beg > c.wg_rows) {
                int32_t p = 0;
                if (lane == 0) p = atomicAdd(&c.s->ngiant, 1);
                p = __shfl(p, 0, 64);
                if (p < kBigCap) {
                    if (lane == 0) c.s->big[p] = it;
                    continue;
                }
            }
            const bool probe = probe_cheaper(no, end - beg);
            const int32_t ks = homo ? -1 : k;
            const int64_t n = probe ? ec_probe_wave(rel, ol, no, adj, beg, end, ks, vals + degoff[it])
                                    : ec_key_wave(rel, ob, adj, beg, end, ks, vals + degoff[it]);
            if (lane == 0) {
                num[it] = (int32_t)n;
                mytot += n;
                fb += 16ull + 4ull * n + (probe ? probe_bytes(no, end - beg) : 12ull * (end - beg));
            }
        }
    }
    __syncthreads();
    // keys with rows above wg_rows: one workgroup each, shared when several
    const int32_t ngiant = min(c.s->ngiant, kBigCap);
    if (can_share && ngiant >= 2) {
        int32_t *items = (int32_t *)slab_alloc(c, 4ll * ngiant + 4);
        if (!items) return;
        for (int32_t i = threadIdx.x; i < ngiant; i += NT) items[i] = c.s->big[i];
        __syncthreads();
        EcJob E2 = E;
        E2.items = items;
        E2.tier = 2;
        if (!ec_shared(c, e, E2, ngiant, 1, NT, ovl, fb, mytot)) return;
    } else if (ngiant > 0) {
        int32_t *items = c.s->big;
        EcJob E2 = E;
        E2.items = items;
        mytot += ec_giant_keys(c, E2, 0, ngiant, fb);
    }
    add_bytes_wave(c, fb);
    int64_t tot;
    block_excl_scan(mytot, c.s->sh, &tot);
    if (threadIdx.x == 0) {
        c.s->ectot[e] = tot;
        c.s->slab_used = (int64_t)((char *)ovl - c.slab);  // the last allocation
    }
    __syncthreads();
}

// Tables of the edges in `mask` whose key vertex has a single candidate with
// a row of at most wg_rows entries (dir as in ec_build), built together: one
// wave per edge and one slab allocation for all of them, instead of the
// barriers and allocations of a full build per edge. Returns the edges built
// (uniform). Uses the dynamic LDS, which no other phase holds meanwhile.
__device__ __forceinline__ uint64_t ec_build_single(Ctx &c, uint64_t mask, int dir) {
    const DevGraph &g = c.g;
    const NQuery &Q = *c.Q;
    const int32_t *off = dir ? g.in_off : g.out_off;
    const int2 *adj = dir ? g.in_adj : g.out_adj;
    int32_t *dsz = (int32_t *)c.dyn;  // [SGM_MAX_QE] bytes of each table, 0: not here
    int32_t *dk = dsz + SGM_MAX_QE;   // [SGM_MAX_QE] the key's candidate
    int32_t *dpos = dk + SGM_MAX_QE;  // [SGM_MAX_QE] byte offset in the allocation
    int32_t *ql = dpos + SGM_MAX_QE;  // [SGM_MAX_QE] edges built here
    int32_t *meta = ql + SGM_MAX_QE;  // [0] edges, [1] bytes
    const int e = threadIdx.x;
    if (e < Q.m) {
        int32_t sz = 0, k = -1;
        if ((mask >> e) & 1ull) {
            const int key = dir ? Q.edst[e] : Q.esrc[e];
            if (c.s->cnt[key] == 1) {
                k = c.L(key)[0];
                const int32_t deg = off[k + 1] - off[k];
                // offsets [2], count [1], values [deg], rounded to 16 bytes
                if (deg <= c.wg_rows) sz = (4 * (3 + deg) + 15) & ~15;
            }
        }
        dsz[e] = sz;
        dk[e] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t nq = 0, tot = 0;
        for (int i = 0; i < Q.m; ++i)
            if (dsz[i]) {
                dpos[i] = tot;
                tot += dsz[i];
                ql[nq++] = i;
            }
        meta[0] = nq;
        meta[1] = tot;
    }
    __syncthreads();
    const int32_t nq = meta[0];
    if (nq == 0) return 0ull;
    char *base = slab_alloc(c, meta[1]);
    if (!base) return 0ull;
    const int lane = threadIdx.x & 63;
    uint64_t fb = 0;
    for (int i = threadIdx.x >> 6; i < nq; i += NW) {
        const int ed = ql[i];
        const int key = dir ? Q.edst[ed] : Q.esrc[ed];
        const int other = dir ? Q.esrc[ed] : Q.edst[ed];
        const int32_t k = dk[ed];
        const int32_t beg = off[k], end = off[k + 1];
        int32_t *degoff = (int32_t *)(base + dpos[ed]);
        int32_t *num = degoff + 2;
        int32_t *vals = degoff + 3;
        const int32_t no = c.s->cnt[other];
        const int32_t rel = Q.elabel[ed];
        const bool probe = probe_cheaper(no, end - beg);
        const int32_t ks = Q.homo ? -1 : k;
        const int64_t n = probe ? ec_probe_wave(rel, c.L(other), no, adj, beg, end, ks, vals)
                                : ec_key_wave(rel, c.B(other), adj, beg, end, ks, vals);
        if (lane == 0) {
            degoff[0] = 0;
            degoff[1] = end - beg;
            num[0] = (int32_t)n;
            c.s->ec_offs[ed] = degoff;
            c.s->ec_cnt[ed] = num;
            c.s->ec_vals[ed] = vals;
            c.s->eckey[ed] = key;
            c.s->ectot[ed] = n;
            fb += 28ull + 4ull * n + (probe ? probe_bytes(no, end - beg) : 12ull * (end - beg));
        }
    }
    add_bytes_wave(c, fb);
    uint64_t built = 0;
    for (int i = 0; i < nq; ++i) built |= 1ull << ql[i];
    __syncthreads();
    return built;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, (uint64_t)__shfl_xor(x, o, 64));
    return x;
}

// Join order of Sec. "Joining Phase", by wave 0 with one query edge per
// lane: start from the source of the edge with the fewest candidate edges;
// bind one new vertex per level through the cheapest edge with exactly one
// bound endpoint (policy 1: first the new vertex with the most edges to
// bound vertices), the earliest edge on ties; all other unused edges between
// the new vertex and bound vertices are checks of that level.
__device__ __forceinline__ void join_order(Ctx &c) {
    if (threadIdx.x >= 64) return;
    const NQuery &Q = *c.Q;
    Smem &s = *c.s;
    const int lane = threadIdx.x;
    const bool has = lane < Q.m;
    const int xs = has ? s.qsrc[lane] : 0, xd = has ? s.qdst[lane] : 0;
    const uint64_t cost = has ? (uint64_t)min(s.ectot[lane], (int64_t)((1ll << 52) - 1)) : 0ull;
    uint32_t vis = 0;   // bound query vertices
    uint64_t used = 0;  // consumed query edges
    int ext = (int)(wave_min_u64(has ? (cost << 6) | (uint64_t)lane : ~0ull) & 63);
    int w = s.qsrc[ext];
    if (lane == 0) s.jorder[0] = w;
    vis |= 1u << w;
    int nc = 0;
    for (int lv = 0; lv < Q.n - 1; ++lv) {
        const bool va = (vis >> xs) & 1u, vb = (vis >> xd) & 1u;
        if (lv > 0) {
            const bool cand = has && !((used >> lane) & 1ull) && va != vb;
            const int wv = va ? xd : xs;  // the endpoint a candidate would bind
            int links = 0;
            if (c.join_policy == 1)
                for (int x = 0; x < Q.n; ++x) {
                    const uint64_t m = __ballot(cand && wv == x);
                    if (wv == x) links = __popcll(m);
                }
            const uint64_t key =
                cand ? ((uint64_t)(63 - links) << 58) | (cost << 6) | (uint64_t)lane : ~0ull;
            ext = (int)(wave_min_u64(key) & 63);
        }
        w = ((vis >> s.qsrc[ext]) & 1u) ? s.qdst[ext] : s.qsrc[ext];
        used |= 1ull << ext;
        const bool chk = has && !((used >> lane) & 1ull) &&
                         ((xs == w && ((vis >> xd) & 1u)) || (xd == w && ((vis >> xs) & 1u)));
        const uint64_t cm = __ballot(chk);
        if (chk) s.chk[nc + __popcll(cm & lanemask_lt(lane))] = lane;
        if (lane == 0) {
            s.lv_ext[lv] = ext;
            s.lv_first[lv] = nc;
            s.lv_nchk[lv] = __popcll(cm);
            s.jorder[lv + 1] = w;
        }
        nc += __popcll(cm);
        used |= cm;
        vis |= 1u << w;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < Q.n) s.jpos[s.jorder[lane]] = lane;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (has) s.eckey[lane] = s.jpos[xs] < s.jpos[xd] ? xs : xd;
}

__device__ __forceinline__ bool ec_contains(const Ctx &c, int e, int32_t keyval, int32_t x) {
    const int kv = c.s->eckey[e];
    const int32_t *kl = c.L(kv);
    const int32_t i = lower_bound_i32(kl, 0, c.s->cnt[kv], keyval);
    if (i >= c.s->cnt[kv] || kl[i] != keyval) return false;
    const int32_t lo = c.s->ec_offs[e][i], hi = lo + c.s->ec_cnt[e][i];
    const int32_t j = lower_bound_i32(c.s->ec_vals[e], lo, hi, x);
    return j < hi && c.s->ec_vals[e][j] == x;
}

// Shared join levels: a chunk is one block of NT parent rows, or 1/nsub of
// its pairs (every nsub-th block of NT pairs) when the level's pairs are
// few rows with long fan-outs; about kJoinChunkPairs pairs per chunk. A
// level of at least kJoinSharePairs pairs is shared with the launch's idle
// workgroups (those that become idle while it runs join in too).
constexpr int64_t kJoinChunkPairs = 16384;
constexpr int64_t kJoinSharePairs = 2 * kJoinChunkPairs;
constexpr int kJoinMaxSub = 64;
// blocks of pairs whose accepted rows take one output reservation (shared
// levels): up to 4 NT pairs, staged per wave in LDS
constexpr int kJoinGroup = 4;

// Pair i of a block: its row rr within the block of parent rows (the last
// whose pair offset is <= pi), its new value x, and whether the extended
// row passes the injectivity test and every check edge of the level
// (Sec. "Joining Phase").
__device__ __forceinline__ bool join_pair(const Smem &s, const JLevel &L, int64_t r0, int64_t pi,
                                          int32_t *rr_out, int32_t *x_out, uint64_t &jb) {
    int32_t a0 = 0, a1 = NT;
    while (a1 - a0 > 1) {
        const int32_t mid = (a0 + a1) >> 1;
        if (s.pairoff[mid] <= pi) a0 = mid;
        else a1 = mid;
    }
    const int32_t x = L.evals[s.rowlo[a0] + (pi - s.pairoff[a0])];
    const int k = L.k;
    const int32_t *row = L.table + (r0 + a0) * k;
    bool ok = true;
    if (!L.homo)
        for (int cc = 0; cc < k; ++cc)
            if (row[cc] == x) ok = false;
    for (int ci = 0; ci < L.nchk && ok; ++ci) {
        // the check edge's values for the row's key vertex hold x
        const JChk &h = L.chk[ci];
        const int32_t kval = row[h.col];
        const int32_t i = lower_bound_i32(h.kl, 0, h.nkl, kval);
        if (i >= h.nkl || h.kl[i] != kval) {
            ok = false;
        } else {
            const int32_t vlo = h.offs[i], vhi = vlo + h.cnt[i];
            const int32_t jx = lower_bound_i32(h.vals, vlo, vhi, x);
            ok = jx < vhi && h.vals[jx] == x;
        }
    }
    jb += 4ull + 4ull * k + 24ull * L.nchk + (ok ? 4ull * (k + 1) : 0ull);
    *rr_out = a0;
    *x_out = x;
    return ok;
}

// Copy a wave's n staged output rows (parent row within the block, new
// value) to out[base, base + n), consecutive lanes on consecutive ints.
__device__ __forceinline__ void join_put(const JLevel &L, int64_t r0, const int32_t *wrr,
                                         const int32_t *wx, int n, int64_t base, int lane) {
    const int k = L.k, w = k + 1;
    // e / w by a 16-bit reciprocal: exact for e < 4096, w <= 16
    const uint32_t inv = (65536u + (uint32_t)w - 1u) / (uint32_t)w;
    int32_t *dst = L.out + base * w;
    for (int e = lane; e < n * w; e += 64) {
        const int rw = (int)(((uint32_t)e * inv) >> 16);
        const int cc = e - rw * w;
        dst[e] = cc < k ? L.table[(r0 + wrr[rw]) * k + cc] : wx[rw];
    }
}

// Rows [r0, r1) of join level L (at most NT of them): each row's fan-out
// (the candidate-edge count of its parent vertex's value), then its pairs
// in blocks of NT, the accepted rows appended to L.out.
// Owner alone (SHARED false): every block of pairs, output places by one
// LDS atomic per wave. SHARED: the blocks sub, sub + nsub, ... only, and
// the accepted rows of up to kJoinGroup of them take their places with one
// device-scope atomic on *gctr.
template <bool SHARED>
__device__ __forceinline__ void join_rows(Ctx &c, const JLevel &L, int64_t r0, int64_t r1,
                                          int32_t sub, int32_t nsub, unsigned long long *gctr,
                                          int32_t *gabort, uint64_t &jb) {
    Smem &s = *c.s;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t r = r0 + threadIdx.x;
    int32_t fan = 0, lo = 0;
    if (r < r1) {
        const int32_t pv = L.table[r * L.k + L.cp];
        const int32_t i = lower_bound_i32(L.pk, 0, L.npk, pv);
        if (i < L.npk && L.pk[i] == pv) {
            lo = L.eoffs[i];
            fan = L.ecnt[i];
        }
        jb += 16ull + 4ull * (32 - __clz(L.npk | 1));
    }
    int64_t tot;
    const int64_t ex = block_excl_scan(fan, s.sh, &tot);
    if (!SHARED && L.rows <= NT && tot > kPairSlack * L.cap) {
        // the level's only block of rows: its pairs bound the level, so a
        // level that could not fit even a much larger slot stops here
        if (threadIdx.x == 0) {
            s.abort_ = kWhySlab;
            s.need = (int64_t)((const char *)L.out - c.slab) + tot * 4 * (L.k + 1);
        }
        __syncthreads();
        return;
    }
    s.pairoff[threadIdx.x] = (int32_t)ex;
    s.rowlo[threadIdx.x] = lo;
    __syncthreads();
    int32_t *wrr = (int32_t *)c.dyn + wid * 512;  // this wave's staged rows
    int32_t *wx = wrr + 256;
    if (!SHARED) {
        for (int64_t pb = 0; pb < tot; pb += NT) {
            const int64_t pi = pb + threadIdx.x;
            int32_t rr = 0, x = 0;
            const bool ok = pi < tot && join_pair(s, L, r0, pi, &rr, &x, jb);
            const uint64_t bm = __ballot(ok);
            const int nok = __popcll(bm);
            int32_t base = 0;
            const int leader = bm ? __builtin_ctzll(bm) : 0;
            if (bm && lane == leader) base = atomicAdd(&s.ctr, nok);
            base = __shfl(base, leader, 64);
            if (ok) {
                const int j = __popcll(bm & lanemask_lt(lane));
                wrr[j] = rr;
                wx[j] = x;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if ((int64_t)base + nok > L.cap) {
                if (lane == 0) s.abort_ = kWhySlab;
            } else {
                join_put(L, r0, wrr, wx, nok, base, lane);
            }
            __builtin_amdgcn_wave_barrier();
        }
    } else {
        const int64_t nblk = (tot + NT - 1) / NT;
        int par = 0;
        for (int64_t i0 = sub; i0 < nblk; i0 += (int64_t)nsub * kJoinGroup, par ^= 1) {
            int wn = 0;
            for (int t = 0; t < kJoinGroup; ++t) {
                const int64_t bi = i0 + (int64_t)t * nsub;
                if (bi >= nblk) break;
                const int64_t pi = bi * NT + threadIdx.x;
                int32_t rr = 0, x = 0;
                const bool ok = pi < tot && join_pair(s, L, r0, pi, &rr, &x, jb);
                const uint64_t bm = __ballot(ok);
                if (ok) {
                    const int j = wn + __popcll(bm & lanemask_lt(lane));
                    wrr[j] = rr;
                    wx[j] = x;
                }
                wn += __popcll(bm);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // one reservation for the group's accepted rows (two buffers: a
            // wave may run one group ahead)
            if (lane == 0) s.wnok[par][wid] = wn;
            __syncthreads();
            if (threadIdx.x == 0) {
                int32_t t = 0;
                for (int w = 0; w < NW; ++w) t += s.wnok[par][w];
                s.wbase[par] = t ? (int64_t)atomicAdd(gctr, (unsigned long long)t) : 0;
            }
            __syncthreads();
            int64_t base = s.wbase[par];
            for (int w = 0; w < wid; ++w) base += s.wnok[par][w];
            if (base + wn > L.cap) {
                if (lane == 0 && wn) atomicExch(gabort, kWhySlab);
            } else {
                join_put(L, r0, wrr, wx, wn, base, lane);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
}

// Chunk ch of a shared level: its block of parent rows and its share of
// that block's pairs.
__device__ __forceinline__ void join_chunk(Ctx &c, const JLevel &L, int32_t ch,
                                           unsigned long long *gctr, int32_t *gabort,
                                           uint64_t &jb) {
    const int64_t b = ch / L.nsub;
    const int64_t r0 = b * NT;
    join_rows<true>(c, L, r0, min(L.rows, r0 + NT), ch % L.nsub, L.nsub, gctr, gabort, jb);
}

// A join level shared through this slot's board entry (kind 2): the level's
// view goes to the entry, its parent rows are cut into nch chunks that the
// owner and idle workgroups claim, output rows are placed through the
// entry's counter; the owner waits for the chunks its helpers claimed (the
// same protocol as a shared filter step) and takes the row count into
// s.ctr.
__device__ __forceinline__ void shared_join(Ctx &c, int32_t nch, uint64_t &jb) {
    HelpJob *j = c.job;
    Smem &s = *c.s;
    {
        const uint64_t *src = (const uint64_t *)&s.jl;
        uint64_t *dst = (uint64_t *)&j->jl;
        for (int i = threadIdx.x; i < (int)(sizeof(JLevel) / 8); i += NT) dst[i] = src[i];
    }
    if (threadIdx.x == 0) {
        j->jrows = 0ull;
        j->abort_ = 0;
        j->bytes = 0ull;
        j->done = 0;
        j->kind = 2;
        j->chunk = 0;
        j->q = c.q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t seq =
            claim_seq(__hip_atomic_load(&j->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) + 1u;
        // the level's view, tables and edge tables before the claim word
        __threadfence();
        atomicExch(&j->claim, claim_word(seq, nch));
        atomicAdd(&c.hctr[0], 1);
    }
    __syncthreads();
    int32_t own = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned long long w = take_chunk(j);
            s.hch = claim_next(w) < claim_nch(w) ? claim_next(w) : -1;
        }
        __syncthreads();
        const int32_t ch = s.hch;
        __syncthreads();
        if (ch < 0) break;
        join_chunk(c, s.jl, ch, &j->jrows, &j->abort_, jb);
        ++own;
    }
    ev(c, SGM_EV_SHARED);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t got = atomicAdd(&j->done, own) + own;
        int64_t n = 0;
        while (got < nch && n < c.help_wait) {
            __builtin_amdgcn_s_sleep(1);
            got = __hip_atomic_load(&j->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ++n;
        }
        if (got < nch) {
            // give up as a filter step does: no further claims, and the
            // slot stays out of use until the next launch clears it
            const uint32_t seq = claim_seq(
                __hip_atomic_load(&j->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            atomicExch(&j->claim, claim_word(seq, 0));
            atomicExch(&j->dirty, 1);
            s.retired = 1;
        }
        // the helpers' rows, written before their reports
        __threadfence();
        atomicSub(&c.hctr[0], 1);
        const unsigned long long placed =
            __hip_atomic_load(&j->jrows, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s.ctr = (int32_t)min((unsigned long long)s.jl.cap, placed);
        const int32_t ab = __hip_atomic_load(&j->abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ab) s.abort_ = ab;
        if (placed > (unsigned long long)s.jl.cap) s.abort_ = kWhySlab;
        if (got < nch) s.abort_ = kWhyHelp;
        add_bytes(c, __hip_atomic_load(&j->bytes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// final ordering helpers
// ---------------------------------------------------------------------------

// Sort key of a row: the ranks of its values within their (sorted) candidate
// lists, concatenated in query-vertex order (s.bitsn bits each; a column of
// a single candidate has rank 0 and no bits). The binary searches of up to
// eight columns advance together, so their probes are independent loads;
// s.kdepth steps bring every search to its end.
__device__ __forceinline__ uint64_t row_key(const Ctx &c, const int32_t *row) {
    const Smem &s = *c.s;
    const int n = c.Q->n;
    const int depth = s.kdepth;
    uint64_t key = 0;
    for (int u0 = 0; u0 < n; u0 += 8) {
        int32_t x[8], lo[8], len[8];
        const int32_t *lst[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int u = u0 + j;
            const bool on = u < n && s.bitsn[u] > 0;
            lst[j] = on ? s.rkl[u] : nullptr;
            x[j] = on ? row[s.jpos[u]] : 0;
            lo[j] = 0;
            len[j] = on ? s.cnt[u] : 0;
        }
        for (int it = 0; it < depth; ++it) {
            int32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = len[j] > 0 ? lst[j][lo[j] + (len[j] >> 1)] : 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t h = len[j] >> 1;
                if (len[j] > 0 && v[j] < x[j]) {
                    lo[j] += h + 1;
                    len[j] -= h + 1;
                } else {
                    len[j] = h;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int u = u0 + j;
            if (u < n && s.bitsn[u] > 0) key = (key << s.bitsn[u]) | (uint64_t)lo[j];
        }
    }
    return key;
}

// Point rkl[u] at the sorted candidate list of every key column, copying
// the lists into LDS while they fit (binary searches then stay on chip).
__device__ __forceinline__ void stage_key_lists(Ctx &c) {
    int32_t *stage = (int32_t *)(c.dyn + kStageOff);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t used = 0;
        for (int u = 0; u < c.Q->n; ++u) {
            const int32_t m = c.s->cnt[u];
            if (c.s->bitsn[u] > 0 && used + m <= kStageInts) {
                c.s->rkl[u] = stage + used;
                used += m;
            } else {
                c.s->rkl[u] = c.L(u);
            }
        }
    }
    __syncthreads();
    for (int u = 0; u < c.Q->n; ++u) {
        int32_t *dst = const_cast<int32_t *>(c.s->rkl[u]);
        if (dst == c.L(u)) continue;
        const int32_t *src = c.L(u);
        for (int32_t i = threadIdx.x; i < c.s->cnt[u]; i += NT) dst[i] = src[i];
    }
    __syncthreads();
}

// One stable 8-bit LSD pass of the whole workgroup. Wave w owns a contiguous
// segment of the input: per-wave digit counts, one scan in (digit, wave)
// order, then every wave places its segment in order without further
// workgroup barriers (64 elements at a time, ranked within the wave by
// matching digits through ballots; four chunks' loads in flight).
__device__ __forceinline__ void wg_radix_pass(Ctx &c, const uint64_t *kin, const int32_t *iin,
                                              uint64_t *kout, int32_t *iout, int64_t n,
                                              int shift) {
    int32_t *cnt = (int32_t *)c.dyn;  // [NW][256] counts, then running offsets
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t seg = ((n + NW - 1) / NW + 63) & ~(int64_t)63;
    const int64_t lo = min(n, wid * seg), hi = min(n, lo + seg);
    __syncthreads();
    for (int i = threadIdx.x; i < NW * 256; i += NT) cnt[i] = 0;
    __syncthreads();
    for (int64_t i = lo + lane; i < hi; i += 64) atomicAdd(&cnt[wid * 256 + ((kin[i] >> shift) & 255)], 1);
    __syncthreads();
    {
        // digit-major exclusive scan; thread d < 256 owns digit d
        int32_t col[NW];
        int64_t sum = 0;
        if (threadIdx.x < 256)
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                col[w] = cnt[w * 256 + threadIdx.x];
                sum += col[w];
            }
        int64_t tot;
        int64_t run = block_excl_scan(sum, c.s->sh, &tot);
        if (threadIdx.x < 256)
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                cnt[w * 256 + threadIdx.x] = (int32_t)run;
                run += col[w];
            }
    }
    __syncthreads();
    int32_t *mine = cnt + wid * 256;
    for (int64_t b = lo; b < hi; b += 256) {
        uint64_t kv[4];
        int32_t iv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = b + q * 64 + lane;
            kv[q] = i < hi ? kin[i] : 0ull;
            iv[q] = i < hi ? iin[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool valid = b + q * 64 + lane < hi;
            const int d = (int)((kv[q] >> shift) & 255);
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint64_t m = __ballot((d >> t) & 1);
                peers &= ((d >> t) & 1) ? m : ~m;
            }
            const int rk = __popcll(peers & lanemask_lt(lane));
            if (valid) {
                const int64_t p = (int64_t)mine[d] + rk;
                kout[p] = kv[q];
                iout[p] = iv[q];
            }
            // every lane has read its offset before the digit's first lane
            // advances it (one wave, program order)
            if (valid && rk == 0) mine[d] += __popcll(peers);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// one query
// ---------------------------------------------------------------------------

__device__ __forceinline__ void clear_slot(Ctx &c, bool full) {
    __syncthreads();
    const int n = c.Q->n;
    const int32_t nwords = c.g.nwords;
    if (full) {
        for (int u = 0; u < n; ++u)
            for (int32_t w = threadIdx.x; w < nwords; w += NT) c.B(u)[w] = 0ull;
        for (int32_t w = threadIdx.x; w < nwords; w += NT) c.scratch[w] = 0ull;
    } else {
        for (int u = 0; u < n; ++u) {
            const int32_t *l = c.L(u);
            uint64_t *b = c.B(u);
            const int32_t cn = c.s->cnt[u];
            for (int32_t i = threadIdx.x; i < cn; i += NT) b[l[i] >> 6] = 0ull;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void run_query(Ctx &c) {
    const NQuery &Q = *c.Q;
    const DevGraph &g = c.g;
    Smem &s = *c.s;
    const int n = Q.n;
    if (threadIdx.x < SGM_MAX_QV) {
        s.cnt[threadIdx.x] = 0;
        s.cand[threadIdx.x] = 0;
        s.level_rows[threadIdx.x] = 0;
        s.jorder[threadIdx.x] = -1;
    }
    if (threadIdx.x < SGM_MAX_QE) {
        s.ectot[threadIdx.x] = 0;
        s.qsrc[threadIdx.x] = threadIdx.x < Q.m ? (int8_t)Q.esrc[threadIdx.x] : 0;
        s.qdst[threadIdx.x] = threadIdx.x < Q.m ? (int8_t)Q.edst[threadIdx.x] : 0;
    }
    if (threadIdx.x < 5) {
        s.t[threadIdx.x] = 0;
        s.pb[threadIdx.x] = 0ull;
    }
    if (threadIdx.x == 0) {
        s.hostord = 0;
        s.keybits = 0;
        s.tableptr = nullptr;
        s.listptr = nullptr;
        s.abort_ = 0;
        s.slab_used = 0;
        s.empty = 0;
        s.status = SGM_OK;
        s.reason = 0;
        s.nrows = 0;
        s.offset = 0;
        s.need = 0;
        s.bytes = 0;
        if (Q.fault) s.status = kFault;
    }
    if (Q.fault) {
        // a failure injected from the host: this query alone ends with a
        // device error, as a fault confined to it would
        __syncthreads();
        return;
    }
    __syncthreads();
    mark(c, 0);
    ev(c, SGM_EV_START);
    // root candidates
    const int root = Q.root;
    if (Q.root_slot < 0) {
        if (threadIdx.x == 0) {
            const int32_t pin = Q.pred[root].pin;
            if (pin >= 0 && pin < g.V && vpred(g, Q.pred[root], pin)) {
                c.B(root)[pin >> 6] |= 1ull << (pin & 63);
                c.L(root)[0] = pin;
                s.cnt[root] = 1;
            }
        }
        __syncthreads();
    } else {
        list_from_bits(c, root, c.rootbits + (int64_t)Q.root_slot * g.nwords, true);
    }
    ev(c, SGM_EV_ROOT);
    // explore along the spanning tree, then refinement rounds
    for (int i = 0; i < Q.n_init && !aborted(c); ++i) {
        filter_step(c, Q.steps[i]);
        ev(c, SGM_EV_EXPLORE);
    }
    const int rounds = Q.refine_rounds < 0 ? 32 : Q.refine_rounds;
    for (int r = 0; r < rounds && !aborted(c) && Q.n_ref > 0; ++r) {
        int removed = 0;
        for (int i = 0; i < Q.n_ref && !aborted(c); ++i) {
            filter_step(c, Q.steps[Q.n_init + i]);
            ev(c, SGM_EV_REFINE);
            removed += s.removed;  // read after the step's final barrier
            __syncthreads();
        }
        if (Q.refine_rounds < 0 && removed == 0) break;
    }
    __syncthreads();
    mark(c, 1);
    if (aborted(c)) {
        clear_slot(c, true);
        if (threadIdx.x == 0) {
            s.status = kNeedWide;
            s.reason = s.abort_;
        }
        return;
    }
    if (threadIdx.x == 0)
        for (int u = 0; u < n; ++u) {
            s.cand[u] = s.cnt[u];
            if (s.cnt[u] == 0) s.empty = 1;
        }
    __syncthreads();
    int64_t rows = 0;
    int32_t *table = nullptr;
    if (!s.empty) {
        for (int u = 0; u < n && !aborted(c); ++u) sort_list(c, u);
        ev(c, SGM_EV_LISTS);
        if (Q.m == 0) {
            table = c.L(0);
            rows = s.cnt[0];
            if (threadIdx.x == 0) {
                s.jorder[0] = 0;
                s.jpos[0] = 0;
            }
            __syncthreads();
        } else if (!aborted(c)) {
            // candidate edges keyed by each edge's source: totals for the order
            const uint64_t all = Q.m == 64 ? ~0ull : (1ull << Q.m) - 1ull;
            const uint64_t one = ec_build_single(c, all, 0);
            if (one) ev(c, SGM_EV_EDGES);
            for (int e = 0; e < Q.m && !aborted(c); ++e) {
                if ((one >> e) & 1ull) continue;
                ec_build(c, e, Q.esrc[e], Q.edst[e], 0);
                ev(c, SGM_EV_EDGES);
            }
            __syncthreads();
            bool none = false, single = true;
            for (int e = 0; e < Q.m; ++e) none |= s.ectot[e] == 0;
            for (int u = 0; u < n; ++u) single &= s.cnt[u] == 1;
            int32_t *one_row = nullptr;
            if (!aborted(c) && !none && single) one_row = (int32_t *)slab_alloc(c, 4ll * n);
            if (one_row) {
                // One candidate per query vertex and its pair in every edge
                // table: those candidates are the only possible row, and a
                // match exactly when they are distinct. The join binds the
                // vertices in index order.
                mark(c, 2);
                if (threadIdx.x == 0) {
                    int64_t r = 1;
                    for (int u = 0; u < n; ++u) {
                        const int32_t x = c.L(u)[0];
                        if (!Q.homo)
                            for (int w = 0; w < u; ++w) r &= (int64_t)(one_row[w] != x);
                        one_row[u] = x;
                        s.jorder[u] = u;
                        s.jpos[u] = u;
                        s.level_rows[u] = r;
                    }
                    s.nrows = r;
                    add_bytes(c, 8ull * n);
                }
                __syncthreads();
                table = one_row;
                rows = s.nrows;
                ev(c, SGM_EV_LEVEL);
            } else if (!aborted(c) && !none) {
                if (threadIdx.x == 0)
                    for (int e = 0; e < Q.m; ++e) s.ecbuilt[e] = s.eckey[e];
                join_order(c);
                __syncthreads();
                ev(c, SGM_EV_ORDER);
                // edges the join looks up by their destination: rebuild keyed so
                uint64_t redo = 0;
                for (int e = 0; e < Q.m; ++e)
                    if (s.eckey[e] != s.ecbuilt[e]) redo |= 1ull << e;
                const uint64_t one2 = aborted(c) ? 0ull : ec_build_single(c, redo, 1);
                if (one2) ev(c, SGM_EV_EDGES);
                for (int e = 0; e < Q.m && !aborted(c); ++e)
                    if (((redo & ~one2) >> e) & 1ull) {
                        ec_build(c, e, Q.edst[e], Q.esrc[e], 1);
                        ev(c, SGM_EV_EDGES);
                    }
                __syncthreads();
                // join levels
                mark(c, 2);
                table = c.L(s.jorder[0]);
                rows = s.cnt[s.jorder[0]];
                if (threadIdx.x == 0) s.level_rows[0] = rows;
                int k = 1;
                for (int lv = 0; lv < n - 1 && !aborted(c) && rows > 0; ++lv) {
                    const int ext = s.lv_ext[lv];
                    const int p = s.eckey[ext];
                    const int cp = s.jpos[p];
                    const int32_t *pk = c.L(p);
                    const int32_t npk = s.cnt[p];
                    const int32_t *eoffs = s.ec_offs[ext];
                    const int32_t *ecnt = s.ec_cnt[ext];
                    const int32_t *evals = s.ec_vals[ext];
                    const int nchk = s.lv_nchk[lv];
                    const int cfirst = s.lv_first[lv];
                    // output capacity: what is left of the slab
                    __syncthreads();
                    const int64_t used0 = (s.slab_used + 255) & ~(int64_t)255;
                    const int64_t left = c.slab_bytes - used0;
                    int64_t cap = left / (4 * (k + 1));
                    if (cap <= 0) {
                        if (threadIdx.x == 0) s.abort_ = kWhySlab;
                        __syncthreads();
                        break;
                    }
                    if (threadIdx.x == 0) s.ctr = 0;
                    __syncthreads();
                    // the level's pairs bound its rows: a level that could not
                    // fit even a much larger slot stops here rather than
                    // after filling this one
                    int64_t pairs = -1;
                    const bool may_share = c.job && c.help_items > 0;
                    // a block of rows whose pairs could reach a shared or a
                    // host-ordered level (rows times the extension edge's
                    // candidate edges bound them) counts them here too
                    if (rows > NT || rows * s.ectot[ext] >= kJoinSharePairs) {
                        int64_t mp = 0;
                        for (int64_t r = threadIdx.x; r < rows; r += NT) {
                            const int32_t pv = table[r * k + cp];
                            const int32_t i = lower_bound_i32(pk, 0, npk, pv);
                            if (i < npk && pk[i] == pv) mp += ecnt[i];
                        }
                        block_excl_scan(mp, s.sh, &pairs);
                        if (pairs > kPairSlack * cap) {
                            if (threadIdx.x == 0) {
                                s.abort_ = kWhySlab;
                                s.need = used0 + pairs * 4 * (k + 1);
                            }
                            __syncthreads();
                            break;
                        }
                    }
                    // A last level that may reach the size the host orders
                    // goes to the top of the slab (its pairs bound its rows),
                    // with room above for the key columns' candidate lists:
                    // the slot's later queries keep the slab below it.
                    int32_t *out = nullptr;
                    if (lv == n - 2 && c.host_order_rows > 0 && pairs >= c.host_order_rows) {
                        int64_t lint = 0;
                        for (int u = 0; u < n; ++u) lint += s.cnt[u];
                        const int64_t tneed = (pairs * 4 * (k + 1) + 255) & ~(int64_t)255;
                        const int64_t lneed = (4 * lint + 256 * (n + 1)) & ~(int64_t)255;
                        const int64_t at = (c.slab_bytes - tneed - lneed) & ~(int64_t)255;
                        if (at >= kPinFloor(c) && at >= used0) {
                            out = (int32_t *)(c.slab + at);
                            cap = pairs;
                            c.below_top = used0;
                            __syncthreads();
                            if (threadIdx.x == 0) s.slab_used = at + pairs * 4 * (k + 1);
                            __syncthreads();
                        }
                    }
                    if (!out) out = (int32_t *)slab_alloc(c, cap * 4 * (k + 1));
                    if (!out) {
                        if (threadIdx.x == 0) s.abort_ = kWhySlab;
                        __syncthreads();
                        break;
                    }
                    // the level's view (parent column, edge tables of its
                    // extension and check edges, output), the same for the
                    // owner and for helpers
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        JLevel &L = s.jl;
                        L.table = table;
                        L.rows = rows;
                        L.k = k;
                        L.cp = cp;
                        L.pk = pk;
                        L.npk = npk;
                        L.eoffs = eoffs;
                        L.ecnt = ecnt;
                        L.evals = evals;
                        L.nchk = nchk;
                        for (int ci = 0; ci < nchk; ++ci) {
                            const int e = s.chk[cfirst + ci];
                            const int kv = s.eckey[e];
                            L.chk[ci] = JChk{c.L(kv), s.ec_offs[e], s.ec_cnt[e], s.ec_vals[e],
                                             s.cnt[kv], s.jpos[kv]};
                        }
                        L.out = out;
                        L.cap = cap;
                        L.homo = Q.homo;
                    }
                    // a level of many pairs is shared (whether or not
                    // workgroups are idle yet: those that become idle join)
                    const int64_t nrb = (rows + NT - 1) / NT;
                    int64_t nsub = 1;
                    if (may_share && pairs >= kJoinSharePairs)
                        nsub = min((int64_t)kJoinMaxSub,
                                   max((int64_t)1, (pairs + nrb * kJoinChunkPairs - 1) /
                                                       (nrb * kJoinChunkPairs)));
                    const bool share = may_share && pairs >= kJoinSharePairs && nrb * nsub <= kMaxChunks;
                    if (threadIdx.x == 0) s.jl.nsub = (int32_t)nsub;
                    __syncthreads();
                    uint64_t jb = 0;  // algorithmic bytes of this thread's rows and pairs
                    if (share) {
                        shared_join(c, (int32_t)(nrb * nsub), jb);
                    } else {
                        for (int64_t rbase = 0; rbase < rows && !aborted(c); rbase += NT)
                            join_rows<false>(c, s.jl, rbase, min(rows, rbase + NT), 0, 1,
                                             nullptr, nullptr, jb);
                    }
                    add_bytes(c, jb);
                    __syncthreads();
                    rows = s.ctr;
                    if (threadIdx.x == 0) s.level_rows[lv + 1] = rows;
                    // give back the unused part of the table allocation
                    __syncthreads();
                    if (threadIdx.x == 0 && !s.abort_)
                        s.slab_used = (int64_t)((char *)out - c.slab) + rows * 4 * (k + 1);
                    __syncthreads();
                    ev(c, SGM_EV_LEVEL);
                    table = out;
                    ++k;
                }
            } else if (none) {
                rows = 0;
            }
        }
    }
    __syncthreads();
    mark(c, 3);
    if (aborted(c)) {
        clear_slot(c, true);
        if (threadIdx.x == 0) {
            s.status = kNeedWide;
            s.reason = s.abort_;
        }
        return;
    }
    if (threadIdx.x == 0) s.nrows = rows;
    if (rows > 0) {
        // ordering: key = concatenated candidate ranks in column order 0..n-1;
        // a projection (thesis Ch. 3, Sec. "GpSense") keys and keeps only
        // its columns
        __syncthreads();
        if (threadIdx.x == 0) {
            int tb = 0, no = 0, depth = 0;
            for (int u = 0; u < n; ++u) {
                const bool kept = Q.proj == 0u || ((Q.proj >> u) & 1u);
                int b = 0;
                while (kept && (1ll << b) < s.cnt[u]) ++b;
                s.bitsn[u] = b;
                tb += b;
                if (kept) s.ocol[no++] = s.jpos[u];
                // a lower bound over m entries ends after bit_length(m) halvings
                if (b > 0) depth = max(depth, 32 - __clz(s.cnt[u]));
            }
            s.ctr = tb;
            s.nout = no;
            s.kdepth = depth;
        }
        __syncthreads();
        if (s.ctr > 64 && rows > 1) {
            clear_slot(c, false);
            if (threadIdx.x == 0) {
                s.status = kNeedWide;
                s.reason = kWhyKey;
            }
            return;
        }
        const int tb = s.ctr;
        const int k = n;
        const int no = s.nout;
        int32_t *idx;
        const uint64_t *skeys = nullptr;  // the sorted keys (rows > 1)
        // A large final table in the slab, with room below it for the slot's
        // later queries: the key columns' sorted candidate lists go beside
        // it and the host orders it (and collapses a projection) with
        // whole-GPU kernels after the launch; one workgroup would spend
        // milliseconds on the keys, the passes and the gather.
        int64_t toff = (int64_t)((const char *)table - c.slab);
        if (c.host_order_rows > 0 && rows >= c.host_order_rows && toff >= 0 &&
            toff < c.slab_bytes) {
            int64_t lint = 0;
            for (int u = 0; u < n; ++u)
                if (s.bitsn[u] > 0) lint += s.cnt[u];
            int32_t *lst = nullptr;
            const int64_t tbytes = (rows * k * 4 + 255) & ~(int64_t)255;
            const int64_t top = ((c.slab_bytes - 4 * lint) & ~(int64_t)255) - tbytes;
            if (toff >= kPinFloor(c)) {
                lst = (int32_t *)slab_alloc(c, 4 * lint);
            } else if (top >= kPinFloor(c) && top > toff) {
                // too low in the slab to keep for the host: move it up to
                // the top, lists above it; overlapping, so the chunks go
                // from the end (every read of a chunk before its writes)
                int32_t *dst = (int32_t *)(c.slab + top);
                const int64_t nint = rows * k;
                for (int64_t end = nint; end > 0; end -= 4 * NT) {
                    const int64_t beg = end - 4 * NT > 0 ? end - 4 * NT : 0;
                    int32_t v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t i = beg + q * NT + threadIdx.x;
                        v[q] = i < end ? table[i] : 0;
                    }
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t i = beg + q * NT + threadIdx.x;
                        if (i < end) dst[i] = v[q];
                    }
                    __syncthreads();
                }
                if (threadIdx.x == 0) add_bytes(c, 8ull * nint);
                table = dst;
                toff = top;
                lst = (int32_t *)(c.slab + top + tbytes);
            }
            if (lst) {
                int64_t o = 0;
                for (int u = 0; u < n; ++u) {
                    if (s.bitsn[u] == 0) continue;
                    const int32_t *src = c.L(u);
                    for (int32_t i = threadIdx.x; i < s.cnt[u]; i += NT) lst[o + i] = src[i];
                    o += s.cnt[u];
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    s.hostord = 1;
                    s.keybits = tb;
                    s.pin_off = toff;
                    s.tableptr = table;
                    s.listptr = lst;
                    add_bytes(c, 8ull * lint);
                }
                __syncthreads();
                ev(c, SGM_EV_SORT);
                ev(c, SGM_EV_OUTPUT);
                clear_slot(c, false);
                mark(c, 4);
                return;
            }
        }
        if (rows > 1) stage_key_lists(c);
        if (c.below_top >= 0 && rows > kRowSortCap) {
            // the last level sits at the slab's top but stayed on this
            // workgroup: its sort buffers go into the slab below it
            __syncthreads();
            if (threadIdx.x == 0) s.slab_used = c.below_top;
            __syncthreads();
            c.slab_bytes = toff;
        }
        if (rows == 1) {
            int32_t *ix = (int32_t *)c.dyn;
            if (threadIdx.x == 0) ix[0] = 0;
            __syncthreads();
            idx = ix;
        } else if (rows <= kRowSortCap) {
            // bitonic network in LDS
            uint64_t *keys = (uint64_t *)c.dyn;
            int32_t *ix = (int32_t *)(c.dyn + sizeof(uint64_t) * kRowSortCap);
            int32_t N = 1;
            while (N < rows) N <<= 1;
            for (int32_t r = threadIdx.x; r < N; r += NT) {
                keys[r] = r < rows ? row_key(c, table + (int64_t)r * k) : ~0ull;
                ix[r] = r;
            }
            __syncthreads();
            for (int32_t size = 2; size <= N; size <<= 1) {
                for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (int32_t i = threadIdx.x; i < N / 2; i += NT) {
                        const int32_t lo = 2 * i - (i & (stride - 1));
                        const int32_t hi = lo + stride;
                        const bool up = (lo & size) == 0;
                        // ties (a key of all ones against the padding)
                        // by row index, so padding stays last
                        const uint64_t x = keys[lo], y = keys[hi];
                        const bool gt = x > y || (x == y && ix[lo] > ix[hi]);
                        if (gt == up) {
                            keys[lo] = y;
                            keys[hi] = x;
                            const int32_t t = ix[lo];
                            ix[lo] = ix[hi];
                            ix[hi] = t;
                        }
                    }
                    __syncthreads();
                }
            }
            idx = ix;
            skeys = keys;
        } else {
            // LSD radix on (key, row) pairs in the slab, 8 bits per pass
            uint64_t *ka = (uint64_t *)slab_alloc(c, 8 * rows);
            uint64_t *kb = (uint64_t *)slab_alloc(c, 8 * rows);
            int32_t *ia = (int32_t *)slab_alloc(c, 4 * rows);
            int32_t *ib = (int32_t *)slab_alloc(c, 4 * rows);
            if (!ka || !kb || !ia || !ib) {
                clear_slot(c, false);
                if (threadIdx.x == 0) {
                    s.status = kNeedWide;
                    s.reason = kWhySlab;
                }
                return;
            }
            if (threadIdx.x == 0) s.unsorted = 0;
            for (int64_t r = threadIdx.x; r < rows; r += NT) {
                ka[r] = row_key(c, table + r * k);
                ia[r] = (int32_t)r;
            }
            __syncthreads();
            // a join that bound the key columns in key order has left the
            // rows in order already: then no pass is needed
            bool down = false;
            for (int64_t r = threadIdx.x; r + 1 < rows; r += NT) down |= ka[r] > ka[r + 1];
            if (down) s.unsorted = 1;
            __syncthreads();
            if (threadIdx.x == 0) add_bytes(c, 8ull * rows);
            const bool passes = s.unsorted != 0;
            for (int sh = 0; passes && sh < tb; sh += 8) {
                wg_radix_pass(c, ka, ia, kb, ib, rows, sh);
                uint64_t *tk = ka;
                ka = kb;
                kb = tk;
                int32_t *ti = ia;
                ia = ib;
                ib = ti;
            }
            if (threadIdx.x == 0 && passes) add_bytes(c, 24ull * rows * ((tb + 7) / 8));
            idx = ia;
            skeys = ka;
        }
        if (Q.proj && rows > 1) {
            // equal projected rows now have equal, adjacent keys: keep the
            // first row of each run (in-place compaction of the order)
            int64_t kept = 0;
            for (int64_t base = 0; base < rows; base += NT) {
                const int64_t i = base + threadIdx.x;
                const bool head = i < rows && (i == 0 || skeys[i] != skeys[i - 1]);
                const int32_t v = i < rows ? idx[i] : 0;
                int64_t tot;
                const int64_t ex = block_excl_scan((int64_t)(head ? 1 : 0), s.sh, &tot);
                if (head) idx[kept + ex] = v;
                kept += tot;
                __syncthreads();
            }
            if (threadIdx.x == 0) add_bytes(c, 16ull * rows);
            rows = kept;
            if (threadIdx.x == 0) s.nrows = rows;
            __syncthreads();
        }
        ev(c, SGM_EV_SORT);
        if (threadIdx.x == 0) {
            const unsigned long long need = (unsigned long long)rows * no;
            const unsigned long long off = atomicAdd(c.out_used, need);
            s.offset = (off + need <= (unsigned long long)c.out_cap) ? (int64_t)off : -1;
        }
        __syncthreads();
        const int64_t off = s.offset;
        if (off < 0) {
            if (threadIdx.x == 0) s.status = kOutFull;
        } else {
            // one wave per 64 output rows: consecutive lanes write
            // consecutive ints of the rows, columns back in query-vertex
            // order; e / no by a 16-bit reciprocal (exact for e < 64 no,
            // no <= 16)
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
            const uint32_t inv = (65536u + (uint32_t)no - 1u) / (uint32_t)no;
            for (int64_t r0 = (int64_t)wid * 64; r0 < rows; r0 += NT) {
                const int32_t my = r0 + lane < rows ? idx[r0 + lane] : 0;
                const int nr = (int)min((int64_t)64, rows - r0);
                int32_t *dst = c.out + off + r0 * no;
                const int ne = nr * no;
                for (int e0 = 0; e0 < ne; e0 += 256) {
                    // four gathers in flight per lane; every lane takes part
                    // in the shuffles
                    int32_t v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int e = e0 + q * 64 + lane;
                        const int r = min(63, (int)(((uint32_t)e * inv) >> 16));
                        const int32_t src = __shfl(my, r, 64);
                        v[q] = e < ne ? table[(int64_t)src * k + s.ocol[e - r * no]] : 0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (e0 + q * 64 + lane < ne) dst[e0 + q * 64 + lane] = v[q];
                }
            }
            if (threadIdx.x == 0) add_bytes(c, 20ull * rows * no);
        }
    }
    ev(c, SGM_EV_OUTPUT);
    clear_slot(c, false);
    mark(c, 4);
}

// at least 4 waves per SIMD (registers <= 128): two workgroups per CU
// slab_cap: the slot's slab below tables its earlier queries of the launch
// left for the host to order (the whole slab otherwise)
__device__ __forceinline__ Ctx slot_ctx(const NArgs &a, Smem &s, unsigned char *dyn, int slot,
                                        int32_t q, int64_t slab_cap) {
    const int32_t nwords = a.g.nwords;
    uint64_t *bits = a.bits + (int64_t)slot * (SGM_MAX_QV + 1) * nwords;
    int32_t *lists = a.lists + (int64_t)slot * SGM_MAX_QV * a.lcap;
    char *slab = a.slab + (int64_t)slot * a.slab_bytes;
    return Ctx{a.g,  a.lcap, slab_cap, a.out, a.out_cap, a.out_used, a.rootbits, &a.qs[q], &s,
               bits, bits + (int64_t)SGM_MAX_QV * nwords, lists, slab, dyn,
               a.trace ? a.trace + (int64_t)q * SGM_TRACE_CAP : nullptr, a.group_lanes,
               a.wg_rows, a.join_policy,
               // while filtering the slab holds the long-row overflow list in
               // [0, 4 lcap) bytes and the marks in [4 lcap, 8 lcap)
               (int32_t *)(slab + 4 * (int64_t)a.lcap), a.board ? a.board + slot : nullptr, a.hctr,
               a.help_items, q, a.nslot, a.ngrid, a.help_wait, a.host_order_rows, -1};
}

// Chunks of the step posted on board entry e, starting with chunk ch, until
// the step has none left; then the chunks are reported done (one release
// fence for all of them).
__device__ __forceinline__ void help_step(const NArgs &a, Smem &s, unsigned char *dyn, int e,
                                          int32_t ch) {
    HelpJob *j = a.board + e;
    // the parameters stay fixed while this workgroup holds unreported chunks
    const NStep st = j->st;
    const int32_t K = j->chunk, G = j->G, n_items = j->n_items, ncount = j->ncount;
    const bool revd = j->revd != 0;
    const int kind = j->kind;
    const int4 *seg = j->seg;
    const int32_t *hul = j->ul;
    const bool nodefer = j->nodefer != 0;
    if ((int)threadIdx.x < ncount) {
        s.nbl[threadIdx.x].v = j->nbl[threadIdx.x].v;
        s.nbl[threadIdx.x].dir = j->nbl[threadIdx.x].dir;
        s.nbl[threadIdx.x].mode = j->nbl[threadIdx.x].mode;
        s.nbl[threadIdx.x].rel = j->nbl[threadIdx.x].rel;
    }
    if (kind == 2) {
        const uint64_t *src = (const uint64_t *)&j->jl;
        uint64_t *dst = (uint64_t *)&s.jl;
        for (int i = threadIdx.x; i < (int)(sizeof(JLevel) / 8); i += NT) dst[i] = src[i];
    }
    __syncthreads();
    Ctx c = slot_ctx(a, s, dyn, e, j->q, a.slab_bytes);
    c.trace = nullptr;
    uint64_t fb = 0;
    int32_t n = 0;
    while (ch >= 0) {
        if (kind == 0) {
            filter_items(c, BoardCtr{j}, st.push != 0, s.nbl, ncount, hul, c.B(st.u), revd, G,
                         ch * K, min(n_items, ch * K + K), fb, nodefer);
        } else if (kind == 1) {
            push_segment(c, BoardCtr{j}, s.nbl, seg[ch], fb);
        } else if (kind == 3) {
            ec_chunk(c, j->ecj, j, ch * K, min(n_items, ch * K + K), G, fb);
        } else if (kind == 4) {
            item_wg_k(c, BoardCtr{j}, st, s.nbl, ncount, hul[ch], c.B(st.u), fb);
        } else {
            join_chunk(c, s.jl, ch, &j->jrows, &j->abort_, fb);
        }
        ++n;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long w = take_chunk(j);
            s.hch = claim_next(w) < claim_nch(w) ? claim_next(w) : -1;
        }
        __syncthreads();
        ch = s.hch;
        __syncthreads();
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) fb += __shfl_xor(fb, o, 64);
    if ((threadIdx.x & 63) == 0 && fb) atomicAdd(&j->bytes, (unsigned long long)fb);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(&j->done, n);
    }
}

// Helpers: claim chunks of posted steps until every slot workgroup has run
// out of queries (or after kHelpIdle empty polls in a row).
__device__ __forceinline__ void help_loop(const NArgs &a, Smem &s, unsigned char *dyn) {
    const int lane = threadIdx.x & 63;
    int64_t idle = 0;
    for (;;) {
        if (threadIdx.x < 64) {
            int32_t e = -2, ch = -1;  // e: -2 nothing found, -1 leave
            const int32_t done =
                __hip_atomic_load(&a.hctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int32_t posted =
                __hip_atomic_load(&a.hctr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (done >= a.nslot) e = -1;
            else if (posted > 0) {
                // entries with an open chunk, 64 at a time from a rotating start
                for (int base = 0; base < a.nslot && e == -2; base += 64) {
                    const int k = base + lane;
                    const int en = (k + (int)blockIdx.x) % a.nslot;
                    bool open = false;
                    if (k < a.nslot) {
                        const unsigned long long w = __hip_atomic_load(
                            &a.board[en].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        open = claim_next(w) < claim_nch(w);
                    }
                    uint64_t m = __ballot(open);
                    while (m && e == -2) {
                        const int l = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        const int cand = (base + l + (int)blockIdx.x) % a.nslot;
                        int32_t got = -1;
                        if (lane == 0) {
                            const unsigned long long w = take_chunk(a.board + cand);
                            if (claim_next(w) < claim_nch(w)) {
                                got = claim_next(w);
                                // the step's parameters and the owner's data
                                __threadfence();
                            }
                        }
                        got = __shfl(got, 0, 64);
                        if (got >= 0) {
                            e = cand;
                            ch = got;
                        }
                    }
                }
            }
            if (lane == 0) {
                s.hq = e;
                s.hch = ch;
            }
        }
        __syncthreads();
        const int32_t e = s.hq, ch = s.hch;
        __syncthreads();
        if (e == -1) break;
        if (e < 0) {
            if (++idle > kHelpIdle) break;
            // quick polls right after work, slower ones while owners run
            // phases they do not share
            if (idle < 64) __builtin_amdgcn_s_sleep(2);
            else __builtin_amdgcn_s_sleep(32);
            continue;
        }
        idle = 0;
        help_step(a, s, dyn, e, ch);
    }
}

__global__ __launch_bounds__(NT, 4) void k_narrow(NArgs a) {
    __shared__ Smem s;
    extern __shared__ unsigned char dyn[];
    const bool help = a.help_items > 0 && a.board != nullptr;
    if ((int)blockIdx.x >= a.nslot) {
        if (help) help_loop(a, s, dyn);
        return;
    }
    if (threadIdx.x == 0) {
        s.retired = 0;
        s.hq = a.board ? __hip_atomic_load(&a.board[blockIdx.x].dirty, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT)
                       : 0;
    }
    __syncthreads();
    if (s.hq) {
        // an earlier launch left this slot after giving up on a shared step
        // (helpers may have written any of its bitmaps since): clear it all
        uint64_t *bits = a.bits + (int64_t)blockIdx.x * (SGM_MAX_QV + 1) * a.g.nwords;
        const int64_t nb = (int64_t)(SGM_MAX_QV + 1) * a.g.nwords;
        for (int64_t w = threadIdx.x; w < nb; w += NT) bits[w] = 0ull;
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicExch(&a.board[blockIdx.x].dirty, 0);
        }
    }
    int64_t slab_cap = a.slab_bytes;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s.q = atomicAdd(a.queue, 1);
        __syncthreads();
        const int32_t q = s.q;
        if (q >= a.nq) break;
        const NQuery &Q = a.qs[q];
        NResult &R = a.res[q];
        if (s.retired) {
            // the slot is out of use: the query is reported for a rerun
            if (threadIdx.x == 0) {
                R.status = kNeedWide;
                R.reason = kWhyHelp;
                R.n_cols = Q.n;
                R.n_rows = 0;
                R.offset = 0;
                for (int u = 0; u < SGM_MAX_QV; ++u) {
                    R.cand[u] = 0;
                    R.level_rows[u] = 0;
                    R.join_order[u] = -1;
                }
                for (int e = 0; e < SGM_MAX_QE; ++e) R.ec[e] = 0;
                R.bytes = 0;
                R.need = 0;
                for (int i = 0; i < 4; ++i) R.ticks[i] = R.pbytes[i] = 0;
                R.host_order = 0;
            }
            continue;
        }
        Ctx c = slot_ctx(a, s, dyn, blockIdx.x, q, slab_cap);
        if (threadIdx.x == 0) s.nev = 0;
        run_query(c);
        __syncthreads();
        if (s.hostord) slab_cap = s.pin_off;  // keep that table until the launch ends
        if (threadIdx.x == 0) {
            R.status = s.status;
            R.reason = s.reason;
            R.n_cols = Q.n;
            R.n_rows = s.status == SGM_OK ? s.nrows : 0;
            R.offset = s.offset;
            for (int u = 0; u < SGM_MAX_QV; ++u) {
                R.cand[u] = u < Q.n ? s.cand[u] : 0;
                R.level_rows[u] = u < Q.n ? s.level_rows[u] : 0;
                R.join_order[u] = u < Q.n ? s.jorder[u] : -1;
            }
            for (int e = 0; e < SGM_MAX_QE; ++e) R.ec[e] = e < Q.m ? s.ectot[e] : 0;
            R.bytes = (int64_t)s.bytes;
            R.need = s.need;
            R.host_order = s.hostord;
            R.key_bits = s.keybits;
            R.table_ptr = (int64_t)(uintptr_t)s.tableptr;
            R.list_ptr = (int64_t)(uintptr_t)s.listptr;
            // phases a query skipped carry the time and bytes of the
            // previous mark
            int64_t prev = s.t[0];
            unsigned long long pbp = 0ull;
            for (int i = 1; i < 5; ++i) {
                const bool hit = s.t[i] != 0;
                const int64_t ti = hit ? s.t[i] : prev;
                const unsigned long long bi = hit ? s.pb[i] : pbp;
                R.ticks[i - 1] = ti - prev;
                R.pbytes[i - 1] = (int64_t)(bi - pbp);
                prev = ti;
                pbp = bi;
            }
        }
    }
    if (help) {
        if (threadIdx.x == 0) atomicAdd(&a.hctr[1], 1);
        help_loop(a, s, dyn);
    }
}

// ---------------------------------------------------------------------------
// root sweep for a batch: one wave per 64-vertex word, one ballot per
// unpinned root
// ---------------------------------------------------------------------------

// Candidate initialisation for the unpinned roots of a batch (Alg. 3.2
// kernel_check, one sweep for all of them): bitmap row j holds the vertices
// that satisfy root predicate j. Predicates come sorted: the n_any of them
// without a type first, the typed ones by type. A block owns a tile of 64
// bitmap words (4096 vertices, 16 per thread, kept in registers after one
// coalesced read). Per chunk of predicates the tile's rows are built in LDS:
// untyped predicates by ballot, typed ones by each vertex OR-ing its bit
// into the rows of the predicates of its own type only (found by binary
// search), so a vertex is tested against about n_pred / (number of types)
// predicates instead of all of them. Rows then leave as 512-byte runs.
constexpr int kSweepTile = 64;    // bitmap words per block
constexpr int kSweepThreads = 256;                     // 4 waves per block
constexpr int kSweepSlots = kSweepTile / (kSweepThreads / 64);  // words per wave
constexpr int kSweepChunk = 64;   // predicates per LDS pass (32 KB of rows)
// LDS row stride in words. Lanes of one wave OR into the same word of the
// rows of different predicates; an unpadded stride of 512 bytes would put all
// of them in one bank, one more word spreads them over the banks.
constexpr int kSweepStride = kSweepTile + 1;

constexpr int kSweepTypes = 1024;  // type tables up to this size are staged in LDS
constexpr int kSweepGroup = 4;     // slots whose typed predicates are walked together
static_assert(kSweepSlots % kSweepGroup == 0, "slot groups must tile the slots");

__global__ __launch_bounds__(kSweepThreads) void k_root_sweep(DevGraph g, const VPred *preds, int32_t n_pred,
                                                    int32_t n_any, uint64_t *rootbits,
                                                    unsigned long long *ctr,
                                                    const int32_t *type_off, int32_t n_types) {
    if (blockIdx.x == 0 && threadIdx.x < 3) ctr[threadIdx.x] = 0ull;
    if (n_pred == 0) return;
    __shared__ uint64_t rows[kSweepChunk * kSweepStride];
    __shared__ VPred pl[kSweepChunk];
    __shared__ int2 pq[kSweepChunk];  // (qout, qin) of the chunk's predicates
    __shared__ int32_t toff[kSweepTypes + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const bool table = n_types > 0 && n_types <= kSweepTypes;
    if (table)
        for (int t = threadIdx.x; t <= n_types; t += kSweepThreads) toff[t] = type_off[t];
    const int32_t w0 = blockIdx.x * kSweepTile;
    // vertex of slot i: word w0 + kSweepSlots * wid + i, bit lane
    int2 vi[kSweepSlots];
#pragma unroll
    for (int i = 0; i < kSweepSlots; ++i) {
        const int64_t v = (int64_t)(w0 + kSweepSlots * wid + i) * 64 + lane;
        vi[i] = v < g.V ? g.vinfo[v] : make_int2(-1, -1);  // type -1: past the end
    }
    for (int32_t c0 = 0; c0 < n_pred; c0 += kSweepChunk) {
        const int cn = min(kSweepChunk, n_pred - c0);
        for (int i = threadIdx.x; i < cn * kSweepStride; i += kSweepThreads) rows[i] = 0ull;
        if ((int)threadIdx.x < cn) {
            const VPred p = preds[c0 + threadIdx.x];
            pl[threadIdx.x] = p;
            pq[threadIdx.x] = make_int2(p.qout, p.qin);
        }
        __syncthreads();
        // untyped predicates: the same test for every lane; lane i keeps
        // the ballot of slot i and the first kSweepSlots lanes store the
        // wave's words
        for (int j = 0; j < min(n_any - c0, cn); ++j) {
            const int2 q = pq[j];
            uint64_t mine = 0;
#pragma unroll
            for (int i = 0; i < kSweepSlots; ++i) {
                const bool ok = vi[i].x >= 0 && (vi[i].y & 255) >= q.x && (vi[i].y >> 8) >= q.y;
                const uint64_t b = __ballot(ok);
                mine = lane == i ? b : mine;
            }
            if (lane < kSweepSlots) rows[j * kSweepStride + kSweepSlots * wid + lane] = mine;
        }
        // typed predicates of this chunk: [t0, cn), sorted by type
        const int t0 = max(0, n_any - c0);
        if (table) {
            // each vertex's range of predicates of its type, all read
            // before any is used (independent LDS reads), packed lo | hi << 16
            int32_t r[kSweepSlots];
#pragma unroll
            for (int i = 0; i < kSweepSlots; ++i) {
                const int32_t t = vi[i].x;
                const bool ok = t >= 0 && t < n_types && t0 < cn;
                const int32_t tc = ok ? t : 0;
                const int32_t lo = max(t0, toff[tc] - c0), hi = min(cn, toff[tc + 1] - c0);
                r[i] = ok && lo < hi ? (lo | (hi << 16)) : 0;
            }
            // kSweepGroup slots walk their ranges side by side, so that
            // their predicate reads and ORs are independent LDS operations
            // in flight together instead of one dependent chain per slot;
            // a slot whose range has ended reads a clamped, unused entry
#pragma unroll
            for (int i0 = 0; i0 < kSweepSlots; i0 += kSweepGroup) {
                int n = 0;
#pragma unroll
                for (int k = 0; k < kSweepGroup; ++k) n = max(n, (r[i0 + k] >> 16) - (r[i0 + k] & 0xffff));
                for (int t = 0; t < n; ++t) {
#pragma unroll
                    for (int k = 0; k < kSweepGroup; ++k) {
                        const int i = i0 + k;
                        const int j = (r[i] & 0xffff) + t;
                        const int2 q = pq[min(j, kSweepChunk - 1)];
                        if (j < (r[i] >> 16) && (vi[i].y & 255) >= q.x && (vi[i].y >> 8) >= q.y)
                            atomicOr((unsigned long long *)&rows[j * kSweepStride + kSweepSlots * wid + i],
                                     1ull << lane);
                    }
                }
            }
        } else {
            // more types than the table holds: binary search per vertex
#pragma unroll
            for (int i = 0; i < kSweepSlots; ++i) {
                const int32_t t = vi[i].x;
                if (t < 0 || t0 >= cn) continue;
                int lo = t0, hi = cn;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (pl[mid].label < t) lo = mid + 1;
                    else hi = mid;
                }
                const int od = vi[i].y & 255, id = vi[i].y >> 8;
                for (int j = lo; j < cn && pl[j].label == t; ++j)
                    if (od >= pq[j].x && id >= pq[j].y)
                        atomicOr((unsigned long long *)&rows[j * kSweepStride + kSweepSlots * wid + i],
                                 1ull << lane);
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < cn * kSweepTile; k += kSweepThreads) {
            const int j = k / kSweepTile, w = k % kSweepTile;
            if (w0 + w < g.nwords) rootbits[(int64_t)(c0 + j) * g.nwords + w0 + w] = rows[j * kSweepStride + w];
        }
        __syncthreads();
    }
}

}  // namespace

size_t narrow_lds_bytes() { return kDynLds; }

void launch_narrow(hipStream_t s, const NArgs &a, int grid) {
    hipLaunchKernelGGL(k_narrow, dim3(grid), dim3(NT), kDynLds, s, a);
}

namespace {
int sweep_grid(const SweepArgs &a) {
    if (a.n_pred == 0) return 1;
    return std::max(1, (a.g.nwords + kSweepTile - 1) / kSweepTile);
}
}  // namespace

void launch_root_sweep(hipStream_t s, const SweepArgs &a) {
    hipLaunchKernelGGL(k_root_sweep, dim3(sweep_grid(a)), dim3(kSweepThreads), 0, s, a.g, a.preds, a.n_pred,
                       a.n_any, a.rootbits, a.ctr, a.type_off, a.n_types);
}

void narrow_node_params(SweepArgs *sa, NArgs *na, int narrow_grid, void **args,
                        hipKernelNodeParams *sweep, hipKernelNodeParams *narrow) {
    args[0] = &sa->g;
    args[1] = &sa->preds;
    args[2] = &sa->n_pred;
    args[3] = &sa->n_any;
    args[4] = &sa->rootbits;
    args[5] = &sa->ctr;
    args[6] = &sa->type_off;
    args[7] = &sa->n_types;
    args[8] = na;
    *sweep = hipKernelNodeParams{};
    sweep->func = reinterpret_cast<void *>(&k_root_sweep);
    sweep->gridDim = dim3(sweep_grid(*sa));
    sweep->blockDim = dim3(kSweepThreads);
    sweep->sharedMemBytes = 0;
    sweep->kernelParams = args;
    sweep->extra = nullptr;
    *narrow = hipKernelNodeParams{};
    narrow->func = reinterpret_cast<void *>(&k_narrow);
    narrow->gridDim = dim3(narrow_grid);
    narrow->blockDim = dim3(NT);
    narrow->sharedMemBytes = kDynLds;
    narrow->kernelParams = args + 8;
    narrow->extra = nullptr;
}

}  // namespace sgm
