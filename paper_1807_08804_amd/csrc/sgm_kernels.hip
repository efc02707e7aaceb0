// HIP kernels (gfx950, wave64) of the filtering-and-joining subgraph
// matcher, and their launchers. Thesis Ch. 3: Alg. 3.1 (pipeline), Alg. 3.2
// (kernel_check / kernel_collect / kernel_explore), Sec. "Candidate Nodes
// Refinement" (prune-only passes), Sec. "Joining Phase" (candidate edges with
// the two-step output scheme, then combination into full matches).
//
// All arithmetic is integer. Candidate sets are bitmaps of 64-bit words, so a
// wave64 ballot over 64 consecutive vertices yields exactly one word.
#include <hip/hip_runtime.h>

#include "sgm_device.h"
#include "sgm_internal.h"

namespace sgm {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void bit_set_atomic(uint64_t *bits, int32_t x) {
    const uint64_t m = 1ull << (x & 63);
    uint64_t *w = bits + (x >> 6);
    // a plain read first avoids most atomics on already-set bits; a stale
    // read only costs one redundant atomic
    if (!(__atomic_load_n(w, __ATOMIC_RELAXED) & m)) atomicOr((unsigned long long *)w, m);
}

__device__ __forceinline__ bool nbr_ok(const DevGraph &g, const NbrDesc &d, int2 e) {
    if (d.rel >= 0 && e.y != d.rel) return false;
    return d.mode == 0 ? bit_test(d.test_bits, e.x) : vpred(g, d.pred, e.x);
}

// rank of x within a candidate set: number of candidates smaller than x
__device__ __forceinline__ int32_t rank_of(const RankRef &r, int32_t x) {
    const uint64_t w = r.bits[x >> 6];
    return r.prefix[x >> 6] + __popcll(w & ((1ull << (x & 63)) - 1ull));
}

// ---------------------------------------------------------------------------
// kernel_check: candidate initialisation sweep (Alg. 3.2, kernel_check)
// ---------------------------------------------------------------------------

// One wave per 64-vertex word: lane i tests vertex 64w+i, the ballot is the
// bitmap word. Reads type and both degree arrays once (coalesced).
__global__ __launch_bounds__(kBlock) void k_check_sweep(DevGraph g, VPred p, uint64_t *bits) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int w = wave; w < g.nwords; w += nwaves) {
        const int32_t v = w * 64 + lane;
        bool ok = false;
        if (v < g.V) ok = vpred(g, p, v);
        const uint64_t b = __ballot(ok);
        if (lane == 0) bits[w] = b;
    }
}

// Pinned (concept) vertex: at most one candidate.
__global__ void k_check_pin(DevGraph g, VPred p, uint64_t *bits) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && p.pin >= 0 && p.pin < g.V && vpred(g, p, p.pin))
        bits[p.pin >> 6] |= 1ull << (p.pin & 63);
}

// ---------------------------------------------------------------------------
// kernel_collect: bitmap -> ascending candidate list + per-word rank prefix
// (Alg. 3.2, kernel_collect: stream compaction by prefix scan)
// ---------------------------------------------------------------------------

// One workgroup (1024 threads) per bitmap; blockIdx.x selects the bitmap.
// Words are taken 1024 at a time (coalesced); a block scan of the word
// popcounts gives each word's output offset.
__global__ __launch_bounds__(1024) void k_collect(const uint64_t *bits_base, int64_t bits_stride,
                                                  int32_t nwords, int32_t *list_base,
                                                  int64_t list_stride, int32_t *count_base,
                                                  int32_t *prefix_base, int64_t prefix_stride,
                                                  const int32_t *slots) {
    const int slot = slots ? slots[blockIdx.x] : (int)blockIdx.x;
    const uint64_t *bits = bits_base + (int64_t)slot * bits_stride;
    int32_t *list = list_base + (int64_t)slot * list_stride;
    int32_t *prefix = prefix_base + (int64_t)slot * prefix_stride;
    __shared__ int32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int32_t carry = 0;
    for (int32_t base = 0; base < nwords; base += 1024) {
        const int32_t w = base + tid;
        uint64_t word = (w < nwords) ? bits[w] : 0ull;
        const int32_t c = __popcll(word);
        const int32_t inc = wave_incl_scan32(c, lane);
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        int32_t wo = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int32_t s = wsum[i];
            if (i < wid) wo += s;
            tot += s;
        }
        const int32_t excl = carry + wo + inc - c;
        if (w < nwords) {
            prefix[w] = excl;
            int32_t pos = excl;
            while (word) {
                const int b = __builtin_ctzll(word);
                list[pos++] = w * 64 + b;
                word &= word - 1ull;
            }
        }
        carry += tot;
        __syncthreads();
    }
    if (tid == 0) {
        count_base[slot] = carry;
        prefix[nwords] = carry;
    }
}

// ---------------------------------------------------------------------------
// kernel_explore / refinement: prune candidates lacking a neighbour
// candidate for some query edge; explore also pushes matching neighbours
// (Alg. 3.2 kernel_explore; Sec. "Candidate Nodes Refinement").
// ---------------------------------------------------------------------------

// G lanes per candidate (low-degree candidates). Candidates with more than
// kBigDegree entries in a scanned direction go to the big list instead.
template <int G>
__global__ __launch_bounds__(kBlock) void k_filter_small(FilterArgs a) {
    const DevGraph &g = a.g;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int gb = lane & ~(G - 1);
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << gb;
    const int gpb = blockDim.x / G;
    const int32_t n = *a.count;
    for (int32_t it = blockIdx.x * gpb + threadIdx.x / G; it < n; it += gridDim.x * gpb) {
        const int32_t up = a.items[it];
        const int32_t ob = g.out_off[up], oe = g.out_off[up + 1];
        const int32_t ib = g.in_off[up], ie = g.in_off[up + 1];
        bool big = false;
        for (int j = 0; j < a.n_nbr; ++j) {
            const int dir = a.nbr[j].dir;
            if ((dir ? ie - ib : oe - ob) > kBigDegree) big = true;
        }
        if (big) {
            if (gl == 0) {
                const int32_t pos = atomicAdd(a.big_count, 1);
                a.big_items[pos] = up;
            }
            continue;
        }
        bool alive = true;
        for (int j = 0; j < a.n_nbr && alive; ++j) {
            const NbrDesc d = a.nbr[j];
            const int2 *adj = d.dir ? g.in_adj : g.out_adj;
            const int32_t beg = d.dir ? ib : ob, end = d.dir ? ie : oe;
            bool found = false;
            for (int32_t base = beg; base < end; base += G) {
                const int32_t i = base + gl;
                bool hit = false;
                if (i < end) hit = nbr_ok(g, d, adj[i]);
                if (__ballot(hit) & gmask) {
                    found = true;
                    break;
                }
            }
            alive = found;
        }
        if (!alive) {
            if (gl == 0) {
                atomicAnd((unsigned long long *)&a.self_bits[up >> 6], ~(1ull << (up & 63)));
                atomicAdd(a.removed, 1ull);
            }
            continue;
        }
        if (!a.do_push) continue;
        for (int j = 0; j < a.n_nbr; ++j) {
            const NbrDesc d = a.nbr[j];
            if (!d.push) continue;
            const int2 *adj = d.dir ? g.in_adj : g.out_adj;
            const int32_t beg = d.dir ? ib : ob, end = d.dir ? ie : oe;
            for (int32_t i = beg + gl; i < end; i += G) {
                const int2 e = adj[i];
                if (nbr_ok(g, d, e)) bit_set_atomic(d.push_bits, e.x);
            }
        }
    }
}

// One workgroup per high-degree candidate.
__global__ __launch_bounds__(kBlock) void k_filter_big(FilterArgs a) {
    const DevGraph &g = a.g;
    const int32_t n = *a.big_count;
    for (int32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const int32_t up = a.big_items[it];
        const int32_t ob = g.out_off[up], oe = g.out_off[up + 1];
        const int32_t ib = g.in_off[up], ie = g.in_off[up + 1];
        bool alive = true;
        for (int j = 0; j < a.n_nbr && alive; ++j) {
            const NbrDesc d = a.nbr[j];
            const int2 *adj = d.dir ? g.in_adj : g.out_adj;
            const int32_t beg = d.dir ? ib : ob, end = d.dir ? ie : oe;
            bool found = false;
            for (int32_t base = beg; base < end; base += blockDim.x) {
                const int32_t i = base + threadIdx.x;
                bool hit = false;
                if (i < end) hit = nbr_ok(g, d, adj[i]);
                if (__syncthreads_or(hit)) {
                    found = true;
                    break;
                }
            }
            alive = found;
        }
        if (!alive) {
            if (threadIdx.x == 0) {
                atomicAnd((unsigned long long *)&a.self_bits[up >> 6], ~(1ull << (up & 63)));
                atomicAdd(a.removed, 1ull);
            }
            continue;
        }
        if (!a.do_push) continue;
        for (int j = 0; j < a.n_nbr; ++j) {
            const NbrDesc d = a.nbr[j];
            if (!d.push) continue;
            const int2 *adj = d.dir ? g.in_adj : g.out_adj;
            const int32_t beg = d.dir ? ib : ob, end = d.dir ? ie : oe;
            for (int32_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
                const int2 e = adj[i];
                if (nbr_ok(g, d, e)) bit_set_atomic(d.push_bits, e.x);
            }
        }
    }
}

// dst &= src; removed (optional) counts the bits cleared
__global__ __launch_bounds__(kBlock) void k_and(uint64_t *dst, const uint64_t *src, int32_t n,
                                                unsigned long long *removed) {
    unsigned long long cut = 0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t d = dst[i];
        cut += __popcll(d & ~src[i]);
        dst[i] = d & src[i];
    }
    if (removed && cut) atomicAdd(removed, cut);
}

// ---------------------------------------------------------------------------
// collect_edge_candidates: two-step output (count, then write at scanned
// offsets), keyed by the candidates of one endpoint (Sec. "Joining Phase")
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool ec_hit(const ECDesc &d, const int2 *adj, int32_t beg, int32_t i,
                                       int32_t key) {
    const int2 e = adj[i];
    if (d.rel >= 0) {
        if (e.y != d.rel) return false;
    } else if (i > beg && adj[i - 1].x == e.x) {
        return false;  // same neighbour under another relation: one pair
    }
    return (e.x != key || d.homomorphic) && bit_test(d.other_bits, e.x);
}

template <int G, bool WRITE>
__global__ __launch_bounds__(kBlock) void k_ec_small(DevGraph g, ECDesc d) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int gb = lane & ~(G - 1);
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << gb;
    const int gpb = blockDim.x / G;
    const int32_t n = *d.key_count;
    const int32_t *off = d.dir ? g.in_off : g.out_off;
    const int2 *adj = d.dir ? g.in_adj : g.out_adj;
    for (int32_t it = blockIdx.x * gpb + threadIdx.x / G; it < n; it += gridDim.x * gpb) {
        const int32_t key = d.keys[it];
        const int32_t beg = off[key], end = off[key + 1];
        if (end - beg > kBigDegree) {
            if (!WRITE && gl == 0) {
                const int32_t pos = atomicAdd(d.big_count, 1);
                d.big_items[pos] = it;
            }
            continue;
        }
        int32_t c = WRITE ? d.offs[it] : 0;
        for (int32_t base = beg; base < end; base += G) {
            const int32_t i = base + gl;
            const bool hit = i < end && ec_hit(d, adj, beg, i, key);
            const uint64_t b = __ballot(hit) & gmask;
            if (WRITE && hit) d.vals[c + __popcll(b & lanemask_lt(lane))] = adj[i].x;
            c += __popcll(b);
        }
        if (!WRITE && gl == 0) {
            d.cnt[it] = c;
            if (c) atomicAdd(d.total, (unsigned long long)c);
        }
    }
}

template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_ec_big(DevGraph g, ECDesc d) {
    __shared__ int32_t wcnt[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int32_t n = *d.big_count;
    const int32_t *off = d.dir ? g.in_off : g.out_off;
    const int2 *adj = d.dir ? g.in_adj : g.out_adj;
    for (int32_t bi = blockIdx.x; bi < n; bi += gridDim.x) {
        const int32_t it = d.big_items[bi];
        const int32_t key = d.keys[it];
        const int32_t beg = off[key], end = off[key + 1];
        int32_t c = WRITE ? d.offs[it] : 0;
        for (int32_t base = beg; base < end; base += blockDim.x) {
            const int32_t i = base + threadIdx.x;
            const bool hit = i < end && ec_hit(d, adj, beg, i, key);
            const uint64_t b = __ballot(hit);
            if (lane == 0) wcnt[wid] = __popcll(b);
            __syncthreads();
            int32_t wo = 0, tot = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                if (w < wid) wo += wcnt[w];
                tot += wcnt[w];
            }
            if (WRITE && hit) d.vals[c + wo + __popcll(b & lanemask_lt(lane))] = adj[i].x;
            c += tot;
            __syncthreads();
        }
        if (!WRITE && threadIdx.x == 0) {
            d.cnt[it] = c;
            if (c) atomicAdd(d.total, (unsigned long long)c);
        }
    }
}

// Transposition of a source-keyed candidate-edge table (outgoing graph
// only): pair i of key index it gets rank[i] = the rank of its value among
// the destination's candidates and src[i] = keys[it]; cnt[rank] counts the
// pairs of each destination candidate. One wave per key.
__global__ __launch_bounds__(kBlock) void k_ec_pairs(const int32_t *keys, const int32_t *key_count,
                                                     const int32_t *offs, const int32_t *vals,
                                                     RankRef rk, int32_t *rank, int32_t *src,
                                                     int32_t *cnt) {
    const int lane = threadIdx.x & 63;
    const int32_t n = *key_count;
    const int32_t nw = (int32_t)((gridDim.x * blockDim.x) >> 6);
    for (int32_t it = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); it < n; it += nw) {
        const int32_t key = keys[it], end = offs[it + 1];
        for (int32_t i = offs[it] + lane; i < end; i += 64) {
            const int32_t r = rank_of(rk, vals[i]);
            rank[i] = r;
            src[i] = key;
            atomicAdd(&cnt[r], 1);
        }
    }
}

// Exclusive scan of n (device count) int32 values by one workgroup;
// out[n] receives the total.
__global__ __launch_bounds__(1024) void k_scan_i32(const int32_t *in, const int32_t *n_dev,
                                                   int32_t *out) {
    __shared__ int32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int32_t n = *n_dev;
    int32_t carry = 0;
    for (int32_t base = 0; base < n; base += 1024) {
        const int32_t i = base + tid;
        const int32_t c = i < n ? in[i] : 0;
        const int32_t inc = wave_incl_scan32(c, lane);
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        int32_t wo = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int32_t s = wsum[w];
            if (w < wid) wo += s;
            tot += s;
        }
        if (i < n) out[i] = carry + wo + inc - c;
        carry += tot;
        __syncthreads();
    }
    if (tid == 0) out[n] = carry;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int64 (three phases)
// ---------------------------------------------------------------------------

constexpr int kScanItems = 8;
constexpr int64_t kScanTile = (int64_t)kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int64_t *in, int64_t n,
                                                        int64_t *part) {
    __shared__ int64_t sh[kBlock / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single workgroup: in-place exclusive scan of part[0..nb), part[nb] = total
__global__ __launch_bounds__(kBlock) void k_scan_partials(int64_t *part, int64_t nb) {
    __shared__ int64_t sh[kBlock / 64 + 1];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        const int64_t x = i < nb ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(x, sh, &tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const int64_t *in, int64_t n,
                                                      const int64_t *part, int64_t *out) {
    __shared__ int64_t sh[kBlock / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t carry = part[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        const int64_t x = i < n ? in[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(x, sh, &tot);
        if (i < n) out[i] = carry + ex;
        carry += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = part[gridDim.x];
}

// ---------------------------------------------------------------------------
// combine_edge_candidates: join levels (Sec. "Joining Phase")
// ---------------------------------------------------------------------------

// per-row fan-out through the extension edge
__global__ __launch_bounds__(kBlock) void k_join_fan(JoinArgs a, int64_t *fan) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.R;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = a.table[r * a.k + a.ext.col];
        const int32_t i = rank_of(a.ext.rank, v);
        fan[r] = a.ext.offs[i + 1] - a.ext.offs[i];
    }
}

constexpr int kJoinItems = 8;
constexpr int64_t kJoinTile = (int64_t)kBlock * kJoinItems;

// Pair t -> (row, j): the last row whose pair offset is <= t.
__device__ __forceinline__ int64_t pair_row(const int64_t *pair_off, int64_t R, int64_t t) {
    int64_t lo = 0, hi = R;  // answer in [0, R)
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pair_off[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Validity of pair t; on success *w = the new vertex's data vertex and *row
// the parent row index.
__device__ __forceinline__ bool join_pair(const JoinArgs &a, int64_t t, int32_t *w,
                                          int64_t *row) {
    const int64_t r = pair_row(a.pair_off, a.R, t);
    const int64_t j = t - a.pair_off[r];
    const int32_t *rp = a.table + r * a.k;
    const int32_t pv = rp[a.ext.col];
    const int32_t pi = rank_of(a.ext.rank, pv);
    const int32_t x = a.ext.vals[a.ext.offs[pi] + j];
    if (!a.homomorphic)
        for (int c = 0; c < a.k; ++c)
            if (rp[c] == x) return false;  // injectivity
    for (int e = 0; e < a.n_chk; ++e) {
        const JoinEdge &ce = a.chk[e];
        const int32_t bi = rank_of(ce.rank, rp[ce.col]);
        const int32_t lo = ce.offs[bi], hi = ce.offs[bi + 1];
        if (lo >= hi) return false;
        int32_t l = lo, h = hi;
        while (l < h) {
            const int32_t mid = (l + h) >> 1;
            if (ce.vals[mid] < x) l = mid + 1;
            else h = mid;
        }
        if (l >= hi || ce.vals[l] != x) return false;
    }
    *w = x;
    *row = r;
    return true;
}

__global__ __launch_bounds__(kBlock) void k_join_count(JoinArgs a) {
    __shared__ int32_t sh[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t base = a.p0 + (int64_t)blockIdx.x * kJoinTile;
    int32_t cnt = 0;
    for (int k = 0; k < kJoinItems; ++k) {
        const int64_t t = base + (int64_t)k * kBlock + threadIdx.x;
        int32_t w;
        int64_t r;
        if (t < a.P && join_pair(a, t, &w, &r)) ++cnt;
    }
    const int32_t inc = wave_incl_scan32(cnt, lane);
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
        a.block_cnt[blockIdx.x] = s;
    }
}

// Write pass: tile rounds in pair order, block-local ordered compaction.
__global__ __launch_bounds__(kBlock) void k_join_write(JoinArgs a) {
    __shared__ int32_t sh[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t base = a.p0 + (int64_t)blockIdx.x * kJoinTile;
    int64_t pos = a.out_base + a.block_cnt[blockIdx.x];
    const int k1 = a.k + 1;
    for (int k = 0; k < kJoinItems; ++k) {
        const int64_t t = base + (int64_t)k * kBlock + threadIdx.x;
        int32_t w = 0;
        int64_t r = 0;
        const bool ok = t < a.P && join_pair(a, t, &w, &r);
        const uint64_t b = __ballot(ok);
        if (lane == 0) sh[wid] = __popcll(b);
        __syncthreads();
        int32_t wo = 0, tot = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            if (i < wid) wo += sh[i];
            tot += sh[i];
        }
        if (ok) {
            const int64_t o = pos + wo + __popcll(b & lanemask_lt(lane));
            int32_t *dst = a.out + o * k1;
            const int32_t *src = a.table + r * a.k;
            for (int c = 0; c < a.k; ++c) dst[c] = src[c];
            dst[a.k] = w;
        }
        pos += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_keys_to_table(const int32_t *keys, int64_t n,
                                                          int32_t *table) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        table[i] = keys[i];
}

// ---------------------------------------------------------------------------
// final ordering: rows ascending in query-vertex column order
// ---------------------------------------------------------------------------

struct ColPos {
    int32_t c[SGM_MAX_QV];
};

__global__ __launch_bounds__(kBlock) void k_iota(int32_t *idx, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        idx[i] = (int32_t)i;
}

__device__ __forceinline__ bool row_less(const int32_t *t, int32_t k, const ColPos &cp, int32_t n,
                                         int32_t a, int32_t b) {
    if (b < 0) return a >= 0;  // padding sorts last
    if (a < 0) return false;
    const int32_t *ra = t + (int64_t)a * k, *rb = t + (int64_t)b * k;
    for (int c = 0; c < n; ++c) {
        const int32_t x = ra[cp.c[c]], y = rb[cp.c[c]];
        if (x != y) return x < y;
    }
    return false;
}

constexpr int kSmallSort = 4096;

// Bitonic sort of up to kSmallSort row indices in one workgroup.
__global__ __launch_bounds__(1024) void k_sort_small(const int32_t *table, int32_t k, ColPos cp,
                                                     int32_t ncols, int32_t n, int32_t *idx) {
    __shared__ int32_t s[kSmallSort];
    int32_t N = 1;
    while (N < n) N <<= 1;
    for (int i = threadIdx.x; i < N; i += blockDim.x) s[i] = i < n ? i : -1;
    __syncthreads();
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < N / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t x = s[lo], y = s[hi];
                const bool swap = up ? row_less(table, k, cp, ncols, y, x)
                                     : row_less(table, k, cp, ncols, x, y);
                if (swap) {
                    s[lo] = y;
                    s[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) idx[i] = s[i];
}

// Radix sort on (key, index) pairs: 8-bit digits, stable.
constexpr int kRadixItems = 8;
constexpr int64_t kRadixTile = (int64_t)kBlock * kRadixItems;

__global__ __launch_bounds__(kBlock) void k_gather_key(const int32_t *table, int32_t k, int32_t col,
                                                       const int32_t *idx, int64_t n,
                                                       int32_t *key) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        key[i] = table[(int64_t)idx[i] * k + col];
}

__global__ __launch_bounds__(kBlock) void k_row_keys(const int32_t *table, int32_t k, KeyCols kc,
                                                     int64_t n, uint64_t *keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t *row = table + i * k;
        uint64_t key = 0;
        for (int u = 0; u < kc.n; ++u) {
            const int b = kc.nbits[u];
            if (b == 0) continue;
            const int32_t x = row[kc.col[u]];
            const uint64_t w = kc.bits[u][x >> 6];
            const int32_t rk = kc.prefix[u][x >> 6] + __popcll(w & ((1ull << (x & 63)) - 1ull));
            key = (key << b) | (uint64_t)rk;
        }
        keys[i] = key;
    }
}

__global__ __launch_bounds__(kBlock) void k_key_half(const uint64_t *keys, const int32_t *idx,
                                                     int64_t n, int hi, int32_t *key) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        key[i] = (int32_t)(uint32_t)(keys[idx[i]] >> (hi ? 32 : 0));
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const int32_t *key, int64_t n, int shift,
                                                       int64_t *hist /* [256][nblocks] */) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const int32_t *key_in,
                                                          const int32_t *idx_in, int64_t n,
                                                          int shift, const int64_t *off,
                                                          int32_t *key_out, int32_t *idx_out) {
    __shared__ int64_t base_d[256];
    __shared__ int32_t wc[kBlock / 64][256];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    base_d[threadIdx.x] = off[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    const int64_t tb = (int64_t)blockIdx.x * kRadixTile;
    for (int k = 0; k < kRadixItems; ++k) {
        for (int w = 0; w < kBlock / 64; ++w) wc[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t i = tb + (int64_t)k * kBlock + threadIdx.x;
        const bool valid = i < n;
        const int32_t kv = valid ? key_in[i] : 0;
        const int d = (kv >> shift) & 255;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const int rk = __popcll(peers & lanemask_lt(lane));
        if (valid && rk == 0) wc[wid][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t p = base_d[d] + rk;
            for (int w = 0; w < wid; ++w) p += wc[w][d];
            key_out[p] = kv;
            idx_out[p] = idx_in[i];
        }
        __syncthreads();
        int64_t add = 0;
        for (int w = 0; w < kBlock / 64; ++w) add += wc[w][threadIdx.x];
        base_d[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_gather_rows(const int32_t *table, int32_t k,
                                                        const int32_t *idx, int64_t n, ColPos cp,
                                                        int32_t ncols, int32_t *out) {
    const int64_t total = n * ncols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / ncols;
        const int c = (int)(t - i * ncols);
        const int32_t r = idx ? idx[i] : (int32_t)i;
        out[t] = table[(int64_t)r * k + cp.c[c]];
    }
}

// Projection (thesis Ch. 3, Sec. "GpSense"): in a table of projected rows
// sorted lexicographically, equal rows are adjacent; head[i] = 1 for the
// first row of each run of equal rows.
__global__ __launch_bounds__(kBlock) void k_row_heads(const int32_t *rows, int32_t k, int64_t n,
                                                      int64_t *head) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t h = 1;
        if (i > 0) {
            h = 0;
            for (int c = 0; c < k; ++c)
                if (rows[i * k + c] != rows[(i - 1) * k + c]) h = 1;
        }
        head[i] = h;
    }
}

// The head rows in order: row i goes to out[pos[i]] (pos = exclusive scan
// of head).
__global__ __launch_bounds__(kBlock) void k_compact_rows(const int32_t *rows, int32_t k, int64_t n,
                                                         const int64_t *head, const int64_t *pos,
                                                         int32_t *out) {
    const int64_t total = n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k;
        if (head[i]) out[pos[i] * k + (t - i * k)] = rows[t];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

constexpr int kGridCap = 256 * 16;  // 16 workgroups per CU on 256 CUs

void launch_check_sweep(hipStream_t s, const DevGraph &g, VPred p, uint64_t *bits) {
    const int grid = grid_for(g.nwords, kBlock / 64, kGridCap);
    hipLaunchKernelGGL(k_check_sweep, dim3(grid), dim3(kBlock), 0, s, g, p, bits);
}

void launch_check_pin(hipStream_t s, const DevGraph &g, VPred p, uint64_t *bits) {
    hipLaunchKernelGGL(k_check_pin, dim3(1), dim3(64), 0, s, g, p, bits);
}

void launch_collect_multi(hipStream_t s, const DevGraph &g, const uint64_t *bits_base,
                          int64_t bits_stride, int32_t *list_base, int64_t list_stride,
                          int32_t *count_base, int32_t *prefix_base, int64_t prefix_stride,
                          const int32_t *slots, int nslots) {
    hipLaunchKernelGGL(k_collect, dim3(nslots), dim3(1024), 0, s, bits_base, bits_stride, g.nwords,
                       list_base, list_stride, count_base, prefix_base, prefix_stride, slots);
}

void launch_filter(hipStream_t s, const FilterArgs &a, int grid_small, int grid_big) {
    hipLaunchKernelGGL(k_filter_small<16>, dim3(grid_small), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_filter_big, dim3(grid_big), dim3(kBlock), 0, s, a);
}

void launch_and(hipStream_t s, uint64_t *dst, const uint64_t *src, int32_t nwords,
                unsigned long long *removed) {
    hipLaunchKernelGGL(k_and, dim3(grid_for(nwords, kBlock, kGridCap)), dim3(kBlock), 0, s, dst,
                       src, nwords, removed);
}

void launch_ec_count(hipStream_t s, const DevGraph &g, const ECDesc &d, int grid_small,
                     int grid_big) {
    hipLaunchKernelGGL((k_ec_small<16, false>), dim3(grid_small), dim3(kBlock), 0, s, g, d);
    hipLaunchKernelGGL((k_ec_big<false>), dim3(grid_big), dim3(kBlock), 0, s, g, d);
}

void launch_ec_write(hipStream_t s, const DevGraph &g, const ECDesc &d, int grid_small,
                     int grid_big) {
    hipLaunchKernelGGL((k_ec_small<16, true>), dim3(grid_small), dim3(kBlock), 0, s, g, d);
    hipLaunchKernelGGL((k_ec_big<true>), dim3(grid_big), dim3(kBlock), 0, s, g, d);
}

void launch_scan_i32(hipStream_t s, const int32_t *in, const int32_t *n, int32_t *out) {
    hipLaunchKernelGGL(k_scan_i32, dim3(1), dim3(1024), 0, s, in, n, out);
}

int64_t scan_tmp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_scan_i64(hipStream_t s, const int64_t *in, int64_t n, int64_t *out, int64_t *tmp) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {  // empty input: out[0] = 0
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, out, (int64_t)0);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, tmp, out);
}

// ---------------------------------------------------------------------------
// expansion of weighted matches into the original graph's matches
// ---------------------------------------------------------------------------

// does g hold the edge s -> t with relation rel (-1: any)? (out-rows are
// sorted by (neighbour, relation))
__device__ __forceinline__ bool has_edge(const DevGraph &g, int32_t s, int32_t t, int32_t rel) {
    int32_t lo = g.out_off[s], hi = g.out_off[s + 1];
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (g.out_adj[mid].x < t) lo = mid + 1;
        else hi = mid;
    }
    for (int32_t i = lo; i < g.out_off[s + 1]; ++i) {
        const int2 e = g.out_adj[i];
        if (e.x != t) return false;
        if (rel < 0 || e.y == rel) return true;
    }
    return false;
}

// One thread per weighted match: a depth-first walk over the members of the
// mapping lists in the query's order; the count pass counts the matches,
// the write pass writes them at the match's offset, in walk order.
template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_expand(ExpandArgs a) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.nw;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t *wr = a.wrows + r * a.n;
        int32_t x[SGM_MAX_QV];    // chosen member per query vertex
        int32_t pos[SGM_MAX_QV];  // next list position per depth
        int64_t c = 0;
        const int64_t o = WRITE ? a.offs[r] : 0;
        int d = 0;
        pos[0] = a.map_off[wr[a.order[0]]];
        while (d >= 0) {
            const int u = a.order[d];
            const int32_t end = a.map_off[wr[u] + 1];
            bool placed = false;
            while (pos[d] < end && !placed) {
                const int32_t m = a.map_ids[pos[d]++];
                bool ok = a.pin[u] < 0 || m == a.pin[u];
                for (int i = 0; i < d && ok; ++i) ok = x[a.order[i]] != m;
                for (int e = a.eb[d]; e < a.eb[d + 1] && ok; ++e) {
                    const int32_t s = a.es[e] == u ? m : x[a.es[e]];
                    const int32_t t = a.ed[e] == u ? m : x[a.ed[e]];
                    ok = has_edge(a.g, s, t, a.el[e]);
                }
                if (ok) {
                    x[u] = m;
                    placed = true;
                }
            }
            if (!placed) {
                --d;
            } else if (d == a.n - 1) {
                if (WRITE)
                    for (int v = 0; v < a.n; ++v) a.out[(o + c) * a.n + v] = x[v];
                ++c;
            } else {
                ++d;
                pos[d] = a.map_off[wr[a.order[d]]];
            }
        }
        if (!WRITE) a.cnt[r] = c;
    }
}

void launch_expand_count(hipStream_t s, const ExpandArgs &a) {
    hipLaunchKernelGGL(k_expand<false>, dim3(grid_for(a.nw, kBlock, kGridCap)), dim3(kBlock), 0, s, a);
}

void launch_expand_write(hipStream_t s, const ExpandArgs &a) {
    hipLaunchKernelGGL(k_expand<true>, dim3(grid_for(a.nw, kBlock, kGridCap)), dim3(kBlock), 0, s, a);
}

void launch_join_fan(hipStream_t s, const JoinArgs &a, int64_t *fan) {
    hipLaunchKernelGGL(k_join_fan, dim3(grid_for(a.R, kBlock, kGridCap)), dim3(kBlock), 0, s, a,
                       fan);
}

int64_t join_tiles(int64_t P) { return (P + kJoinTile - 1) / kJoinTile; }

void launch_join_count(hipStream_t s, const JoinArgs &a) {
    const int64_t nb = join_tiles(a.P - a.p0);
    if (nb) hipLaunchKernelGGL(k_join_count, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
}

void launch_join_write(hipStream_t s, const JoinArgs &a) {
    const int64_t nb = join_tiles(a.P - a.p0);
    if (nb) hipLaunchKernelGGL(k_join_write, dim3((unsigned)nb), dim3(kBlock), 0, s, a);
}

void launch_keys_to_table(hipStream_t s, const int32_t *keys, const int32_t *, int64_t n,
                          int32_t *table) {
    hipLaunchKernelGGL(k_keys_to_table, dim3(grid_for(n, kBlock, kGridCap)), dim3(kBlock), 0, s,
                       keys, n, table);
}

void launch_iota(hipStream_t s, int32_t *idx, int64_t n) {
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kBlock, kGridCap)), dim3(kBlock), 0, s, idx, n);
}

void launch_sort_small(hipStream_t s, const int32_t *table, int32_t k, const int32_t *colpos,
                       int32_t ncols, int32_t n, int32_t *idx) {
    ColPos cp{};
    for (int c = 0; c < SGM_MAX_QV; ++c) cp.c[c] = c < ncols ? colpos[c] : 0;
    hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(1024), 0, s, table, k, cp, ncols, n, idx);
}

int64_t small_sort_limit() { return kSmallSort; }

int64_t radix_tiles(int64_t n) { return (n + kRadixTile - 1) / kRadixTile; }

void launch_ec_pairs(hipStream_t s, const int32_t *keys, const int32_t *key_count, int64_t n_keys,
                     const int32_t *offs, const int32_t *vals, RankRef rk, int32_t *rank,
                     int32_t *src, int32_t *cnt) {
    hipLaunchKernelGGL(k_ec_pairs, dim3(grid_for(n_keys * 64, kBlock, kGridCap)), dim3(kBlock), 0,
                       s, keys, key_count, offs, vals, rk, rank, src, cnt);
}

void launch_gather_key(hipStream_t s, const int32_t *table, int32_t k, int32_t col,
                       const int32_t *idx, int64_t n, int32_t *key) {
    hipLaunchKernelGGL(k_gather_key, dim3(grid_for(n, kBlock, kGridCap)), dim3(kBlock), 0, s,
                       table, k, col, idx, n, key);
}

// Ordering keys from the key columns' sorted candidate lists: the rank of
// each key column's value (binary search in its list), nbits[c] bits per
// column, the first column highest. One thread per row.
__global__ __launch_bounds__(kBlock) void k_row_keys_lists(const int32_t *table, int32_t k,
                                                           ListKeys lk, int64_t n,
                                                           uint64_t *keys) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t *row = table + r * k;
        uint64_t key = 0;
        for (int c = 0; c < lk.n; ++c) {
            const int32_t rk = lower_bound_i32(lk.list + lk.off[c], 0, lk.cnt[c], row[lk.col[c]]);
            key = (key << lk.nbits[c]) | (uint64_t)rk;
        }
        keys[r] = key;
    }
}

void launch_row_keys_lists(hipStream_t s, const int32_t *table, int32_t k, const ListKeys &lk,
                           int64_t n, uint64_t *keys) {
    hipLaunchKernelGGL(k_row_keys_lists, dim3(grid_for(n, kBlock, kGridCap)), dim3(kBlock), 0, s,
                       table, k, lk, n, keys);
}

void launch_row_keys(hipStream_t s, const int32_t *table, int32_t k, const KeyCols &kc, int64_t n,
                     uint64_t *keys) {
    hipLaunchKernelGGL(k_row_keys, dim3(grid_for(n, kBlock, kGridCap)), dim3(kBlock), 0, s, table,
                       k, kc, n, keys);
}

void launch_key_half(hipStream_t s, const uint64_t *keys, const int32_t *idx, int64_t n, int hi,
                     int32_t *key) {
    hipLaunchKernelGGL(k_key_half, dim3(grid_for(n, kBlock, kGridCap)), dim3(kBlock), 0, s, keys,
                       idx, n, hi, key);
}

void launch_radix_hist(hipStream_t s, const int32_t *key, int64_t n, int shift, int64_t *hist) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)radix_tiles(n)), dim3(kBlock), 0, s, key, n,
                       shift, hist);
}

void launch_radix_scatter(hipStream_t s, const int32_t *key_in, const int32_t *idx_in, int64_t n,
                          int shift, const int64_t *off, int32_t *key_out, int32_t *idx_out) {
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)radix_tiles(n)), dim3(kBlock), 0, s, key_in,
                       idx_in, n, shift, off, key_out, idx_out);
}

void launch_gather_rows(hipStream_t s, const int32_t *table, int32_t k, const int32_t *idx,
                        int64_t n, const int32_t *colpos, int32_t ncols, int32_t *out) {
    ColPos cp{};
    for (int c = 0; c < SGM_MAX_QV; ++c) cp.c[c] = c < ncols ? colpos[c] : 0;
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(n * ncols, kBlock, kGridCap)), dim3(kBlock), 0,
                       s, table, k, idx, n, cp, ncols, out);
}

void launch_unique_rows(hipStream_t s, const int32_t *rows, int32_t k, int64_t n, int64_t *head,
                        int64_t *pos, int64_t *tmp, int32_t *out) {
    hipLaunchKernelGGL(k_row_heads, dim3(grid_for(n, kBlock, kGridCap)), dim3(kBlock), 0, s, rows,
                       k, n, head);
    launch_scan_i64(s, head, n, pos, tmp);
    hipLaunchKernelGGL(k_compact_rows, dim3(grid_for(n * k, kBlock, kGridCap)), dim3(kBlock), 0, s,
                       rows, k, n, head, pos, out);
}

}  // namespace sgm
