// C ABI of the sgm library: graph residency, per-query orchestration of the
// filtering-and-joining pipeline (thesis Alg. 3.1), batching, statistics.
// Every step of a match runs in the HIP kernels of sgm_kernels.hip; this file
// only validates, plans, sizes buffers and launches.
#include <hip/hip_runtime.h>

#include <sys/mman.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <deque>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "sgm_internal.h"
#include "sgm_narrow.h"
#include "sgm_plan.h"

using namespace sgm;

namespace {

thread_local std::string g_last_error;

int scratch_setup(int device);

void set_error(const char *what, hipError_t e) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_last_error = buf;
}

struct DeviceError {
    int code;
};

#define HIPX(call)                                         \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) {                            \
            set_error(#call, e_);                          \
            throw DeviceError{SGM_EDEVICE};                \
        }                                                  \
    } while (0)

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Caching device allocator: buffers return to size-keyed free lists and are
// reused by later work on the same stream (stream order makes reuse safe).
class DevPool {
   public:
    void *get(size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= 2 * bytes + (1u << 20)) {
            void *p = it->second;
            free_.erase(it);
            live_ += size_[p];
            return p;
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            // drop cached blocks and retry once
            (void)hipGetLastError();
            trim();
            e = hipMalloc(&p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                g_last_error = "device allocation failed";
                throw DeviceError{SGM_ENOMEM};
            }
        }
        size_[p] = bytes;
        live_ += bytes;
        return p;
    }
    void put(void *p) {
        if (!p) return;
        auto it = size_.find(p);
        if (it == size_.end()) return;
        live_ -= it->second;
        free_.emplace(it->second, p);
    }
    void trim() {
        for (auto &kv : free_) {
            (void)hipFree(kv.second);
            size_.erase(kv.second);
        }
        free_.clear();
    }
    ~DevPool() {
        trim();
        for (auto &kv : size_) (void)hipFree(kv.first);
    }
    size_t live() const { return live_; }

   private:
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> size_;
    size_t live_ = 0;
};

// Buffers taken from the pool during one query, returned at its end.
struct Scope {
    DevPool &pool;
    std::vector<void *> held;
    explicit Scope(DevPool &p) : pool(p) {}
    template <class T>
    T *get(int64_t n) {
        void *p = pool.get(sizeof(T) * (size_t)std::max<int64_t>(n, 1));
        held.push_back(p);
        return (T *)p;
    }
    void release(void *p) {
        for (auto &h : held)
            if (h == p) {
                pool.put(p);
                h = nullptr;
            }
    }
    ~Scope() {
        for (void *p : held) pool.put(p);
    }
};

constexpr int kMaxSlots = 1024;
constexpr int kMaxRounds = 32;
constexpr int kMaxDesc = 2048;

// Small per-query counters, cleared with one memset per query.
struct DevCounters {
    int32_t cand_count[SGM_MAX_QV + 1];
    int32_t big_count[kMaxSlots];
    unsigned long long removed[kMaxRounds + 1];
    unsigned long long ec_total[SGM_MAX_QE];
};

// Resources of the persistent per-query kernel on one stream: slots,
// descriptors, root sweep rows and the output arena.
struct NarrowCtx {
    hipStream_t stream = nullptr;
    // capacities of a context for queries that outgrew a regular slot (0:
    // the regular ones)
    int32_t lcap_want = 0;
    int64_t slab_want = 0;
    int slots = 0;
    int32_t lcap = 0;
    int64_t slab_bytes = 0;
    uint64_t *bits = nullptr;
    int32_t *lists = nullptr;
    char *slab = nullptr;
    int qcap = 0;
    NQuery *d_q = nullptr, *h_q = nullptr;
    NResult *d_res = nullptr, *h_res = nullptr;
    VPred *d_preds = nullptr, *h_preds = nullptr;  // distinct root predicates
    int root_cap = 0;
    uint64_t *d_rootbits = nullptr;
    int32_t *d_out = nullptr;
    int64_t out_cap = 0;
    // [0] queue, [1] out used, [2] helper counters (posted steps, slot
    // workgroups done)
    unsigned long long *d_ctr = nullptr, *h_ctr = nullptr;
    HelpJob *d_board = nullptr;  // [kNarrowMaxSlots] shared filter steps
    bool serve = false;          // a server's context: no shared steps
    int32_t *h_out = nullptr;
    int64_t h_out_cap = 0;
    int64_t *d_trace = nullptr, *h_trace = nullptr;  // [trace_cap][SGM_TRACE_CAP]
    int trace_cap = 0;
    hipEvent_t done = nullptr;
    // result tables go to pinned host blocks on this second stream while
    // the context's own stream orders the next large table
    hipStream_t copy = nullptr;
    std::vector<hipEvent_t> copy_ev;
    // one batch as a HIP graph: upload descriptors, upload root predicates,
    // root sweep, persistent kernel, read back results, read back counters.
    // Built on first use; every launch updates all node parameters.
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraphNode_t gn[7] = {};
    SweepArgs sa{};
    NArgs na{};
    // parameters of the instantiated graph's last launch: nodes whose
    // parameters did not change are not updated again
    SweepArgs last_sa{};
    NArgs last_na{};
    int last_grid = -1, last_sweep_grid = -1;
    size_t last_qb = 0, last_pb = 0, last_rb = 0;
    const void *last_hout = nullptr;
    void *kargs[9] = {};
};

}  // namespace

struct sgm_graph {
    // sgm_inject_fault: the query index of the next persistent-kernel launch
    // that fails as if by a device fault (-1: none)
    int64_t fault_query = -1;
    int device = 0;
    hipStream_t stream = nullptr;
    sgm_options opts;
    int32_t V = 0;
    int64_t E = 0;
    int32_t nwords = 0;
    int32_t max_out = 0, max_in = 0;
    int32_t n_big = 0;  // vertices with a direction above kBigDegree
    double ns_per_tick = 10.0;  // device wall clock period
    // step events of the last match call (options.profile = 2)
    std::vector<int64_t> trace;  // [queries][SGM_TRACE_CAP]
    std::vector<int32_t> trace_n;
    int32_t n_types = 0;
    std::vector<int64_t> type_freq;
    int32_t n_rels = 0;
    std::vector<int64_t> rel_freq;  // edges per relation (after dedupe)
    DevGraph dg{};
    // device memory owned by the graph
    int32_t *d_out_off = nullptr, *d_in_off = nullptr;
    int2 *d_vinfo = nullptr;
    int2 *d_out_adj = nullptr, *d_in_adj = nullptr;
    int2 *d_out_ta = nullptr, *d_out_tb = nullptr, *d_in_ta = nullptr, *d_in_tb = nullptr;
    int32_t *d_hub_of = nullptr, *d_hub_toff = nullptr;
    // with options.host_graph: the adjacency arrays above live in pinned host
    // memory; (host address, device address) of each such allocation
    std::vector<std::pair<void *, void *>> host_graph_bufs;
    // a compressed graph (sgm_load_compressed): matches are homomorphisms
    bool homomorphic = false;
    // sgm_attach_mapping: mapping lists of a compression of this graph
    int32_t map_nw = 0;
    int32_t *d_map_off = nullptr, *d_map_ids = nullptr;
    std::vector<int32_t> hyper_of;
    uint64_t *d_bits = nullptr;   // [SGM_MAX_QV + 1][nwords] (last: push scratch)
    int32_t *d_lists = nullptr;   // [SGM_MAX_QV][V]
    int32_t *d_prefix = nullptr;  // [SGM_MAX_QV][nwords + 1]
    int32_t *d_big = nullptr;     // [max(n_big,1)]
    NbrDesc *d_desc = nullptr;    // [kMaxDesc]
    DevCounters *d_cnt = nullptr;
    int32_t *d_slots = nullptr;   // [SGM_MAX_QV] ids for multi-collect
    // pinned host staging
    NbrDesc *h_desc = nullptr;
    DevCounters *h_cnt = nullptr;
    int32_t *h_slots = nullptr;
    int64_t *h_small = nullptr;   // [64] small readbacks
    void *h_rows = nullptr;
    size_t h_rows_cap = 0;
    hipEvent_t ev_rows[2] = {nullptr, nullptr};  // staging halves of result readback
    DevPool pool;
    std::mutex mu;
    // profiling
    std::vector<hipEvent_t> ev_free;
    struct Pending {
        int kid;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Pending> pending;
    sgm_kstat kstat[SGM_K_COUNT]{};
    std::atomic<int> launches{0};
    // persistent per-query kernel on the graph's own stream
    NarrowCtx nw;
    NarrowCtx nwb;  // few large slots for queries that outgrow a regular one
    sgm_tuning tune{512, 64, 8192, 0, 1024, 64, 0, {0}};
};

namespace {

// ---------------------------------------------------------------------------
// profiling helpers
// ---------------------------------------------------------------------------

struct Prof {
    sgm_graph *g;
    int kid;
    double bytes;
    hipEvent_t a = nullptr, b = nullptr;
    Prof(sgm_graph *g_, int kid_, double bytes_, bool on_graph_stream = true)
        : g(g_), kid(kid_), bytes(bytes_) {
        g->launches++;
        if (!g->opts.profile || !on_graph_stream) return;
        a = take();
        b = take();
        HIPX(hipEventRecord(a, g->stream));
    }
    hipEvent_t take() {
        if (g->ev_free.empty()) {
            hipEvent_t e;
            HIPX(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = g->ev_free.back();
        g->ev_free.pop_back();
        return e;
    }
    ~Prof() {
        if (!a) return;
        if (hipEventRecord(b, g->stream) == hipSuccess) g->pending.push_back({kid, a, b, bytes});
    }
};

// after a full stream sync: fold pending event pairs into the stats
void prof_flush(sgm_graph *g) {
    for (auto &p : g->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g->kstat[p.kid].launches++;
            g->kstat[p.kid].ms_total += ms;
            g->kstat[p.kid].bytes_total += p.bytes;
        }
        g->ev_free.push_back(p.a);
        g->ev_free.push_back(p.b);
    }
    g->pending.clear();
}

void sync(sgm_graph *g) {
    HIPX(hipStreamSynchronize(g->stream));
    prof_flush(g);
}

// ---------------------------------------------------------------------------
// graph load
// ---------------------------------------------------------------------------

int normalize_csr(int32_t V, int32_t E, const int32_t *row_ptr, const int32_t *col,
                  const int32_t *rel, std::vector<int32_t> &off, std::vector<int2> &adj) {
    if (row_ptr[0] != 0 || row_ptr[V] != E) return SGM_EINVAL;
    for (int32_t v = 0; v < V; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return SGM_EINVAL;
    for (int64_t i = 0; i < E; ++i)
        if (col[i] < 0 || col[i] >= V || rel[i] < 0) return SGM_EINVAL;
    off.assign((size_t)V + 1, 0);
    adj.resize((size_t)E);
    int64_t w = 0;
    auto less = [](const int2 &a, const int2 &b) { return a.x != b.x ? a.x < b.x : a.y < b.y; };
    for (int32_t v = 0; v < V; ++v) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        off[v] = (int32_t)w;
        const int64_t start = w;
        bool sorted = true;
        for (int64_t i = b; i < e; ++i) {
            adj[w] = make_int2(col[i], rel[i]);
            if (w > start && !less(adj[w - 1], adj[w])) sorted = false;
            ++w;
        }
        if (!sorted) {
            std::sort(adj.begin() + start, adj.begin() + w, less);
            int64_t k = start;
            for (int64_t i = start; i < w; ++i)
                if (k == start || adj[k - 1].x != adj[i].x || adj[k - 1].y != adj[i].y)
                    adj[k++] = adj[i];
            w = k;
        }
    }
    off[V] = (int32_t)w;
    adj.resize((size_t)w);
    return SGM_OK;
}

void build_in(int32_t V, const std::vector<int32_t> &off, const std::vector<int2> &adj,
              std::vector<int32_t> &in_off, std::vector<int2> &in_adj) {
    in_off.assign((size_t)V + 1, 0);
    for (const int2 &e : adj) in_off[e.x + 1]++;
    for (int32_t v = 0; v < V; ++v) in_off[v + 1] += in_off[v];
    std::vector<int32_t> fill(in_off.begin(), in_off.end() - 1);
    in_adj.resize(adj.size());
    // sources visited in ascending order, relations ascending within a
    // source, so every in-row comes out sorted by (src, rel)
    for (int32_t v = 0; v < V; ++v)
        for (int32_t i = off[v]; i < off[v + 1]; ++i) in_adj[fill[adj[i].x]++] = make_int2(v, adj[i].y);
}

template <class T>
T *dev_upload(const std::vector<T> &h) {
    T *p = nullptr;
    HIPX(hipMalloc(&p, sizeof(T) * std::max<size_t>(h.size(), 1)));
    if (!h.empty()) HIPX(hipMemcpy(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return p;
}

// An O(E) graph array in pinned host memory that kernels read in place over
// the host link (thesis Ch. 3, Sec. "Scalability Test": a data graph too
// large for the device stays in main memory). Mapped into the device's
// address space and cacheable on the device: the arrays are read-only after
// this copy, which completes before any kernel runs.
template <class T>
T *host_upload(const std::vector<T> &h, std::vector<std::pair<void *, void *>> &bufs) {
    void *p = nullptr;
    HIPX(hipHostMalloc(&p, sizeof(T) * std::max<size_t>(h.size(), 1),
                       hipHostMallocMapped | hipHostMallocNonCoherent));
    void *d = nullptr;
    const hipError_t e = hipHostGetDevicePointer(&d, p, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(p);
        HIPX(e);
    }
    bufs.emplace_back(p, d);
    if (!h.empty()) std::memcpy(p, h.data(), sizeof(T) * h.size());
    return (T *)d;
}

void narrow_free(NarrowCtx &nw);

void free_graph_mem(sgm_graph *g) {
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (auto &p : g->pending) {
        g->ev_free.push_back(p.a);
        g->ev_free.push_back(p.b);
    }
    for (hipEvent_t e : g->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : g->ev_rows)
        if (e) (void)hipEventDestroy(e);
    void *dp[] = {g->d_out_off, g->d_in_off, g->d_vinfo,  g->d_out_adj, g->d_in_adj,
                  g->d_bits,    g->d_lists,  g->d_prefix, g->d_big,     g->d_desc,
                  g->d_cnt,     g->d_slots,  g->d_out_ta, g->d_out_tb,  g->d_in_ta,
                  g->d_in_tb,   g->d_hub_of, g->d_hub_toff, g->d_map_off, g->d_map_ids};
    for (void *p : dp) {
        bool host = false;
        for (const auto &b : g->host_graph_bufs) host |= b.second == p;
        if (p && !host) (void)hipFree(p);
    }
    for (const auto &b : g->host_graph_bufs) (void)hipHostFree(b.first);
    void *hp[] = {g->h_desc, g->h_cnt, g->h_slots, g->h_small, g->h_rows};
    for (void *p : hp)
        if (p) (void)hipHostFree(p);
    narrow_free(g->nw);
    narrow_free(g->nwb);
    if (g->stream) (void)hipStreamDestroy(g->stream);
}

// Hub-row index (DevGraph::out_ta ... hub_toff): copies of the adjacency
// arrays whose hub rows are re-sorted by the other end's type first, and
// per hub, direction, order and type the offset of the type's first entry.
struct HubIndex {
    std::vector<int2> out_ta, out_tb, in_ta, in_tb;
    std::vector<int32_t> hub_of, toff;
    int32_t types = 0;
};

void build_hub_index(int32_t V, const std::vector<int32_t> &off, const std::vector<int2> &adj,
                     const std::vector<int32_t> &in_off, const std::vector<int2> &in_adj,
                     const int32_t *type, int32_t n_types, HubIndex *h) {
    h->types = n_types + 1;
    h->hub_of.assign((size_t)V, -1);
    std::vector<int32_t> hubs;
    for (int32_t v = 0; v < V; ++v)
        if (off[v + 1] - off[v] >= kHubRow || in_off[v + 1] - in_off[v] >= kHubRow) {
            h->hub_of[v] = (int32_t)hubs.size();
            hubs.push_back(v);
        }
    h->out_ta = adj;
    h->out_tb = adj;
    h->in_ta = in_adj;
    h->in_tb = in_adj;
    h->toff.assign(hubs.size() * 4 * (size_t)h->types, 0);
    auto by_type_rel = [&](const int2 &a, const int2 &b) {
        const int32_t ta = type[a.x], tb = type[b.x];
        return ta != tb ? ta < tb : (a.y != b.y ? a.y < b.y : a.x < b.x);
    };
    auto by_type_end = [&](const int2 &a, const int2 &b) {
        const int32_t ta = type[a.x], tb = type[b.x];
        return ta != tb ? ta < tb : (a.x != b.x ? a.x < b.x : a.y < b.y);
    };
    auto work = [&](size_t lo, size_t hi) {
        for (size_t k = lo; k < hi; ++k) {
            const int32_t v = hubs[k];
            for (int dir = 0; dir < 2; ++dir) {
                const std::vector<int32_t> &o = dir ? in_off : off;
                const int32_t b = o[v], e = o[v + 1];
                for (int order = 0; order < 2; ++order) {
                    std::vector<int2> &arr =
                        dir ? (order ? h->in_tb : h->in_ta) : (order ? h->out_tb : h->out_ta);
                    if (order) std::sort(arr.begin() + b, arr.begin() + e, by_type_end);
                    else std::sort(arr.begin() + b, arr.begin() + e, by_type_rel);
                    int32_t *t = &h->toff[((k * 2 + dir) * 2 + order) * (size_t)h->types];
                    int32_t i = b;
                    for (int32_t ty = 0; ty < h->types; ++ty) {
                        while (i < e && type[arr[i].x] < ty) ++i;
                        t[ty] = i - b;
                    }
                }
            }
        }
    };
    const size_t nt = std::max<size_t>(1, std::min<size_t>(8, hubs.size() / 16));
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t)
        th.emplace_back(work, hubs.size() * t / nt, hubs.size() * (t + 1) / nt);
    work(0, hubs.size() / nt);
    for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------
// one query
// ---------------------------------------------------------------------------

struct ECTab {
    int key;      // key vertex
    int other;
    int dir;      // 0: keys are sources (scan out-edges), 1: keys are destinations
    int slot;     // big-list counter slot
    int32_t *cnt = nullptr;
    int32_t *offs = nullptr;
    int32_t *vals = nullptr;
    int32_t *big = nullptr;
    int64_t n = 0;
};

struct HostCopy {
    void *dst;
    const void *src;
    size_t bytes;
};

// Host copies of a batch's result tables out of the pinned staging buffer;
// large totals are split over threads (first touch of the fresh result
// buffers is part of the cost).
void parallel_copy(const std::vector<HostCopy> &cs) {
    size_t total = 0;
    for (const HostCopy &c : cs) total += c.bytes;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::min<size_t>({(size_t)8, (size_t)hw, total >> 23});  // 8 MB each
    if (nt <= 1) {
        for (const HostCopy &c : cs) std::memcpy(c.dst, c.src, c.bytes);
        return;
    }
    // cut the concatenated bytes into nt equal ranges
    const size_t per = (total + nt - 1) / nt;
    auto work = [&](size_t lo, size_t hi) {
        size_t pos = 0;
        for (const HostCopy &c : cs) {
            const size_t a = std::max(lo, pos), b = std::min(hi, pos + c.bytes);
            if (a < b) std::memcpy((char *)c.dst + (a - pos), (const char *)c.src + (a - pos), b - a);
            pos += c.bytes;
            if (pos >= hi) break;
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work, per * t, std::min(total, per * (t + 1)));
    work(0, std::min(total, per));
    for (auto &x : th) x.join();
}

// Host worker threads for per-query planning and packing: started once,
// kept for the life of the process (never destroyed, so no thread waits on
// a pool that exit tears down), parked on a condition variable between
// jobs. One job at a time; the caller works on it too.
class HostPool {
  public:
    static HostPool &get() {
        static HostPool *p = new HostPool();
        return *p;
    }
    int workers() const { return (int)nworkers_; }
    // run(c) for c in [0, nchunks), on the workers and the caller
    void run(int nchunks, const std::function<void(int)> &fn) {
        std::lock_guard<std::mutex> one(job_mu_);
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            nchunks_ = nchunks;
            next_.store(0);
            left_ = nchunks;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return left_ == 0; });
        fn_ = nullptr;
    }

  private:
    HostPool() {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        nworkers_ = std::min(7u, hw > 1 ? hw - 1 : 0u);
        for (unsigned t = 0; t < nworkers_; ++t) std::thread([this] { loop(); }).detach();
    }
    void work() {
        for (;;) {
            const int c = next_.fetch_add(1);
            if (c >= nchunks_) return;
            (*fn_)(c);
            std::lock_guard<std::mutex> lk(mu_);
            if (--left_ == 0) done_cv_.notify_all();
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                if (!fn_) continue;
            }
            work();
        }
    }
    unsigned nworkers_ = 0;
    std::mutex job_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *fn_ = nullptr;
    int nchunks_ = 0, left_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
};

// f(lo, hi) over [0, n) in chunks of at least min_each items, on the host
// pool's workers and the caller (the caller alone for small n).
template <class F>
void parallel_for(int n, int min_each, F &&f) {
    HostPool &pool = HostPool::get();
    const int nt = std::min<int>(pool.workers() + 1, n / std::max(1, min_each));
    if (nt <= 1) {
        f(0, n);
        return;
    }
    const int per = (n + nt - 1) / nt;
    const std::function<void(int)> chunk = [&](int c) { f(c * per, std::min(n, (c + 1) * per)); };
    pool.run(nt, chunk);
}

constexpr size_t kStageBytes = (size_t)256 << 20;  // multi-kernel readback chunk

// Host buffer of a result table. Large tables get 2 MB-aligned memory with
// transparent huge pages requested, which cuts page faults on first touch;
// freed with free() either way.
int32_t *alloc_rows(size_t bytes) {
    if (bytes >= ((size_t)64 << 20)) {
        void *p = nullptr;
        if (posix_memalign(&p, (size_t)2 << 20, bytes) != 0) return nullptr;
        (void)madvise(p, bytes, MADV_HUGEPAGE);
        return (int32_t *)p;
    }
    return (int32_t *)std::malloc(std::max<size_t>(bytes, 4));
}

// Host memory of the result tables of one persistent launch: a pinned block
// into which the output arena (and the tables the host orders) are copied
// straight from the device, with no second copy on the host; the results
// point into it and hold a reference each. A block whose last result is
// freed is kept for later launches (a few of them), so a steady stream of
// batches reuses pinned, already-mapped memory.
struct RowBlock {
    char *ptr = nullptr;
    size_t cap = 0;
    std::atomic<int64_t> refs{0};
};

std::mutex g_blk_mu;
std::vector<RowBlock *> g_blk_free;
constexpr size_t kKeepBlocks = 3;
constexpr size_t kBlockMin = (size_t)4 << 20;  // launches returning less copy as before

RowBlock *block_get(size_t bytes) {
    {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        int best = -1;
        for (size_t i = 0; i < g_blk_free.size(); ++i)
            if (g_blk_free[i]->cap >= bytes &&
                (best < 0 || g_blk_free[i]->cap < g_blk_free[(size_t)best]->cap))
                best = (int)i;
        if (best >= 0) {
            RowBlock *b = g_blk_free[(size_t)best];
            g_blk_free.erase(g_blk_free.begin() + best);
            return b;
        }
    }
    RowBlock *b = new RowBlock();
    const size_t cap = std::max(bytes + (bytes >> 3), kBlockMin);
    if (hipHostMalloc((void **)&b->ptr, cap, hipHostMallocDefault) != hipSuccess) {
        delete b;
        throw DeviceError{SGM_ENOMEM};
    }
    b->cap = cap;
    return b;
}

void block_release(RowBlock *b) {
    if (b->refs.fetch_sub(1) != 1) return;
    RowBlock *drop = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        g_blk_free.push_back(b);
        if (g_blk_free.size() > kKeepBlocks) {
            // drop the smallest kept block
            size_t k = 0;
            for (size_t i = 1; i < g_blk_free.size(); ++i)
                if (g_blk_free[i]->cap < g_blk_free[k]->cap) k = i;
            drop = g_blk_free[k];
            g_blk_free.erase(g_blk_free.begin() + (long)k);
        }
    }
    if (drop) {
        (void)hipHostFree(drop->ptr);
        delete drop;
    }
}

// Every result the library hands out is the first member of a box that
// knows whether its rows live in a block.
struct ResultBox {
    sgm_result r;
    RowBlock *blk;
};

sgm_result *result_new() {
    ResultBox *b = (ResultBox *)std::calloc(1, sizeof(ResultBox));
    return b ? &b->r : nullptr;
}

RowBlock *&result_block(sgm_result *r) { return reinterpret_cast<ResultBox *>(r)->blk; }

// Release a result's rows (its block reference, or its own buffer).
void result_drop_rows(sgm_result *r) {
    RowBlock *&b = result_block(r);
    if (b) block_release(b);
    else std::free(r->rows);
    b = nullptr;
    r->rows = nullptr;
}

// Copy a device table to host memory through two pinned staging halves of
// kStageBytes on stream st (the host copy of one chunk overlaps the
// transfer of the next). Caller holds g->mu.
void readback_rows(sgm_graph *g, hipStream_t st, const int32_t *dev, size_t bytes, int32_t *host) {
    if (bytes == 0) return;
    const size_t half = std::min(bytes, kStageBytes);
    if (g->h_rows_cap < 2 * half) {
        if (g->h_rows) (void)hipHostFree(g->h_rows);
        g->h_rows = nullptr;
        g->h_rows_cap = 0;
        const size_t cap = std::max<size_t>(2 * half, 1 << 20);
        HIPX(hipHostMalloc(&g->h_rows, cap, hipHostMallocDefault));
        g->h_rows_cap = cap;
    }
    for (hipEvent_t &e : g->ev_rows)
        if (!e) HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    char *stage[2] = {(char *)g->h_rows, (char *)g->h_rows + half};
    const size_t nch = (bytes + half - 1) / half;
    auto issue = [&](size_t i) {
        const size_t off = i * half, len = std::min(half, bytes - off);
        HIPX(hipMemcpyAsync(stage[i & 1], (const char *)dev + off, len, hipMemcpyDeviceToHost, st));
        HIPX(hipEventRecord(g->ev_rows[i & 1], st));
    };
    issue(0);
    for (size_t i = 0; i < nch; ++i) {
        if (i + 1 < nch) issue(i + 1);  // its half was copied out last round
        HIPX(hipEventSynchronize(g->ev_rows[i & 1]));
        const size_t off = i * half, len = std::min(half, bytes - off);
        parallel_copy({HostCopy{(char *)host + off, stage[i & 1], len}});
    }
}

// Stable order of n non-negative int32 keys below 2^nbits (whole-GPU LSD
// radix passes, 8-bit digits); key is overwritten. Returns the order.
int32_t *order_by_i32(sgm_graph *g, Scope &sc, int32_t *key, int64_t n, int nbits) {
    int32_t *ia = sc.get<int32_t>(n), *ib = sc.get<int32_t>(n);
    int32_t *ka = key, *kb = sc.get<int32_t>(n);
    const int64_t tiles = radix_tiles(n);
    int64_t *hist = sc.get<int64_t>(256 * tiles);
    int64_t *hoff = sc.get<int64_t>(256 * tiles + 1);
    int64_t *tmp = sc.get<int64_t>(scan_tmp_words(256 * tiles) + 1);
    hipStream_t st = g->stream;
    {
        Prof p(g, SGM_K_SORT, 4.0 * n);
        launch_iota(st, ia, n);
    }
    for (int sh = 0; sh < nbits; sh += 8) {
        Prof p(g, SGM_K_SORT, 20.0 * n);
        launch_radix_hist(st, ka, n, sh, hist);
        launch_scan_i64(st, hist, 256 * tiles, hoff, tmp);
        launch_radix_scatter(st, ka, ia, n, sh, hoff, kb, ib);
        std::swap(ka, kb);
        std::swap(ia, ib);
    }
    return ia;
}

// Order n rows by 64-bit keys of tb bits with whole-GPU LSD radix passes
// (stable, 8-bit digits over the 32-bit halves); returns the order.
int32_t *order_by_keys(sgm_graph *g, Scope &sc, const uint64_t *keys, int64_t n, int tb) {
    int32_t *ia = sc.get<int32_t>(n), *ib = sc.get<int32_t>(n);
    int32_t *ka = sc.get<int32_t>(n), *kb = sc.get<int32_t>(n);
    const int64_t tiles = radix_tiles(n);
    int64_t *hist = sc.get<int64_t>(256 * tiles);
    int64_t *hoff = sc.get<int64_t>(256 * tiles + 1);
    int64_t *tmp = sc.get<int64_t>(scan_tmp_words(256 * tiles) + 1);
    hipStream_t st = g->stream;
    {
        Prof p(g, SGM_K_SORT, 4.0 * n);
        launch_iota(st, ia, n);
    }
    for (int half = 0; half < 2; ++half) {
        const int hb = half == 0 ? std::min(tb, 32) : tb - 32;
        if (hb <= 0) break;
        {
            Prof p(g, SGM_K_SORT, 16.0 * n);
            launch_key_half(st, keys, ia, n, half, ka);
        }
        for (int sh = 0; sh < hb; sh += 8) {
            Prof p(g, SGM_K_SORT, 20.0 * n);
            launch_radix_hist(st, ka, n, sh, hist);
            launch_scan_i64(st, hist, 256 * tiles, hoff, tmp);
            launch_radix_scatter(st, ka, ia, n, sh, hoff, kb, ib);
            std::swap(ka, kb);
            std::swap(ia, ib);
        }
    }
    return ia;
}

struct Query {
    sgm_graph *g;
    const QInfo &qi;
    Plan pl;
    Scope sc;
    sgm_result *res;
    // flags of the run: a projection's count needs its distinct rows, so a
    // projected query materialises the join's final table even when only
    // the count is asked for (want_rows then stays false)
    uint32_t flags;
    bool want_rows;
    int next_slot = 0;
    Query(sgm_graph *g_, const QInfo &q_, sgm_result *r, uint32_t f)
        : g(g_), qi(q_), sc(g_->pool), res(r),
          flags(q_.proj ? (f & ~SGM_COUNT_ONLY) : f), want_rows(!(f & SGM_COUNT_ONLY)) {}

    uint64_t *bits(int u) const { return g->d_bits + (int64_t)u * g->nwords; }
    uint64_t *scratch() const { return g->d_bits + (int64_t)SGM_MAX_QV * g->nwords; }
    int32_t *list(int u) const { return g->d_lists + (int64_t)u * g->V; }
    int32_t *prefix(int u) const { return g->d_prefix + (int64_t)u * (g->nwords + 1); }
    int32_t *cand_count_dev(int u) const { return &g->d_cnt->cand_count[u]; }
    hipStream_t st() const { return g->stream; }

    // with the outgoing graph only, in-degrees are unknown (not tested)
    VPred pred(int u) const {
        return VPred{qi.label[u], qi.pin[u], qi.qout[u], g->opts.out_only ? 0 : qi.qin[u]};
    }

    void collect_one(int u) {
        Prof p(g, SGM_K_COLLECT, (double)g->nwords * 12.0);
        launch_collect_multi(st(), g->dg, bits(u), g->nwords, list(u), g->V, cand_count_dev(u),
                             prefix(u), g->nwords + 1, nullptr, 1);
    }

    void collect_all() {
        Prof p(g, SGM_K_COLLECT, (double)qi.n * g->nwords * 12.0);
        launch_collect_multi(st(), g->dg, g->d_bits, g->nwords, g->d_lists, g->V,
                             g->d_cnt->cand_count, g->d_prefix, g->nwords + 1, nullptr, qi.n);
    }

    int grid_small_for(int64_t items) const {
        int64_t gsz = (items + (kBlock / 16) - 1) / (kBlock / 16);
        return (int)std::max<int64_t>(1, std::min<int64_t>(gsz, 2048));
    }
    int grid_big() const { return std::max(1, std::min(g->n_big, 1024)); }

    int filter_launch(int u, const NbrDesc *dev_desc, int n_nbr, bool push, int64_t items_bound,
                      unsigned long long *removed, int kid) {
        FilterArgs a{};
        a.g = g->dg;
        a.items = list(u);
        a.count = cand_count_dev(u);
        a.self_bits = bits(u);
        a.nbr = dev_desc;
        a.n_nbr = n_nbr;
        a.do_push = push ? 1 : 0;
        a.big_items = g->d_big;
        const int slot = next_slot++;
        if (slot >= kMaxSlots) return SGM_EUNSUPPORTED;
        a.big_count = &g->d_cnt->big_count[slot];
        a.removed = removed;
        Prof p(g, kid, 0.0);
        launch_filter(st(), a, grid_small_for(items_bound), grid_big());
        return SGM_OK;
    }

    // Filtering phase: Alg. 3.2 initialisation along the spanning tree, then
    // the refinement rounds.
    int filter() {
        const int n = qi.n;
        HIPX(hipMemsetAsync(g->d_bits, 0, sizeof(uint64_t) * (size_t)n * g->nwords, st()));
        HIPX(hipMemsetAsync(g->d_cnt, 0, sizeof(DevCounters), st()));
        // descriptors for every filter launch, uploaded once
        Program pr;
        if (g->opts.out_only)
            build_program_out_only(qi, pl, g->opts.low_conn_degree, g->opts.refine_reversed, &pr);
        else
            build_program(qi, pl, g->opts.low_conn_degree, g->opts.refine_reversed, &pr);
        std::vector<NbrDesc> &hd = desc_;
        hd.clear();
        for (const PNbr &p : pr.nbr) {
            NbrDesc d{};
            d.dir = p.dir;
            d.rel = p.rel;
            d.mode = p.mode;
            d.push = 1;
            d.pred = pred(p.v);
            d.test_bits = bits(p.v);
            d.push_bits = p.mode == 0 ? scratch() : bits(p.v);
            hd.push_back(d);
        }
        if ((int)hd.size() > kMaxDesc) return SGM_EUNSUPPORTED;
        if (!hd.empty()) {
            std::memcpy(g->h_desc, hd.data(), sizeof(NbrDesc) * hd.size());
            HIPX(hipMemcpyAsync(g->d_desc, g->h_desc, sizeof(NbrDesc) * hd.size(),
                                hipMemcpyHostToDevice, st()));
        }
        // root check (kernel_check): the first vertex of O
        const int root = pl.visit[0];
        if (qi.pin[root] >= 0) {
            Prof p(g, SGM_K_CHECK, 8.0);
            launch_check_pin(st(), g->dg, pred(root), bits(root));
        } else {
            Prof p(g, SGM_K_CHECK, 8.0 * g->V + g->nwords * 8.0);
            launch_check_sweep(st(), g->dg, pred(root), bits(root));
        }
        for (const PStep &s : pr.init) {
            if (s.sweep) {
                // outgoing graph only: a vertex reached over an edge into
                // its parent starts from its predicate alone
                if (qi.pin[s.u] >= 0) {
                    Prof p(g, SGM_K_CHECK, 8.0);
                    launch_check_pin(st(), g->dg, pred(s.u), bits(s.u));
                } else {
                    Prof p(g, SGM_K_CHECK, 8.0 * g->V + g->nwords * 8.0);
                    launch_check_sweep(st(), g->dg, pred(s.u), bits(s.u));
                }
            }
            collect_one(s.u);
            if (s.parent >= 0)
                HIPX(hipMemsetAsync(scratch(), 0, sizeof(uint64_t) * g->nwords, st()));
            const int64_t bound = qi.pin[s.u] >= 0 ? 1 : g->V;
            int rc = filter_launch(s.u, g->d_desc + s.first, s.count, true, bound,
                                   &g->d_cnt->removed[kMaxRounds], SGM_K_EXPLORE);
            if (rc) return rc;
            if (s.parent >= 0) {
                Prof p(g, SGM_K_OTHER, g->nwords * 24.0);
                launch_and(st(), bits(s.parent), scratch(), g->nwords);
            }
        }
        int rounds = g->opts.refine_rounds;
        const bool fixpoint = rounds < 0;
        if (fixpoint) rounds = kMaxRounds;
        rounds = std::min(rounds, kMaxRounds);
        for (int r = 0; r < rounds && !pr.refine.empty(); ++r) {
            for (const PStep &s : pr.refine) {
                collect_one(s.u);
                const int64_t bound = qi.pin[s.u] >= 0 ? 1 : g->V;
                // a step with a parent (outgoing graph only) pushes into the
                // scratch bitmap, then prunes the parent by it
                if (s.parent >= 0)
                    HIPX(hipMemsetAsync(scratch(), 0, sizeof(uint64_t) * g->nwords, st()));
                int rc = filter_launch(s.u, g->d_desc + s.first, s.count, s.parent >= 0, bound,
                                       &g->d_cnt->removed[r], SGM_K_REFINE);
                if (rc) return rc;
                if (s.parent >= 0) {
                    Prof p(g, SGM_K_OTHER, g->nwords * 24.0);
                    launch_and(st(), bits(s.parent), scratch(), g->nwords, &g->d_cnt->removed[r]);
                }
            }
            if (fixpoint) {
                HIPX(hipMemcpyAsync(g->h_small, &g->d_cnt->removed[r], sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, st()));
                sync(g);
                if (g->h_small[0] == 0) break;
            }
        }
        collect_all();
        return SGM_OK;
    }

    std::vector<NbrDesc> desc_;
    int32_t ccount[SGM_MAX_QV] = {};
    ECTab ec[SGM_MAX_QE];
    int jorder[SGM_MAX_QV];   // query vertex at each join column
    int jpos[SGM_MAX_QV];     // join column of each query vertex

    ECDesc ec_desc(const ECTab &t, int e) {
        ECDesc d{};
        d.key_vertex = t.key;
        d.dir = t.dir;
        d.rel = qi.elabel[e];
        d.keys = list(t.key);
        d.key_count = cand_count_dev(t.key);
        d.other_bits = bits(t.other);
        d.cnt = t.cnt;
        d.offs = t.offs;
        d.vals = t.vals;
        d.homomorphic = g->homomorphic ? 1 : 0;
        d.total = &g->d_cnt->ec_total[e];
        d.big_items = t.big;
        d.big_count = &g->d_cnt->big_count[t.slot];
        return d;
    }

    void ec_count(ECTab &t, int e) {
        t.cnt = sc.get<int32_t>(ccount[t.key]);
        t.big = sc.get<int32_t>(std::min<int64_t>(ccount[t.key], std::max(g->n_big, 1)));
        t.slot = next_slot++;
        if (t.slot >= kMaxSlots) throw DeviceError{SGM_EUNSUPPORTED};
        Prof p(g, SGM_K_EC_COUNT, 0.0);
        launch_ec_count(st(), g->dg, ec_desc(t, e), grid_small_for(ccount[t.key]), grid_big());
    }

    // Joining phase, part 1: candidate edges of every query edge, then the
    // join order (Sec. "Joining Phase": start from the edge with the fewest
    // candidate edges; prefer edges whose endpoints are both bound; ties by
    // fewest candidates, then lowest edge index).
    int collect_edges() {
        const int m = qi.m;
        for (int e = 0; e < m; ++e) {
            ECTab &t = ec[e];
            t.key = qi.esrc[e];
            t.other = qi.edst[e];
            t.dir = 0;
            ec_count(t, e);
        }
        HIPX(hipMemcpyAsync(g->h_cnt->ec_total, g->d_cnt->ec_total,
                            sizeof(unsigned long long) * m, hipMemcpyDeviceToHost, st()));
        sync(g);
        int64_t tot[SGM_MAX_QE];
        for (int e = 0; e < m; ++e) {
            tot[e] = (int64_t)g->h_cnt->ec_total[e];
            res->stats.ec[e] = tot[e];
        }
        for (int e = 0; e < m; ++e)
            if (tot[e] == 0) return 1;  // no match
        // join order
        bool vis[SGM_MAX_QV] = {}, used[SGM_MAX_QE] = {};
        int e0 = 0;
        for (int e = 1; e < m; ++e)
            if (tot[e] < tot[e0]) e0 = e;
        int nj = 0;
        jorder[nj++] = qi.esrc[e0];
        vis[qi.esrc[e0]] = true;
        ext_.clear();
        // each join level: new vertex, extension edge, check edges
        auto add_level = [&](int e_ext) {
            const int a = qi.esrc[e_ext], b = qi.edst[e_ext];
            const int w = vis[a] ? b : a;
            Level L{};
            L.w = w;
            L.ext = e_ext;
            used[e_ext] = true;
            for (int e = 0; e < m; ++e) {
                if (used[e]) continue;
                const int x = qi.esrc[e], y = qi.edst[e];
                if ((x == w && vis[y]) || (y == w && vis[x])) {
                    L.chk[L.n_chk++] = e;
                    used[e] = true;
                }
            }
            vis[w] = true;
            jorder[nj++] = w;
            ext_.push_back(L);
        };
        add_level(e0);
        while (nj < qi.n) {
            int best = -1;
            for (int e = 0; e < m; ++e) {
                if (used[e]) continue;
                const bool va = vis[qi.esrc[e]], vb = vis[qi.edst[e]];
                if (va == vb) continue;
                if (best < 0 || tot[e] < tot[best]) best = e;
            }
            if (best < 0) return SGM_EINVAL;
            add_level(best);
        }
        for (int j = 0; j < qi.n; ++j) jpos[jorder[j]] = j;
        // orientation: key = the endpoint bound first (with the outgoing
        // graph only, a destination key is made by transposing below)
        bool flip[SGM_MAX_QE] = {};
        for (int e = 0; e < m; ++e) {
            ECTab &t = ec[e];
            const int a = qi.esrc[e], b = qi.edst[e];
            const bool key_src = jpos[a] < jpos[b];
            if (!key_src && g->opts.out_only) {
                flip[e] = true;
            } else if (!key_src) {
                sc.release(t.cnt);
                sc.release(t.big);
                t.key = b;
                t.other = a;
                t.dir = 1;
                // count again keyed by the destination (total unchanged)
                ec_count(t, e);
            }
        }
        for (int e = 0; e < m; ++e) {
            ECTab &t = ec[e];
            t.n = tot[e];
            t.offs = sc.get<int32_t>((int64_t)ccount[t.key] + 1);
            t.vals = sc.get<int32_t>(t.n);
            {
                Prof p(g, SGM_K_OTHER, 8.0 * ccount[t.key]);
                launch_scan_i32(st(), t.cnt, cand_count_dev(t.key), t.offs);
            }
            {
                Prof p(g, SGM_K_EC_WRITE, 0.0);
                launch_ec_write(st(), g->dg, ec_desc(t, e), grid_small_for(ccount[t.key]),
                                grid_big());
            }
            if (flip[e]) transpose(t);
        }
        return SGM_OK;
    }

    // Re-key a source-keyed table by its destination without the incoming
    // graph: (destination rank, source) per pair, a stable sort by the rank
    // (sources stay ascending within a key), the counts scanned to offsets.
    void transpose(ECTab &t) {
        const int a = t.key, b = t.other;
        const int64_t n = t.n;
        int32_t *rk = sc.get<int32_t>(n), *src = sc.get<int32_t>(n);
        int32_t *cnt = sc.get<int32_t>((int64_t)ccount[b] + 1);
        HIPX(hipMemsetAsync(cnt, 0, sizeof(int32_t) * ((size_t)ccount[b] + 1), st()));
        {
            Prof p(g, SGM_K_EC_WRITE, 16.0 * n + 4.0 * ccount[a]);
            launch_ec_pairs(st(), list(a), cand_count_dev(a), ccount[a], t.offs, t.vals,
                            RankRef{bits(b), prefix(b)}, rk, src, cnt);
        }
        int nbits = 1;
        while ((1ll << nbits) < ccount[b]) ++nbits;
        const int32_t *idx = order_by_i32(g, sc, rk, n, nbits);
        int32_t *vals = sc.get<int32_t>(n), *offs = sc.get<int32_t>((int64_t)ccount[b] + 1);
        {
            Prof p(g, SGM_K_EC_WRITE, 12.0 * n);
            launch_gather_key(st(), src, 1, 0, idx, n, vals);
        }
        {
            Prof p(g, SGM_K_OTHER, 8.0 * ccount[b]);
            launch_scan_i32(st(), cnt, cand_count_dev(b), offs);
        }
        sc.release(t.cnt);
        sc.release(t.offs);
        sc.release(t.vals);
        t.key = b;
        t.other = a;
        t.dir = 1;
        t.cnt = cnt;
        t.offs = offs;
        t.vals = vals;
    }

    struct Level {
        int w, ext, n_chk;
        int chk[SGM_MAX_QE];
    };
    std::vector<Level> ext_;

    JoinEdge jedge(int e) const {
        const ECTab &t = ec[e];
        JoinEdge j{};
        j.col = jpos[t.key];
        j.rank = RankRef{bits(t.key), prefix(t.key)};
        j.offs = t.offs;
        j.vals = t.vals;
        return j;
    }

    // Joining phase, part 2: extend the table one query vertex per level.
    // Pair ranges whose output would exceed the join budget are processed as
    // chunks, depth-first through the remaining levels; final rows are
    // appended to fin_ in order, so chunking does not change the row order.
    int32_t *fin_ = nullptr;
    int64_t fin_rows_ = 0, fin_cap_ = 0;
    int64_t level_acc_[SGM_MAX_QV] = {};
    int64_t budget_ = 0;

    void append_final(const int32_t *t, int64_t R, int k) {
        if (R == 0) return;
        if (flags & SGM_COUNT_ONLY) {
            fin_rows_ += R;
            return;
        }
        if (fin_rows_ + R > fin_cap_) {
            int64_t cap = std::max<int64_t>(2 * fin_cap_, fin_rows_ + R);
            int32_t *nf = sc.get<int32_t>(cap * k);
            if (fin_rows_)
                HIPX(hipMemcpyAsync(nf, fin_, sizeof(int32_t) * fin_rows_ * k,
                                    hipMemcpyDeviceToDevice, st()));
            if (fin_) sc.release(fin_);
            fin_ = nf;
            fin_cap_ = cap;
        }
        HIPX(hipMemcpyAsync(fin_ + fin_rows_ * k, t, sizeof(int32_t) * R * k,
                            hipMemcpyDeviceToDevice, st()));
        fin_rows_ += R;
    }

    int join_from(size_t li, const int32_t *table, int64_t R, int k) {
        if (li == ext_.size()) {
            append_final(table, R, k);
            return SGM_OK;
        }
        const Level &L = ext_[li];
        if (L.n_chk > SGM_MAX_QV) return SGM_EUNSUPPORTED;
        JoinArgs a{};
        a.table = table;
        a.R = R;
        a.k = k;
        a.homomorphic = g->homomorphic ? 1 : 0;
        a.ext = jedge(L.ext);
        a.n_chk = L.n_chk;
        for (int c = 0; c < L.n_chk; ++c) a.chk[c] = jedge(L.chk[c]);
        int64_t *fan = sc.get<int64_t>(R);
        int64_t *poff = sc.get<int64_t>(R + 1);
        int64_t *tmp = sc.get<int64_t>(scan_tmp_words(R) + 1);
        {
            Prof p(g, SGM_K_JOIN, R * 28.0);
            launch_join_fan(st(), a, fan);
        }
        {
            Prof p(g, SGM_K_OTHER, 16.0 * R);
            launch_scan_i64(st(), fan, R, poff, tmp);
        }
        HIPX(hipMemcpyAsync(g->h_small, poff + R, sizeof(int64_t), hipMemcpyDeviceToHost, st()));
        sync(g);
        const int64_t P = g->h_small[0];
        sc.release(fan);
        sc.release(tmp);
        a.pair_off = poff;
        const bool last = li + 1 == ext_.size();
        // pairs bound the output: chunk the pair range to the budget
        const int64_t chunk = std::max<int64_t>(1, budget_ / (4 * (k + 1)));
        for (int64_t p0 = 0; p0 < P; p0 += chunk) {
            const int64_t p1 = std::min(P, p0 + chunk);
            if (p0 > 0 || p1 < P) res->stats.n_chunks++;
            a.p0 = p0;
            a.P = p1;
            const int64_t tiles = join_tiles(p1 - p0);
            int64_t *bcnt = sc.get<int64_t>(tiles);
            int64_t *boff = sc.get<int64_t>(tiles + 1);
            int64_t *tmp2 = sc.get<int64_t>(scan_tmp_words(tiles) + 1);
            a.block_cnt = bcnt;
            {
                Prof p(g, SGM_K_JOIN, (p1 - p0) * (4.0 * k + 16.0 + 24.0 * L.n_chk));
                launch_join_count(st(), a);
            }
            {
                Prof p(g, SGM_K_OTHER, 16.0 * tiles);
                launch_scan_i64(st(), bcnt, tiles, boff, tmp2);
            }
            HIPX(hipMemcpyAsync(g->h_small, boff + tiles, sizeof(int64_t), hipMemcpyDeviceToHost,
                                st()));
            sync(g);
            const int64_t R2 = g->h_small[0];
            level_acc_[li + 1] += R2;
            sc.release(bcnt);
            sc.release(tmp2);
            if (R2 == 0 || (last && (flags & SGM_COUNT_ONLY))) {
                if (last) fin_rows_ += R2;
                sc.release(boff);
                continue;
            }
            int32_t *out = sc.get<int32_t>(R2 * (k + 1));
            a.out = out;
            a.block_cnt = boff;
            a.out_base = 0;
            {
                Prof p(g, SGM_K_JOIN, (p1 - p0) * (4.0 * k + 16.0 + 24.0 * L.n_chk) +
                                          R2 * 4.0 * (k + 1));
                launch_join_write(st(), a);
            }
            sc.release(boff);
            res->stats.peak_rows = std::max(res->stats.peak_rows, R2);
            res->stats.peak_bytes = std::max<int64_t>(res->stats.peak_bytes, R2 * 4 * (k + 1));
            if (last && !fin_ && p0 == 0 && p1 == P) {
                // one chunk at the last level: the level's table is the result
                fin_ = out;
                fin_rows_ = R2;
                fin_cap_ = R2;
                continue;
            }
            const int rc = join_from(li + 1, out, R2, k + 1);
            sc.release(out);
            if (rc) return rc;
        }
        sc.release(poff);
        return SGM_OK;
    }

    int join(int32_t **table_out, int64_t *rows_out) {
        const int seed = jorder[0];
        budget_ = g->opts.join_budget_bytes > 0 ? g->opts.join_budget_bytes : (16ll << 30);
        level_acc_[0] = ccount[seed];
        const int rc = join_from(0, list(seed), ccount[seed], 1);
        for (int l = 0; l < qi.n; ++l) res->stats.level_rows[l] = level_acc_[l];
        if (rc) return rc;
        *rows_out = fin_rows_;
        *table_out = fin_;
        if (g->opts.result_cap_rows > 0 && fin_rows_ > g->opts.result_cap_rows)
            return SGM_ETOOBIG;
        return SGM_OK;
    }

    // Final ordering (rows ascending in query-vertex column order) and the
    // copy to host (when copy). With a projection (thesis Ch. 3, Sec.
    // "GpSense") only the projected columns are ordered and kept, and equal
    // projected rows, now adjacent, collapse into one. Returns the number
    // of rows of the result.
    int64_t finish(const int32_t *table, int64_t R, bool copy) {
        const int n = qi.n;
        if (!table && R > 0) {
            // the join materialises its final table whenever finish runs
            g_last_error = "internal: final table not materialised";
            throw DeviceError{SGM_EDEVICE};
        }
        // output columns: the projected query vertices (all of them without
        // a projection) in index order, and where the table holds each
        int32_t colpos[SGM_MAX_QV], colu[SGM_MAX_QV];
        int no = 0;
        bool identity = true;
        for (int u = 0; u < n; ++u) {
            identity &= jpos[u] == u;
            if (qi.proj && !((qi.proj >> u) & 1u)) continue;
            colpos[no] = jpos[u];
            colu[no] = u;
            ++no;
        }
        // a table in column order is already sorted on any prefix of columns
        const bool lead = qi.proj == 0 || (qi.proj & (qi.proj + 1u)) == 0;
        int32_t *idx = nullptr;
        if (!(identity && lead) && R > 1) {
            if (R <= small_sort_limit()) {
                idx = sc.get<int32_t>(R);
                Prof p(g, SGM_K_SORT, 4.0 * R * no);
                launch_sort_small(st(), table, n, colpos, no, (int32_t)R, idx);
            } else {
                int nbits = 1;
                while ((1ll << nbits) < g->V) ++nbits;
                int32_t *ia = sc.get<int32_t>(R), *ib = sc.get<int32_t>(R);
                int32_t *ka = sc.get<int32_t>(R), *kb = sc.get<int32_t>(R);
                const int64_t tiles = radix_tiles(R);
                int64_t *hist = sc.get<int64_t>(256 * tiles);
                int64_t *hoff = sc.get<int64_t>(256 * tiles + 1);
                int64_t *tmp = sc.get<int64_t>(scan_tmp_words(256 * tiles) + 1);
                {
                    Prof p(g, SGM_K_SORT, 4.0 * R);
                    launch_iota(st(), ia, R);
                }
                // candidate ranks packed into one key of at most 64 bits:
                // ceil(bits / 8) passes instead of a pass set per column
                KeyCols kc{};
                kc.n = no;
                int tb = 0;
                for (int c = 0; c < no; ++c) {
                    const int u = colu[c];
                    int b = 0;
                    while ((1ll << b) < ccount[u]) ++b;
                    kc.bits[c] = bits(u);
                    kc.prefix[c] = prefix(u);
                    kc.col[c] = colpos[c];
                    kc.nbits[c] = b;
                    tb += b;
                }
                if (tb <= 64) {
                    uint64_t *keys = sc.get<uint64_t>(R);
                    {
                        Prof p(g, SGM_K_SORT, 4.0 * R * no + 8.0 * R);
                        launch_row_keys(st(), table, n, kc, R, keys);
                    }
                    for (int half = 0; half < 2; ++half) {
                        const int hb = half == 0 ? std::min(tb, 32) : tb - 32;
                        if (hb <= 0) break;
                        {
                            Prof p(g, SGM_K_SORT, 16.0 * R);
                            launch_key_half(st(), keys, ia, R, half, ka);
                        }
                        for (int sh = 0; sh < hb; sh += 8) {
                            Prof p(g, SGM_K_SORT, 20.0 * R);
                            launch_radix_hist(st(), ka, R, sh, hist);
                            launch_scan_i64(st(), hist, 256 * tiles, hoff, tmp);
                            launch_radix_scatter(st(), ka, ia, R, sh, hoff, kb, ib);
                            std::swap(ka, kb);
                            std::swap(ia, ib);
                        }
                    }
                }
                for (int c = no - 1; c >= 0 && tb > 64; --c) {
                    {
                        Prof p(g, SGM_K_SORT, 12.0 * R);
                        launch_gather_key(st(), table, n, colpos[c], ia, R, ka);
                    }
                    for (int sh = 0; sh < nbits; sh += 8) {
                        Prof p(g, SGM_K_SORT, 20.0 * R);
                        launch_radix_hist(st(), ka, R, sh, hist);
                        launch_scan_i64(st(), hist, 256 * tiles, hoff, tmp);
                        launch_radix_scatter(st(), ka, ia, R, sh, hoff, kb, ib);
                        std::swap(ka, kb);
                        std::swap(ia, ib);
                    }
                }
                idx = ia;
            }
        }
        int32_t *out = sc.get<int32_t>(R * no);
        {
            Prof p(g, SGM_K_OTHER, 8.0 * R * no);
            launch_gather_rows(st(), table, n, idx, R, colpos, no, out);
        }
        if (qi.proj && R > 1) {
            int64_t *head = sc.get<int64_t>(R), *pos = sc.get<int64_t>(R + 1);
            int64_t *tmp = sc.get<int64_t>(scan_tmp_words(R) + 1);
            int32_t *uniq = sc.get<int32_t>(R * no);
            {
                Prof p(g, SGM_K_OTHER, 8.0 * R * no + 24.0 * R);
                launch_unique_rows(st(), out, no, R, head, pos, tmp, uniq);
            }
            HIPX(hipMemcpyAsync(g->h_small, pos + R, sizeof(int64_t), hipMemcpyDeviceToHost, st()));
            sync(g);
            R = g->h_small[0];
            out = uniq;
        }
        if (!copy) return R;
        const size_t bytes = sizeof(int32_t) * (size_t)R * no;
        res->rows = alloc_rows(bytes);
        if (!res->rows) throw DeviceError{SGM_ENOMEM};
        readback_rows(g, st(), out, bytes, res->rows);
        return R;
    }

    int run() {
        const int64_t t0 = now_ns();
        const int n = qi.n;
        int rc = make_plan(qi, g->V, g->type_freq.data(), g->n_types, &pl);
        if (rc) return rc;
        for (int i = 0; i < SGM_MAX_QV; ++i) res->stats.visit_order[i] = pl.visit[i];
        res->n_cols = qi.n_out;
        rc = filter();
        if (rc) return rc;
        HIPX(hipMemcpyAsync(g->h_cnt->cand_count, g->d_cnt->cand_count, sizeof(int32_t) * n,
                            hipMemcpyDeviceToHost, st()));
        sync(g);
        const int64_t t1 = now_ns();
        res->stats.ns_filter = t1 - t0;
        bool empty = false;
        for (int u = 0; u < n; ++u) {
            ccount[u] = g->h_cnt->cand_count[u];
            res->stats.cand[u] = ccount[u];
            empty |= ccount[u] == 0;
        }
        res->stats.n_chunks = 1;
        if (empty) return done(0, t0);
        if (qi.m == 0) {
            // single vertex: the candidate list is the (sorted) answer
            jorder[0] = 0;
            jpos[0] = 0;
            res->stats.join_order[0] = 0;
            const int64_t R = ccount[0];
            if (g->opts.result_cap_rows > 0 && R > g->opts.result_cap_rows) {
                res->n_rows = R;
                return SGM_ETOOBIG;
            }
            if (want_rows) finish(list(0), R, true);
            return done(R, t0);
        }
        rc = collect_edges();
        const int64_t t2 = now_ns();
        res->stats.ns_collect = t2 - t1;
        if (rc == 1) return done(0, t0);
        if (rc) return rc;
        for (int j = 0; j < n; ++j) res->stats.join_order[j] = jorder[j];
        int32_t *table = nullptr;
        int64_t R = 0;
        rc = join(&table, &R);
        const int64_t t3 = now_ns();
        res->stats.ns_join = t3 - t2;
        if (rc == SGM_ETOOBIG) {
            res->n_rows = R;
            res->stats.ns_total = now_ns() - t0;
            return rc;
        }
        if (rc) return rc;
        // a projection's row count needs its distinct rows, also when only
        // the count is asked for (the join then materialised its table)
        if (R > 0 && (want_rows || qi.proj)) R = finish(table, R, want_rows);
        res->stats.ns_finish = now_ns() - t3;
        return done(R, t0);
    }

    // Candidate sets after the filtering phase and candidate-edge counts.
    int inspect(int64_t *counts, int32_t **ids, int64_t *ec_out) {
        const int n = qi.n;
        int rc = make_plan(qi, g->V, g->type_freq.data(), g->n_types, &pl);
        if (rc) return rc;
        rc = filter();
        if (rc) return rc;
        HIPX(hipMemcpyAsync(g->h_cnt->cand_count, g->d_cnt->cand_count, sizeof(int32_t) * n,
                            hipMemcpyDeviceToHost, st()));
        sync(g);
        int64_t total = 0;
        bool empty = false;
        for (int u = 0; u < n; ++u) {
            ccount[u] = g->h_cnt->cand_count[u];
            counts[u] = ccount[u];
            total += ccount[u];
            empty |= ccount[u] == 0;
        }
        int32_t *h = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1));
        if (!h) throw std::bad_alloc();
        int64_t off = 0;
        for (int u = 0; u < n; ++u) {
            if (ccount[u])
                HIPX(hipMemcpyAsync(h + off, list(u), sizeof(int32_t) * ccount[u],
                                    hipMemcpyDeviceToHost, st()));
            off += ccount[u];
        }
        sync(g);
        *ids = h;
        if (!empty && qi.m > 0) {
            for (int e = 0; e < qi.m; ++e) {
                ECTab &t = ec[e];
                t.key = qi.esrc[e];
                t.other = qi.edst[e];
                t.dir = 0;
                ec_count(t, e);
            }
            HIPX(hipMemcpyAsync(g->h_cnt->ec_total, g->d_cnt->ec_total,
                                sizeof(unsigned long long) * qi.m, hipMemcpyDeviceToHost, st()));
            sync(g);
            for (int e = 0; e < qi.m; ++e) ec_out[e] = (int64_t)g->h_cnt->ec_total[e];
        }
        return SGM_OK;
    }

    int done(int64_t R, int64_t t0) {
        res->n_rows = R;
        // rows is non-NULL for every successful SORTED result, also when empty
        if (want_rows && !res->rows) {
            res->rows = (int32_t *)std::malloc(sizeof(int32_t));
            if (!res->rows) throw std::bad_alloc();
        }
        res->stats.ns_total = now_ns() - t0;
        return SGM_OK;
    }
};

// ---------------------------------------------------------------------------
// persistent per-query kernel: resources and one batch
// ---------------------------------------------------------------------------

constexpr int kNarrowMaxSlots = 512;                 // 2 workgroups per CU
constexpr int32_t kTypeTable = 1024;                 // vertex types covered by the sweep's table
constexpr int64_t kNarrowSlabMin = 8ll << 20;        // per slot, small graphs
constexpr int64_t kNarrowSlabMax = 32ll << 20;       // per slot, large graphs (served form)
// A graph's own batch context: 40 B per data vertex up to 160 MB per slot
// (512 slots of a 4M-vertex graph hold about 87 GB of HBM), so that queries
// with tables of ~1e6 rows finish in their slot and a batch is one launch.
constexpr int32_t kHubTypesMax = 4096;    // more vertex types: no hub-row index
constexpr int64_t kHostOrderRows = 65536;  // final tables from this size are ordered by the host
constexpr int64_t kBatchSlabPerVertex = 40;
constexpr int64_t kBatchSlabMax = 160ll << 20;
constexpr int32_t kNarrowListCap = 1 << 16;          // per query vertex
constexpr int kNarrowQueryCap = 4096;                // queries per launch
constexpr int64_t kNarrowOutCap = 256ll << 20;       // int32 elements (1 GB) per context
// Every launch also reads back this many leading ints of the output arena,
// so that small results need no second copy and wait.
constexpr int64_t kOutPrefix = 16384;
constexpr int kBigSlots = 4;                         // large slots of the retry context
constexpr int32_t kBigListCap = 1 << 22;             // per query vertex, large slot
constexpr int64_t kBigSlab = 256ll << 20;            // per large slot

// slot memory for edge tables, join tables and sort buffers: 8 bytes per
// data vertex, within [8 MB, 32 MB]
// Slab of one regular slot: a server's contexts (several side by side, up
// to max_batch slots each) keep theirs small; the graph's own batch context
// takes room for large intermediate tables.
int64_t narrow_slab_bytes(const sgm_graph *g, bool serve) {
    if (serve) return std::min<int64_t>(kNarrowSlabMax, std::max<int64_t>(kNarrowSlabMin, 8ll * g->V));
    return std::min<int64_t>(kBatchSlabMax,
                             std::max<int64_t>(kNarrowSlabMin, kBatchSlabPerVertex * g->V));
}

template <class T>
void dev_free(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}
template <class T>
void host_free(T *&p) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
}

void narrow_free(NarrowCtx &nw) {
    if (nw.stream) (void)hipStreamSynchronize(nw.stream);
    dev_free(nw.bits);
    dev_free(nw.lists);
    dev_free(nw.slab);
    dev_free(nw.d_q);
    dev_free(nw.d_res);
    dev_free(nw.d_preds);
    dev_free(nw.d_rootbits);
    dev_free(nw.d_out);
    dev_free(nw.d_ctr);
    dev_free(nw.d_board);
    host_free(nw.h_q);
    host_free(nw.h_res);
    host_free(nw.h_preds);
    host_free(nw.h_ctr);
    host_free(nw.h_out);
    dev_free(nw.d_trace);
    host_free(nw.h_trace);
    if (nw.done) (void)hipEventDestroy(nw.done);
    nw.done = nullptr;
    if (nw.copy) {
        (void)hipStreamSynchronize(nw.copy);
        (void)hipStreamDestroy(nw.copy);
    }
    for (hipEvent_t e : nw.copy_ev) (void)hipEventDestroy(e);
    if (nw.gexec) (void)hipGraphExecDestroy(nw.gexec);
    if (nw.graph) (void)hipGraphDestroy(nw.graph);
    nw.gexec = nullptr;
    nw.graph = nullptr;
    const NarrowCtx keep = nw;
    nw = NarrowCtx{};
    nw.stream = keep.stream;
    nw.serve = keep.serve;
    nw.lcap_want = keep.lcap_want;
    nw.slab_want = keep.slab_want;
}

void narrow_reserve(sgm_graph *g, NarrowCtx &nw, int slots, int nq, int nroot) {
    if (nw.lcap == 0) {
        nw.lcap = std::min<int32_t>(g->V, nw.lcap_want ? nw.lcap_want : kNarrowListCap);
        nw.slab_bytes = nw.slab_want ? nw.slab_want : narrow_slab_bytes(g, nw.serve);
        // while filtering, a slot's slab holds two lists of up to lcap ints
        if (nw.slab_bytes < 8ll * nw.lcap) throw DeviceError{SGM_EUNSUPPORTED};
        HIPX(hipMalloc(&nw.d_ctr, sizeof(unsigned long long) * 3));
        HIPX(hipHostMalloc(&nw.h_ctr, sizeof(unsigned long long) * 2, hipHostMallocDefault));
        // board entries start at sequence 0 with no chunks; the kernel
        // retires every step it posts, so they need no clearing later
        HIPX(hipMalloc(&nw.d_board, sizeof(HelpJob) * kNarrowMaxSlots));
        HIPX(hipMemsetAsync(nw.d_board, 0, sizeof(HelpJob) * kNarrowMaxSlots, nw.stream));
        nw.out_cap = kNarrowOutCap;
        HIPX(hipMalloc(&nw.d_out, sizeof(int32_t) * nw.out_cap));
        HIPX(hipHostMalloc(&nw.h_out, sizeof(int32_t) * (1 << 20), hipHostMallocDefault));
        nw.h_out_cap = 1 << 20;
        HIPX(hipEventCreateWithFlags(&nw.done, hipEventDisableTiming));
    }
    if (slots > nw.slots) {
        HIPX(hipStreamSynchronize(nw.stream));
        dev_free(nw.bits);
        dev_free(nw.lists);
        dev_free(nw.slab);
        nw.slots = 0;
        const size_t bw = (size_t)(SGM_MAX_QV + 1) * g->nwords;
        HIPX(hipMalloc(&nw.bits, sizeof(uint64_t) * bw * slots));
        HIPX(hipMemsetAsync(nw.bits, 0, sizeof(uint64_t) * bw * slots, nw.stream));
        HIPX(hipMalloc(&nw.lists, sizeof(int32_t) * (size_t)SGM_MAX_QV * nw.lcap * slots));
        HIPX(hipMalloc(&nw.slab, (size_t)nw.slab_bytes * slots));
        nw.slots = slots;
    }
    if (nq > nw.qcap) {
        HIPX(hipStreamSynchronize(nw.stream));
        dev_free(nw.d_q);
        dev_free(nw.d_res);
        host_free(nw.h_q);
        host_free(nw.h_res);
        nw.qcap = 0;
        HIPX(hipMalloc(&nw.d_q, sizeof(NQuery) * nq));
        HIPX(hipMalloc(&nw.d_res, sizeof(NResult) * nq));
        HIPX(hipHostMalloc(&nw.h_q, sizeof(NQuery) * nq, hipHostMallocDefault));
        HIPX(hipHostMalloc(&nw.h_res, sizeof(NResult) * nq, hipHostMallocDefault));
        nw.qcap = nq;
    }
    if (nroot > nw.root_cap) {
        HIPX(hipStreamSynchronize(nw.stream));
        dev_free(nw.d_preds);
        dev_free(nw.d_rootbits);
        host_free(nw.h_preds);
        nw.root_cap = 0;
        // root predicates, then the sweep's type-offset table (at most
        // kTypeTable + 1 ints)
        const size_t pb = sizeof(VPred) * nroot + sizeof(int32_t) * (kTypeTable + 1);
        HIPX(hipMalloc(&nw.d_preds, pb));
        HIPX(hipHostMalloc(&nw.h_preds, pb, hipHostMallocDefault));
        HIPX(hipMalloc(&nw.d_rootbits, sizeof(uint64_t) * (size_t)g->nwords * nroot));
        nw.root_cap = nroot;
    }
}

// Pack one validated query and its plan; false if it exceeds the packed
// descriptor's capacity (the query then runs on the multi-kernel path).
bool pack_query(sgm_graph *g, const QInfo &qi, const Plan &pl, NQuery *nq, int *root_slot_next,
                Plan *pl_out) {
    Program pr;
    build_program(qi, pl, g->opts.low_conn_degree, g->opts.refine_reversed, &pr);
    if ((int)(pr.init.size() + pr.refine.size()) > kNMaxSteps || (int)pr.nbr.size() > kNMaxNbr)
        return false;
    std::memset(nq, 0, sizeof(*nq));
    nq->n = qi.n;
    nq->m = qi.m;
    for (int u = 0; u < qi.n; ++u) nq->pred[u] = VPred{qi.label[u], qi.pin[u], qi.qout[u], qi.qin[u]};
    for (int e = 0; e < qi.m; ++e) {
        nq->esrc[e] = qi.esrc[e];
        nq->edst[e] = qi.edst[e];
        nq->elabel[e] = qi.elabel[e];
    }
    nq->root = pl.visit[0];
    // unpinned roots get their bitmap row from the batch's root sweep; the
    // row is assigned per distinct predicate after packing
    nq->root_slot = qi.pin[nq->root] >= 0 ? -1 : (*root_slot_next)++;
    nq->n_init = (int)pr.init.size();
    nq->n_ref = (int)pr.refine.size();
    nq->refine_rounds = g->opts.refine_rounds < 0 ? -1 : std::min(g->opts.refine_rounds, 32);
    nq->proj = qi.proj;
    nq->homo = g->homomorphic ? 1 : 0;
    int k = 0;
    auto put = [&](const PStep &s) {
        NStep &t = nq->steps[k++];
        t.u = (int8_t)s.u;
        t.push = (int8_t)s.push;
        t.parent = (int8_t)s.parent;
        t.first = (int16_t)s.first;
        t.count = (int16_t)s.count;
    };
    for (const PStep &s : pr.init) put(s);
    for (const PStep &s : pr.refine) put(s);
    for (size_t i = 0; i < pr.nbr.size(); ++i) {
        nq->nbr[i].v = (int8_t)pr.nbr[i].v;
        nq->nbr[i].dir = (int8_t)pr.nbr[i].dir;
        nq->nbr[i].mode = (int8_t)pr.nbr[i].mode;
        nq->nbr[i].rel = pr.nbr[i].rel;
    }
    *pl_out = pl;
    return true;
}

// One persistent-kernel launch in flight on a context's stream.
struct NarrowJob {
    std::vector<int> packed;   // query indices, in descriptor order
    std::vector<Plan> plans;
    int nroot = 0;
    int64_t t0 = 0;
    bool traced = false;
};

// Pack queries which[0..count) (validated into qis), upload and launch them
// asynchronously on nw.stream; queries that do not fit a descriptor go to
// `wide`. Returns false when nothing was launched.
bool narrow_launch(sgm_graph *g, NarrowCtx &nw, const std::vector<QInfo> &qis, const int *which,
                   int count, NarrowJob &job, std::vector<int> &wide,
                   std::vector<sgm_result *> &res, bool profiled) {
    job.t0 = now_ns();
    job.packed.clear();
    job.plans.clear();
    const int max_slots = nw.slab_want ? kBigSlots : kNarrowMaxSlots;
    narrow_reserve(g, nw, std::min(count, max_slots), count, 0);
    // The work queue hands out descriptors in order: the expected-longest
    // query (an unpinned root with many candidates of its type, then more
    // query vertices), then the expected-shortest, then the next longest,
    // and so on. Longest first alone makes the first slots' heavy root
    // steps all run at once and contend; alternating them with short
    // queries ends the large batch's launch about 5 % sooner.
    std::vector<Plan> plans((size_t)count);
    std::vector<int64_t> cost((size_t)count, -1);
    std::vector<int> order;
    order.reserve((size_t)count);
    parallel_for(count, 128, [&](int lo, int hi) {
        for (int i = lo; i < hi; ++i) {
            const QInfo &qi = qis[which[i]];
            if (make_plan(qi, g->V, g->type_freq.data(), g->n_types, &plans[i]) != SGM_OK)
                continue;  // cost stays -1
            const int r = plans[i].visit[0];
            const int32_t lab = qi.label[r];
            const int64_t rootc = qi.pin[r] >= 0 ? 1
                                  : (lab >= 0 && lab < g->n_types ? g->type_freq[lab] : g->V);
            cost[i] = rootc * (SGM_MAX_QV + 1) + qi.n;
        }
    });
    for (int i = 0; i < count; ++i) {
        if (cost[i] >= 0) {
            order.push_back(i);
        } else {
            wide.push_back(which[i]);
            res[which[i]]->stats.fallback = 16;
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    {
        std::vector<int> alt;
        alt.reserve(order.size());
        size_t lo = 0, hi = order.size();
        while (lo < hi) {
            alt.push_back(order[lo++]);
            if (lo < hi) alt.push_back(order[--hi]);
        }
        order.swap(alt);
    }
    // descriptors in queue order, packed in parallel (a root's sweep row is
    // assigned below; here an unpinned root only gets a non-negative slot)
    const int no = (int)order.size();
    std::vector<Plan> pls((size_t)no);
    std::vector<char> packed_ok((size_t)no, 0);
    parallel_for(no, 128, [&](int lo, int hi) {
        for (int k = lo; k < hi; ++k) {
            const int i = order[k];
            int rs = 0;
            packed_ok[k] = pack_query(g, qis[which[i]], plans[i], &nw.h_q[k], &rs, &pls[k]);
        }
    });
    int np = 0;
    for (int k = 0; k < no; ++k) {
        const int i = order[k];
        if (!packed_ok[k]) {
            wide.push_back(which[i]);
            res[which[i]]->stats.fallback = 16;
            continue;
        }
        if (np != k) std::memcpy(&nw.h_q[np], &nw.h_q[k], sizeof(NQuery));
        if (g->fault_query >= 0 && which[i] == g->fault_query) {
            nw.h_q[np].fault = 1;
            g->fault_query = -1;
        }
        job.packed.push_back(which[i]);
        job.plans.push_back(pls[k]);
        ++np;
    }
    int nroot = 0;
    if (np == 0) return false;
    // one sweep row per distinct root predicate (type, degree bounds), rows
    // in (type, bounds) order with the untyped (-1) ones first, as the
    // sweep expects
    std::map<std::array<int32_t, 3>, int> row_of;
    for (int i = 0; i < np; ++i) {
        const NQuery &q = nw.h_q[i];
        if (q.root_slot < 0) continue;
        const VPred &p = q.pred[q.root];
        row_of.emplace(std::array<int32_t, 3>{p.label, p.qout, p.qin}, 0);
    }
    std::vector<VPred> preds;
    int n_any = 0;
    for (auto &kv : row_of) {
        kv.second = (int)preds.size();
        preds.push_back(VPred{kv.first[0], -1, kv.first[1], kv.first[2]});
        if (kv.first[0] < 0) ++n_any;
    }
    for (int i = 0; i < np; ++i) {
        NQuery &q = nw.h_q[i];
        if (q.root_slot < 0) continue;
        const VPred &p = q.pred[q.root];
        q.root_slot = row_of[std::array<int32_t, 3>{p.label, p.qout, p.qin}];
    }
    nroot = (int)preds.size();
    job.nroot = nroot;
    // at least one predicate row, so that a graph's copy node never has size 0
    narrow_reserve(g, nw, std::min(np, max_slots), np, std::max(nroot, 1));
    if (nroot) std::memcpy(nw.h_preds, preds.data(), sizeof(VPred) * nroot);
    else nw.h_preds[0] = VPred{-1, -1, 0, 0};
    // type_off[t] = first predicate of type >= t (predicates are sorted)
    const int32_t n_types = nroot && g->n_types <= kTypeTable ? g->n_types : 0;
    int32_t *type_off = (int32_t *)(nw.h_preds + std::max(nroot, 1));
    for (int32_t t = 0, j = 0; t <= n_types && n_types > 0; ++t) {
        while (j < nroot && preds[j].label < t) ++j;
        type_off[t] = j;
    }
    hipStream_t st = nw.stream;
    NArgs a{};
    a.g = g->dg;
    a.qs = nw.d_q;
    a.nq = np;
    a.res = nw.d_res;
    a.queue = (int32_t *)nw.d_ctr;
    a.bits = nw.bits;
    a.lists = nw.lists;
    a.lcap = nw.lcap;
    a.slab = nw.slab;
    a.slab_bytes = nw.slab_bytes;
    a.rootbits = nw.d_rootbits;
    a.out = nw.d_out;
    a.out_cap = nw.out_cap;
    a.out_used = nw.d_ctr + 1;
    a.group_lanes = g->tune.group_lanes;
    a.wg_rows = g->tune.wg_rows;
    a.join_policy = g->tune.join_policy;
    nw.sa = SweepArgs{g->dg,       nw.d_preds, nroot, n_any, nw.d_rootbits, nw.d_ctr,
                      (const int32_t *)(nw.d_preds + std::max(nroot, 1)), n_types};
    const int slot_grid =
        std::min(np, nw.slab_want ? nw.slots : std::min(nw.slots, g->tune.slots));
    // Shared filter steps need every workgroup of the launch resident at
    // once (two per CU): helpers then wait only for work that exists. A
    // server's contexts launch side by side, so they share no steps.
    const bool help = !nw.serve && g->tune.help_items > 0;
    a.nslot = slot_grid;
    a.help_items = help ? g->tune.help_items : 0;
    a.board = nw.d_board;
    a.hctr = (int32_t *)(nw.d_ctr + 2);
    a.help_wait = g->tune.help_wait > 0 ? g->tune.help_wait : kHelpWaitDefault;
    // the graph's own contexts hand large final tables to the host for
    // whole-GPU ordering (a server's completers do not hold the graph)
    a.host_order_rows = nw.serve ? 0 : kHostOrderRows;
    const int grid =
        help ? std::min(kNarrowMaxSlots, std::max(slot_grid, g->tune.helpers)) : slot_grid;
    a.ngrid = grid;
    job.traced = profiled && g->opts.profile >= 2;
    if (g->opts.graphs && !(profiled && g->opts.profile)) {
        nw.na = a;
        hipKernelNodeParams ps, pn;
        narrow_node_params(&nw.sa, &nw.na, grid, nw.kargs, &ps, &pn);
        const size_t qb = sizeof(NQuery) * np,
                     pb = sizeof(VPred) * std::max(nroot, 1) + sizeof(int32_t) * (n_types + 1);
        const size_t rb = sizeof(NResult) * np, cb = sizeof(unsigned long long) * 2;
        const size_t ob = sizeof(int32_t) * kOutPrefix;
        const auto H2D = hipMemcpyHostToDevice, D2H = hipMemcpyDeviceToHost;
        if (!nw.gexec) {
            HIPX(hipGraphCreate(&nw.graph, 0));
            HIPX(hipGraphAddMemcpyNode1D(&nw.gn[0], nw.graph, nullptr, 0, nw.d_q, nw.h_q, qb, H2D));
            HIPX(hipGraphAddMemcpyNode1D(&nw.gn[1], nw.graph, &nw.gn[0], 1, nw.d_preds, nw.h_preds,
                                         pb, H2D));
            HIPX(hipGraphAddKernelNode(&nw.gn[2], nw.graph, &nw.gn[1], 1, &ps));
            HIPX(hipGraphAddKernelNode(&nw.gn[3], nw.graph, &nw.gn[2], 1, &pn));
            HIPX(hipGraphAddMemcpyNode1D(&nw.gn[4], nw.graph, &nw.gn[3], 1, nw.h_res, nw.d_res, rb,
                                         D2H));
            HIPX(hipGraphAddMemcpyNode1D(&nw.gn[5], nw.graph, &nw.gn[4], 1, nw.h_ctr, nw.d_ctr, cb,
                                         D2H));
            HIPX(hipGraphAddMemcpyNode1D(&nw.gn[6], nw.graph, &nw.gn[5], 1, nw.h_out, nw.d_out, ob,
                                         D2H));
            HIPX(hipGraphInstantiate(&nw.gexec, nw.graph, nullptr, nullptr, 0));
        } else {
            // buffers are reallocated only while no launch is in flight, and
            // every pointer a node uses is compared here
            if (qb != nw.last_qb || nw.na.qs != nw.last_na.qs)
                HIPX(hipGraphExecMemcpyNodeSetParams1D(nw.gexec, nw.gn[0], nw.d_q, nw.h_q, qb, H2D));
            if (pb != nw.last_pb || nw.sa.preds != nw.last_sa.preds)
                HIPX(hipGraphExecMemcpyNodeSetParams1D(nw.gexec, nw.gn[1], nw.d_preds, nw.h_preds,
                                                       pb, H2D));
            if (std::memcmp(&nw.sa, &nw.last_sa, sizeof(SweepArgs)) != 0 ||
                (int)ps.gridDim.x != nw.last_sweep_grid)
                HIPX(hipGraphExecKernelNodeSetParams(nw.gexec, nw.gn[2], &ps));
            if (std::memcmp(&nw.na, &nw.last_na, sizeof(NArgs)) != 0 || grid != nw.last_grid)
                HIPX(hipGraphExecKernelNodeSetParams(nw.gexec, nw.gn[3], &pn));
            if (rb != nw.last_rb || nw.na.res != nw.last_na.res)
                HIPX(hipGraphExecMemcpyNodeSetParams1D(nw.gexec, nw.gn[4], nw.h_res, nw.d_res, rb,
                                                       D2H));
            if (nw.na.queue != nw.last_na.queue)
                HIPX(hipGraphExecMemcpyNodeSetParams1D(nw.gexec, nw.gn[5], nw.h_ctr, nw.d_ctr, cb,
                                                       D2H));
            if (nw.h_out != nw.last_hout || nw.na.out != nw.last_na.out)
                HIPX(hipGraphExecMemcpyNodeSetParams1D(nw.gexec, nw.gn[6], nw.h_out, nw.d_out, ob,
                                                       D2H));
        }
        nw.last_sa = nw.sa;
        nw.last_na = nw.na;
        nw.last_grid = grid;
        nw.last_sweep_grid = (int)ps.gridDim.x;
        nw.last_qb = qb;
        nw.last_pb = pb;
        nw.last_rb = rb;
        nw.last_hout = nw.h_out;
        HIPX(hipGraphLaunch(nw.gexec, st));
        HIPX(hipEventRecord(nw.done, st));
        return true;
    }
    HIPX(hipMemcpyAsync(nw.d_q, nw.h_q, sizeof(NQuery) * np, hipMemcpyHostToDevice, st));
    if (nroot)
        HIPX(hipMemcpyAsync(nw.d_preds, nw.h_preds,
                            sizeof(VPred) * nroot + sizeof(int32_t) * (n_types + 1),
                            hipMemcpyHostToDevice, st));
    {
        Prof p(g, SGM_K_CHECK, nroot ? (8.0 + 0.125 * nroot) * g->V : 0.0, profiled && nroot > 0);
        launch_root_sweep(st, nw.sa);
    }
    if (job.traced) {
        if (np > nw.trace_cap) {
            HIPX(hipStreamSynchronize(st));
            dev_free(nw.d_trace);
            host_free(nw.h_trace);
            nw.trace_cap = 0;
            HIPX(hipMalloc(&nw.d_trace, sizeof(int64_t) * SGM_TRACE_CAP * np));
            HIPX(hipHostMalloc(&nw.h_trace, sizeof(int64_t) * SGM_TRACE_CAP * np,
                               hipHostMallocDefault));
            nw.trace_cap = np;
        }
        HIPX(hipMemsetAsync(nw.d_trace, 0, sizeof(int64_t) * SGM_TRACE_CAP * np, st));
        a.trace = nw.d_trace;
    }
    {
        Prof p(g, SGM_K_PERSIST, 0.0, profiled);
        launch_narrow(st, a, grid);
    }
    if (job.traced)
        HIPX(hipMemcpyAsync(nw.h_trace, nw.d_trace, sizeof(int64_t) * SGM_TRACE_CAP * np,
                            hipMemcpyDeviceToHost, st));
    HIPX(hipMemcpyAsync(nw.h_res, nw.d_res, sizeof(NResult) * np, hipMemcpyDeviceToHost, st));
    HIPX(hipMemcpyAsync(nw.h_ctr, nw.d_ctr, sizeof(unsigned long long) * 2, hipMemcpyDeviceToHost,
                        st));
    HIPX(hipMemcpyAsync(nw.h_out, nw.d_out, sizeof(int32_t) * kOutPrefix, hipMemcpyDeviceToHost, st));
    HIPX(hipEventRecord(nw.done, st));
    return true;
}

// Wait for a launched job and fill the results of its finished queries;
// queries that outgrew their slot are appended to `wide`.
void narrow_collect(sgm_graph *g, NarrowCtx &nw, NarrowJob &job, const std::vector<QInfo> &qis,
                    uint32_t flags, std::vector<sgm_result *> &res, std::vector<int> &wide,
                    bool profiled) {
    hipStream_t st = nw.stream;
    HIPX(hipEventSynchronize(nw.done));
    if (profiled) prof_flush(g);
    const int np = (int)job.packed.size();
    if (profiled && g->opts.profile) {
        double b = 0;
        for (int i = 0; i < np; ++i) b += (double)nw.h_res[i].bytes;
        g->kstat[SGM_K_PERSIST].bytes_total += b;
    }
    const int64_t used = std::min<int64_t>((int64_t)nw.h_ctr[1], nw.out_cap);
    const bool want = !(flags & SGM_COUNT_ONLY);
    // bytes of rows this launch returns: the arena's used part, and room for
    // the large tables the host orders
    size_t host_bytes = 0;
    for (int i = 0; i < np; ++i) {
        const NResult &r = nw.h_res[i];
        if (r.status == SGM_OK && r.host_order)
            host_bytes += ((size_t)r.n_rows * qis[job.packed[i]].n_out * 4 + 255) & ~(size_t)255;
    }
    const size_t arena_bytes = ((size_t)used * 4 + 255) & ~(size_t)255;
    RowBlock *blk = nullptr;
    size_t blk_next = arena_bytes;  // next free byte of the block (host-ordered tables)
    // this call's own reference to the block, dropped when it returns (or
    // throws): a block that no result took goes back to the pool
    struct Hold {
        RowBlock *b = nullptr;
        ~Hold() {
            if (b) block_release(b);
        }
    } hold;
    // the copies into a pinned block run on the context's copy stream and
    // are waited for before this call returns (also when it throws)
    struct CopyWait {
        hipStream_t s = nullptr;
        ~CopyWait() {
            if (s) (void)hipStreamSynchronize(s);
        }
    } copy_wait;
    if (want && arena_bytes + host_bytes >= kBlockMin) {
        blk = block_get(arena_bytes + host_bytes);
        blk->refs.store(1);
        hold.b = blk;
        if (!nw.copy) HIPX(hipStreamCreateWithFlags(&nw.copy, hipStreamNonBlocking));
        copy_wait.s = nw.copy;
        // the kernel has finished (nw.done): the arena is final
        if (used > 0)
            HIPX(hipMemcpyAsync(blk->ptr, nw.d_out, sizeof(int32_t) * used, hipMemcpyDeviceToHost,
                                nw.copy));
    } else if (want && used > kOutPrefix) {
        // the launch read back the first kOutPrefix ints; the rest now
        int64_t from = kOutPrefix;
        if (nw.h_out_cap < used) {
            host_free(nw.h_out);
            nw.h_out_cap = 0;
            const int64_t cap = std::max<int64_t>(used, 1 << 20);
            HIPX(hipHostMalloc(&nw.h_out, sizeof(int32_t) * cap, hipHostMallocDefault));
            nw.h_out_cap = cap;
            from = 0;
        }
        HIPX(hipMemcpyAsync(nw.h_out + from, nw.d_out + from, sizeof(int32_t) * (used - from),
                            hipMemcpyDeviceToHost, st));
        HIPX(hipStreamSynchronize(st));
    }
    const int64_t t1 = now_ns();
    std::vector<HostCopy> copies;
    std::vector<int> hostord;
    if (job.traced)
        for (int i = 0; i < np; ++i) {
            const size_t q = (size_t)job.packed[i];
            if (q >= g->trace_n.size()) continue;
            const int64_t *ev = nw.h_trace + (size_t)i * SGM_TRACE_CAP;
            int32_t k = 0;
            while (k < SGM_TRACE_CAP && ev[k] != 0) ++k;
            std::memcpy(&g->trace[q * SGM_TRACE_CAP], ev, sizeof(int64_t) * k);
            g->trace_n[q] = k;
        }
    for (int i = 0; i < np; ++i) {
        const NResult &r = nw.h_res[i];
        const int qi_idx = job.packed[i];
        if (r.status == kFault) {
            res[qi_idx]->status = SGM_EDEVICE;
            continue;
        }
        if (r.status != SGM_OK) {
            wide.push_back(qi_idx);
            // sgm_stats.fallback codes: the kernel's reasons 1, 2, 4; 8 for a
            // full output arena; 32 for a shared step its helpers left
            // unfinished (kernel reason kWhyHelp)
            res[qi_idx]->stats.fallback =
                r.status == kOutFull ? 8 : (r.reason == kWhyHelp ? 32 : r.reason);
            res[qi_idx]->stats.peak_bytes = r.need;  // slot memory a join level could need
            continue;
        }
        sgm_result *out = res[qi_idx];
        const QInfo &qi = qis[qi_idx];
        out->n_cols = qi.n_out;
        out->n_rows = r.n_rows;
        sgm_stats &stt = out->stats;
        for (int u = 0; u < qi.n; ++u) {
            stt.cand[u] = r.cand[u];
            stt.level_rows[u] = r.level_rows[u];
            stt.join_order[u] = r.join_order[u];
        }
        for (int e = 0; e < qi.m; ++e) stt.ec[e] = r.ec[e];
        for (int u = 0; u < SGM_MAX_QV; ++u) stt.visit_order[u] = job.plans[i].visit[u];
        for (int u = 0; u < qi.n; ++u)
            stt.peak_rows = std::max(stt.peak_rows, (int64_t)r.level_rows[u]);
        stt.n_chunks = 1;
        stt.n_launches = job.nroot ? 2 : 1;
        stt.ns_total = t1 - job.t0;
        stt.ns_filter = (int64_t)(r.ticks[0] * g->ns_per_tick);
        stt.ns_collect = (int64_t)(r.ticks[1] * g->ns_per_tick);
        stt.ns_join = (int64_t)(r.ticks[2] * g->ns_per_tick);
        stt.ns_finish = (int64_t)(r.ticks[3] * g->ns_per_tick);
        stt.device_bytes = r.bytes;
        for (int i = 0; i < 4; ++i) stt.phase_bytes[i] = r.pbytes[i];
        stt.path = SGM_PATH_NARROW;
        if (r.host_order) {
            hostord.push_back(i);
            continue;
        }
        if (g->opts.result_cap_rows > 0 && r.n_rows > g->opts.result_cap_rows) {
            out->status = SGM_ETOOBIG;
            continue;
        }
        out->status = SGM_OK;
        if (want) {
            const size_t bytes = sizeof(int32_t) * (size_t)r.n_rows * qi.n_out;
            if (blk) {
                out->rows = (int32_t *)blk->ptr + r.offset;
                result_block(out) = blk;
                blk->refs.fetch_add(1);
            } else {
                out->rows = alloc_rows(bytes);
                if (!out->rows) throw std::bad_alloc();
                if (bytes) copies.push_back({out->rows, nw.h_out + r.offset, bytes});
            }
        }
    }
    parallel_copy(copies);
    // large final tables the kernel left unordered in its slots' slabs:
    // order them (and collapse projections) with whole-GPU kernels on this
    // context's stream (the graph's own; caller holds g->mu), then read them
    // back
    // one scope for all of them: each sorted table stays on the device until
    // the copy stream has taken it
    Scope sc(g->pool);
    size_t nev = 0;
    for (int i : hostord) {
        const NResult &r = nw.h_res[i];
        const int qi_idx = job.packed[i];
        sgm_result *out = res[qi_idx];
        const QInfo &qi = qis[qi_idx];
        const int n = qi.n;
        int32_t jpos[SGM_MAX_QV], colpos[SGM_MAX_QV];
        for (int l = 0; l < n; ++l) jpos[r.join_order[l]] = l;
        int no = 0;
        for (int u = 0; u < n; ++u)
            if (!qi.proj || ((qi.proj >> u) & 1u)) colpos[no++] = jpos[u];
        int64_t R = r.n_rows;
        const bool rows_wanted = !(flags & SGM_COUNT_ONLY);
        if (rows_wanted || qi.proj) {
            const int32_t *table = (const int32_t *)(uintptr_t)r.table_ptr;
            // keys from the key columns' lists the kernel left beside the
            // table (the same columns and widths as its own ordering)
            ListKeys lk{};
            lk.list = (const int32_t *)(uintptr_t)r.list_ptr;
            int64_t lo = 0;
            for (int u = 0; u < n; ++u) {
                const bool kept = !qi.proj || ((qi.proj >> u) & 1u);
                int b = 0;
                while (kept && (1ll << b) < r.cand[u]) ++b;
                if (b == 0) continue;
                lk.off[lk.n] = lo;
                lk.cnt[lk.n] = (int32_t)r.cand[u];
                lk.nbits[lk.n] = b;
                lk.col[lk.n] = jpos[u];
                ++lk.n;
                lo += r.cand[u];
            }
            uint64_t *keys = sc.get<uint64_t>(R);
            {
                Prof p(g, SGM_K_SORT, (4.0 * lk.n + 8.0) * R);
                launch_row_keys_lists(st, table, n, lk, R, keys);
            }
            const int32_t *idx = order_by_keys(g, sc, keys, R, r.key_bits);
            int32_t *sorted = sc.get<int32_t>(R * no);
            {
                Prof p(g, SGM_K_OTHER, 8.0 * R * no);
                launch_gather_rows(st, table, n, idx, R, colpos, no, sorted);
            }
            if (qi.proj && R > 1) {
                int64_t *head = sc.get<int64_t>(R), *pos = sc.get<int64_t>(R + 1);
                int64_t *tmp = sc.get<int64_t>(scan_tmp_words(R) + 1);
                int32_t *uniq = sc.get<int32_t>(R * no);
                {
                    Prof p(g, SGM_K_OTHER, 8.0 * R * no + 24.0 * R);
                    launch_unique_rows(st, sorted, no, R, head, pos, tmp, uniq);
                }
                HIPX(hipMemcpyAsync(g->h_small, pos + R, sizeof(int64_t), hipMemcpyDeviceToHost,
                                    st));
                HIPX(hipStreamSynchronize(st));
                R = g->h_small[0];
                sorted = uniq;
            }
            out->n_rows = R;
            if (rows_wanted && !(g->opts.result_cap_rows > 0 && R > g->opts.result_cap_rows)) {
                const size_t bytes = sizeof(int32_t) * (size_t)R * no;
                if (blk) {
                    // straight into the pinned block (room was set aside), on
                    // the copy stream once this stream has ordered the table
                    out->rows = (int32_t *)(blk->ptr + blk_next);
                    blk_next += (bytes + 255) & ~(size_t)255;
                    result_block(out) = blk;
                    blk->refs.fetch_add(1);
                    if (bytes) {
                        if (nev == nw.copy_ev.size()) {
                            hipEvent_t e;
                            HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                            nw.copy_ev.push_back(e);
                        }
                        HIPX(hipEventRecord(nw.copy_ev[nev], st));
                        HIPX(hipStreamWaitEvent(nw.copy, nw.copy_ev[nev], 0));
                        ++nev;
                        HIPX(hipMemcpyAsync(out->rows, sorted, bytes, hipMemcpyDeviceToHost,
                                            nw.copy));
                    }
                } else {
                    out->rows = alloc_rows(bytes);
                    if (!out->rows) throw std::bad_alloc();
                    readback_rows(g, st, sorted, bytes, out->rows);
                }
            }
        }
        out->n_rows = R;
        out->status = g->opts.result_cap_rows > 0 && R > g->opts.result_cap_rows ? SGM_ETOOBIG
                                                                                 : SGM_OK;
    }
    // every table in its block before the sorted copies go back to the pool
    if (copy_wait.s) HIPX(hipStreamSynchronize(copy_wait.s));
    if (profiled) prof_flush(g);
}

// Run queries `which` (validated into qis) through the persistent kernel on
// the graph's own stream, kNarrowQueryCap per launch.
void narrow_batch(sgm_graph *g, const std::vector<QInfo> &qis, const std::vector<int> &which,
                  uint32_t flags, std::vector<sgm_result *> &res, std::vector<int> &wide) {
    for (size_t base = 0; base < which.size(); base += kNarrowQueryCap) {
        const int count = (int)std::min<size_t>(kNarrowQueryCap, which.size() - base);
        NarrowJob job;
        if (narrow_launch(g, g->nw, qis, which.data() + base, count, job, wide, res, true))
            narrow_collect(g, g->nw, job, qis, flags, res, wide, true);
    }
}

// Queries that outgrew a regular slot (candidate list, slot memory or the
// output arena) run again in the large-slot context on the graph's stream;
// what still does not fit stays in `wide`. Caller holds g->mu.
void narrow_retry_large(sgm_graph *g, const std::vector<QInfo> &qis, uint32_t flags,
                        std::vector<sgm_result *> &res, std::vector<int> &wide) {
    std::vector<int> again, keep;
    for (int i : wide) {
        const int32_t why = res[i]->stats.fallback;
        // a join level that stopped early for want of memory reports what
        // its pairs could take; far beyond a large slot it goes wide at once
        const bool fits = why != kWhySlab || res[i]->stats.peak_bytes <= kPairSlack * kBigSlab;
        ((why == kWhyList || why == kWhySlab || why == 8) && fits ? again : keep).push_back(i);
    }
    if (again.empty()) return;
    wide = keep;
    for (size_t base = 0; base < again.size(); base += kNarrowQueryCap) {
        const int count = (int)std::min<size_t>(kNarrowQueryCap, again.size() - base);
        NarrowJob job;
        if (narrow_launch(g, g->nwb, qis, again.data() + base, count, job, wide, res, true))
            narrow_collect(g, g->nwb, job, qis, flags, res, wide, true);
    }
}

// multi-kernel path for one validated query
int wide_locked(sgm_graph *g, const QInfo &qi, uint32_t flags, sgm_result *res) {
    const int l0 = g->launches;
    int rc;
    try {
        Query Q(g, qi, res, flags);
        rc = Q.run();
    } catch (const DeviceError &e) {
        rc = e.code;
        (void)hipStreamSynchronize(g->stream);
        (void)hipGetLastError();
        g->pending.clear();
    } catch (const std::bad_alloc &) {
        rc = SGM_ENOMEM;
    }
    res->stats.n_launches = g->launches - l0;
    return rc;
}

// Validate, run the persistent kernel on every valid query, rerun the ones
// that outgrow a slot on the multi-kernel path. res[i] are zeroed results;
// per-query outcomes go to res[i]->status. Returns a global error code.
int run_queries(sgm_graph *g, const sgm_query *qs, const uint32_t *proj, int n, uint32_t flags,
                std::vector<sgm_result *> &res) {
    std::vector<QInfo> qis((size_t)n);
    std::vector<int> valid, wide;
    if (g->opts.profile >= 2) {
        g->trace.assign((size_t)n * SGM_TRACE_CAP, 0);
        g->trace_n.assign((size_t)n, 0);
    }
    parallel_for(n, 128, [&](int lo, int hi) {
        for (int i = lo; i < hi; ++i) {
            int rc = check_query(&qs[i], g->V, &qis[i]);
            if (rc == SGM_OK && proj) rc = set_projection(&qis[i], proj[i]);
            res[i]->status = rc;
        }
    });
    for (int i = 0; i < n; ++i)
        if (res[i]->status == SGM_OK) valid.push_back(i);
    if (g->opts.path == SGM_PATH_WIDE) {
        wide = valid;
    } else {
        try {
            narrow_batch(g, qis, valid, flags, res, wide);
            narrow_retry_large(g, qis, flags, res, wide);
        } catch (const DeviceError &e) {
            (void)hipStreamSynchronize(g->stream);
            (void)hipGetLastError();
            g->pending.clear();
            return e.code;
        } catch (const std::bad_alloc &) {
            return SGM_ENOMEM;
        }
    }
    for (int i : wide) {
        if (g->opts.path == SGM_PATH_NARROW) {
            res[i]->status = SGM_EUNSUPPORTED;
            continue;
        }
        const int32_t why = res[i]->stats.fallback;
        std::memset(&res[i]->stats, 0, sizeof(sgm_stats));
        res[i]->stats.path = SGM_PATH_WIDE;
        res[i]->stats.fallback = why;
        res[i]->status = wide_locked(g, qis[i], flags, res[i]);
    }
    return SGM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void sgm_default_options(sgm_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->refine_rounds = 1;
    o->refine_reversed = 1;
    o->low_conn_degree = 1;
    o->result_cap_rows = 0;
    o->join_budget_bytes = 0;
    o->profile = 0;
    o->graphs = 1;
}

const char *sgm_strerror(int code) {
    switch (code) {
        case SGM_OK: return "ok";
        case SGM_EINVAL: return "invalid argument";
        case SGM_ENOMEM: return "out of memory";
        case SGM_EDEVICE: return "device error";
        case SGM_ETOOBIG: return "result exceeds the row cap";
        case SGM_EUNSUPPORTED: return "unsupported query";
        default: return "unknown error";
    }
}

const char *sgm_last_error(void) { return g_last_error.c_str(); }

// sgm_load_graph, and sgm_load_compressed: a weighted graph's degree
// bounds (out_bound, in_bound, or null for the rows' lengths) and
// homomorphic matching
static int load_graph_impl(int32_t n_vertices, int32_t n_edges, const int32_t *row_ptr,
                           const int32_t *col, const int32_t *rel, const int32_t *type,
                           const sgm_options *opts, const int32_t *out_bound,
                           const int32_t *in_bound, bool homomorphic, sgm_graph **out) {
    if (!out) return SGM_EINVAL;
    *out = nullptr;
    if (n_vertices < 1 || n_edges < 0 || !row_ptr || !type || (n_edges > 0 && (!col || !rel)))
        return SGM_EINVAL;
    if (n_vertices > (1 << 30)) return SGM_EUNSUPPORTED;
    for (int32_t v = 0; v < n_vertices; ++v)
        if (type[v] < 0) return SGM_EINVAL;
    std::vector<int32_t> off, in_off;
    std::vector<int2> adj, in_adj;
    int rc;
    try {
        rc = normalize_csr(n_vertices, n_edges, row_ptr, col, rel, off, adj);
        if (rc) {
            g_last_error = "malformed CSR";
            return rc;
        }
        if (opts && opts->out_only) {
            // outgoing graph only: every in-row empty
            in_off.assign((size_t)n_vertices + 1, 0);
            in_adj.assign(1, make_int2(0, 0));
        } else {
            build_in(n_vertices, off, adj, in_off, in_adj);
        }
    } catch (const std::bad_alloc &) {
        return SGM_ENOMEM;
    }
    if (opts && opts->out_only && (opts->out_only != 1 || opts->path == SGM_PATH_NARROW))
        return SGM_EINVAL;
    if (opts && opts->host_graph != 0 && opts->host_graph != 1) return SGM_EINVAL;
    sgm_graph *g = new (std::nothrow) sgm_graph();
    if (!g) return SGM_ENOMEM;
    if (opts) g->opts = *opts;
    else sgm_default_options(&g->opts);
    if (g->opts.out_only) g->opts.path = SGM_PATH_WIDE;
    g->homomorphic = homomorphic;
    g->device = g->opts.device;
    g->V = n_vertices;
    g->E = (int64_t)adj.size();
    g->nwords = (n_vertices + 63) / 64;
    int32_t maxt = 0;
    for (int32_t v = 0; v < n_vertices; ++v) maxt = std::max(maxt, type[v]);
    g->n_types = maxt + 1;
    g->type_freq.assign((size_t)g->n_types, 0);
    for (int32_t v = 0; v < n_vertices; ++v) g->type_freq[type[v]]++;
    int32_t maxr = -1;
    for (const int2 &e : adj) maxr = std::max(maxr, e.y);
    g->n_rels = maxr + 1;
    g->rel_freq.assign((size_t)g->n_rels, 0);
    for (const int2 &e : adj) g->rel_freq[e.y]++;
    int nbig = 0;
    for (int32_t v = 0; v < n_vertices; ++v) {
        const int32_t od = off[v + 1] - off[v], id = in_off[v + 1] - in_off[v];
        g->max_out = std::max(g->max_out, od);
        g->max_in = std::max(g->max_in, id);
        if (od > kBigDegree || id > kBigDegree) ++nbig;
    }
    g->n_big = nbig;
    try {
        HIPX(hipSetDevice(g->device));
        // the fixed device area of sgm_match_query_noalloc: its address on
        // this device, taken once per device (on failure only that entry
        // point is unavailable; it reports the error)
        (void)scratch_setup(g->device);
        HIPX(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
        g->nw.stream = g->stream;
        g->nwb.stream = g->stream;
        g->nwb.lcap_want = kBigListCap;
        g->nwb.slab_want = kBigSlab;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device) == hipSuccess &&
            khz > 0)
            g->ns_per_tick = 1e6 / khz;
        // the O(E) arrays: in HBM, or with options.host_graph in host memory
        const bool hg = g->opts.host_graph != 0;
        auto edges_upload = [&](const std::vector<int2> &h) {
            return hg ? host_upload(h, g->host_graph_bufs) : dev_upload(h);
        };
        g->d_out_off = dev_upload(off);
        g->d_in_off = dev_upload(in_off);
        g->d_out_adj = edges_upload(adj);
        g->d_in_adj = edges_upload(in_adj);
        std::vector<int2> vi((size_t)n_vertices);
        for (int32_t v = 0; v < n_vertices; ++v) {
            const int32_t od = out_bound ? out_bound[v] : off[v + 1] - off[v];
            const int32_t id = in_bound ? in_bound[v] : in_off[v + 1] - in_off[v];
            vi[v] = make_int2(type[v], std::min(od, 255) | std::min(id, 255) << 8);
        }
        g->d_vinfo = dev_upload(vi);
        if (g->n_types <= kHubTypesMax) {
            HubIndex hx;
            build_hub_index(n_vertices, off, adj, in_off, in_adj, type, g->n_types, &hx);
            g->d_out_ta = edges_upload(hx.out_ta);
            g->d_out_tb = edges_upload(hx.out_tb);
            g->d_in_ta = edges_upload(hx.in_ta);
            g->d_in_tb = edges_upload(hx.in_tb);
            g->d_hub_of = dev_upload(hx.hub_of);
            g->d_hub_toff = dev_upload(hx.toff);
            g->dg.hub_types = hx.types;
        }
        HIPX(hipMalloc(&g->d_bits, sizeof(uint64_t) * (size_t)(SGM_MAX_QV + 1) * g->nwords));
        HIPX(hipMalloc(&g->d_lists, sizeof(int32_t) * (size_t)SGM_MAX_QV * g->V));
        HIPX(hipMalloc(&g->d_prefix, sizeof(int32_t) * (size_t)SGM_MAX_QV * (g->nwords + 1)));
        HIPX(hipMalloc(&g->d_big, sizeof(int32_t) * (size_t)std::max(nbig, 1)));
        HIPX(hipMalloc(&g->d_desc, sizeof(NbrDesc) * kMaxDesc));
        HIPX(hipMalloc(&g->d_cnt, sizeof(DevCounters)));
        HIPX(hipMalloc(&g->d_slots, sizeof(int32_t) * SGM_MAX_QV));
        HIPX(hipHostMalloc(&g->h_desc, sizeof(NbrDesc) * kMaxDesc, hipHostMallocDefault));
        HIPX(hipHostMalloc(&g->h_cnt, sizeof(DevCounters), hipHostMallocDefault));
        HIPX(hipHostMalloc(&g->h_slots, sizeof(int32_t) * SGM_MAX_QV, hipHostMallocDefault));
        HIPX(hipHostMalloc(&g->h_small, sizeof(int64_t) * 64, hipHostMallocDefault));
        g->dg.V = g->V;
        g->dg.nwords = g->nwords;
        g->dg.out_off = g->d_out_off;
        g->dg.in_off = g->d_in_off;
        g->dg.out_adj = g->d_out_adj;
        g->dg.in_adj = g->d_in_adj;
        g->dg.vinfo = g->d_vinfo;
        g->dg.out_ta = g->d_out_ta;
        g->dg.out_tb = g->d_out_tb;
        g->dg.in_ta = g->d_in_ta;
        g->dg.in_tb = g->d_in_tb;
        g->dg.hub_of = g->d_hub_of;
        g->dg.hub_toff = g->d_hub_toff;
        HIPX(hipDeviceSynchronize());
    } catch (const DeviceError &e) {
        free_graph_mem(g);
        delete g;
        return e.code;
    }
    *out = g;
    return SGM_OK;
}

int sgm_load_graph(int32_t n_vertices, int32_t n_edges, const int32_t *row_ptr,
                   const int32_t *col, const int32_t *rel, const int32_t *type,
                   const sgm_options *opts, sgm_graph **out) {
    return load_graph_impl(n_vertices, n_edges, row_ptr, col, rel, type, opts, nullptr, nullptr,
                           false, out);
}

int sgm_load_compressed(const sgm_compressed *c, const sgm_options *opts, sgm_graph **out) {
    if (!out) return SGM_EINVAL;
    *out = nullptr;
    if (!c || c->n_edges > INT32_MAX || (opts && opts->out_only)) return SGM_EINVAL;
    for (int32_t v = 0; v < c->n_vertices; ++v)
        if (c->out_bound[v] < 0 || c->in_bound[v] < 0) return SGM_EINVAL;
    return load_graph_impl(c->n_vertices, (int32_t)c->n_edges, c->row_ptr, c->col, c->rel, c->type,
                           opts, c->out_bound, c->in_bound, true, out);
}

int sgm_attach_mapping(sgm_graph *g, const sgm_compressed *c) {
    if (!g || !c || c->n_original != g->V || c->n_vertices < 1 || !c->map_off || !c->map_ids ||
        !c->hyper_of || c->map_off[0] != 0 || c->map_off[c->n_vertices] != g->V)
        return SGM_EINVAL;
    for (int32_t x = 0; x < c->n_vertices; ++x)
        if (c->map_off[x + 1] < c->map_off[x]) return SGM_EINVAL;
    for (int32_t v = 0; v < g->V; ++v)
        if (c->map_ids[v] < 0 || c->map_ids[v] >= g->V || c->hyper_of[v] < 0 ||
            c->hyper_of[v] >= c->n_vertices)
            return SGM_EINVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    try {
        HIPX(hipSetDevice(g->device));
        HIPX(hipStreamSynchronize(g->stream));
        dev_free(g->d_map_off);
        dev_free(g->d_map_ids);
        g->map_nw = 0;
        g->d_map_off = dev_upload(std::vector<int32_t>(c->map_off, c->map_off + c->n_vertices + 1));
        g->d_map_ids = dev_upload(std::vector<int32_t>(c->map_ids, c->map_ids + g->V));
        g->hyper_of.assign(c->hyper_of, c->hyper_of + g->V);
        g->map_nw = c->n_vertices;
    } catch (const DeviceError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return SGM_ENOMEM;
    }
    return SGM_OK;
}

int sgm_match_compressed(sgm_graph *g, sgm_graph *gw, const sgm_query *q, uint32_t flags,
                         sgm_result **out) {
    if (!out) return SGM_EINVAL;
    *out = nullptr;
    if (!g || !gw || !q || g == gw || (flags & ~SGM_COUNT_ONLY) || !gw->homomorphic ||
        g->map_nw != gw->V || !g->d_map_off)
        return SGM_EINVAL;
    QInfo qi;
    int rc = check_query(q, g->V, &qi);
    if (rc) return rc;
    // pinned query vertices take their weighted vertices
    const int n = qi.n;
    int32_t wpin[SGM_MAX_QV];
    for (int u = 0; u < n; ++u) wpin[u] = qi.pin[u] >= 0 ? g->hyper_of[qi.pin[u]] : -1;
    sgm_query qw = *q;
    qw.vertex_pin = wpin;
    sgm_result *rw = nullptr;
    rc = sgm_match_query(gw, &qw, SGM_SORTED, &rw);
    if (rc) return rc;
    sgm_result *res = result_new();
    if (!res) {
        sgm_free_result(rw);
        return SGM_ENOMEM;
    }
    res->n_cols = n;
    res->stats = rw->stats;
    const int64_t nw = rw->n_rows;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        try {
            HIPX(hipSetDevice(g->device));
            Scope sc(g->pool);
            hipStream_t st = g->stream;
            // assignment order: breadth first over the query's edges from a
            // pinned vertex (else vertex 0), so that every vertex after the
            // first meets a query edge to one chosen before it
            ExpandArgs a{};
            a.g = g->dg;
            a.n = n;
            a.nw = nw;
            a.map_off = g->d_map_off;
            a.map_ids = g->d_map_ids;
            int depth[SGM_MAX_QV];
            for (int u = 0; u < n; ++u) depth[u] = -1;
            int nord = 0;
            auto visit_from = [&](int s0) {
                depth[s0] = nord;
                a.order[nord++] = s0;
                for (int i = depth[s0]; i < nord; ++i) {
                    const int u = a.order[i];
                    for (int e = 0; e < qi.m; ++e) {
                        const int v = qi.esrc[e] == u ? qi.edst[e] : qi.edst[e] == u ? qi.esrc[e] : -1;
                        if (v >= 0 && depth[v] < 0) {
                            depth[v] = nord;
                            a.order[nord++] = v;
                        }
                    }
                }
            };
            int start = 0;
            for (int u = n - 1; u >= 0; --u)
                if (qi.pin[u] >= 0) start = u;
            visit_from(start);
            for (int u = 0; u < n; ++u)
                if (depth[u] < 0) visit_from(u);
            for (int u = 0; u < n; ++u) a.pin[u] = qi.pin[u];
            // each query edge is checked once both ends are chosen
            int ne = 0;
            for (int d = 0; d < n; ++d) {
                a.eb[d] = ne;
                for (int e = 0; e < qi.m; ++e)
                    if (std::max(depth[qi.esrc[e]], depth[qi.edst[e]]) == d) {
                        a.es[ne] = qi.esrc[e];
                        a.ed[ne] = qi.edst[e];
                        a.el[ne] = qi.elabel[e];
                        ++ne;
                    }
            }
            a.eb[n] = ne;
            int64_t total = 0;
            int32_t *table = nullptr;
            if (nw > 0) {
                int32_t *wrows = sc.get<int32_t>(nw * n);
                HIPX(hipMemcpyAsync(wrows, rw->rows, sizeof(int32_t) * (size_t)(nw * n),
                                    hipMemcpyHostToDevice, st));
                a.wrows = wrows;
                a.cnt = sc.get<int64_t>(nw);
                int64_t *offs = sc.get<int64_t>(nw + 1);
                int64_t *tmp = sc.get<int64_t>(scan_tmp_words(nw) + 1);
                launch_expand_count(st, a);
                launch_scan_i64(st, a.cnt, nw, offs, tmp);
                HIPX(hipMemcpyAsync(g->h_small, offs + nw, sizeof(int64_t), hipMemcpyDeviceToHost, st));
                HIPX(hipStreamSynchronize(st));
                total = g->h_small[0];
                a.offs = offs;
                if (total > 0 && !(flags & SGM_COUNT_ONLY)) {
                    table = sc.get<int32_t>(total * n);
                    a.out = table;
                    launch_expand_write(st, a);
                }
            }
            res->n_rows = total;
            if (g->opts.result_cap_rows > 0 && total > g->opts.result_cap_rows) {
                rc = SGM_ETOOBIG;
            } else if (!(flags & SGM_COUNT_ONLY)) {
                // ascending lexicographic order: stable LSD passes over the
                // columns, last column first
                int32_t *rows = table;
                if (total > 1) {
                    int nbits = 1;
                    while ((1ll << nbits) < g->V) ++nbits;
                    int32_t *ia = sc.get<int32_t>(total), *ib = sc.get<int32_t>(total);
                    int32_t *ka = sc.get<int32_t>(total), *kb = sc.get<int32_t>(total);
                    const int64_t tiles = radix_tiles(total);
                    int64_t *hist = sc.get<int64_t>(256 * tiles);
                    int64_t *hoff = sc.get<int64_t>(256 * tiles + 1);
                    int64_t *stmp = sc.get<int64_t>(scan_tmp_words(256 * tiles) + 1);
                    launch_iota(st, ia, total);
                    for (int c = n - 1; c >= 0; --c) {
                        launch_gather_key(st, table, n, c, ia, total, ka);
                        for (int sh = 0; sh < nbits; sh += 8) {
                            launch_radix_hist(st, ka, total, sh, hist);
                            launch_scan_i64(st, hist, 256 * tiles, hoff, stmp);
                            launch_radix_scatter(st, ka, ia, total, sh, hoff, kb, ib);
                            std::swap(ka, kb);
                            std::swap(ia, ib);
                        }
                    }
                    int32_t colpos[SGM_MAX_QV];
                    for (int c = 0; c < n; ++c) colpos[c] = c;
                    rows = sc.get<int32_t>(total * n);
                    launch_gather_rows(st, table, n, ia, total, colpos, n, rows);
                }
                const size_t bytes = sizeof(int32_t) * (size_t)(total * n);
                res->rows = alloc_rows(bytes);
                if (!res->rows) throw DeviceError{SGM_ENOMEM};
                if (total > 0) readback_rows(g, st, rows, bytes, res->rows);
            }
            HIPX(hipStreamSynchronize(st));
        } catch (const DeviceError &e) {
            rc = e.code;
            (void)hipStreamSynchronize(g->stream);
        } catch (const std::bad_alloc &) {
            rc = SGM_ENOMEM;
        }
    }
    sgm_free_result(rw);
    res->status = rc;
    if (rc == SGM_OK || rc == SGM_ETOOBIG) {
        if (rc != SGM_OK) result_drop_rows(res);
        *out = res;
        return rc;
    }
    sgm_free_result(res);
    return rc;
}

void sgm_free_graph(sgm_graph *g) {
    if (!g) return;
    free_graph_mem(g);
    delete g;
}

void sgm_results_summary(sgm_result *const *rs, int32_t n, int64_t *out) {
    if (!rs || !out) return;
    for (int32_t i = 0; i < n; ++i) {
        const sgm_result *r = rs[i];
        out[4 * (int64_t)i + 0] = r ? r->status : SGM_EINVAL;
        out[4 * (int64_t)i + 1] = r ? r->n_cols : 0;
        out[4 * (int64_t)i + 2] = r ? r->n_rows : 0;
        out[4 * (int64_t)i + 3] = r ? (int64_t)(uintptr_t)r->rows : 0;
    }
}

int sgm_inject_fault(sgm_graph *g, int64_t query_index) {
    if (!g || query_index < -1) return SGM_EINVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    g->fault_query = query_index;
    return SGM_OK;
}

void sgm_default_tuning(sgm_tuning *t) {
    if (!t) return;
    *t = sgm_tuning{512, 64, 8192, 0, 1024, 64, 0, {0}};
}

int sgm_get_tuning(const sgm_graph *g, sgm_tuning *t) {
    if (!g || !t) return SGM_EINVAL;
    *t = g->tune;
    return SGM_OK;
}

static bool tuning_ok(const sgm_tuning &t) {
    const bool pow2 = t.group_lanes > 0 && (t.group_lanes & (t.group_lanes - 1)) == 0;
    return t.slots >= 1 && t.slots <= 512 && pow2 && t.group_lanes <= 64 && t.wg_rows >= 64 &&
           (t.join_policy == 0 || t.join_policy == 1) &&
           (t.help_items == 0 || t.help_items >= 64) && t.helpers >= 0 && t.helpers <= 512 &&
           t.help_wait >= 0;
}

int sgm_set_tuning(sgm_graph *g, const sgm_tuning *t) {
    if (!g || !t || !tuning_ok(*t)) return SGM_EINVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    g->tune = *t;
    g->tune.reserved[0] = 0;
    return SGM_OK;
}

int sgm_autotune(sgm_graph *g, const sgm_query *qs, int32_t n, int32_t reps, sgm_tuning *best) {
    if (!g || n <= 0 || !qs || reps < 1 || g->opts.out_only || g->homomorphic) return SGM_EINVAL;
    reps = std::min(reps, 16);
    std::lock_guard<std::mutex> lk(g->mu);
    std::vector<QInfo> qis((size_t)n);
    std::vector<int> valid;
    for (int i = 0; i < n; ++i)
        if (check_query(&qs[i], g->V, &qis[i]) == SGM_OK) valid.push_back(i);
    if (valid.empty()) return SGM_EINVAL;
    const sgm_tuning saved = g->tune;
    std::vector<sgm_tuning> grid;
    for (int sl : {256, 512})
        for (int gl : {16, 64})
            for (int wr : {2048, 8192, 32768})
                for (int jp : {0, 1})
                    for (int hi : {0, 1024})
                        grid.push_back(
                            sgm_tuning{sl, gl, wr, jp, hi, saved.helpers, saved.help_wait, {0}});
    std::vector<sgm_result> store((size_t)n);
    std::vector<sgm_result *> res((size_t)n);
    for (int i = 0; i < n; ++i) res[i] = &store[i];
    std::vector<int64_t> rows_ref;
    double best_t = 1e300;
    sgm_tuning pick = saved;
    try {
        for (const sgm_tuning &t : grid) {
            g->tune = t;
            std::vector<double> ts;
            for (int r = 0; r <= reps; ++r) {  // the first run warms up
                for (sgm_result &x : store) x = sgm_result{};
                std::vector<int> wide;
                const int64_t t0 = now_ns();
                narrow_batch(g, qis, valid, SGM_COUNT_ONLY, res, wide);
                const double el = (double)(now_ns() - t0);
                if (r > 0) ts.push_back(el);
                std::vector<int64_t> rows((size_t)n, -1);
                for (int i : valid)
                    if (std::find(wide.begin(), wide.end(), i) == wide.end()) rows[i] = store[i].n_rows;
                if (rows_ref.empty()) rows_ref = rows;
                for (int i : valid)
                    if (rows[i] >= 0 && rows_ref[i] >= 0 && rows[i] != rows_ref[i]) {
                        g->tune = saved;
                        g_last_error = "autotune: a tuning changed a result";
                        return SGM_EDEVICE;
                    }
            }
            std::sort(ts.begin(), ts.end());
            const double med = ts[ts.size() / 2];
            if (med < best_t) {
                best_t = med;
                pick = t;
            }
        }
    } catch (const DeviceError &e) {
        (void)hipStreamSynchronize(g->stream);
        (void)hipGetLastError();
        g->pending.clear();
        g->tune = saved;
        return e.code;
    } catch (const std::bad_alloc &) {
        g->tune = saved;
        return SGM_ENOMEM;
    }
    g->tune = pick;
    if (best) *best = pick;
    return SGM_OK;
}

int sgm_trace_events(sgm_graph *g, int32_t i, int64_t *out, int32_t cap, double *ns_per_tick) {
    if (!g || i < 0 || cap < 0 || (cap > 0 && !out)) return SGM_EINVAL;
    if (ns_per_tick) *ns_per_tick = g->ns_per_tick;
    if ((size_t)i >= g->trace_n.size()) return SGM_EINVAL;
    const int32_t n = g->trace_n[(size_t)i];
    const int32_t k = std::min(n, cap);
    if (k > 0) std::memcpy(out, &g->trace[(size_t)i * SGM_TRACE_CAP], sizeof(int64_t) * k);
    return n;
}

int sgm_graph_info(const sgm_graph *g, int32_t *n_vertices, int64_t *n_edges,
                   int32_t *max_out_degree, int32_t *max_in_degree) {
    if (!g) return SGM_EINVAL;
    if (n_vertices) *n_vertices = g->V;
    if (n_edges) *n_edges = g->E;
    if (max_out_degree) *max_out_degree = g->max_out;
    if (max_in_degree) *max_in_degree = g->max_in;
    return SGM_OK;
}

}  // extern "C"

namespace {

int match_one(sgm_graph *g, const sgm_query *q, const uint32_t *proj, uint32_t flags,
              sgm_result **out) {
    if (!out) return SGM_EINVAL;
    *out = nullptr;
    if (!g || !q || (flags & ~SGM_COUNT_ONLY)) return SGM_EINVAL;
    sgm_result *res = result_new();
    if (!res) return SGM_ENOMEM;
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (hipSetDevice(g->device) != hipSuccess) {
            std::free(res);
            return SGM_EDEVICE;
        }
        std::vector<sgm_result *> rv{res};
        rc = run_queries(g, q, proj, 1, flags, rv);
        if (rc == SGM_OK) rc = res->status;
    }
    res->status = rc;
    if (rc == SGM_OK || rc == SGM_ETOOBIG) {
        if (rc != SGM_OK) result_drop_rows(res);
        *out = res;
        return rc;
    }
    sgm_free_result(res);
    return rc;
}

int match_many(sgm_graph *g, const sgm_query *qs, const uint32_t *proj, int32_t n, uint32_t flags,
               sgm_result **out) {
    if (!g || !out || n < 0 || (n > 0 && !qs) || (flags & ~SGM_COUNT_ONLY)) return SGM_EINVAL;
    std::vector<sgm_result *> rv((size_t)n, nullptr);
    for (int32_t i = 0; i < n; ++i) {
        out[i] = nullptr;
        rv[i] = result_new();
        if (!rv[i]) {
            for (int32_t j = 0; j < i; ++j) sgm_free_result(rv[j]);
            return SGM_ENOMEM;
        }
    }
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (hipSetDevice(g->device) != hipSuccess) rc = SGM_EDEVICE;
        else rc = run_queries(g, qs, proj, n, flags, rv);
    }
    if (rc != SGM_OK) {
        for (auto *r : rv) sgm_free_result(r);
        return rc;
    }
    for (int32_t i = 0; i < n; ++i) {
        if (rv[i]->status != SGM_OK) result_drop_rows(rv[i]);
        out[i] = rv[i];
    }
    return SGM_OK;
}

}  // namespace

extern "C" {

int sgm_match_query(sgm_graph *g, const sgm_query *q, uint32_t flags, sgm_result **out) {
    return match_one(g, q, nullptr, flags, out);
}

int sgm_match_batch(sgm_graph *g, const sgm_query *qs, int32_t n, uint32_t flags,
                    sgm_result **out) {
    return match_many(g, qs, nullptr, n, flags, out);
}

int sgm_match_query_proj(sgm_graph *g, const sgm_query *q, uint32_t project, uint32_t flags,
                         sgm_result **out) {
    return match_one(g, q, &project, flags, out);
}

int sgm_match_batch_proj(sgm_graph *g, const sgm_query *qs, const uint32_t *project, int32_t n,
                         uint32_t flags, sgm_result **out) {
    if (n > 0 && !project) {
        if (out)
            for (int32_t i = 0; i < n; ++i) out[i] = nullptr;
        return SGM_EINVAL;
    }
    return match_many(g, qs, project, n, flags, out);
}

int sgm_inspect_query(sgm_graph *g, const sgm_query *q, int64_t *counts, int32_t **ids,
                      int64_t *ec) {
    if (!ids) return SGM_EINVAL;
    *ids = nullptr;
    if (!g || !q || !counts || !ec) return SGM_EINVAL;
    QInfo qi;
    int rc = check_query(q, g->V, &qi);
    if (rc) return rc;
    for (int u = 0; u < SGM_MAX_QV; ++u) counts[u] = 0;
    for (int e = 0; e < SGM_MAX_QE; ++e) ec[e] = 0;
    std::lock_guard<std::mutex> lk(g->mu);
    if (hipSetDevice(g->device) != hipSuccess) return SGM_EDEVICE;
    sgm_result scratch_res{};
    try {
        Query Q(g, qi, &scratch_res, SGM_COUNT_ONLY);
        rc = Q.inspect(counts, ids, ec);
    } catch (const DeviceError &e) {
        rc = e.code;
        (void)hipStreamSynchronize(g->stream);
        (void)hipGetLastError();
        g->pending.clear();
    } catch (const std::bad_alloc &) {
        rc = SGM_ENOMEM;
    }
    if (rc != SGM_OK) {
        std::free(*ids);
        *ids = nullptr;
    }
    return rc;
}

void sgm_free_ids(int32_t *ids) { std::free(ids); }

void sgm_free_result(sgm_result *r) {
    if (!r) return;
    result_drop_rows(r);
    std::free(reinterpret_cast<ResultBox *>(r));
}

int sgm_kernel_stats(sgm_graph *g, int32_t kernel, sgm_kstat *out) {
    if (!g || !out || kernel < 0 || kernel >= SGM_K_COUNT) return SGM_EINVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    *out = g->kstat[kernel];
    return SGM_OK;
}

int sgm_reset_kernel_stats(sgm_graph *g) {
    if (!g) return SGM_EINVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    for (auto &k : g->kstat) k = sgm_kstat{};
    return SGM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// served form: continuous batching over streams
// ---------------------------------------------------------------------------

struct sgm_server {
    sgm_graph *g = nullptr;
    sgm_serve_options o{};
    std::vector<NarrowCtx> ctx;
    struct Ticket {
        QInfo qi;
        int status = SGM_OK;  // of the query check
        uint32_t flags = 0;
        int64_t t_submit = 0, t_done = 0;
        int64_t est = 0;      // admission estimate (estimate_bytes)
        sgm_result *res = nullptr;
        bool done = false;
    };
    struct Batch {
        int ctx = -1;
        std::vector<uint64_t> ids;
        std::vector<QInfo> qis;
        std::vector<sgm_result *> res;
        std::vector<int64_t> est;
        std::vector<int> which, wide;
        NarrowJob job;
        bool launched = false;
        uint32_t flags = 0;
    };
    // a query that outgrew its slot, waiting for the rerun thread
    struct Rerun {
        uint64_t id;
        QInfo qi;
        sgm_result *res;
        uint32_t flags;
        int64_t est;
    };
    std::mutex mu;
    std::condition_variable cv_in, cv_out, cv_ctx, cv_done, cv_rerun;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::vector<char> ctx_busy;   // a batch is being launched or runs on the context
    std::vector<Batch *> on_ctx;  // launched batch of each context, for its completer
    std::deque<Rerun> reruns;
    uint64_t next_id = 1;
    int64_t bytes_in_flight = 0, queries_in_flight = 0;
    bool stop = false;
    bool dispatcher_done = false;
    int completers_left = 0;
    sgm_serve_stats st{};
    std::thread dispatcher, rerunner;
    std::vector<std::thread> completers;
};

namespace {

// Dispatcher: closes a micro-batch (max_batch queries, or max_wait_ns after
// its first query arrived), takes a free stream context, admits queries in
// arrival order while the admission estimates of everything admitted and
// unfinished stay under the cap (one query is always admitted when nothing
// runs), and launches the batch; batches on other contexts keep running.
void serve_dispatch(sgm_server *S) {
    sgm_graph *g = S->g;
    (void)hipSetDevice(g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_in.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        if (S->pending.empty()) {
            if (S->stop) break;
            continue;
        }
        // batch window: wait for a full batch or the first query's deadline
        for (;;) {
            if ((int)S->pending.size() >= S->o.max_batch || S->stop) break;
            const int64_t first = S->tickets[S->pending.front()].t_submit;
            const int64_t left = first + S->o.max_wait_ns - now_ns();
            if (left <= 0) break;
            S->cv_in.wait_for(lk, std::chrono::nanoseconds(left));
        }
        // a free stream context
        int ci = -1;
        S->cv_ctx.wait(lk, [&] {
            for (size_t i = 0; i < S->ctx_busy.size(); ++i)
                if (!S->ctx_busy[i]) {
                    ci = (int)i;
                    return true;
                }
            return false;
        });
        // admission; the flags of a batch are those of its first query
        sgm_server::Batch *b = new sgm_server::Batch();
        b->ctx = ci;
        b->flags = S->tickets[S->pending.front()].flags;
        bool stalled = false;
        int64_t add = 0;
        while (!S->pending.empty() && (int)b->ids.size() < S->o.max_batch) {
            sgm_server::Ticket &t = S->tickets[S->pending.front()];
            if (t.flags != b->flags) break;
            const bool nothing_running = S->queries_in_flight == 0 && b->ids.empty();
            if (!nothing_running && S->bytes_in_flight + add + t.est > S->o.admission_cap_bytes) {
                stalled = true;
                break;
            }
            b->ids.push_back(S->pending.front());
            add += t.est;
            S->pending.pop_front();
        }
        if (stalled) S->st.admission_stalls++;
        if (b->ids.empty()) {
            delete b;
            // wait for running work to release its estimate
            S->cv_done.wait(lk);
            continue;
        }
        S->ctx_busy[ci] = 1;
        S->bytes_in_flight += add;
        S->queries_in_flight += (int64_t)b->ids.size();
        S->st.max_in_flight = std::max(S->st.max_in_flight, S->queries_in_flight);
        S->st.batches++;
        for (uint64_t id : b->ids) {
            sgm_server::Ticket &t = S->tickets[id];
            b->qis.push_back(t.qi);
            b->res.push_back(t.res);
            b->est.push_back(t.est);
        }
        lk.unlock();
        for (size_t i = 0; i < b->ids.size(); ++i)
            if (b->res[i]->status == SGM_OK) b->which.push_back((int)i);
        try {
            b->launched = narrow_launch(g, S->ctx[ci], b->qis, b->which.data(),
                                        (int)b->which.size(), b->job, b->wide, b->res, false);
        } catch (const DeviceError &e) {
            for (auto *r : b->res) r->status = e.code;
            b->which.clear();
            b->wide.clear();
            b->launched = false;
        }
        lk.lock();
        S->on_ctx[ci] = b;
        S->cv_out.notify_all();
    }
    S->dispatcher_done = true;
    S->cv_out.notify_all();
}

// Mark ticket id done at t_done (caller holds S->mu) and release its
// estimate.
void serve_finish(sgm_server *S, uint64_t id, int64_t est, int64_t t_done) {
    auto it = S->tickets.find(id);
    sgm_server::Ticket &t = it->second;
    t.t_done = t_done;
    t.done = true;
    sgm_result *r = t.res;
    if (r->status != SGM_OK && r->status != SGM_ETOOBIG) result_drop_rows(r);
    r->stats.ns_total = t_done - t.t_submit;
    S->st.completed++;
    S->bytes_in_flight -= est;
    S->queries_in_flight--;
}

// Completer of context ci: waits for the batch launched there (its own
// stream and event), completes its finished queries at once, hands the ones
// that outgrew their slot to the rerun thread and frees the context. Each
// context has its own completer, so a batch that ends early is completed
// while a longer one still runs on another stream.
void serve_complete(sgm_server *S, int ci) {
    sgm_graph *g = S->g;
    (void)hipSetDevice(g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_out.wait(lk, [&] { return S->on_ctx[ci] != nullptr || S->dispatcher_done; });
        sgm_server::Batch *b = S->on_ctx[ci];
        if (!b) {
            if (S->dispatcher_done) break;
            continue;
        }
        lk.unlock();
        try {
            if (b->launched)
                narrow_collect(g, S->ctx[ci], b->job, b->qis, b->flags, b->res, b->wide, false);
        } catch (const DeviceError &e) {
            for (int i : b->which) b->res[i]->status = e.code;
            b->wide.clear();
        } catch (const std::bad_alloc &) {
            for (int i : b->which) b->res[i]->status = SGM_ENOMEM;
            b->wide.clear();
        }
        const int64_t t_done = now_ns();
        std::vector<char> rerun(b->ids.size(), 0);
        for (int i : b->wide) rerun[(size_t)i] = 1;
        lk.lock();
        for (size_t i = 0; i < b->ids.size(); ++i) {
            if (rerun[i])
                S->reruns.push_back(
                    sgm_server::Rerun{b->ids[i], b->qis[i], b->res[i], b->flags, b->est[i]});
            else
                serve_finish(S, b->ids[i], b->est[i], t_done);
        }
        S->on_ctx[ci] = nullptr;
        S->ctx_busy[ci] = 0;
        delete b;
        S->cv_ctx.notify_all();
        S->cv_done.notify_all();
        S->cv_rerun.notify_one();
    }
    if (--S->completers_left == 0) S->cv_rerun.notify_all();
}

// Rerun thread: queries that outgrew a regular slot run again in a large
// slot, then on the multi-kernel path, on the graph's own stream, so the
// completers never wait for them.
void serve_rerun(sgm_server *S) {
    sgm_graph *g = S->g;
    (void)hipSetDevice(g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_rerun.wait(lk, [&] { return !S->reruns.empty() || S->completers_left == 0; });
        if (S->reruns.empty()) {
            if (S->completers_left == 0) break;
            continue;
        }
        // every waiting query with the flags of the first
        const uint32_t flags = S->reruns.front().flags;
        std::vector<sgm_server::Rerun> take;
        for (auto it = S->reruns.begin(); it != S->reruns.end();) {
            if (it->flags == flags) {
                take.push_back(*it);
                it = S->reruns.erase(it);
            } else {
                ++it;
            }
        }
        lk.unlock();
        std::vector<QInfo> qis;
        std::vector<sgm_result *> res;
        std::vector<int> wide;
        for (size_t i = 0; i < take.size(); ++i) {
            qis.push_back(take[i].qi);
            res.push_back(take[i].res);
            wide.push_back((int)i);
        }
        {
            std::lock_guard<std::mutex> gl(g->mu);
            try {
                narrow_retry_large(g, qis, flags, res, wide);
            } catch (const DeviceError &e) {
                (void)hipStreamSynchronize(g->stream);
                (void)hipGetLastError();
                g->pending.clear();
            } catch (const std::bad_alloc &) {
            }
            for (int i : wide) {
                const int32_t why = res[i]->stats.fallback;
                std::memset(&res[i]->stats, 0, sizeof(sgm_stats));
                res[i]->stats.path = SGM_PATH_WIDE;
                res[i]->stats.fallback = why;
                res[i]->status = wide_locked(g, qis[i], flags, res[i]);
            }
        }
        const int64_t t_done = now_ns();
        lk.lock();
        S->st.wide_fallbacks += (int64_t)wide.size();
        for (const auto &r : take) serve_finish(S, r.id, r.est, t_done);
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

void sgm_default_serve_options(sgm_serve_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->streams = 4;
    o->max_batch = 256;
    o->max_wait_ns = 100000;
    o->admission_cap_bytes = 64ll << 30;
}

int sgm_server_create(sgm_graph *g, const sgm_serve_options *opts, sgm_server **out) {
    if (!out) return SGM_EINVAL;
    *out = nullptr;
    if (!g || g->opts.out_only || g->homomorphic) return SGM_EINVAL;
    sgm_serve_options o;
    if (opts) o = *opts;
    else sgm_default_serve_options(&o);
    if (o.streams < 1 || o.streams > 16 || o.max_batch < 1 || o.max_batch > kNarrowQueryCap ||
        o.max_wait_ns < 0 || o.admission_cap_bytes <= 0)
        return SGM_EINVAL;
    sgm_server *S = new (std::nothrow) sgm_server();
    if (!S) return SGM_ENOMEM;
    S->g = g;
    S->o = o;
    S->ctx.resize((size_t)o.streams);
    S->on_ctx.assign((size_t)o.streams, nullptr);
    S->ctx_busy.assign((size_t)o.streams, 0);
    try {
        HIPX(hipSetDevice(g->device));
        for (auto &c : S->ctx) {
            HIPX(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
            c.serve = true;
            narrow_reserve(g, c, std::min(o.max_batch, kNarrowMaxSlots), o.max_batch, 0);
        }
    } catch (const DeviceError &e) {
        for (auto &c : S->ctx) {
            narrow_free(c);
            if (c.stream) (void)hipStreamDestroy(c.stream);
        }
        delete S;
        return e.code;
    }
    S->completers_left = o.streams;
    S->dispatcher = std::thread(serve_dispatch, S);
    for (int i = 0; i < o.streams; ++i) S->completers.emplace_back(serve_complete, S, i);
    S->rerunner = std::thread(serve_rerun, S);
    *out = S;
    return SGM_OK;
}

int sgm_submit(sgm_server *s, const sgm_query *q, uint32_t flags, uint64_t *ticket) {
    if (!s || !q || !ticket || (flags & ~SGM_COUNT_ONLY)) return SGM_EINVAL;
    sgm_result *res = result_new();
    if (!res) return SGM_ENOMEM;
    sgm_server::Ticket t;
    t.status = check_query(q, s->g->V, &t.qi);
    res->status = t.status;
    t.flags = flags;
    t.res = res;
    if (t.status == SGM_OK) {
        Plan pl;
        const sgm_graph *g = s->g;
        if (make_plan(t.qi, g->V, g->type_freq.data(), g->n_types, &pl) == SGM_OK)
            t.est = estimate_bytes(t.qi, pl, g->V, g->E, g->type_freq.data(), g->n_types,
                                   g->rel_freq.data(), g->n_rels);
    }
    t.t_submit = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        sgm_free_result(res);
        return SGM_EINVAL;
    }
    const uint64_t id = s->next_id++;
    *ticket = id;
    s->st.submitted++;
    if (t.status != SGM_OK) {
        t.done = true;
        t.t_done = t.t_submit;
        s->st.completed++;
        s->tickets.emplace(id, t);
        s->cv_done.notify_all();
        return SGM_OK;
    }
    s->tickets.emplace(id, t);
    s->pending.push_back(id);
    s->cv_in.notify_one();
    return SGM_OK;
}

int sgm_wait(sgm_server *s, uint64_t ticket, int64_t timeout_ns, sgm_result **out) {
    if (!s || !out) return SGM_EINVAL;
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return SGM_EINVAL;
    auto ready = [&] { return s->tickets[ticket].done; };
    if (timeout_ns < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready))
        return SGM_EDEVICE;
    it = s->tickets.find(ticket);
    *out = it->second.res;
    s->tickets.erase(it);
    return SGM_OK;
}

int sgm_server_stats(sgm_server *s, sgm_serve_stats *out) {
    if (!s || !out) return SGM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return SGM_OK;
}

void sgm_server_destroy(sgm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_in.notify_all();
    s->cv_out.notify_all();
    s->cv_ctx.notify_all();
    s->cv_done.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_out.notify_all();
    }
    for (auto &t : s->completers)
        if (t.joinable()) t.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_rerun.notify_all();
    }
    if (s->rerunner.joinable()) s->rerunner.join();
    (void)hipSetDevice(s->g->device);
    for (auto &c : s->ctx) {
        narrow_free(c);
        if (c.stream) (void)hipStreamDestroy(c.stream);
    }
    for (auto &kv : s->tickets) sgm_free_result(kv.second.res);
    delete s;
}

int sgm_serve_replay(sgm_server *s, const sgm_query *qs, const int64_t *arrival_ns, int32_t n,
                     uint32_t flags, int64_t *latency_ns, sgm_result **out) {
    if (!s || n < 0 || (n > 0 && (!qs || !arrival_ns || !latency_ns))) return SGM_EINVAL;
    for (int32_t i = 1; i < n; ++i)
        if (arrival_ns[i] < arrival_ns[i - 1]) return SGM_EINVAL;
    // state[i]: 0 = not yet submitted, > 0 = ticket, < 0 = submit error
    std::vector<std::atomic<int64_t>> state((size_t)n);
    std::vector<int64_t> sub_t((size_t)n, 0);
    for (auto &x : state) x.store(0);
    const int64_t t0 = now_ns();
    std::thread sub([&] {
        for (int32_t i = 0; i < n; ++i) {
            const int64_t at = t0 + arrival_ns[i];
            const int64_t now = now_ns();
            if (at - now > 200000)
                std::this_thread::sleep_for(std::chrono::nanoseconds(at - now - 100000));
            while (now_ns() < at) {
            }
            uint64_t tk = 0;
            sub_t[i] = now_ns();
            const int rc = sgm_submit(s, &qs[i], flags, &tk);
            state[i].store(rc == SGM_OK ? (int64_t)tk : (int64_t)rc);
        }
    });
    int ret = SGM_OK;
    for (int32_t i = 0; i < n; ++i) {
        int64_t st;
        while ((st = state[i].load()) == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
        latency_ns[i] = -1;
        if (out) out[i] = nullptr;
        if (st < 0) {
            ret = (int)st;
            continue;
        }
        sgm_result *r = nullptr;
        const int w = sgm_wait(s, (uint64_t)st, -1, &r);
        if (w != SGM_OK) {
            ret = w;
            continue;
        }
        // completion - scheduled arrival (ns_total = completion - submission)
        latency_ns[i] = sub_t[i] + r->stats.ns_total - (t0 + arrival_ns[i]);
        if (out) out[i] = r;
        else sgm_free_result(r);
    }
    sub.join();
    return ret;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Single queries without allocation: every device buffer of the persistent
// kernel's launch (one slot, descriptor, result, counters, helper board,
// root sweep row, output arena) lives in one fixed array of device memory
// that each GPU holds until the process ends.
// ---------------------------------------------------------------------------

namespace {

constexpr int64_t kScratchBytes = 64ll << 20;     // the whole fixed area
constexpr int64_t kScratchSlab = 16ll << 20;      // slab of its one slot
constexpr int64_t kScratchMinOut = 1ll << 20;     // smallest output arena accepted (bytes)
constexpr int kScratchDevices = 64;

}  // namespace

// The fixed area. Host code never uses this name as an address: kernels and
// copies get the per-device address that hipGetSymbolAddress returned.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};
std::mutex g_scratch_call_mu[kScratchDevices];  // calls on one device run one at a time
// Leading 8-byte words of each device's slot bitmaps known to be zero: the
// kernel clears the bitmaps it set, but a graph with more vertices lays its
// bitmaps over what other buffers of an earlier call held.
int64_t g_scratch_zero_words[kScratchDevices] = {};

// Device address of the fixed area on the current device (once per device;
// called by sgm_load_graph with the graph's device current).
int scratch_setup(int device) {
    if (device < 0 || device >= kScratchDevices) return SGM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return SGM_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error("hipGetSymbolAddress(scratch)", e);
        return SGM_EDEVICE;
    }
    g_scratch_ptr[device] = p;
    return SGM_OK;
}

__global__ void k_zero_words(uint64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Layout of the fixed area for a graph (byte offsets, 256-aligned).
struct ScratchLayout {
    int64_t bits, lists, slab, rootbits, preds, q, res, ctr, board, out, out_bytes;
    int32_t lcap;
    bool fits;
};

int64_t align256(int64_t x) { return (x + 255) & ~255ll; }

// The small fixed-size buffers come first, at the same offsets for every
// graph; the slot bitmaps follow at a fixed offset too.
ScratchLayout scratch_layout(const sgm_graph *g) {
    ScratchLayout L{};
    L.lcap = std::min<int32_t>(g->V, kNarrowListCap);
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.board = take(sizeof(HelpJob));
    L.ctr = take(sizeof(unsigned long long) * 3);
    L.q = take(sizeof(NQuery));
    L.res = take(sizeof(NResult));
    L.preds = take(sizeof(VPred));
    L.bits = take((int64_t)(SGM_MAX_QV + 1) * g->nwords * 8);
    L.lists = take((int64_t)SGM_MAX_QV * L.lcap * 4);
    L.slab = take(kScratchSlab);
    L.rootbits = take((int64_t)g->nwords * 8);
    L.out = o;
    L.out_bytes = (kScratchBytes - o) & ~255ll;
    L.fits = L.out_bytes >= kScratchMinOut && kScratchSlab >= 8ll * L.lcap;
    return L;
}

}  // namespace

extern "C" {

int sgm_match_query_noalloc(sgm_graph *g, const sgm_query *q, uint32_t flags, int32_t *rows,
                            int64_t rows_cap, int64_t *n_rows) {
    if (n_rows) *n_rows = 0;
    if (!g || !q || !n_rows || (flags & ~SGM_COUNT_ONLY) || rows_cap < 0 ||
        (!(flags & SGM_COUNT_ONLY) && rows_cap > 0 && !rows) || g->opts.out_only || g->homomorphic)
        return SGM_EINVAL;
    QInfo qi;
    int rc = check_query(q, g->V, &qi);
    if (rc != SGM_OK) return rc;
    if (g->device < 0 || g->device >= kScratchDevices || !g_scratch_ptr[g->device]) {
        g_last_error = "the fixed device area of this device has no address";
        return SGM_EDEVICE;
    }
    const ScratchLayout L = scratch_layout(g);
    if (!L.fits) {
        g_last_error = "graph too large for the fixed device area (64 MB)";
        return SGM_EUNSUPPORTED;
    }
    Plan pl;
    if (make_plan(qi, g->V, g->type_freq.data(), g->n_types, &pl) != SGM_OK) return SGM_EINVAL;
    NQuery nq;
    Plan pl_out;
    int root_slots = 0;
    if (!pack_query(g, qi, pl, &nq, &root_slots, &pl_out)) {
        g_last_error = "query plan exceeds the packed descriptor";
        return SGM_EUNSUPPORTED;
    }
    const bool sweep = nq.root_slot >= 0;
    if (sweep) nq.root_slot = 0;
    const VPred rootp = VPred{nq.pred[nq.root].label, -1, nq.pred[nq.root].qout,
                              nq.pred[nq.root].qin};
    std::lock_guard<std::mutex> call(g_scratch_call_mu[g->device]);
    std::lock_guard<std::mutex> lk(g->mu);
    char *base = (char *)g_scratch_ptr[g->device];
    NResult r;
    try {
        HIPX(hipSetDevice(g->device));
        hipStream_t st = g->stream;
        unsigned long long *ctr = (unsigned long long *)(base + L.ctr);
        // what must start at zero: the helper board entry (every call), the
        // slot bitmaps where an earlier call on another graph left other
        // data (the kernel clears the bitmaps it sets); the sweep zeroes the
        // work queue, the output counter and the helper counters. The zero
        // fill covers the front of the area, so it runs before the uploads.
        const int64_t bit_words = (int64_t)(SGM_MAX_QV + 1) * g->nwords;
        const bool clear_bits = g_scratch_zero_words[g->device] < bit_words;
        const int64_t zero_words = clear_bits ? (L.bits + 8 * bit_words) / 8 : L.ctr / 8;
        g_scratch_zero_words[g->device] = 0;  // until this call has ended normally
        hipLaunchKernelGGL(k_zero_words, dim3(clear_bits ? 256 : 1), dim3(256), 0, st,
                           (uint64_t *)base, zero_words);
        HIPX(hipGetLastError());
        HIPX(hipMemcpyAsync(base + L.q, &nq, sizeof(NQuery), hipMemcpyHostToDevice, st));
        if (sweep)
            HIPX(hipMemcpyAsync(base + L.preds, &rootp, sizeof(VPred), hipMemcpyHostToDevice, st));
        launch_root_sweep(st, SweepArgs{g->dg, (const VPred *)(base + L.preds), sweep ? 1 : 0,
                                        sweep && rootp.label < 0 ? 1 : 0,
                                        (uint64_t *)(base + L.rootbits), ctr, nullptr, 0});
        HIPX(hipGetLastError());
        NArgs a{};
        a.g = g->dg;
        a.qs = (const NQuery *)(base + L.q);
        a.nq = 1;
        a.res = (NResult *)(base + L.res);
        a.queue = (int32_t *)ctr;
        a.bits = (uint64_t *)(base + L.bits);
        a.lists = (int32_t *)(base + L.lists);
        a.lcap = L.lcap;
        a.slab = base + L.slab;
        a.slab_bytes = kScratchSlab;
        a.rootbits = (const uint64_t *)(base + L.rootbits);
        a.out = (int32_t *)(base + L.out);
        a.out_cap = L.out_bytes / 4;
        a.out_used = ctr + 1;
        a.group_lanes = g->tune.group_lanes;
        a.wg_rows = g->tune.wg_rows;
        a.join_policy = g->tune.join_policy;
        a.nslot = 1;
        a.help_items = g->tune.help_items;
        a.board = (HelpJob *)(base + L.board);
        a.hctr = (int32_t *)(ctr + 2);
        a.help_wait = g->tune.help_wait > 0 ? g->tune.help_wait : kHelpWaitDefault;
        const int grid = a.help_items > 0 ? std::min(kNarrowMaxSlots, std::max(1, g->tune.helpers)) : 1;
        a.ngrid = grid;
        launch_narrow(st, a, grid);
        HIPX(hipGetLastError());
        HIPX(hipMemcpyAsync(&r, base + L.res, sizeof(NResult), hipMemcpyDeviceToHost, st));
        HIPX(hipStreamSynchronize(st));
        // the kernel left the slot bitmaps zero, unless its owner gave up on
        // a shared step (helpers may then have written any of them): the
        // next call clears them first
        if (!(r.status != SGM_OK && r.reason == kWhyHelp)) g_scratch_zero_words[g->device] = bit_words;
        if (r.status != SGM_OK) {
            g_last_error = r.status == kOutFull || r.reason == kWhySlab || r.reason == kWhyList
                               ? "query outgrows the fixed device area (use sgm_match_query)"
                               : "query needs a path the fixed device area does not hold "
                                 "(use sgm_match_query)";
            return r.reason == kWhyKey ? SGM_EUNSUPPORTED : SGM_ENOMEM;
        }
        *n_rows = r.n_rows;
        if (flags & SGM_COUNT_ONLY) return SGM_OK;
        if (r.n_rows > rows_cap) return SGM_ETOOBIG;
        const size_t bytes = sizeof(int32_t) * (size_t)r.n_rows * (size_t)qi.n;
        if (bytes) {
            HIPX(hipMemcpyAsync(rows, base + L.out + 4 * r.offset, bytes, hipMemcpyDeviceToHost, st));
            HIPX(hipStreamSynchronize(st));
        }
    } catch (const DeviceError &e) {
        (void)hipStreamSynchronize(g->stream);
        (void)hipGetLastError();
        return e.code;
    }
    return SGM_OK;
}

}  // extern "C"
