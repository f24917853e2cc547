// C ABI of libcoremaint: host orchestration of the device graph store, the
// initial decomposition and the batched maintenance drivers.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <initializer_list>
#include <mutex>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/coremaint.h"
#include "cm_launch.h"

using namespace cm;

namespace {

// A named host-side range of the library's work (validation, reservation,
// maintenance launches, compaction, the public calls), shown by
// `rocprofv3 --marker-trace`; without a profiler a push / pop is a call
// into a no-op table.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct cm_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    cm_config cfg{};
    Tune tune{};
    int num_cu = 0;
    int coop_maint = 0;   // cooperative grid of the maintenance kernel
    int coop_dec = 0;     // cooperative grid of the decomposition kernel
    int grid_reg = 0;     // grid of regular grid-stride kernels

    DevGraph g{};
    DevBatch b{};
    DevQueues q{};
    Ctl *ctl = nullptr;       // device
    Bar *bar = nullptr;       // device grid-barrier state
    Ctl *hctl = nullptr;      // pinned host mirror
    int32_t batch_cap = 0;    // capacity of batch arrays
    int32_t hash_cap = 0;     // allocated hash slots
    int32_t scan_cap = 0;
    int32_t *src_buf = nullptr, *dst_buf = nullptr;  // device staging of host inputs
    int64_t *scan_tmp = nullptr;
    int64_t scan_tmp_cap = 0;
    int64_t *i64_scratch = nullptr;   // small device scratch (totals)
    unsigned long long *u64_scratch = nullptr;
    unsigned long long *hu64 = nullptr;  // pinned host scratch
    int32_t *firstidx = nullptr;      // [n_cap] vertex-deletion duplicate check
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // plain form: outcomes of the maintenance launches in flight (pinned) and
    // their start / end events
    static constexpr int LSLOTS = 4;
    LaunchOut *lout = nullptr;
    hipEvent_t lev[LSLOTS][2] = {};
    int coop_prog = 0;        // cooperative grid of the batch program kernel
    // batch programs (cm_run_batches)
    ProgDesc *d_prog = nullptr;
    ProgDesc *h_prog = nullptr;       // pinned
    ProgBatch *d_pbatch = nullptr;
    ProgOut *d_pout = nullptr;
    int32_t prog_cap = 0;
    int32_t *d_isrc = nullptr, *d_idst = nullptr, *d_isub = nullptr;  // staged host items
    int64_t items_cap = 0;
    unsigned long long *d_sub_bad = nullptr;
    int32_t sub_cap = 0;
    DebugLog dl{};            // iteration log (cfg.debug), allocated by cm_create
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<char> graph_key;
    // serving (cm_serve_*): pinned request ring read by a persistent launch
    bool serving = false;
    bool serve_live = false;        // a serving launch is in flight
    cm_serve_config scfg{};
    int coop_serve = 0;
    ServeHdr *shdr = nullptr;       // pinned
    ProgBatch *sring = nullptr;     // pinned [ring_requests]
    ProgOut *sout = nullptr;        // pinned [ring_requests]
    int32_t *d_bsub = nullptr;      // request index of each item of a fused batch [batch_cap]
    int32_t *ssrc = nullptr, *sdst = nullptr;  // pinned payload [ring_items]
    int64_t s_next = 0;             // tickets issued (= batches published)
    int64_t s_done = 0;             // batches finished (host view)
    int64_t s_first = 0;            // first batch of the live launch
    int64_t s_pay_tail = 0;         // payload slots handed out (monotonic)
    std::vector<int64_t> s_pstart;  // per ring slot: monotonic payload start
    std::vector<int64_t> s_bytes;   // per ring slot: bytes charged to the budget
    std::vector<int32_t> s_nids;    // per ring slot: ids in use after the batch
    int64_t s_inflight = 0;         // bytes charged by unfinished requests
    int32_t s_n_ids = 0;            // ids handed out (host view, pending insertions included)
    bool s_grow = false;            // vertex capacity must grow at the next stop
    int64_t s_pending_ins = 0;      // items of unfinished insertions (repack sizing)
    std::vector<cm_batch_stats> s_results;

    bool loaded = false;
    bool decomposed = false;
    bool poisoned = false;
    int clock_khz = 0;        // device wall clock rate
    bool no_alloc = false;    // inside cm_update_edges_noalloc: the pool may not grow
    void *na_scratch = nullptr;  // this device's address of the allocation-free scratch array
    int64_t m = 0;
    int32_t n_alive = 0;
    int32_t epoch = 0;
    int32_t bstamp = 0;
    std::string err;
};

// ---------------------------------------------------------------------------
// Allocation-free edge updates (cm_update_edges_noalloc): the batch arrays,
// the batch hash and the locate-scan queue of one call live in this
// file-scope device array instead of buffers the handle allocates.  Every
// GPU holds its own copy at its own address, looked up once per device.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t NA_ITEMS = CM_NOALLOC_MAX_ITEMS;  // largest batch
constexpr int64_t NA_HASH = 2 * NA_ITEMS;           // hash slots for it (power of two)
constexpr int64_t NA_SCAN = (int64_t)1 << 20;       // locate-scan chunk items
constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
// layout: int32 err, eu, ev, hslot, rem0, rem1, sel, esel [NA_ITEMS]; int64 su, sv [NA_ITEMS];
// u64 hkey [NA_HASH]; int32 hval [NA_HASH]; int64 scanq [NA_SCAN]
constexpr size_t NA_I32 = na_align(sizeof(int32_t) * NA_ITEMS);
constexpr size_t NA_I64 = na_align(sizeof(int64_t) * NA_ITEMS);
constexpr size_t NA_BYTES = 8 * NA_I32 + 2 * NA_I64 + na_align(sizeof(unsigned long long) * NA_HASH) +
                            na_align(sizeof(int32_t) * NA_HASH) + na_align(sizeof(int64_t) * NA_SCAN);
constexpr int NA_DEVICES = 64;
std::mutex na_mu;
void *na_addr[NA_DEVICES] = {};
}  // namespace

__device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
// Address of this device's scratch array (the device must be current);
// resolved once per device.
hipError_t na_lookup(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= NA_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(na_mu);
    if (!na_addr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        na_addr[device] = p;
    }
    *out = na_addr[device];
    return hipSuccess;
}
}  // namespace

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace {

struct Fail {
    int code;
};

void serve_free(cm_graph *g);

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) {                                                        \
            g->poisoned = true;                                                        \
            g->err = std::string("HIP error ") + hipGetErrorString(_e) + " at " #expr; \
            throw Fail{CM_E_DEVICE};                                                   \
        }                                                                              \
    } while (0)

template <class T>
void dev_alloc(cm_graph *g, T **p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        g->err = "device allocation of " + std::to_string(sizeof(T) * (size_t)count) + " bytes failed";
        throw Fail{CM_E_NOMEM};
    }
}

template <class T>
void dev_free(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Refuse to launch with a missing buffer (a null device pointer would make
// the kernel fault).
void require_ptrs(cm_graph *g, std::initializer_list<const void *> ps, const char *what) {
    for (const void *p : ps) {
        if (!p) {
            g->poisoned = true;
            g->err = std::string("internal: missing device buffer for ") + what;
            throw Fail{CM_E_INTERNAL};
        }
    }
}

KArgs make_args(cm_graph *g) {
    require_ptrs(g, {g->ctl, g->bar, g->i64_scratch, g->u64_scratch}, "control block");
    if (g->loaded) {
        const DevGraph &d = g->g;
        require_ptrs(g, {d.off, d.len, d.cap, d.nbr, d.core, d.mcd, d.stamp.p, d.chg, d.cd.p, d.dec,
                         d.done, d.matched, d.claim, d.bmark, d.gain},
                     "graph arrays");
        const DevQueues &q = g->q;
        require_ptrs(g, {q.fq[0], q.fq[1], q.fh[0], q.fh[1], q.eq[0], q.eq[1],
                         q.eh[0], q.eh[1], q.cand, q.chg, q.chh, q.touched, g->b.vlist, g->b.reloc,
                         g->b.reloc_off, g->b.reloc_cap, g->scan_tmp, g->firstidx},
                     "queues");
    }
    KArgs a{};
    a.g = g->g;
    a.b = g->b;
    a.q = g->q;
    a.t = g->tune;
    a.ctl = g->ctl;
    a.bar = g->bar;
    a.dl = g->dl;
    return a;
}

// Bounds of the kernels' waits, in device wall-clock ticks: a grid barrier
// wait may last BAR_WAIT_MS plus `extra_ms` (a serving launch's idle wait,
// during which one thread waits for the host while the others sit at the
// barrier), a workgroup's chain of local steps runs at most LOCAL_SLICE_MS
// before it passes a barrier.
constexpr unsigned long long BAR_WAIT_MS = 10000, LOCAL_SLICE_MS = 20;
void set_bar_bounds(cm_graph *g, int64_t extra_ms) {
    const unsigned long long khz = (unsigned long long)g->clock_khz;
    const unsigned long long v[2] = {(BAR_WAIT_MS + (unsigned long long)std::max<int64_t>(extra_ms, 0)) * khz,
                                     LOCAL_SLICE_MS * khz};
    HIPCHK(hipMemcpyAsync(&g->bar->wait_ticks[0], &v[0], sizeof(v[0]), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(&g->bar->slice_ticks[0], &v[1], sizeof(v[1]), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
}

// Batch stamps (bmark values) restart before they could overflow: the host
// clears the marks between calls.
void bstamp_guard(cm_graph *g) {
    if (g->bstamp < (1 << 29) || !g->g.bmark) return;
    HIPCHK(fill_i32(g->g.bmark, 0, g->g.n_cap, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    g->bstamp = 0;
}

// Debug mode: every update call starts an empty iteration log.
void debug_reset(cm_graph *g) {
    bstamp_guard(g);
    if (g->dl.n) HIPCHK(fill_u64(g->dl.n, 0ull, 2, g->stream));
}

void sync_ctl(cm_graph *g) {
    HIPCHK(hipMemcpyAsync(g->hctl, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
}

// After a cooperative launch: a grid barrier that gave up waiting (a
// workgroup never arrived) poisons the handle.
void check_abort(cm_graph *g) {
    unsigned int ab = 0;
    HIPCHK(hipMemcpyAsync(&ab, &g->bar->abort[0], sizeof(ab), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    if (ab) {
        g->poisoned = true;
        g->err = "internal: grid barrier wait gave up";
        throw Fail{CM_E_INTERNAL};
    }
}

void check_overflow(cm_graph *g) {
    if (g->hctl->overflow) {
        g->poisoned = true;
        g->err = "internal queue overflow (code " + std::to_string(g->hctl->overflow) + ")";
        throw Fail{CM_E_INTERNAL};
    }
}

// Per-vertex arrays (re)allocation to n_cap ids, keeping the first n_keep.
void alloc_vertex_arrays(cm_graph *g, int32_t n_cap, int32_t n_keep) {
    DevGraph ng = g->g;
    ng.n_cap = n_cap;
    hipStream_t st = g->stream;
    auto grow32 = [&](int32_t *&dst, int32_t *old, int32_t fillv, int per = 1) {
        dev_alloc(g, &dst, (int64_t)per * n_cap);
        HIPCHK(fill_i32(dst, fillv, (int64_t)per * n_cap, st));
        if (old && n_keep > 0)
            HIPCHK(hipMemcpyAsync(dst, old, sizeof(int32_t) * (size_t)per * (size_t)n_keep,
                                  hipMemcpyDeviceToDevice, st));
    };
    grow32(ng.len, g->g.len, 0);
    grow32(ng.cap, g->g.cap, 0);
    grow32(ng.core, g->g.core, -1);
    grow32(ng.mcd, g->g.mcd, 0);
    grow32(ng.stamp.p, g->g.stamp.p, 0, 2);  // (stamp, cd) records: two words per id
    grow32(ng.chg, g->g.chg, 0);
    ng.cd.p = ng.stamp.p + 1;
    grow32(ng.dec, g->g.dec, 0);
    grow32(ng.done, g->g.done, 0);
    grow32((int32_t *&)ng.matched, (int32_t *)g->g.matched, 0);
    grow32(ng.bmark, g->g.bmark, 0);
    grow32(ng.gain, g->g.gain, 0);
    if (g->tune.sublists) grow32(ng.slen, g->g.slen, 0);
    if (g->tune.uplists) grow32(ng.ubl, g->g.ubl, -1);
    dev_alloc(g, &ng.off, n_cap);
    HIPCHK(fill_i64(ng.off, 0, n_cap, st));
    if (g->g.off && n_keep > 0)
        HIPCHK(hipMemcpyAsync(ng.off, g->g.off, sizeof(int64_t) * (size_t)n_keep, hipMemcpyDeviceToDevice, st));
    dev_alloc(g, &ng.claim, n_cap);
    HIPCHK(fill_u64(ng.claim, ~0ull, n_cap, st));
    if (g->g.claim && n_keep > 0)
        HIPCHK(hipMemcpyAsync(ng.claim, g->g.claim, sizeof(unsigned long long) * (size_t)n_keep,
                              hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    DevGraph old = g->g;
    dev_free(old.len); dev_free(old.cap); dev_free(old.core); dev_free(old.mcd);
    dev_free(old.stamp.p); dev_free(old.chg); dev_free(old.dec);
    dev_free(old.done); dev_free(old.matched); dev_free(old.bmark); dev_free(old.gain);
    dev_free(old.off); dev_free(old.claim); dev_free(old.slen); dev_free(old.ubl);
    ng.nbr = g->g.nbr;
    ng.sub = g->g.sub;
    ng.upl = g->g.upl;
    ng.pool_size = g->g.pool_size;
    ng.n_ids = g->g.n_ids;
    g->g = ng;

    // vertex-sized batch / queue arrays
    dev_free(g->b.vlist); dev_free(g->b.reloc); dev_free(g->b.reloc_off); dev_free(g->b.reloc_cap);
    dev_alloc(g, &g->b.vlist, n_cap);
    dev_alloc(g, &g->b.reloc, n_cap);
    dev_alloc(g, &g->b.reloc_off, n_cap);
    dev_alloc(g, &g->b.reloc_cap, n_cap);
    for (int i = 0; i < 2; ++i) {
        dev_free(g->q.fq[i]); dev_free(g->q.eq[i]);
        dev_alloc(g, &g->q.fq[i], n_cap);
        dev_alloc(g, &g->q.eq[i], n_cap);
    }
    dev_free(g->q.cand); dev_free(g->q.chg); dev_free(g->q.touched);
    dev_alloc(g, &g->q.cand, n_cap);
    dev_alloc(g, &g->q.chg, n_cap);
    dev_alloc(g, &g->q.touched, n_cap);
    g->q.vcap = n_cap;
    dev_free(g->firstidx);
    dev_alloc(g, &g->firstidx, n_cap);
    HIPCHK(fill_i32(g->firstidx, INT_MAX, n_cap, st));
    int64_t need_tmp = scan_tmp_len(n_cap);
    if (need_tmp > g->scan_tmp_cap) {
        dev_free(g->scan_tmp);
        dev_alloc(g, &g->scan_tmp, need_tmp);
        g->scan_tmp_cap = need_tmp;
    }
}

// Chunk queues sized for n_cap + pool/chunk items.
void alloc_chunk_queues(cm_graph *g) {
    int64_t h = (int64_t)g->g.n_cap + g->g.pool_size / std::max(1, g->tune.chunk) + 1024;
    if (h > INT_MAX) h = INT_MAX;
    if (h > g->q.hcap) {
        for (int i = 0; i < 2; ++i) {
            dev_free(g->q.fh[i]); dev_free(g->q.eh[i]);
            dev_alloc(g, &g->q.fh[i], h);
            dev_alloc(g, &g->q.eh[i], h);
        }
        dev_free(g->q.chh);
        dev_alloc(g, &g->q.chh, h);
        g->q.hcap = (int32_t)h;
    }
    if (g->tune.async_steps) {
        // an asynchronous step holds every item it creates: vertices (each at
        // most once) plus two chunk items per chunk of a claimed list
        const int64_t ac = std::min<int64_t>((int64_t)g->g.n_cap + 2 * (int64_t)g->q.hcap, INT_MAX);
        if (ac > g->q.acap) {
            for (int i = 0; i < 2; ++i) {
                dev_free(g->q.aq[i]);
                dev_alloc(g, &g->q.aq[i], ac);
                HIPCHK(fill_u64(g->q.aq[i], ~0ull, ac, g->stream));
            }
            g->q.acap = (int32_t)ac;
        }
    }
}

void ensure_vertex_capacity(cm_graph *g, int64_t need) {
    if (need <= g->g.n_cap) return;
    if (g->cfg.vertex_capacity > 0 && need > g->cfg.vertex_capacity) {
        g->err = "vertex capacity exceeded";
        throw Fail{CM_E_CAPACITY};
    }
    if (need > INT_MAX - 1) {
        g->err = "vertex ids exceed int32";
        throw Fail{CM_E_CAPACITY};
    }
    int64_t nc = std::max<int64_t>(need, (int64_t)g->g.n_cap + g->g.n_cap / 2 + 1024);
    if (g->cfg.vertex_capacity > 0) nc = std::min<int64_t>(nc, g->cfg.vertex_capacity);
    nc = std::min<int64_t>(nc, INT_MAX - 1);
    alloc_vertex_arrays(g, (int32_t)nc, g->g.n_ids);
    alloc_chunk_queues(g);
}

void ensure_batch(cm_graph *g, int64_t s) {
    if (s > INT_MAX / 2) {
        g->err = "batch too large";
        throw Fail{CM_E_ARG};
    }
    if (s > g->batch_cap) {
        int64_t c = std::max<int64_t>(s, 1024);
        DevBatch &b = g->b;
        dev_free(b.err); dev_free(b.eu); dev_free(b.ev); dev_free(b.su); dev_free(b.sv);
        dev_free(b.hslot); dev_free(b.rem[0]); dev_free(b.rem[1]); dev_free(b.sel); dev_free(b.esel);
        dev_free(g->src_buf); dev_free(g->dst_buf);
        dev_alloc(g, &b.err, c); dev_alloc(g, &b.eu, c); dev_alloc(g, &b.ev, c);
        dev_alloc(g, &b.su, c); dev_alloc(g, &b.sv, c); dev_alloc(g, &b.hslot, c);
        dev_alloc(g, &b.rem[0], c); dev_alloc(g, &b.rem[1], c); dev_alloc(g, &b.sel, c);
        dev_alloc(g, &b.esel, c);
        HIPCHK(fill_i32(b.esel, 0, c, g->stream));
        dev_alloc(g, &g->src_buf, c); dev_alloc(g, &g->dst_buf, c);
        b.cap = (int32_t)c;
        g->batch_cap = (int32_t)c;
    }
    int64_t hc = next_pow2(std::max<int64_t>(2 * s, 1024));
    if (hc > g->hash_cap) {
        dev_free(g->b.hkey); dev_free(g->b.hval);
        dev_alloc(g, &g->b.hkey, hc);
        dev_alloc(g, &g->b.hval, hc);
        g->hash_cap = (int32_t)hc;
    }
    g->b.hcap = (int32_t)hc;
    HIPCHK(fill_u64(g->b.hkey, ~0ull, hc, g->stream));
    HIPCHK(fill_i32(g->b.hval, INT_MAX, hc, g->stream));
    int64_t sc = 2 * s + g->g.pool_size / std::max(1, g->tune.chunk) + 1024;
    sc = std::min<int64_t>(sc, INT_MAX);
    if (sc > g->scan_cap) {
        dev_free(g->b.scanq);
        dev_alloc(g, &g->b.scanq, sc);
        g->scan_cap = (int32_t)sc;
    }
    g->b.scap = g->scan_cap;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Build (or rebuild) the adjacency pool so that every live list gets slack;
// lists keep their order, tombstones are dropped.  extra = slots to add to
// the pool beyond the packed size.
void repack(cm_graph *g, int64_t extra) {
    Range range("coremaint.repack");
    hipStream_t st = g->stream;
    KArgs a = make_args(g);
    int32_t *cnt = g->g.gain;  // gain is zero between batches; used as scratch here
    HIPCHK(count_live(a, cnt, g->grid_reg, st));
    int64_t *caps64 = nullptr, *newoff = nullptr;
    dev_alloc(g, &caps64, g->g.n_cap);
    dev_alloc(g, &newoff, g->g.n_cap);
    HIPCHK(caps_from_counts(cnt, g->g.n_ids, g->g.n_cap, caps64, g->g.cap, st));
    HIPCHK(exclusive_scan_i64(caps64, newoff, g->g.n_cap, g->scan_tmp, g->i64_scratch, st));
    int64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, g->i64_scratch, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int64_t pool = total + std::max<int64_t>(extra, total / 4) + 4096;
    if (g->cfg.edge_capacity_hint > pool) pool = g->cfg.edge_capacity_hint;
    int32_t *newnbr = nullptr;
    dev_alloc(g, &newnbr, pool);
    if (g->tune.sublists) {
        // supporter lists live only within an iteration: nothing to copy
        dev_free(g->g.sub);
        dev_alloc(g, &g->g.sub, pool);
    }
    if (g->tune.uplists) {
        // every up-list is invalidated with the move (repack_finish)
        dev_free(g->g.upl);
        dev_alloc(g, &g->g.upl, pool);
    }
    HIPCHK(repack_copy(a, newoff, newnbr, g->grid_reg, st));
    HIPCHK(repack_finish(a, newoff, cnt, g->grid_reg, st));
    HIPCHK(fill_i32(cnt, 0, g->g.n_cap, st));
    HIPCHK(hipStreamSynchronize(st));
    dev_free(caps64);
    dev_free(newoff);
    dev_free(g->g.nbr);
    g->g.nbr = newnbr;
    g->g.pool_size = pool;
    unsigned long long tail = (unsigned long long)total;
    HIPCHK(ctl_set_pool(g->ctl, tail, st));
    HIPCHK(hipStreamSynchronize(st));
    g->hctl->pool_tail = tail;
    g->hctl->garbage = 0;
    alloc_chunk_queues(g);
}

int finish(cm_graph *g, int code, cm_batch_stats *stats, double t0) {
    if (stats) {
        stats->status = code;
        stats->ms_total = now_ms() - t0;
    }
    if (code == CM_OK) g->err.clear();
    return code;
}

void fill_stats(cm_graph *g, cm_batch_stats *st, int64_t applied, int64_t dropped, int64_t first_bad) {
    if (!st) return;
    const Ctl &c = *g->hctl;
    st->iterations = (int32_t)c.st_iters;
    st->first_bad = first_bad;
    st->applied = applied;
    st->dropped = dropped;
    st->remaining_sum = (int64_t)c.st_remaining;
    st->candidates = (int64_t)c.st_candidates;
    st->evicted = (int64_t)c.st_evicted;
    st->changed = (int64_t)c.st_changed;
    st->scanned = (int64_t)c.st_scanned;
    st->rounds = (int64_t)c.st_rounds;
    st->grid_steps = (int64_t)c.st_grid_steps;
    st->local_steps = (int64_t)c.st_local_steps;
    st->cand_degree = (int64_t)c.st_cdeg;
    st->evicted_degree = (int64_t)c.st_edeg;
    st->changed_degree = (int64_t)c.st_hdeg;
}

// Algorithmic bytes of a batch: what the method itself must move, from the
// sets Algorithms 1-7 define, counted once per access (no cache effects) and
// independent of how many list entries the kernels happen to scan:
//  partition, per remaining edge per iteration: edge 8 + two core gathers 8
//    + claim atomic and read 8 + compaction 8 = 32
//  validation and apply, per applied edge: 2 x (length atomic 4 + entry 4 +
//    slot 4) + SD deltas 8 + validation 8 = 40
//  per insertion candidate (CSD count) and per evicted / peeled vertex
//    (counter decrements): offset and length 16 + per list entry id, core
//    and SD or counter 12
//  per vertex whose core moved: per list entry 20 (SD recount: id + core;
//    neighbour delta: core + atomic + id)
int64_t alg_bytes(unsigned long long remaining, unsigned long long applied, unsigned long long icand,
                  unsigned long long cdeg, unsigned long long evicted, unsigned long long edeg,
                  unsigned long long hdeg) {
    return (int64_t)(32ull * remaining + 40ull * applied + 16ull * icand + 12ull * cdeg + 16ull * evicted +
                     12ull * edeg + 20ull * hdeg);
}
int64_t alg_bytes(const Ctl &c) {
    return alg_bytes(c.st_remaining, c.st_selected, c.st_icand, c.st_cdeg, c.st_evicted, c.st_edeg, c.st_hdeg);
}
int64_t alg_bytes(const ProgOut &o) {
    return alg_bytes(o.remaining, o.selected, o.icand, o.cdeg, o.evicted, o.edeg, o.hdeg);
}

// Validate a batch already staged in g->b.src_in/dst_in (s items).  Returns
// the number of valid items; in strict mode throws on the first bad item.
int64_t validate(cm_graph *g, int64_t s, bool inserting, bool strict, int64_t *first_bad,
                 int cur, cm_batch_stats *stats, bool packed) {
    Range range("coremaint.validate");
    hipStream_t st = g->stream;
    g->bstamp += 2;
    HIPCHK(ctl_batch_reset(g->ctl, cur, st));
    KArgs a = make_args(g);
    a.inserting = inserting ? 1 : 0;
    a.s = (int32_t)s;
    a.bstamp = g->bstamp;
    a.cur = cur;
    a.strict = strict ? 1 : 0;
    if (!packed) a.b.sub_in = nullptr;
    HIPCHK(validate_batch(a, g->grid_reg, st));
    sync_ctl(g);
    check_overflow(g);
    int32_t fb = g->hctl->first_bad;
    *first_bad = fb == INT_MAX ? -1 : fb;
    if (stats) stats->first_bad = *first_bad;
    if (fb != INT_MAX && strict && !packed) {
        int32_t code = 0;
        HIPCHK(hipMemcpyAsync(&code, g->b.err + fb, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        g->err = std::string("invalid batch item ") + std::to_string(fb) + ": " + cm_strerror(code);
        throw Fail{code};
    }
    return g->hctl->rem_count[cur];
}

// Make room for an insertion batch (validated list `cur`) before any
// mutation: lists that cannot take their new edges move to spill blocks;
// if the pool is full it is repacked into a larger one and the step redone.
void reserve(cm_graph *g, int cur) {
    Range range("coremaint.reserve");
    hipStream_t st = g->stream;
    for (int attempt = 0; attempt < 4; ++attempt) {
        KArgs a = make_args(g);
        a.inserting = 1;
        a.bstamp = g->bstamp;
        a.cur = cur;
        // clear counters used by the reservation (keep validation results)
        HIPCHK(ctl_reserve_reset(g->ctl, st));
        HIPCHK(reserve_gain(a, g->grid_reg, st));
        HIPCHK(reserve_alloc_copy(a, g->grid_reg, st));
        sync_ctl(g);
        check_overflow(g);
        if (!g->hctl->pool_fail) return;
        if (g->no_alloc) {
            g->err = "adjacency pool full (the allocation-free call cannot grow it; nothing was applied)";
            throw Fail{CM_E_CAPACITY};
        }
        // pool exhausted: repack with room for this batch, then redo
        int64_t extra = 4 * (int64_t)g->hctl->rem_count[cur] + (int64_t)g->g.pool_size / 2;
        repack(g, extra);
        g->bstamp += 2;
    }
    g->err = "adjacency pool could not be grown";
    throw Fail{CM_E_NOMEM};
}

// Plain form: one cooperative launch per superior edge set.  The next
// launch is queued before the host reads the outcome of the current one
// (from its pinned LaunchOut slot, after its end event), so the device does
// not idle while the host decides; a launch that finds no edges left runs no
// iteration and changes nothing, so the last queued launch of a batch is an
// empty one.
void run_plain(cm_graph *g, KArgs a, double &kms, int &launches) {
    hipStream_t st = g->stream;
    constexpr int depth = 2;  // launches in flight
    int64_t issued = 0, consumed = 0;
    auto issue = [&]() {
        const int s = (int)(issued % cm_graph::LSLOTS);
        a.lout = &g->lout[s];
        HIPCHK(hipEventRecord(g->lev[s][0], st));
        HIPCHK(maintain_coop(a, g->coop_maint, st));
        HIPCHK(hipEventRecord(g->lev[s][1], st));
        ++issued;
    };
    // wait for launch `consumed`, account for it and return its outcome
    auto take = [&]() {
        const int s = (int)(consumed % cm_graph::LSLOTS);
        HIPCHK(hipEventSynchronize(g->lev[s][1]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g->lev[s][0], g->lev[s][1]));
        kms += ms;
        ++launches;
        ++consumed;
        const LaunchOut o = g->lout[s];
        if (o.aborted) {
            g->poisoned = true;
            g->err = "internal: grid barrier wait gave up";
            throw Fail{CM_E_INTERNAL};
        }
        if (o.overflow) {
            g->poisoned = true;
            g->err = "internal queue overflow (code " + std::to_string(o.overflow) + ")";
            throw Fail{CM_E_INTERNAL};
        }
        return o;
    };
    issue();
    for (;;) {
        if (issued - consumed < depth) issue();
        const LaunchOut o = take();
        if (o.rem_next == 0) break;
        if (o.iters == 0) {
            g->poisoned = true;
            g->err = "maintenance launch made no progress";
            throw Fail{CM_E_INTERNAL};
        }
    }
    while (consumed < issued) {
        const LaunchOut o = take();
        if (o.iters != 0) {  // a launch queued after the last set found edges
            g->poisoned = true;
            g->err = "internal: a queued maintenance launch ran after the batch ended";
            throw Fail{CM_E_INTERNAL};
        }
    }
    sync_ctl(g);
}

// Run the iterations of a validated batch (list `cur`) to completion.
void run_maintenance(cm_graph *g, bool inserting, cm_batch_stats *stats) {
    Range range("coremaint.maintain");
    hipStream_t st = g->stream;
    KArgs a = make_args(g);
    a.inserting = inserting ? 1 : 0;
    a.max_iters = g->cfg.mode == CM_MODE_PERSISTENT ? INT_MAX : 1;
    double kms = 0.0;
    int launches = 0;
    if (g->cfg.mode != CM_MODE_PERSISTENT) {
        run_plain(g, a, kms, launches);
        g->epoch = g->hctl->epoch;
    } else {
        for (;;) {
            if (g->cfg.timing) HIPCHK(hipEventRecord(g->ev0, st));
            HIPCHK(maintain_coop(a, g->coop_maint, st));
            if (g->cfg.timing) HIPCHK(hipEventRecord(g->ev1, st));
            ++launches;
            sync_ctl(g);
            check_abort(g);
            check_overflow(g);
            if (g->cfg.timing) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
                kms += ms;
            }
            g->epoch = g->hctl->epoch;
            int nxt = (g->epoch + 1) & 1;
            if (g->hctl->rem_count[nxt] == 0) break;
            if (g->hctl->iters_done == 0) {
                g->poisoned = true;
                g->err = "maintenance launch made no progress";
                throw Fail{CM_E_INTERNAL};
            }
        }
    }
    if (stats) {
        stats->launches = launches;
        stats->kernel_ms = kms;
        stats->alg_bytes = alg_bytes(*g->hctl);
    }
}

// Shared body of edge insertion / deletion on staged device inputs.
int64_t edge_batch(cm_graph *g, int64_t s, bool inserting, cm_batch_stats *stats, int64_t *dropped,
                   bool strict_override, bool strict_value, bool packed = false) {
    hipStream_t st = g->stream;
    bool strict = strict_override ? strict_value : g->cfg.strict != 0;
    int cur = (g->epoch + 1) & 1;
    int64_t fb = -1;
    int64_t valid = validate(g, s, inserting, strict, &fb, cur, stats, packed);
    *dropped = s - valid;
    if (stats) stats->first_bad = fb;
    if (valid == 0) {
        if (stats) fill_stats(g, stats, 0, *dropped, fb);
        return 0;
    }
    if (stats) {
        stats->group = 1;
        stats->first_stamp = g->epoch + 1;
    }
    KArgs a = make_args(g);
    a.inserting = inserting ? 1 : 0;
    a.cur = cur;
    if (inserting) {
        reserve(g, cur);
    } else {
        HIPCHK(ctl_reserve_reset(g->ctl, st));
        a.bstamp = g->bstamp;
        HIPCHK(reserve_gain(a, g->grid_reg, st));  // endpoints + tombstone counts
    }
    run_maintenance(g, inserting, stats);
    if (!inserting) {
        Range range("coremaint.compact");
        KArgs c = make_args(g);
        HIPCHK(delete_compact(c, g->grid_reg, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    // statistics of the whole batch are in the mirror read by the last sync
    sync_ctl(g);
    if (stats) {
        int32_t launches = stats->launches;
        double kms = stats->kernel_ms;
        int64_t ab = stats->alg_bytes;
        fill_stats(g, stats, valid, *dropped, fb);
        stats->launches = launches;
        stats->kernel_ms = kms;
        stats->alg_bytes = ab;
    }
    g->m += inserting ? valid : -valid;
    return valid;
}

// Launch the batch program (device descriptor already written): directly as
// a cooperative kernel, or by replaying an instantiated hipGraph whose single
// cooperative kernel node carries the current KArgs (rebuilt when any buffer
// address or size in KArgs changed).  Returns 1 when the graph was used.
int launch_program(cm_graph *g, const KArgs &a) {
    hipStream_t st = g->stream;
    if (!g->cfg.use_graph) {
        HIPCHK(program_coop(a, g->coop_prog, st));
        return 0;
    }
    std::vector<char> key(sizeof(KArgs) + sizeof(int));
    std::memcpy(key.data(), &a, sizeof(KArgs));
    std::memcpy(key.data() + sizeof(KArgs), &g->coop_prog, sizeof(int));
    if (!g->gexec || key != g->graph_key) {
        if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        g->gexec = nullptr;
        g->graph = nullptr;
        KArgs copy = a;
        void *args[] = {&copy};
        hipKernelNodeParams p{};
        p.func = const_cast<void *>(program_kernel());
        p.gridDim = dim3(g->coop_prog);
        p.blockDim = dim3(COOP_THREADS);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        HIPCHK(hipGraphCreate(&g->graph, 0));
        HIPCHK(hipGraphAddKernelNode(&node, g->graph, nullptr, 0, &p));
        hipKernelNodeAttrValue v;
        std::memset(&v, 0, sizeof(v));
        v.cooperative = 1;
        HIPCHK(hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v));
        HIPCHK(hipGraphInstantiate(&g->gexec, g->graph, nullptr, nullptr, 0));
        g->graph_key = key;
    }
    HIPCHK(hipGraphLaunch(g->gexec, st));
    return 1;
}

// Run the batch program pb (items in ds / dd [/ dsub], device memory) in
// persistent launches: one launch, or more when the adjacency pool must be
// repacked (the launch stops before mutating the batch that ran out; the
// host repacks and relaunches from there).  out receives every batch's
// outcome.
void program_execute(cm_graph *g, const std::vector<ProgBatch> &pb, const int32_t *ds, const int32_t *dd,
                     const int32_t *dsub, bool strict, std::vector<ProgOut> &out, int *used_graph_out,
                     double *kms_out, int *launches_out) {
    hipStream_t st = g->stream;
    const int32_t nb = (int32_t)pb.size();
    out.assign((size_t)nb, ProgOut{});
    if (nb > g->prog_cap) {
        dev_free(g->d_pbatch);
        dev_free(g->d_pout);
        int32_t c = std::max(nb, 64);
        dev_alloc(g, &g->d_pbatch, c);
        dev_alloc(g, &g->d_pout, c);
        g->prog_cap = c;
    }
    HIPCHK(hipMemcpyAsync(g->d_pbatch, pb.data(), sizeof(ProgBatch) * (size_t)nb, hipMemcpyHostToDevice, st));
    int32_t first = 0;
    int used_graph = 0;
    double kms = 0.0;
    int launches = 0;
    for (int attempt = 0; attempt < 8; ++attempt) {
        ProgDesc *hd = g->h_prog;
        std::memset(hd, 0, sizeof(ProgDesc));
        hd->gsrc = g->src_buf;
        hd->gdst = g->dst_buf;
        hd->gcap = g->batch_cap;
        hd->firstidx = g->firstidx;
        hd->batches = g->d_pbatch;
        hd->out = g->d_pout;
        hd->src = ds;
        hd->dst = dd;
        hd->sub = dsub;
        hd->sub_bad = dsub ? g->d_sub_bad : nullptr;
        hd->nb = nb;
        hd->first = first;
        hd->strict = strict ? 1 : 0;
        hd->bstamp0 = g->bstamp + 2;
        hd->stop = first;
        hd->pool_fail = 0;
        g->bstamp += 2 * (nb - first) + 2;
        HIPCHK(hipMemcpyAsync(g->d_prog, hd, sizeof(ProgDesc), hipMemcpyHostToDevice, st));
        KArgs a = make_args(g);
        a.prog = g->d_prog;
        if (g->cfg.timing) HIPCHK(hipEventRecord(g->ev0, st));
        used_graph |= launch_program(g, a);
        if (g->cfg.timing) HIPCHK(hipEventRecord(g->ev1, st));
        ++launches;
        HIPCHK(hipMemcpyAsync(g->h_prog, g->d_prog, sizeof(ProgDesc), hipMemcpyDeviceToHost, st));
        sync_ctl(g);
        check_abort(g);
        check_overflow(g);
        if (g->cfg.timing) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
            kms += ms;
        }
        g->epoch = g->hctl->epoch;
        int32_t stop = g->h_prog->stop;
        if (stop > first)
            HIPCHK(hipMemcpy(out.data() + first, g->d_pout + first, sizeof(ProgOut) * (size_t)(stop - first),
                             hipMemcpyDeviceToHost));
        if (!g->h_prog->pool_fail) {
            if (stop != nb) {
                g->poisoned = true;
                g->err = "batch program stopped early";
                throw Fail{CM_E_INTERNAL};
            }
            break;
        }
        // adjacency pool exhausted at batch `stop`: repack with room, resume there
        int64_t pending = 0;
        for (int32_t j = stop; j < nb; ++j)
            if (pb[j].kind == 0 || pb[j].kind == 2) pending += pb[j].s;
        repack(g, 4 * pending + g->g.pool_size / 2);
        first = stop;
        if (attempt == 7) {
            g->err = "adjacency pool could not be grown";
            throw Fail{CM_E_NOMEM};
        }
    }
    *used_graph_out = used_graph;
    *kms_out = kms;
    *launches_out = launches;
}

// Outcome of one program batch as the one-call statistics.
void stats_from_out(cm_graph *g, const ProgOut &o, int64_t items, int launches, double kms, cm_batch_stats *r) {
    if (!r) return;
    r->status = o.status;
    r->iterations = o.iterations;
    r->first_bad = o.first_bad;
    r->applied = o.valid;
    r->dropped = o.status == 0 ? items - o.valid : 0;
    r->remaining_sum = (int64_t)o.remaining;
    r->candidates = (int64_t)o.candidates;
    r->evicted = (int64_t)o.evicted;
    r->changed = (int64_t)o.changed;
    r->scanned = (int64_t)o.scanned;
    r->rounds = (int64_t)o.rounds;
    r->local_steps = (int64_t)o.steps;
    r->group = 1;
    r->first_stamp = o.ep0;
    r->alg_bytes = alg_bytes(o);
    r->cand_degree = (int64_t)o.cdeg;
    r->evicted_degree = (int64_t)o.edeg;
    r->changed_degree = (int64_t)o.hdeg;
    r->launches = launches;
    r->kernel_ms = kms;
}

template <class T>
void grow_dev(cm_graph *g, T *&p, int64_t &cap_io, int64_t need) {
    if (need <= cap_io && p) return;
    dev_free(p);
    int64_t c = std::max<int64_t>(need, 1024);
    dev_alloc(g, &p, c);
    cap_io = c;
}

void stage_inputs(cm_graph *g, int64_t s, const int32_t *src, const int32_t *dst, int on_device) {
    if (on_device) {
        g->b.src_in = const_cast<int32_t *>(src);
        g->b.dst_in = const_cast<int32_t *>(dst);
    } else {
        HIPCHK(hipMemcpyAsync(g->src_buf, src, sizeof(int32_t) * (size_t)s, hipMemcpyHostToDevice, g->stream));
        HIPCHK(hipMemcpyAsync(g->dst_buf, dst, sizeof(int32_t) * (size_t)s, hipMemcpyHostToDevice, g->stream));
        g->b.src_in = g->src_buf;
        g->b.dst_in = g->dst_buf;
    }
}

void require_ready(cm_graph *g, bool need_cores) {
    if (g->poisoned) {
        throw Fail{CM_E_DEVICE};
    }
    if (g->serving) {
        g->err = "the graph is being served (call cm_serve_stop first)";
        throw Fail{CM_E_STATE};
    }
    if (!g->loaded || (need_cores && !g->decomposed)) {
        g->err = need_cores ? "no decomposed graph (call cm_load_graph and cm_core_decompose)"
                            : "no graph loaded";
        throw Fail{CM_E_STATE};
    }
}

void release_all(cm_graph *g) {
    DevGraph &d = g->g;
    dev_free(d.off); dev_free(d.len); dev_free(d.cap); dev_free(d.nbr); dev_free(d.core);
    dev_free(d.mcd); dev_free(d.stamp.p); dev_free(d.chg); d.cd.p = nullptr; dev_free(d.dec);
    dev_free(d.done); dev_free(d.matched); dev_free(d.claim); dev_free(d.bmark); dev_free(d.gain);
    dev_free(d.sub); dev_free(d.slen); dev_free(d.upl); dev_free(d.ubl);
    DevBatch &b = g->b;
    dev_free(b.err); dev_free(b.eu); dev_free(b.ev); dev_free(b.su); dev_free(b.sv);
    dev_free(b.hslot); dev_free(b.rem[0]); dev_free(b.rem[1]); dev_free(b.sel); dev_free(b.esel);
    dev_free(b.hkey); dev_free(b.hval); dev_free(b.vlist); dev_free(b.scanq); dev_free(b.reloc);
    dev_free(b.reloc_off); dev_free(b.reloc_cap);
    DevQueues &q = g->q;
    for (int i = 0; i < 2; ++i) {
        dev_free(q.fq[i]); dev_free(q.fh[i]); dev_free(q.eq[i]); dev_free(q.eh[i]);
    }
    dev_free(q.cand); dev_free(q.chg); dev_free(q.chh); dev_free(q.touched);
    dev_free(q.aq[0]); dev_free(q.aq[1]);
    dev_free(g->d_pbatch); dev_free(g->d_pout); dev_free(g->d_isrc); dev_free(g->d_idst);
    dev_free(g->d_isub); dev_free(g->d_sub_bad);
    g->prog_cap = 0; g->items_cap = 0; g->sub_cap = 0;
    if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->gexec = nullptr; g->graph = nullptr; g->graph_key.clear();
    // (the small scratch buffers allocated by cm_create stay until cm_destroy)
    dev_free(g->src_buf); dev_free(g->dst_buf); dev_free(g->scan_tmp); dev_free(g->firstidx);
    g->g = DevGraph{};
    g->b = DevBatch{};
    g->q = DevQueues{};
    g->batch_cap = g->hash_cap = g->scan_cap = 0;
    g->scan_tmp_cap = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void cm_config_default(cm_config *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->strict = 1;
    cfg->mode = CM_MODE_PLAIN;
}

const char *cm_strerror(int status) {
    switch (status) {
    case CM_OK: return "ok";
    case CM_E_BUSY: return "request must wait (serving ring, payload space or budget full)";
    case CM_E_ARG: return "invalid argument";
    case CM_E_RANGE: return "vertex id out of range";
    case CM_E_SELF_LOOP: return "self-loop";
    case CM_E_DUP: return "duplicate item in batch";
    case CM_E_EXISTS: return "edge already exists";
    case CM_E_MISSING: return "edge does not exist";
    case CM_E_DEAD: return "vertex was deleted";
    case CM_E_NOMEM: return "out of memory";
    case CM_E_CAPACITY: return "capacity exceeded";
    case CM_E_STATE: return "invalid state";
    case CM_E_DEVICE: return "device error";
    case CM_E_INTERNAL: return "internal error";
    case CM_E_IO: return "snapshot file error";
    default: return "unknown status";
    }
}

const char *cm_last_error(const cm_graph *g) { return g ? g->err.c_str() : ""; }

int cm_create(const cm_config *cfg, cm_graph **out) {
    if (!out) return CM_E_ARG;
    *out = nullptr;
    cm_graph *g = new (std::nothrow) cm_graph();
    if (!g) return CM_E_NOMEM;
    try {
        if (cfg) g->cfg = *cfg;
        else cm_config_default(&g->cfg);
        if (g->cfg.mode != CM_MODE_PLAIN && g->cfg.mode != CM_MODE_PERSISTENT) {
            delete g;
            return CM_E_ARG;
        }
        HIPCHK(hipGetDevice(&g->device));
        HIPCHK(na_lookup(g->device, &g->na_scratch));
        g->stream = (hipStream_t)g->cfg.stream;
        HIPCHK(hipDeviceGetAttribute(&g->num_cu, hipDeviceAttributeMultiprocessorCount, g->device));
        int coop_ok = 0;
        HIPCHK(hipDeviceGetAttribute(&coop_ok, hipDeviceAttributeCooperativeLaunch, g->device));
        if (!coop_ok) {
            g->err = "device does not support cooperative launches";
            throw Fail{CM_E_DEVICE};
        }
        g->tune.small_deg = g->cfg.small_degree > 0 ? g->cfg.small_degree : 4;
        g->tune.large_deg = g->cfg.large_degree > 0 ? g->cfg.large_degree : 256;
        g->tune.chunk = g->cfg.chunk > 0 ? g->cfg.chunk : 256;
        g->tune.rounds = g->cfg.partition_rounds > 0 ? std::min(g->cfg.partition_rounds, 8) : 2;
        g->tune.local_edges = g->cfg.local_edges > 0 ? g->cfg.local_edges : 2048;
        g->tune.local_items = g->cfg.local_items > 0 ? g->cfg.local_items : 128;
        g->tune.local_work = g->cfg.local_work > 0 ? g->cfg.local_work : 16384;
        g->tune.async_steps = g->cfg.async_steps ? 1 : 0;
        g->tune.single_edge = g->cfg.single_edge ? 1 : 0;
        if (g->cfg.expand_mode < 0 || g->cfg.expand_mode > 4) {
            g->err = "expand_mode must be 0 .. 4";
            throw Fail{CM_E_ARG};
        }
        g->tune.prune = g->cfg.expand_mode == 1 ? 1 : 0;
        g->tune.sublists = (g->cfg.expand_mode == 0 || g->cfg.expand_mode >= 3) && !g->tune.async_steps ? 1 : 0;
        g->tune.uplists = (g->cfg.expand_mode == 0 || g->cfg.expand_mode == 4) && !g->tune.async_steps ? 1 : 0;
        if (g->cfg.stamp_limit < 0) {
            g->err = "stamp_limit must be >= 0";
            throw Fail{CM_E_ARG};
        }
        g->tune.stamp_limit = g->cfg.stamp_limit > 0 ? std::min(g->cfg.stamp_limit, EPOCH_REWIND) : EPOCH_REWIND;
        if (g->tune.single_edge) g->tune.rounds = 1;
        if (g->tune.large_deg < g->tune.small_deg) g->tune.large_deg = g->tune.small_deg;
        int bpc_m = 0, bpc_d = 0;
        HIPCHK(coop_occupancy(0, &bpc_m));
        HIPCHK(coop_occupancy(1, &bpc_d));
        int want = g->cfg.blocks_per_cu > 0 ? g->cfg.blocks_per_cu : 1;
        g->coop_maint = g->num_cu * std::max(1, std::min(want, bpc_m));
        g->coop_dec = g->num_cu * std::max(1, std::min(want, bpc_d));
        g->grid_reg = g->num_cu * 8;
        int bpc_p = 0;
        HIPCHK(coop_occupancy(2, &bpc_p));
        g->coop_prog = g->num_cu * std::max(1, std::min(want, bpc_p));
        dev_alloc(g, &g->d_prog, 1);
        HIPCHK(hipHostMalloc((void **)&g->h_prog, sizeof(ProgDesc), hipHostMallocDefault));
        std::memset(g->h_prog, 0, sizeof(ProgDesc));
        dev_alloc(g, &g->ctl, 1);
        HIPCHK(hipMemsetAsync(g->ctl, 0, sizeof(Ctl), g->stream));
        dev_alloc(g, &g->bar, 1);
        HIPCHK(hipMemsetAsync(g->bar, 0, sizeof(Bar), g->stream));
        HIPCHK(hipDeviceGetAttribute(&g->clock_khz, hipDeviceAttributeWallClockRate, g->device));
        if (g->clock_khz <= 0) {
            g->err = "device wall clock rate unknown";
            throw Fail{CM_E_DEVICE};
        }
        set_bar_bounds(g, 0);
        HIPCHK(hipHostMalloc((void **)&g->hctl, sizeof(Ctl), hipHostMallocDefault));
        std::memset(g->hctl, 0, sizeof(Ctl));
        HIPCHK(hipHostMalloc((void **)&g->hu64, 4 * sizeof(unsigned long long), hipHostMallocDefault));
        dev_alloc(g, &g->i64_scratch, 4);
        dev_alloc(g, &g->u64_scratch, 4);
        HIPCHK(hipEventCreate(&g->ev0));
        HIPCHK(hipEventCreate(&g->ev1));
        if (g->cfg.debug < 0) {
            g->err = "debug must be >= 0";
            throw Fail{CM_E_ARG};
        }
        if (g->cfg.debug) {
            g->dl.cap = g->cfg.debug > 1 ? (int64_t)g->cfg.debug : ((int64_t)1 << 20);
            dev_alloc(g, &g->dl.sel, 3 * g->dl.cap);
            dev_alloc(g, &g->dl.chg, 3 * g->dl.cap);
            dev_alloc(g, &g->dl.n, 2);
            HIPCHK(fill_u64(g->dl.n, 0ull, 2, g->stream));
        }
        HIPCHK(hipHostMalloc((void **)&g->lout, sizeof(LaunchOut) * cm_graph::LSLOTS, hipHostMallocDefault));
        std::memset(g->lout, 0, sizeof(LaunchOut) * cm_graph::LSLOTS);
        for (auto &pr : g->lev)
            for (auto &e : pr) HIPCHK(hipEventCreate(&e));
        HIPCHK(hipStreamSynchronize(g->stream));
    } catch (const Fail &f) {
        cm_destroy(g);
        return f.code;
    }
    *out = g;
    return CM_OK;
}

void cm_destroy(cm_graph *g) {
    if (!g) return;
    if (g->serving && g->shdr) __atomic_store_n(&g->shdr->stop, 1, __ATOMIC_RELEASE);
    (void)hipStreamSynchronize(g->stream);
    serve_free(g);
    release_all(g);
    dev_free(g->i64_scratch);
    dev_free(g->u64_scratch);
    dev_free(g->d_prog);
    if (g->h_prog) (void)hipHostFree(g->h_prog);
    if (g->ctl) (void)hipFree(g->ctl);
    if (g->bar) (void)hipFree(g->bar);
    if (g->hctl) (void)hipHostFree(g->hctl);
    if (g->hu64) (void)hipHostFree(g->hu64);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    for (auto &pr : g->lev)
        for (auto &e : pr)
            if (e) (void)hipEventDestroy(e);
    if (g->lout) (void)hipHostFree(g->lout);
    dev_free(g->dl.sel);
    dev_free(g->dl.chg);
    dev_free(g->dl.n);
    delete g;
}

int cm_load_graph(cm_graph *g, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                  int on_device) {
    Range range("cm_load_graph");
    if (!g || n < 0 || m < 0 || (m > 0 && (!src || !dst))) return CM_E_ARG;
    if (g->poisoned) return CM_E_DEVICE;
    if (g->serving) return CM_E_STATE;
    hipStream_t st = g->stream;
    try {
        release_all(g);
        g->loaded = g->decomposed = false;
        g->m = 0;
        int32_t n_cap = std::max<int32_t>(n + 1, g->cfg.vertex_capacity > 0 ? g->cfg.vertex_capacity
                                                                           : n + n / 8 + 1024);
        alloc_vertex_arrays(g, n_cap, 0);
        g->g.n_ids = n;
        // stage edges on the device
        int32_t *ds = nullptr, *dd = nullptr;
        bool own = false;
        if (on_device) {
            ds = const_cast<int32_t *>(src);
            dd = const_cast<int32_t *>(dst);
        } else if (m > 0) {
            dev_alloc(g, &ds, m);
            dev_alloc(g, &dd, m);
            own = true;
            HIPCHK(hipMemcpyAsync(ds, src, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(dd, dst, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, st));
        }
        int rc = CM_OK;
        if (m > 0) {
            // range / self-loop / duplicate check
            int64_t hc = next_pow2(2 * m);
            unsigned long long *hkey = nullptr;
            int64_t *hval = nullptr;
            dev_alloc(g, &hkey, hc);
            dev_alloc(g, &hval, hc);
            HIPCHK(fill_u64(hkey, ~0ull, hc, st));
            HIPCHK(fill_i64(hval, INT64_MAX, hc, st));
            HIPCHK(fill_u64(g->u64_scratch, ~0ull, 1, st));
            HIPCHK(load_check(ds, dd, m, n, hkey, hval, (uint32_t)(hc - 1), g->u64_scratch, st));
            HIPCHK(hipMemcpyAsync(g->hu64, g->u64_scratch, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            dev_free(hkey);
            dev_free(hval);
            unsigned long long fb = g->hu64[0];
            if (fb != ~0ull) {
                rc = -(int)(fb & 0xff);
                g->err = std::string("invalid edge ") + std::to_string((long long)(fb >> 8)) + ": " +
                         cm_strerror(rc);
            }
        }
        if (rc == CM_OK) {
            // alive ids get core 0 until decomposed
            HIPCHK(fill_i32(g->g.core, 0, n, st));
            HIPCHK(fill_i32(g->g.len, 0, g->g.n_cap, st));
            if (m > 0) HIPCHK(count_deg(ds, dd, m, g->g.len, st));
            int64_t *caps64 = nullptr;
            dev_alloc(g, &caps64, g->g.n_cap);
            HIPCHK(caps_from_counts(g->g.len, n, g->g.n_cap, caps64, g->g.cap, st));
            HIPCHK(exclusive_scan_i64(caps64, g->g.off, g->g.n_cap, g->scan_tmp, g->i64_scratch, st));
            int64_t total = 0;
            HIPCHK(hipMemcpyAsync(&total, g->i64_scratch, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            dev_free(caps64);
            int64_t pool = total + total / 4 + 4096;
            if (g->cfg.edge_capacity_hint > pool) pool = g->cfg.edge_capacity_hint;
            dev_alloc(g, &g->g.nbr, pool);
            if (g->tune.sublists) dev_alloc(g, &g->g.sub, pool);
            if (g->tune.uplists) dev_alloc(g, &g->g.upl, pool);
            g->g.pool_size = pool;
            HIPCHK(fill_i32(g->g.len, 0, g->g.n_cap, st));
            if (m > 0) HIPCHK(scatter_edges(ds, dd, m, g->g.off, g->g.len, g->g.nbr, st));
            // control block
            HIPCHK(hipMemsetAsync(g->ctl, 0, sizeof(Ctl), st));
            unsigned long long tail = (unsigned long long)total;
            HIPCHK(ctl_set_pool(g->ctl, tail, st));
            HIPCHK(hipStreamSynchronize(st));
            std::memset(g->hctl, 0, sizeof(Ctl));
            g->hctl->pool_tail = tail;
            g->epoch = 0;
            alloc_chunk_queues(g);
            g->m = m;
            g->n_alive = n;
            g->loaded = true;
        }
        if (own) {
            dev_free(ds);
            dev_free(dd);
        }
        if (rc != CM_OK) {
            release_all(g);
            return rc;
        }
    } catch (const Fail &f) {
        return f.code;
    }
    g->err.clear();
    return CM_OK;
}

int cm_core_decompose(cm_graph *g, cm_batch_stats *stats) {
    Range range("cm_core_decompose");
    if (!g) return CM_E_ARG;
    double t0 = now_ms();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    try {
        require_ready(g, false);
        hipStream_t st = g->stream;
        HIPCHK(ctl_batch_reset(g->ctl, 0, st));
        KArgs a = make_args(g);
        HIPCHK(dec_prep(a, g->grid_reg, st));
        if (g->cfg.timing) HIPCHK(hipEventRecord(g->ev0, st));
        HIPCHK(decompose_coop(a, g->coop_dec, st));
        if (g->cfg.timing) HIPCHK(hipEventRecord(g->ev1, st));
        HIPCHK(mcd_init(a, g->grid_reg, st));
        sync_ctl(g);
        check_abort(g);
        check_overflow(g);
        if (stats) {
            stats->scanned = (int64_t)g->hctl->st_scanned;
            stats->iterations = g->hctl->dec_rounds;
            stats->rounds = g->hctl->dec_rounds;
            stats->grid_steps = (int64_t)g->hctl->st_grid_steps;
            stats->local_steps = (int64_t)g->hctl->st_local_steps;
            stats->launches = 1;
            if (g->cfg.timing) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
                stats->kernel_ms = ms;
            }
            // per adjacency entry: id 4 + core 4 + degree atomic 4; per vertex 16
            stats->alg_bytes = 12 * stats->scanned + 16 * (int64_t)g->n_alive;
        }
        g->decomposed = true;
    } catch (const Fail &f) {
        return finish(g, f.code, stats, t0);
    }
    return finish(g, CM_OK, stats, t0);
}

static int edge_call(cm_graph *g, int64_t s, const int32_t *src, const int32_t *dst, int on_device,
                     cm_batch_stats *stats, bool inserting) {
    Range range(inserting ? "cm_insert_edges" : "cm_delete_edges");
    if (!g) return CM_E_ARG;
    double t0 = now_ms();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->first_bad = -1;
    }
    if (s < 0 || (s > 0 && (!src || !dst))) return finish(g, CM_E_ARG, stats, t0);
    try {
        require_ready(g, true);
        debug_reset(g);
        if (s == 0) return finish(g, CM_OK, stats, t0);
        ensure_batch(g, s);
        stage_inputs(g, s, src, dst, on_device);
        int64_t dropped = 0;
        edge_batch(g, s, inserting, stats, &dropped, false, false);
    } catch (const Fail &f) {
        return finish(g, f.code, stats, t0);
    }
    return finish(g, CM_OK, stats, t0);
}

int cm_insert_edges(cm_graph *g, int64_t s, const int32_t *src, const int32_t *dst, int on_device,
                    cm_batch_stats *stats) {
    return edge_call(g, s, src, dst, on_device, stats, true);
}

int cm_delete_edges(cm_graph *g, int64_t s, const int32_t *src, const int32_t *dst, int on_device,
                    cm_batch_stats *stats) {
    return edge_call(g, s, src, dst, on_device, stats, false);
}

int cm_update_edges_noalloc(cm_graph *g, int32_t kind, int64_t s, const int32_t *src, const int32_t *dst,
                            cm_batch_stats *stats) {
    if (!g) return CM_E_ARG;
    double t0 = now_ms();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->first_bad = -1;
    }
    if ((kind != CM_BATCH_INSERT && kind != CM_BATCH_DELETE) || s < 0 || (s > 0 && (!src || !dst)))
        return finish(g, CM_E_ARG, stats, t0);
    if (s > CM_NOALLOC_MAX_ITEMS) {
        g->err = "batch larger than CM_NOALLOC_MAX_ITEMS";
        return finish(g, CM_E_CAPACITY, stats, t0);
    }
    try {
        require_ready(g, true);
        debug_reset(g);
        if (s == 0) return finish(g, CM_OK, stats, t0);
        if (!g->na_scratch) {
            g->err = "allocation-free scratch not resolved on this device";
            throw Fail{CM_E_DEVICE};
        }
        // every list the locate scan may queue: one chunk item per chunk of a
        // distinct endpoint's list
        const int64_t scan_need = 2 * s + g->g.pool_size / std::max(1, g->tune.chunk) + 1024;
        if (scan_need > NA_SCAN) {
            g->err = "graph too large for the allocation-free locate-scan queue";
            throw Fail{CM_E_CAPACITY};
        }
        hipStream_t st = g->stream;
        unsigned char *base = (unsigned char *)g->na_scratch;
        size_t at = 0;
        auto carve = [&](size_t bytes) {
            unsigned char *p = base + at;
            at += bytes;
            return (void *)p;
        };
        DevBatch nb = g->b;  // vertex-sized arrays (vlist, reloc) stay the handle's own
        nb.cap = (int32_t)NA_ITEMS;
        nb.err = (int32_t *)carve(NA_I32);
        nb.eu = (int32_t *)carve(NA_I32);
        nb.ev = (int32_t *)carve(NA_I32);
        nb.hslot = (int32_t *)carve(NA_I32);
        nb.rem[0] = (int32_t *)carve(NA_I32);
        nb.rem[1] = (int32_t *)carve(NA_I32);
        nb.sel = (int32_t *)carve(NA_I32);
        nb.esel = (int32_t *)carve(NA_I32);
        nb.su = (int64_t *)carve(NA_I64);
        nb.sv = (int64_t *)carve(NA_I64);
        nb.hkey = (unsigned long long *)carve(na_align(sizeof(unsigned long long) * NA_HASH));
        nb.hval = (int32_t *)carve(na_align(sizeof(int32_t) * NA_HASH));
        nb.scanq = (int64_t *)carve(na_align(sizeof(int64_t) * NA_SCAN));
        nb.scap = (int32_t)NA_SCAN;
        nb.hcap = (int32_t)next_pow2(std::max<int64_t>(2 * s, 1024));
        nb.src_in = const_cast<int32_t *>(src);
        nb.dst_in = const_cast<int32_t *>(dst);
        nb.sub_in = nullptr;
        // the array keeps the last call's contents (any handle's): clear the
        // hash and the selection stamps this call reads
        HIPCHK(fill_u64(nb.hkey, ~0ull, nb.hcap, st));
        HIPCHK(fill_i32(nb.hval, INT_MAX, nb.hcap, st));
        HIPCHK(fill_i32(nb.esel, 0, s, st));
        const DevBatch saved = g->b;
        g->b = nb;
        g->no_alloc = true;
        try {
            int64_t dropped = 0;
            edge_batch(g, s, kind == CM_BATCH_INSERT, stats, &dropped, false, false);
        } catch (...) {
            g->b = saved;
            g->no_alloc = false;
            throw;
        }
        g->b = saved;
        g->no_alloc = false;
    } catch (const Fail &f) {
        return finish(g, f.code, stats, t0);
    }
    return finish(g, CM_OK, stats, t0);
}

int cm_insert_vertices(cm_graph *g, int32_t c, const int64_t *off, const int32_t *nbrs, int on_device,
                       int32_t *first_new_id, cm_batch_stats *stats) {
    Range range("cm_insert_vertices");
    if (!g) return CM_E_ARG;
    double t0 = now_ms();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->first_bad = -1;
    }
    if (c < 0 || (c > 0 && !off)) return finish(g, CM_E_ARG, stats, t0);
    int32_t first = -1;
    bool created = false;
    bool counted = false;
    try {
        require_ready(g, true);
        debug_reset(g);
        hipStream_t st = g->stream;
        first = g->g.n_ids;
        if (first_new_id) *first_new_id = first;
        if (c == 0) return finish(g, CM_OK, stats, t0);
        // offsets to the host to size the batch
        std::vector<int64_t> hoff(2);
        int64_t total = 0;
        int64_t *doff = nullptr;
        bool own_off = false;
        if (on_device) {
            HIPCHK(hipMemcpyAsync(&total, off + c, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            int64_t first_off = 0;
            HIPCHK(hipMemcpyAsync(&first_off, off, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (first_off != 0) { g->err = "off[0] must be 0"; throw Fail{CM_E_ARG}; }
            doff = const_cast<int64_t *>(off);
        } else {
            if (off[0] != 0) { g->err = "off[0] must be 0"; throw Fail{CM_E_ARG}; }
            for (int32_t i = 0; i < c; ++i)
                if (off[i + 1] < off[i]) { g->err = "offsets must be non-decreasing"; throw Fail{CM_E_ARG}; }
            total = off[c];
            dev_alloc(g, &doff, (int64_t)c + 1);
            own_off = true;
            HIPCHK(hipMemcpyAsync(doff, off, sizeof(int64_t) * ((size_t)c + 1), hipMemcpyHostToDevice, st));
        }
        if (on_device) {
            HIPCHK(fill_u64(g->u64_scratch, ~0ull, 1, st));
            HIPCHK(vins_check_off(doff, c, g->u64_scratch, st));
            HIPCHK(hipMemcpyAsync(g->hu64, g->u64_scratch, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (g->hu64[0] != ~0ull) { g->err = "offsets must be non-decreasing"; throw Fail{CM_E_ARG}; }
        }
        if (total < 0 || (total > 0 && !nbrs)) { g->err = "bad neighbour list"; throw Fail{CM_E_ARG}; }
        ensure_vertex_capacity(g, (int64_t)first + c);
        ensure_batch(g, std::max<int64_t>(total, 1));
        // new ids exist (core 0) while the batch is validated
        KArgs a = make_args(g);
        HIPCHK(vins_init(a, first, c, st));
        g->g.n_ids = first + c;
        created = true;
        if (total > 0) {
            HIPCHK(vins_expand(doff, c, first, g->src_buf, g->grid_reg, st));
            if (on_device) {
                HIPCHK(hipMemcpyAsync(g->dst_buf, nbrs, sizeof(int32_t) * (size_t)total, hipMemcpyDeviceToDevice, st));
            } else {
                HIPCHK(hipMemcpyAsync(g->dst_buf, nbrs, sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice, st));
            }
            g->b.src_in = g->src_buf;
            g->b.dst_in = g->dst_buf;
        }
        if (own_off) dev_free(doff);
        if (total > 0 && g->cfg.mode == CM_MODE_PERSISTENT) {
            // one persistent launch: the new vertices enter as stars
            std::vector<ProgBatch> pb(1);
            pb[0].off = 0;
            pb[0].s = (int32_t)total;
            pb[0].kind = 2;
            pb[0].v0 = first;
            pb[0].nv = c;
            pb[0].n_ids = first + c;
            std::vector<ProgOut> out;
            int used = 0, launches = 0;
            double kms = 0.0;
            program_execute(g, pb, g->src_buf, g->dst_buf, nullptr, g->cfg.strict != 0, out, &used, &kms, &launches);
            stats_from_out(g, out[0], total, launches, kms, stats);
            if (out[0].status != 0) {
                g->err = std::string("invalid neighbour item ") + std::to_string(out[0].first_bad) + ": " +
                         cm_strerror(out[0].status);
                throw Fail{out[0].status};
            }
            g->m += out[0].valid;
            g->n_alive += c;
        } else {
            g->n_alive += c;
            counted = true;
            if (total > 0) {
                int64_t dropped = 0;
                edge_batch(g, total, true, stats, &dropped, false, false);
            }
        }
        created = false;
    } catch (const Fail &f) {
        if (created && !g->poisoned) {
            KArgs a = make_args(g);
            (void)vins_revert(a, first, c, g->stream);
            (void)hipStreamSynchronize(g->stream);
            g->g.n_ids = first;
            if (counted) g->n_alive -= c;
        }
        return finish(g, f.code, stats, t0);
    }
    return finish(g, CM_OK, stats, t0);
}

int cm_delete_vertices(cm_graph *g, int32_t c, const int32_t *ids, int on_device, cm_batch_stats *stats) {
    Range range("cm_delete_vertices");
    if (!g) return CM_E_ARG;
    double t0 = now_ms();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->first_bad = -1;
    }
    if (c < 0 || (c > 0 && !ids)) return finish(g, CM_E_ARG, stats, t0);
    try {
        require_ready(g, true);
        debug_reset(g);
        if (c == 0) return finish(g, CM_OK, stats, t0);
        hipStream_t st = g->stream;
        int32_t *dids = nullptr;
        bool own = false;
        if (on_device) {
            dids = const_cast<int32_t *>(ids);
        } else {
            dev_alloc(g, &dids, c);
            own = true;
            HIPCHK(hipMemcpyAsync(dids, ids, sizeof(int32_t) * (size_t)c, hipMemcpyHostToDevice, st));
        }
        KArgs a = make_args(g);
        HIPCHK(fill_u64(g->u64_scratch, ~0ull, 1, st));
        HIPCHK(fill_u64(g->u64_scratch + 1, 0ull, 1, st));
        HIPCHK(vdel_check(a, dids, c, g->firstidx, g->u64_scratch, g->u64_scratch + 1, st));
        HIPCHK(hipMemcpyAsync(g->hu64, g->u64_scratch, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        unsigned long long fb = g->hu64[0];
        int64_t total = (int64_t)g->hu64[1];
        if (fb != ~0ull) {
            int code = -(int)(fb & 0xff);
            int64_t idx = (int64_t)(fb >> 8);
            if (stats) stats->first_bad = idx;
            if (g->cfg.strict) {
                if (own) dev_free(dids);
                g->err = std::string("invalid vertex item ") + std::to_string((long long)idx) + ": " +
                         cm_strerror(code);
                return finish(g, code, stats, t0);
            }
            // filter mode: keep the valid, first occurrences only
            std::vector<int32_t> h(c);
            HIPCHK(hipMemcpy(h.data(), dids, sizeof(int32_t) * (size_t)c, hipMemcpyDeviceToHost));
            std::vector<int32_t> core_h(g->g.n_ids);
            HIPCHK(hipMemcpy(core_h.data(), g->g.core, sizeof(int32_t) * (size_t)g->g.n_ids, hipMemcpyDeviceToHost));
            std::vector<int32_t> keep;
            std::vector<char> seen(g->g.n_ids, 0);
            for (int32_t i = 0; i < c; ++i) {
                int32_t x = h[i];
                if (x < 0 || x >= g->g.n_ids || core_h[x] < 0 || seen[x]) continue;
                seen[x] = 1;
                keep.push_back(x);
            }
            if (stats) stats->dropped = c - (int64_t)keep.size();
            if (own) dev_free(dids);
            dev_alloc(g, &dids, std::max<int64_t>(1, (int64_t)keep.size()));
            own = true;
            c = (int32_t)keep.size();
            if (c > 0)
                HIPCHK(hipMemcpy(dids, keep.data(), sizeof(int32_t) * (size_t)c, hipMemcpyHostToDevice));
            HIPCHK(fill_u64(g->u64_scratch + 1, 0ull, 1, st));
            HIPCHK(fill_u64(g->u64_scratch, ~0ull, 1, st));
            HIPCHK(vdel_check(a, dids, c, g->firstidx, g->u64_scratch, g->u64_scratch + 1, st));
            HIPCHK(hipMemcpyAsync(g->hu64, g->u64_scratch, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            total = (int64_t)g->hu64[1];
        }
        if (g->cfg.mode == CM_MODE_PERSISTENT && c > 0) {
            // one persistent launch: the ids leave as stars
            ensure_batch(g, std::max<int64_t>(std::max<int64_t>(total, c), 1));
            std::vector<ProgBatch> pb(1);
            pb[0].off = 0;
            pb[0].s = c;
            pb[0].kind = 3;
            pb[0].n_ids = g->g.n_ids;
            std::vector<ProgOut> out;
            int used = 0, launches = 0;
            double kms = 0.0;
            const int64_t fb_host = stats ? stats->first_bad : -1;
            const int64_t dropped_host = stats ? stats->dropped : 0;
            program_execute(g, pb, dids, nullptr, nullptr, true, out, &used, &kms, &launches);
            stats_from_out(g, out[0], total, launches, kms, stats);
            if (stats) {
                stats->first_bad = fb_host;
                stats->dropped = dropped_host;
            }
            if (out[0].status != 0) {
                if (own) dev_free(dids);
                g->err = std::string("vertex deletion failed: ") + cm_strerror(out[0].status);
                return finish(g, out[0].status, stats, t0);
            }
            g->m -= out[0].valid;
            if (own) dev_free(dids);
            g->n_alive -= c;
            return finish(g, CM_OK, stats, t0);
        }
        if (total > 0) {
            ensure_batch(g, total);
            HIPCHK(fill_u64(g->u64_scratch + 2, 0ull, 1, st));
            KArgs a2 = make_args(g);
            HIPCHK(vdel_gather(a2, dids, c, g->src_buf, g->dst_buf, total, g->u64_scratch + 2, g->grid_reg, st));
            g->b.src_in = g->src_buf;
            g->b.dst_in = g->dst_buf;
            int64_t dropped = 0;
            // an edge between two deleted ids is gathered twice: drop the copy
            edge_batch(g, total, false, stats, &dropped, true, false);
            if (stats) stats->dropped = 0;
        }
        KArgs a3 = make_args(g);
        HIPCHK(vdel_finish(a3, dids, c, st));
        HIPCHK(hipStreamSynchronize(st));
        if (own) dev_free(dids);
        g->n_alive -= c;
    } catch (const Fail &f) {
        return finish(g, f.code, stats, t0);
    }
    return finish(g, CM_OK, stats, t0);
}

int cm_get_cores(cm_graph *g, int32_t *out, int32_t n, int on_device) {
    if (!g || n < 0 || (n > 0 && !out)) return CM_E_ARG;
    try {
        require_ready(g, false);
        if (n > g->g.n_ids) return CM_E_ARG;
        if (n == 0) return CM_OK;
        HIPCHK(hipMemcpyAsync(out, g->g.core, sizeof(int32_t) * (size_t)n,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_get_superior_degrees(cm_graph *g, int32_t *out, int32_t n, int on_device) {
    if (!g || n < 0 || (n > 0 && !out)) return CM_E_ARG;
    try {
        require_ready(g, true);
        if (n > g->g.n_ids) return CM_E_ARG;
        if (n == 0) return CM_OK;
        HIPCHK(hipMemcpyAsync(out, g->g.mcd, sizeof(int32_t) * (size_t)n,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

// ---------------------------------------------------------------------------
// Serving: continuous batching through a pinned request ring
// ---------------------------------------------------------------------------
void cm_serve_config_default(cm_serve_config *c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->ring_requests = 4096;
    c->idle_ms = 20;
    c->ring_items = (int64_t)1 << 24;
    c->max_items = (int64_t)1 << 22;
    c->budget_bytes = (int64_t)1 << 30;
    c->vertex_headroom = 1 << 20;
}

}  // extern "C"

namespace {

void serve_free(cm_graph *g) {
    if (g->shdr) (void)hipHostFree(g->shdr);
    if (g->sring) (void)hipHostFree(g->sring);
    if (g->sout) (void)hipHostFree(g->sout);
    if (g->ssrc) (void)hipHostFree(g->ssrc);
    if (g->sdst) (void)hipHostFree(g->sdst);
    g->shdr = nullptr;
    g->sring = nullptr;
    g->sout = nullptr;
    g->ssrc = g->sdst = nullptr;
    dev_free(g->d_bsub);
}

template <class T>
T *host_dev_ptr(cm_graph *g, T *p) {
    void *d = nullptr;
    HIPCHK(hipHostGetDevicePointer(&d, p, 0));
    return (T *)d;
}

// Copy the finished batches' outcomes out of the ring and settle accounts.
void serve_collect(cm_graph *g) {
    const long long head = __atomic_load_n(&g->shdr->head, __ATOMIC_ACQUIRE);
    const int32_t R = g->scfg.ring_requests;
    for (long long t = g->s_done; t < head; ++t) {
        const int32_t slot = (int32_t)(t % R);
        const ProgOut &o = g->sout[slot];
        const ProgBatch &b = g->sring[slot];
        cm_batch_stats &r = g->s_results[t];
        std::memset(&r, 0, sizeof(r));
        r.status = o.status;
        r.iterations = o.iterations;
        r.first_bad = o.first_bad;
        r.applied = o.valid;
        r.remaining_sum = (int64_t)o.remaining;
        r.candidates = (int64_t)o.candidates;
        r.evicted = (int64_t)o.evicted;
        r.changed = (int64_t)o.changed;
        r.scanned = (int64_t)o.scanned;
        r.rounds = (int64_t)o.rounds;
        r.local_steps = (int64_t)o.steps;
        r.group = o.group;
        r.first_stamp = o.ep0;
        r.alg_bytes = alg_bytes(o);
        r.cand_degree = (int64_t)o.cdeg;
        r.evicted_degree = (int64_t)o.edeg;
        r.changed_degree = (int64_t)o.hdeg;
        if (o.status == 0) {
            const bool ins = b.kind == 0 || b.kind == 2;
            g->m += ins ? o.valid : -(int64_t)o.valid;
            if (b.kind == 2) g->n_alive += o.vdone;
            if (b.kind == 3) g->n_alive -= o.vdone;
        }
        if (b.kind == 0 || b.kind == 2) g->s_pending_ins -= b.s;
        g->s_inflight -= g->s_bytes[slot];
        g->g.n_ids = std::max(g->g.n_ids, g->s_nids[slot]);
    }
    g->s_done = std::max<int64_t>(g->s_done, head);
}

void serve_launch(cm_graph *g) {
    hipStream_t st = g->stream;
    bstamp_guard(g);
    ProgDesc *hd = g->h_prog;
    std::memset(hd, 0, sizeof(ProgDesc));
    hd->batches = host_dev_ptr(g, g->sring);
    hd->out = host_dev_ptr(g, g->sout);
    hd->src = host_dev_ptr(g, g->ssrc);
    hd->dst = host_dev_ptr(g, g->sdst);
    hd->gsrc = g->src_buf;
    hd->gdst = g->dst_buf;
    hd->gcap = g->batch_cap;
    hd->firstidx = g->firstidx;
    hd->hdr = host_dev_ptr(g, g->shdr);
    hd->bsub = g->d_bsub;
    hd->sub_bad = g->d_sub_bad;
    hd->fuse = std::max(1, g->scfg.fuse);
    int khz = 0;
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device));
    hd->idle_ticks = (unsigned long long)std::max(1, g->scfg.idle_ms) * (unsigned long long)std::max(khz, 1);
    hd->ring = g->scfg.ring_requests;
    hd->sfirst = g->s_done;
    hd->strict = g->cfg.strict ? 1 : 0;
    hd->bstamp0 = g->bstamp + 2;
    g->shdr->exit_at = g->s_done;
    __atomic_store_n(&g->shdr->exit_reason, 0, __ATOMIC_RELEASE);
    g->s_first = g->s_done;
    HIPCHK(hipMemcpyAsync(g->d_prog, hd, sizeof(ProgDesc), hipMemcpyHostToDevice, st));
    KArgs a = make_args(g);
    a.prog = g->d_prog;
    HIPCHK(serve_coop(a, g->coop_serve, st));
    g->serve_live = true;
}

// After the serving launch has left: settle, then handle why it left.
void serve_after_exit(cm_graph *g) {
    HIPCHK(hipStreamSynchronize(g->stream));
    g->serve_live = false;
    serve_collect(g);
    sync_ctl(g);
    check_abort(g);
    check_overflow(g);
    g->epoch = g->hctl->epoch;
    const long long at = g->shdr->exit_at;
    g->bstamp += 2 * (int32_t)(at - g->s_first) + 2;
    const int32_t reason = __atomic_load_n(&g->shdr->exit_reason, __ATOMIC_ACQUIRE);
    if (reason == SV_POOL) {
        repack(g, 4 * std::max<int64_t>(g->s_pending_ins, 0) + g->g.pool_size / 2);
    } else if (reason == SV_TOOBIG || reason == SV_ABORT) {
        g->poisoned = true;
        g->err = reason == SV_TOOBIG ? "internal: served batch larger than the staged capacity"
                                     : "internal: serving launch aborted";
        throw Fail{CM_E_INTERNAL};
    }
    __atomic_store_n(&g->shdr->stop, 0, __ATOMIC_RELEASE);
    if (g->s_grow) {
        // ids of unfinished insertions are kept too (their slots are re-initialised on activation)
        int32_t keep = g->g.n_ids;
        g->g.n_ids = g->s_n_ids;
        ensure_vertex_capacity(g, (int64_t)g->s_n_ids + std::max(g->scfg.vertex_headroom, 1024));
        g->g.n_ids = keep;
        g->s_grow = false;
    }
}

// Poll the live launch; relaunch when work is pending and none is live.
void serve_pump(cm_graph *g) {
    serve_collect(g);
    if (g->serve_live && __atomic_load_n(&g->shdr->exit_reason, __ATOMIC_ACQUIRE) != 0) serve_after_exit(g);
    if (!g->serve_live && g->s_done < g->s_next) serve_launch(g);
}

void serve_require(cm_graph *g) {
    if (g->poisoned) throw Fail{CM_E_DEVICE};
    if (!g->serving) {
        g->err = "not serving (call cm_serve_start)";
        throw Fail{CM_E_STATE};
    }
}

// Reserve a ring slot and `items` payload slots; false when the request must
// wait (ring, payload or budget full).  On success returns the payload
// position.
bool serve_admit(cm_graph *g, int64_t items, int64_t bytes, int64_t *pos_out) {
    const int32_t R = g->scfg.ring_requests;
    const int64_t P = g->scfg.ring_items;
    if (g->s_next - g->s_done >= R) return false;
    if (g->s_next > g->s_done && g->s_inflight + bytes > g->scfg.budget_bytes) return false;
    // payload: contiguous [pos, pos + items) on the ring, wrapping to 0 if needed
    int64_t start = g->s_pay_tail;
    int64_t pos = start % P;
    if (pos + items > P) start += P - pos;
    const int64_t oldest = g->s_next > g->s_done ? g->s_pstart[g->s_done % R] : g->s_pay_tail;
    if (start + items - oldest > P) return false;
    *pos_out = start;
    return true;
}

void serve_publish(cm_graph *g, const ProgBatch &b, int64_t start, int64_t bytes, int32_t nids_after,
                   int64_t *ticket) {
    const int32_t R = g->scfg.ring_requests;
    const int64_t t = g->s_next;
    const int32_t slot = (int32_t)(t % R);
    g->sring[slot] = b;
    g->s_pstart[slot] = start;
    g->s_bytes[slot] = bytes;
    g->s_nids[slot] = nids_after;
    g->s_pay_tail = start + std::max<int64_t>(b.s, 0);
    g->s_inflight += bytes;
    if (b.kind == 0 || b.kind == 2) g->s_pending_ins += b.s;
    if ((int64_t)g->s_results.size() <= t) g->s_results.resize((size_t)std::max<int64_t>(t + 1, 2 * (int64_t)g->s_results.size()));
    std::atomic_thread_fence(std::memory_order_release);
    __atomic_store_n(&g->shdr->tail, (long long)(t + 1), __ATOMIC_RELEASE);
    g->s_next = t + 1;
    if (ticket) *ticket = t;
}

// Device bytes a request may claim while unfinished: its payload plus, for
// insertions, room for both list entries of every edge and a relocated list.
int64_t serve_bytes(int32_t kind, int64_t items) {
    return 8 * items + ((kind == 0 || kind == 2) ? 32 * items : 0);
}

}  // namespace

extern "C" {

int cm_serve_start(cm_graph *g, const cm_serve_config *cfg) {
    Range range("cm_serve_start");
    if (!g) return CM_E_ARG;
    try {
        require_ready(g, true);
        cm_serve_config c;
        if (cfg) c = *cfg;
        else cm_serve_config_default(&c);
        if (c.ring_requests < 1 || c.ring_items < 1 || c.max_items < 1 || c.max_items > c.ring_items ||
            c.max_items > INT_MAX / 4 || c.idle_ms < 1 || c.budget_bytes < 1 || c.vertex_headroom < 0 ||
            c.fuse < 0 || c.fuse > FUSE_MAX) {
            g->err = "bad serving configuration";
            throw Fail{CM_E_ARG};
        }
        g->scfg = c;
        ensure_batch(g, c.max_items);
        ensure_vertex_capacity(g, (int64_t)g->g.n_ids + c.vertex_headroom);
        HIPCHK(hipStreamSynchronize(g->stream));
        int bpc = 0;
        HIPCHK(coop_occupancy(3, &bpc));
        int want = g->cfg.blocks_per_cu > 0 ? g->cfg.blocks_per_cu : 1;
        g->coop_serve = g->num_cu * std::max(1, std::min(want, bpc));
        serve_free(g);
        dev_alloc(g, &g->d_bsub, g->batch_cap);
        {
            int64_t cap = g->sub_cap;
            grow_dev(g, g->d_sub_bad, cap, FUSE_MAX);
            g->sub_cap = (int32_t)cap;
        }
        debug_reset(g);
        set_bar_bounds(g, c.idle_ms);
        HIPCHK(hipHostMalloc((void **)&g->shdr, sizeof(ServeHdr), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&g->sring, sizeof(ProgBatch) * (size_t)c.ring_requests, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&g->sout, sizeof(ProgOut) * (size_t)c.ring_requests, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&g->ssrc, sizeof(int32_t) * (size_t)c.ring_items, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&g->sdst, sizeof(int32_t) * (size_t)c.ring_items, hipHostMallocDefault));
        std::memset(g->shdr, 0, sizeof(ServeHdr));
        std::memset(g->sring, 0, sizeof(ProgBatch) * (size_t)c.ring_requests);
        std::memset(g->sout, 0, sizeof(ProgOut) * (size_t)c.ring_requests);
        g->s_pstart.assign((size_t)c.ring_requests, 0);
        g->s_bytes.assign((size_t)c.ring_requests, 0);
        g->s_nids.assign((size_t)c.ring_requests, 0);
        g->s_results.clear();
        g->s_results.resize(1024);
        g->s_next = g->s_done = g->s_first = g->s_pay_tail = 0;
        g->s_inflight = 0;
        g->s_pending_ins = 0;
        g->s_n_ids = g->g.n_ids;
        g->s_grow = false;
        g->serve_live = false;
        g->serving = true;
    } catch (const Fail &f) {
        serve_free(g);
        return f.code;
    }
    g->err.clear();
    return CM_OK;
}

int cm_serve_submit_edges(cm_graph *g, int32_t session, int32_t kind, int64_t s, const int32_t *src,
                          const int32_t *dst, int64_t *ticket) {
    if (!g || (kind != CM_REQ_INSERT_EDGES && kind != CM_REQ_DELETE_EDGES) || s < 0 ||
        (s > 0 && (!src || !dst)))
        return CM_E_ARG;
    try {
        serve_require(g);
        if (s > g->scfg.max_items) { g->err = "request larger than max_items"; return CM_E_CAPACITY; }
        const int64_t bytes = serve_bytes(kind, s);
        int64_t start = 0;
        if (!serve_admit(g, s, bytes, &start)) {
            serve_pump(g);
            if (!serve_admit(g, s, bytes, &start)) return CM_E_BUSY;
        }
        const int64_t pos = start % g->scfg.ring_items;
        if (s > 0) {
            std::memcpy(g->ssrc + pos, src, sizeof(int32_t) * (size_t)s);
            std::memcpy(g->sdst + pos, dst, sizeof(int32_t) * (size_t)s);
        }
        ProgBatch b{};
        b.off = pos;
        b.s = (int32_t)s;
        b.kind = kind;
        b.n_ids = g->s_n_ids;
        b.session = session < 0 ? -1 : session;
        serve_publish(g, b, start, bytes, g->s_n_ids, ticket);
        serve_pump(g);
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_serve_submit_insert_vertices(cm_graph *g, int32_t c, const int64_t *off, const int32_t *nbrs,
                                    int32_t *first_new_id, int64_t *ticket) {
    if (!g || c < 0 || (c > 0 && !off)) return CM_E_ARG;
    try {
        serve_require(g);
        if (c > 0 && off[0] != 0) { g->err = "off[0] must be 0"; return CM_E_ARG; }
        for (int32_t i = 0; i < c; ++i)
            if (off[i + 1] < off[i]) { g->err = "offsets must be non-decreasing"; return CM_E_ARG; }
        const int64_t total = c > 0 ? off[c] : 0;
        if (total > 0 && !nbrs) return CM_E_ARG;
        if (total > g->scfg.max_items) { g->err = "request larger than max_items"; return CM_E_CAPACITY; }
        if ((int64_t)g->s_n_ids + c > INT_MAX - 1) { g->err = "vertex ids exceed int32"; return CM_E_CAPACITY; }
        if ((int64_t)g->s_n_ids + c > g->g.n_cap) {
            // the ids must exist before the request is admitted
            if (g->serve_live) {
                g->s_grow = true;
                __atomic_store_n(&g->shdr->stop, 1, __ATOMIC_RELEASE);
                serve_pump(g);
                if (g->serve_live) return CM_E_BUSY;
            }
            int32_t keep = g->g.n_ids;
            g->g.n_ids = g->s_n_ids;
            ensure_vertex_capacity(g, (int64_t)g->s_n_ids + c + g->scfg.vertex_headroom);
            g->g.n_ids = keep;
            g->s_grow = false;
        }
        const int64_t bytes = serve_bytes(CM_REQ_INSERT_VERTICES, total);
        int64_t start = 0;
        if (!serve_admit(g, total, bytes, &start)) {
            serve_pump(g);
            if (!serve_admit(g, total, bytes, &start)) return CM_E_BUSY;
        }
        const int64_t pos = start % g->scfg.ring_items;
        const int32_t v0 = g->s_n_ids;
        for (int32_t i = 0; i < c; ++i)
            for (int64_t j = off[i]; j < off[i + 1]; ++j) {
                g->ssrc[pos + j] = v0 + i;
                g->sdst[pos + j] = nbrs[j];
            }
        ProgBatch b{};
        b.off = pos;
        b.s = (int32_t)total;
        b.kind = CM_REQ_INSERT_VERTICES;
        b.session = -1;
        b.v0 = v0;
        b.nv = c;
        b.n_ids = v0 + c;
        g->s_n_ids = v0 + c;
        if (first_new_id) *first_new_id = v0;
        serve_publish(g, b, start, bytes, v0 + c, ticket);
        serve_pump(g);
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_serve_submit_delete_vertices(cm_graph *g, int32_t c, const int32_t *ids, int64_t *ticket) {
    if (!g || c < 0 || (c > 0 && !ids)) return CM_E_ARG;
    try {
        serve_require(g);
        if (c > g->scfg.max_items) { g->err = "request larger than max_items"; return CM_E_CAPACITY; }
        const int64_t bytes = serve_bytes(CM_REQ_DELETE_VERTICES, c);
        int64_t start = 0;
        if (!serve_admit(g, c, bytes, &start)) {
            serve_pump(g);
            if (!serve_admit(g, c, bytes, &start)) return CM_E_BUSY;
        }
        const int64_t pos = start % g->scfg.ring_items;
        if (c > 0) std::memcpy(g->ssrc + pos, ids, sizeof(int32_t) * (size_t)c);
        ProgBatch b{};
        b.off = pos;
        b.s = c;
        b.kind = CM_REQ_DELETE_VERTICES;
        b.session = -1;
        b.n_ids = g->s_n_ids;
        serve_publish(g, b, start, bytes, g->s_n_ids, ticket);
        serve_pump(g);
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_serve_poll(cm_graph *g, int64_t *finished) {
    if (!g) return CM_E_ARG;
    try {
        serve_require(g);
        serve_pump(g);
        if (finished) *finished = g->s_done;
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_serve_result(cm_graph *g, int64_t ticket, cm_batch_stats *out) {
    if (!g || !out || ticket < 0) return CM_E_ARG;
    if (ticket >= g->s_done) return CM_E_BUSY;
    *out = g->s_results[(size_t)ticket];
    return CM_OK;
}

int cm_serve_stop(cm_graph *g) {
    Range range("cm_serve_stop");
    if (!g) return CM_E_ARG;
    if (!g->serving) return CM_OK;
    try {
        // finish every admitted request, then end the launch
        const double t0 = now_ms();
        while (g->s_done < g->s_next) {
            serve_pump(g);
            if (now_ms() - t0 > 600000.0) {
                g->poisoned = true;
                g->err = "serving did not drain";
                throw Fail{CM_E_INTERNAL};
            }
        }
        if (g->serve_live) {
            __atomic_store_n(&g->shdr->stop, 1, __ATOMIC_RELEASE);
            while (__atomic_load_n(&g->shdr->exit_reason, __ATOMIC_ACQUIRE) == 0) {
                if (now_ms() - t0 > 600000.0) {
                    g->poisoned = true;
                    g->err = "serving launch did not stop";
                    throw Fail{CM_E_INTERNAL};
                }
            }
            serve_after_exit(g);
        }
        g->g.n_ids = std::max(g->g.n_ids, g->s_n_ids);
        g->serving = false;
        serve_free(g);
        set_bar_bounds(g, 0);
    } catch (const Fail &f) {
        g->serving = false;
        return f.code;
    }
    return CM_OK;
}

}  // extern "C"

namespace {

// Snapshot file: header, then int32 core[n_ids], int32 SD[n_ids], and the m
// edges as int32 src[m], int32 dst[m] (each undirected edge once, (min, max)).
struct SnapHeader {
    char magic[8];
    int32_t version;
    int32_t n_ids;
    int32_t n_alive;
    int32_t pad;
    int64_t m;
    uint64_t checksum;  // word-wise FNV-1a of the payload
};
constexpr char SNAP_MAGIC[8] = {'C', 'M', 'S', 'N', 'A', 'P', '0', '1'};
constexpr int32_t SNAP_VERSION = 1;

void fnv_words(uint64_t &h, const int32_t *p, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        h ^= (uint64_t)(uint32_t)p[i];
        h *= 0x100000001b3ull;
    }
}

}  // namespace

extern "C" {

int cm_snapshot(cm_graph *g, const char *path) {
    Range range("cm_snapshot");
    if (!g || !path) return CM_E_ARG;
    try {
        require_ready(g, true);
        hipStream_t st = g->stream;
        const int32_t n = g->g.n_ids;
        const int64_t m = g->m;
        std::vector<int32_t> core((size_t)std::max(n, 1)), sd((size_t)std::max(n, 1));
        std::vector<int32_t> xs((size_t)std::max<int64_t>(m, 1)), ys((size_t)std::max<int64_t>(m, 1));
        if (n > 0) {
            HIPCHK(hipMemcpyAsync(core.data(), g->g.core, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(sd.data(), g->g.mcd, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st));
        }
        if (m > 0) {
            int32_t *dx = nullptr, *dy = nullptr;
            dev_alloc(g, &dx, m);
            dev_alloc(g, &dy, m);
            HIPCHK(fill_u64(g->u64_scratch, 0ull, 1, st));
            KArgs a = make_args(g);
            HIPCHK(export_edges(a, dx, dy, m, g->u64_scratch, g->grid_reg, st));
            HIPCHK(hipMemcpyAsync(xs.data(), dx, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(ys.data(), dy, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            dev_free(dx);
            dev_free(dy);
        }
        HIPCHK(hipStreamSynchronize(st));
        for (int32_t v = 0; v < n; ++v)
            if (core[(size_t)v] < 0) sd[(size_t)v] = 0;
        SnapHeader h{};
        std::memcpy(h.magic, SNAP_MAGIC, 8);
        h.version = SNAP_VERSION;
        h.n_ids = n;
        h.n_alive = g->n_alive;
        h.m = m;
        uint64_t cs = 0xcbf29ce484222325ull;
        fnv_words(cs, core.data(), (size_t)n);
        fnv_words(cs, sd.data(), (size_t)n);
        fnv_words(cs, xs.data(), (size_t)m);
        fnv_words(cs, ys.data(), (size_t)m);
        h.checksum = cs;
        FILE *f = std::fopen(path, "wb");
        if (!f) {
            g->err = std::string("cannot open ") + path + " for writing";
            return CM_E_IO;
        }
        bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
        ok = ok && std::fwrite(core.data(), sizeof(int32_t), (size_t)n, f) == (size_t)n;
        ok = ok && std::fwrite(sd.data(), sizeof(int32_t), (size_t)n, f) == (size_t)n;
        ok = ok && std::fwrite(xs.data(), sizeof(int32_t), (size_t)m, f) == (size_t)m;
        ok = ok && std::fwrite(ys.data(), sizeof(int32_t), (size_t)m, f) == (size_t)m;
        ok = (std::fclose(f) == 0) && ok;
        if (!ok) {
            g->err = std::string("write to ") + path + " failed";
            return CM_E_IO;
        }
    } catch (const Fail &f) {
        return f.code;
    }
    g->err.clear();
    return CM_OK;
}

int cm_restore(const cm_config *cfg, const char *path, cm_graph **out) {
    Range range("cm_restore");
    if (!path || !out) return CM_E_ARG;
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return CM_E_IO;
    SnapHeader h{};
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && std::memcmp(h.magic, SNAP_MAGIC, 8) == 0 &&
              h.version == SNAP_VERSION && h.n_ids >= 0 && h.n_ids < INT_MAX - 1 && h.m >= 0 &&
              h.n_alive >= 0 && h.n_alive <= h.n_ids;
    std::vector<int32_t> core, sd, xs, ys;
    if (ok) {
        // the payload must be exactly the size the header announces
        const long here = std::ftell(f);
        ok = here >= 0 && std::fseek(f, 0, SEEK_END) == 0;
        const long end = ok ? std::ftell(f) : -1;
        ok = ok && end >= here && (uint64_t)(end - here) == 4ull * (2ull * (uint64_t)h.n_ids + 2ull * (uint64_t)h.m) &&
             std::fseek(f, here, SEEK_SET) == 0;
    }
    if (ok) {
        const size_t n = (size_t)h.n_ids, m = (size_t)h.m;
        core.resize(std::max<size_t>(n, 1));
        sd.resize(std::max<size_t>(n, 1));
        xs.resize(std::max<size_t>(m, 1));
        ys.resize(std::max<size_t>(m, 1));
        ok = std::fread(core.data(), sizeof(int32_t), n, f) == n && std::fread(sd.data(), sizeof(int32_t), n, f) == n &&
             std::fread(xs.data(), sizeof(int32_t), m, f) == m && std::fread(ys.data(), sizeof(int32_t), m, f) == m;
        if (ok) {
            uint64_t cs = 0xcbf29ce484222325ull;
            fnv_words(cs, core.data(), n);
            fnv_words(cs, sd.data(), n);
            fnv_words(cs, xs.data(), m);
            fnv_words(cs, ys.data(), m);
            ok = cs == h.checksum;
        }
        // consistency: cores in range, dead ids hold no edge, the alive count matches
        int64_t alive = 0;
        for (size_t v = 0; ok && v < n; ++v) {
            ok = core[v] >= -1 && core[v] < h.n_ids && sd[v] >= 0 && (core[v] >= 0 || sd[v] == 0);
            alive += core[v] >= 0;
        }
        ok = ok && alive == h.n_alive;
        for (size_t e = 0; ok && e < m; ++e)
            ok = xs[e] >= 0 && xs[e] < h.n_ids && ys[e] >= 0 && ys[e] < h.n_ids && core[(size_t)xs[e]] >= 0 &&
                 core[(size_t)ys[e]] >= 0;
    }
    std::fclose(f);
    if (!ok) return CM_E_IO;
    cm_graph *g = nullptr;
    int rc = cm_create(cfg, &g);
    if (rc != CM_OK) return rc;
    rc = cm_load_graph(g, h.n_ids, h.m, xs.data(), ys.data(), 0);
    if (rc != CM_OK) {
        cm_destroy(g);
        return rc == CM_E_NOMEM || rc == CM_E_DEVICE ? rc : CM_E_IO;
    }
    try {
        hipStream_t st = g->stream;
        if (h.n_ids > 0) {
            HIPCHK(hipMemcpyAsync(g->g.core, core.data(), sizeof(int32_t) * (size_t)h.n_ids, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(g->g.mcd, sd.data(), sizeof(int32_t) * (size_t)h.n_ids, hipMemcpyHostToDevice, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        g->n_alive = h.n_alive;
        g->decomposed = true;
    } catch (const Fail &fl) {
        cm_destroy(g);
        return fl.code;
    }
    *out = g;
    return CM_OK;
}

int cm_debug_log(cm_graph *g, int64_t *n_sel, int32_t *sel, int64_t sel_cap, int64_t *n_chg, int32_t *chg,
                 int64_t chg_cap) {
    if (!g || sel_cap < 0 || chg_cap < 0 || (sel_cap > 0 && !sel) || (chg_cap > 0 && !chg)) return CM_E_ARG;
    if (!g->dl.n) {
        g->err = "the iteration log needs cm_config.debug";
        return CM_E_STATE;
    }
    if (g->serving) {
        g->err = "the graph is being served (call cm_serve_stop first)";
        return CM_E_STATE;
    }
    try {
        hipStream_t st = g->stream;
        unsigned long long cnt[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(cnt, g->dl.n, sizeof(cnt), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (n_sel) *n_sel = (int64_t)cnt[0];
        if (n_chg) *n_chg = (int64_t)cnt[1];
        const int64_t ks = std::min<int64_t>(std::min<int64_t>((int64_t)cnt[0], g->dl.cap), sel_cap);
        const int64_t kc = std::min<int64_t>(std::min<int64_t>((int64_t)cnt[1], g->dl.cap), chg_cap);
        if (ks > 0)
            HIPCHK(hipMemcpyAsync(sel, g->dl.sel, sizeof(int32_t) * 3 * (size_t)ks, hipMemcpyDeviceToHost, st));
        if (kc > 0)
            HIPCHK(hipMemcpyAsync(chg, g->dl.chg, sizeof(int32_t) * 3 * (size_t)kc, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if ((int64_t)cnt[0] > g->dl.cap || (int64_t)cnt[1] > g->dl.cap) {
            g->err = "the iteration log overflowed its capacity";
            return CM_E_CAPACITY;
        }
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_phase_times(cm_graph *g, double *ms, int64_t *counts, int32_t n, int reset) {
    if (!g || n < 0 || n > PH_SLOTS || (n > 0 && !ms)) return CM_E_ARG;
    try {
        if (!g->ctl) return CM_E_STATE;
        int khz = 0;
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device));
        if (khz <= 0) { g->err = "device wall clock rate unknown"; throw Fail{CM_E_DEVICE}; }
        unsigned long long buf[2 * PH_SLOTS];
        HIPCHK(hipMemcpyAsync(buf, &g->ctl->ph_ticks[0], sizeof(buf), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        for (int32_t i = 0; i < n; ++i) {
            ms[i] = (double)buf[i] / (double)khz;
            if (counts) counts[i] = (int64_t)buf[PH_SLOTS + i];
        }
        if (reset) {
            std::memset(buf, 0, sizeof(buf));
            HIPCHK(hipMemcpyAsync(&g->ctl->ph_ticks[0], buf, sizeof(buf), hipMemcpyHostToDevice, g->stream));
            HIPCHK(hipStreamSynchronize(g->stream));
        }
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_num_vertices(cm_graph *g, int32_t *n_ids, int32_t *n_alive) {
    if (!g) return CM_E_ARG;
    if (n_ids) *n_ids = g->g.n_ids;
    if (n_alive) *n_alive = g->n_alive;
    return CM_OK;
}

int cm_num_edges(cm_graph *g, int64_t *m) {
    if (!g || !m) return CM_E_ARG;
    *m = g->m;
    return CM_OK;
}

int cm_export_edges(cm_graph *g, int32_t *src, int32_t *dst, int64_t cap, int64_t *m_out, int on_device) {
    if (!g || cap < 0 || (cap > 0 && (!src || !dst))) return CM_E_ARG;
    try {
        require_ready(g, false);
        if (m_out) *m_out = g->m;
        if (cap < g->m) return CM_E_ARG;
        if (g->m == 0) return CM_OK;
        hipStream_t st = g->stream;
        int32_t *xs = src, *ys = dst;
        bool own = !on_device;
        if (own) {
            dev_alloc(g, &xs, g->m);
            dev_alloc(g, &ys, g->m);
        }
        HIPCHK(fill_u64(g->u64_scratch, 0ull, 1, st));
        KArgs a = make_args(g);
        HIPCHK(export_edges(a, xs, ys, g->m, g->u64_scratch, g->grid_reg, st));
        if (own) {
            HIPCHK(hipMemcpyAsync(src, xs, sizeof(int32_t) * (size_t)g->m, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(dst, ys, sizeof(int32_t) * (size_t)g->m, hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        if (own) {
            dev_free(xs);
            dev_free(ys);
        }
    } catch (const Fail &f) {
        return f.code;
    }
    return CM_OK;
}

int cm_run_batches(cm_graph *g, int32_t nb, const int32_t *kinds, const int64_t *offsets,
                   const int32_t *src, const int32_t *dst, const int32_t *sub, int32_t nsub,
                   int on_device, cm_batch_stats *results, int32_t *sub_status) {
    Range range("cm_run_batches");
    if (!g || nb < 0 || nb > (1 << 28) || (nb > 0 && (!kinds || !offsets))) return CM_E_ARG;
    if (nsub < 0 || (sub && nsub == 0)) return CM_E_ARG;
    double t0 = now_ms();
    if (results)
        for (int32_t j = 0; j < nb; ++j) {
            std::memset(&results[j], 0, sizeof(cm_batch_stats));
            results[j].first_bad = -1;
        }
    if (sub_status)
        for (int32_t b = 0; b < nsub; ++b) sub_status[b] = CM_OK;
    try {
        require_ready(g, true);
        debug_reset(g);
        if (nb == 0) return CM_OK;
        if (offsets[0] != 0) { g->err = "offsets[0] must be 0"; throw Fail{CM_E_ARG}; }
        int64_t max_s = 0;
        for (int32_t j = 0; j < nb; ++j) {
            int64_t sj = offsets[j + 1] - offsets[j];
            if (sj < 0) { g->err = "offsets must be non-decreasing"; throw Fail{CM_E_ARG}; }
            if (kinds[j] != CM_BATCH_INSERT && kinds[j] != CM_BATCH_DELETE) {
                g->err = "unknown batch kind";
                throw Fail{CM_E_ARG};
            }
            max_s = std::max(max_s, sj);
        }
        const int64_t total = offsets[nb];
        if (total > 0 && (!src || !dst)) throw Fail{CM_E_ARG};
        if (max_s > INT_MAX / 2) { g->err = "batch too large"; throw Fail{CM_E_ARG}; }
        hipStream_t st = g->stream;
        ensure_batch(g, std::max<int64_t>(max_s, 1));
        // items on the device
        const int32_t *ds = src, *dd = dst, *dsub = sub;
        if (!on_device && total > 0) {
            if (total > g->items_cap) {
                dev_free(g->d_isrc); dev_free(g->d_idst); dev_free(g->d_isub);
                int64_t c = std::max<int64_t>(total, 1024);
                dev_alloc(g, &g->d_isrc, c);
                dev_alloc(g, &g->d_idst, c);
                dev_alloc(g, &g->d_isub, c);
                g->items_cap = c;
            }
            HIPCHK(hipMemcpyAsync(g->d_isrc, src, sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(g->d_idst, dst, sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice, st));
            if (sub)
                HIPCHK(hipMemcpyAsync(g->d_isub, sub, sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice, st));
            ds = g->d_isrc;
            dd = g->d_idst;
            dsub = sub ? g->d_isub : nullptr;
        }
        if (sub) {
            int64_t cap = g->sub_cap;
            grow_dev(g, g->d_sub_bad, cap, nsub);
            g->sub_cap = (int32_t)cap;
            HIPCHK(fill_u64(g->d_sub_bad, ~0ull, nsub, st));
        }
        g->b.sub_bad = g->d_sub_bad;
        const bool strict = g->cfg.strict != 0;

        if (g->cfg.mode == CM_MODE_PLAIN) {
            for (int32_t j = 0; j < nb; ++j) {
                int64_t sj = offsets[j + 1] - offsets[j];
                if (sj == 0) continue;
                ensure_batch(g, sj);  // no reallocation (max size done above); clears the batch hash
                g->b.src_in = const_cast<int32_t *>(ds + offsets[j]);
                g->b.dst_in = const_cast<int32_t *>(dd + offsets[j]);
                g->b.sub_in = dsub ? dsub + offsets[j] : nullptr;
                cm_batch_stats tmp;
                std::memset(&tmp, 0, sizeof(tmp));
                tmp.first_bad = -1;
                const double tb = now_ms();
                int64_t dropped = 0;
                try {
                    edge_batch(g, sj, kinds[j] == CM_BATCH_INSERT, &tmp, &dropped, false, false, dsub != nullptr);
                } catch (const Fail &f) {
                    if (g->poisoned || f.code > CM_E_RANGE || f.code < CM_E_DEAD) throw;
                    tmp.status = f.code;
                }
                tmp.ms_total = now_ms() - tb;
                if (results) results[j] = tmp;
            }
            g->b.sub_in = nullptr;
        } else {
            std::vector<ProgBatch> pb(nb);
            for (int32_t j = 0; j < nb; ++j) {
                pb[j].off = offsets[j];
                pb[j].s = (int32_t)(offsets[j + 1] - offsets[j]);
                pb[j].kind = kinds[j];
            }
            std::vector<ProgOut> out(nb);
            int used_graph = 0;
            double kms = 0.0;
            int launches = 0;
            program_execute(g, pb, ds, dd, dsub, strict, out, &used_graph, &kms, &launches);
            for (int32_t j = 0; j < nb; ++j) {
                const ProgOut &o = out[j];
                if (o.status == 0) g->m += kinds[j] == CM_BATCH_INSERT ? o.valid : -(int64_t)o.valid;
                if (!results) continue;
                cm_batch_stats &r = results[j];
                r.status = o.status;
                r.iterations = o.iterations;
                r.first_bad = o.first_bad;
                r.applied = o.valid;
                r.dropped = o.status == 0 ? (offsets[j + 1] - offsets[j]) - o.valid : 0;
                r.remaining_sum = (int64_t)o.remaining;
                r.candidates = (int64_t)o.candidates;
                r.evicted = (int64_t)o.evicted;
                r.changed = (int64_t)o.changed;
                r.scanned = (int64_t)o.scanned;
                r.rounds = (int64_t)o.rounds;
                r.local_steps = (int64_t)o.steps;
                r.alg_bytes = alg_bytes(o);
                r.cand_degree = (int64_t)o.cdeg;
                r.evicted_degree = (int64_t)o.edeg;
                r.changed_degree = (int64_t)o.hdeg;
                r.launches = j == 0 ? launches : 0;
                r.graph_launch = used_graph;
                r.group = 1;
                r.first_stamp = o.ep0;
                r.kernel_ms = j == 0 ? kms : 0.0;
            }
        }
        g->b.sub_in = nullptr;
        if (sub && sub_status) {
            std::vector<unsigned long long> sb(nsub);
            HIPCHK(hipMemcpy(sb.data(), g->d_sub_bad, sizeof(unsigned long long) * (size_t)nsub, hipMemcpyDeviceToHost));
            for (int32_t b = 0; b < nsub; ++b)
                sub_status[b] = sb[b] == ~0ull ? CM_OK : -(int)(sb[b] & 0xff);
        }
        if (results && nb > 0 && g->cfg.mode != CM_MODE_PLAIN) results[0].ms_total = now_ms() - t0;
    } catch (const Fail &f) {
        g->b.sub_in = nullptr;
        return f.code;
    }
    g->err.clear();
    return CM_OK;
}

}  // extern "C"
