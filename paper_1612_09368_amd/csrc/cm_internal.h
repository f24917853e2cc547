// Internal device-side layout and helpers of libcoremaint (gfx950, wave64).
//
// Graph store ("slack CSR with per-vertex spill blocks"): vertex v owns the
// contiguous slot range nbr[off[v] .. off[v] + cap[v]); the first len[v]
// slots are used, entries < 0 are tombstones left by deletions inside a
// batch.  A list that outgrows its slack moves to a fresh block carved from
// the tail of the same pool (its spill block); the old range becomes garbage
// that the next repack reclaims.  Every list stays contiguous, so one wave
// reads a list with coalesced loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cm_keys.h"

namespace cm {

constexpr int WAVE = 64;
constexpr int32_t TOMB = -1;             // deleted adjacency slot
constexpr uint64_t EMPTY_KEY = ~0ull;    // empty hash slot

// One batch of a batch program: items [off, off + s) of the program's
// src/dst (and of sub, when it packs independent batches).
struct ProgBatch {
    int64_t off;
    int32_t s;
    int32_t kind;        // 0 insert edges, 1 delete edges, 2 insert vertices, 3 delete vertices
    int32_t v0;          // kind 2: first new id
    int32_t nv;          // kind 2: new ids [v0, v0 + nv); items are their edges (new id, neighbour)
    int32_t n_ids;       // ids in use for this batch (0: the launch's); kind 3: items are ids
    int32_t session;     // serving: independent session of the request (-1: none)
    int32_t nsub;        // serving: requests fused into this batch (0: one request); item i then
                         // belongs to request bsub[i] of the group
    int32_t pad;
};

// Most requests one served batch may fuse.
constexpr int FUSE_MAX = 32;

// ---------------------------------------------------------------------------
// Control block: counters shared by all workgroups of a launch.  Rotating
// queue tails use three slots: in round r the tail r%3 is read, (r+1)%3
// receives pushes and (r+2)%3 is cleared for the next round.
// ---------------------------------------------------------------------------
struct Ctl {
    int32_t rem_count[2];    // remaining-edge lists, ping-pong by epoch parity
    int32_t sel_count;       // selected edges of the current iteration
    int32_t fq_tail[3];      // expansion: normal vertices
    int32_t fh_tail[3];      // expansion: chunks of long lists
    int32_t eq_tail[3];      // eviction / peel / decomposition: normal vertices
    int32_t eh_tail[3];      // eviction / peel / decomposition: chunks of long lists
    int32_t cand_count;      // candidates of the iteration (insert)
    int32_t chg_count;       // changed vertices (normal)
    int32_t chh_count;       // changed vertices (chunks)
    int32_t touched_count;   // vertices whose peel counter was touched (delete)
    int32_t overflow;        // a queue push went past its capacity (bug guard)
    int32_t epoch;           // last iteration stamp used
    int32_t iters_done;      // iterations run by the last launch
    int32_t pool_fail;       // adjacency pool exhausted during reservation
    int32_t first_bad;       // smallest invalid batch index
    int32_t valid_count;     // valid batch items
    int32_t scan_tail;       // locate-scan chunk queue
    int32_t vlist_count;     // distinct endpoints of the batch
    int32_t reloc_count;     // lists relocated to spill blocks
    int32_t changed_count;   // vertices whose core moved (current iteration)
    int32_t rm_count[3];     // decomposition: remaining vertices (rotating)
    int32_t min_deg[3];      // decomposition: smallest remaining degree (rotating)
    int32_t kmax;            // decomposition: largest core number
    int32_t dec_rounds;      // decomposition: frontier rounds
    int32_t ipub[2][4];      // iteration step machine: (step, round, force grid) published by workgroup 0
    int32_t dpub[2][6];      // decomposition step machine: (step, k, j, f, kmax, force grid)
    unsigned long long pool_tail;     // next free adjacency slot
    unsigned long long garbage;       // slots abandoned by relocations
    // statistics (summed over the iterations of a batch)
    unsigned long long st_iters;
    unsigned long long st_remaining;
    unsigned long long st_selected;
    unsigned long long st_candidates;
    unsigned long long st_evicted;
    unsigned long long st_changed;
    unsigned long long st_scanned;
    unsigned long long st_rounds;       // cascade rounds (expansion, eviction, peel)
    unsigned long long st_grid_steps;   // steps run by the whole grid
    unsigned long long st_local_steps;  // steps run inside one workgroup
    unsigned long long st_icand;        // insertion candidates visited
    unsigned long long st_cdeg;         // list entries of the insertion candidates
    unsigned long long st_edeg;         // list entries of the evicted / peeled vertices
    unsigned long long st_hdeg;         // list entries of the vertices whose core moved
    // phase clock (device wall clock ticks, summed until the host clears them;
    // written by global thread 0 only): indices are StepKind for grid steps,
    // then PH_LOCAL .. PH_COMPACT below
    unsigned long long ph_ticks[16];
    unsigned long long ph_count[16];
    // vertex deletion inside a batch program
    unsigned long long vd_total;  // list slots of the valid ids
    int32_t vd_tail;              // gathered edges
    int32_t vd_bad;               // smallest invalid id index
    int32_t vd_count;             // valid ids
    int32_t aq_tail[2];           // asynchronous queues: slots handed out
    int32_t aq_head[2];           //   slots taken by consumers
    int32_t aq_pend[2];           //   items pushed and not finished
    unsigned long long one_key;   // single-edge regime: largest complemented claim key of the iteration
    int32_t sv_decision;          // serving: decision of the waiting thread
    ProgBatch sv_batch;           // serving: descriptor of the current batch
    int32_t sv_gn;                // serving: requests fused into the current batch
    int32_t sv_goff[FUSE_MAX + 1];  // serving: item offsets of the fused requests in the batch
};

// Phase-clock slots after the step kinds (0 .. 7).
constexpr int PH_LOCAL = 8;      // a chain of steps run inside workgroup 0 (plus its barrier)
constexpr int PH_VALIDATE = 9;   // batch validation in a batch program
constexpr int PH_RESERVE = 10;   // capacity reservation in a batch program
constexpr int PH_COMPACT = 11;   // tombstone compaction in a batch program
constexpr int PH_SLOTS = 16;

// Grid barrier state: one arrival counter per group of workgroups (a group is
// the workgroups that share blockIdx % NGRP, i.e. one XCD under round-robin
// dispatch), one counter for the groups, one generation word; each on its
// own 128-byte line.
constexpr int NGRP = 8;
constexpr int XSLOTS = 16;  // XCC ids a workgroup can report
struct Bar {
    unsigned int grp[XSLOTS * 32];  // arrival counters (per group, 128-byte apart)
    unsigned int top[32];
    unsigned int gen[32];
    unsigned int abort[32];   // set when a wait gives up; later barriers return at once
    unsigned long long xreg[XSLOTS * 16];  // per XCC: (launch epoch << 32) | workgroups on it
    unsigned long long wait_ticks[16];   // [0]: device wall-clock ticks a barrier wait may last
    unsigned long long slice_ticks[16];  // [0]: ticks one workgroup's chain of local steps may run
};

// One of two int32 fields that share an 8-byte record per vertex (the
// record array holds field 0 of vertex v at 2v and field 1 at 2v + 1), so
// that a kernel touching both fields of a random vertex fetches one cache
// line instead of two.
struct Paired {
    int32_t *p;  // &field of vertex 0
    __device__ __forceinline__ int32_t &operator[](int64_t v) const { return p[2 * v]; }
};

// Per-vertex device arrays plus the adjacency pool.
struct DevGraph {
    int32_t n_cap;       // allocated ids
    int32_t n_ids;       // ids in use
    int64_t pool_size;   // slots in nbr
    int64_t *off;        // [n_cap] first slot of the list
    int32_t *len;        // [n_cap] used slots (incl. tombstones)
    int32_t *cap;        // [n_cap] reserved slots
    int32_t *nbr;        // [pool_size]
    int32_t *core;       // [n_cap] core number; -1 = dead id
    int32_t *mcd;        // [n_cap] superior degree SD (neighbours with core >= own)
    Paired stamp;        // [n_cap] iteration stamp: candidate (insert) / peeled (delete); paired with cd
    int32_t *chg;        // [n_cap] iteration stamp: core moved this iteration
    Paired cd;           // [n_cap] insertion counter (CSD, then decremented); in the same record as
                         // stamp, which every access to a candidate's counter checks first
    int32_t *dec;        // [n_cap] deletion peel counter (zero between iterations)
    int32_t *done;       // [n_cap] finished chunks of a long list (zero between uses)
    uint32_t *matched;   // [n_cap] selection round stamp
    unsigned long long *claim;  // [n_cap] selection claim key (smaller wins)
    int32_t *bmark;      // [n_cap] batch stamp (validation scans, reservation)
    int32_t *gain;       // [n_cap] edges a batch adds to the list (zero between uses)
    // Supporter runs of an insertion iteration (null when off): while the
    // expansion counts a candidate's CSD it also writes the neighbours that
    // are level-k candidates-to-be (core == k, SD > k), compacted from the
    // start of the candidate's own slot range of `sub`; the eviction then
    // walks those alone instead of the whole list.  slen = the run's length
    // (zeroed when the candidate is claimed; the chunks of a long list
    // reserve their slots in it with atomics).
    int32_t *sub;        // [pool_size] same slot ranges as nbr
    int32_t *slen;       // [n_cap] length of the candidate's supporter run
    // Up-lists of long lists (null when off), kept across iterations and
    // batches: per chunk of a list split into chunks, the neighbours whose
    // core was at least the owner's when the list was last scanned whole,
    // compacted into the chunk's slot range of `upl` (a negative entry ends
    // a chunk holding fewer than its slots).  ubl = the list length at that
    // scan (slots from ubl on were appended later and are read from nbr), or
    // -1 when the up-list is invalid.  Every change that could put a
    // neighbour into the owner's up-set outside it -- a neighbour rising to
    // the owner's core, the owner's core falling, an edge of the owner
    // deleted, the list moved -- makes it invalid; a neighbour that falls, or
    // the owner rising, only leaves extra entries, which every reader tests.
    int32_t *upl;        // [pool_size] same slot ranges as nbr
    int32_t *ubl;        // [n_cap]
};

// Edges of one batch after validation.
struct DevBatch {
    int32_t cap;         // capacity in edges
    int32_t *src_in;     // raw input (device copy or caller pointer)
    int32_t *dst_in;
    int32_t *err;        // [cap] per-item status
    int32_t *eu;         // [cap] canonical endpoints, eu < ev
    int32_t *ev;
    int64_t *su;         // [cap] slot of ev in N(eu) (delete), -1 if not found
    int64_t *sv;         // [cap] slot of eu in N(ev) (delete)
    int32_t *hslot;      // [cap] hash slot of the item
    int32_t *rem[2];     // remaining edge indices, ping-pong
    int32_t *sel;        // selected edge indices of an iteration
    int32_t *esel;       // [cap] iteration stamp of selection
    int32_t hcap;        // hash slots (power of two)
    unsigned long long *hkey;  // [hcap]
    int32_t *hval;       // [hcap] smallest item index with that key
    int32_t *vlist;      // [n_cap] distinct batch endpoints (reservation / compaction)
    int64_t *scanq;      // [scap] (vertex, chunk) locate-scan items
    int32_t scap;
    const int32_t *sub_in;  // sub-batch id per item (packed batches) or null
    unsigned long long *sub_bad;  // per sub-batch min of (item << 8 | -code)
    int32_t *reloc;      // [n_cap] relocated vertices
    int64_t *reloc_off;  // [n_cap] their new first slot
    int32_t *reloc_cap;  // [n_cap] their new capacity
};

// Frontier queues of an iteration.  Long lists (len > large) enter the
// chunk queues as (vertex << 32 | chunk) items so that their work spreads
// over many waves.
struct DevQueues {
    int32_t vcap;        // capacity of vertex queues
    int32_t hcap;        // capacity of chunk queues
    int32_t *fq[2];
    int64_t *fh[2];
    int32_t *eq[2];
    int64_t *eh[2];
    int32_t *cand;
    int32_t *chg;
    int64_t *chh;
    int32_t *touched;
    int32_t acap;                 // capacity of the asynchronous work queues
    unsigned long long *aq[2];    // asynchronous steps: 0 expansion, 1 eviction / peel
};

struct Tune {
    int32_t small_deg;   // list length walked by one lane (whole-graph passes, asynchronous cascades)
    int32_t large_deg;   // longer lists are chunked
    int32_t chunk;       // chunk length
    int32_t rounds;      // selection rounds per iteration
    int32_t local_edges; // partition / apply steps up to this many edges run in one workgroup
    int32_t local_items; // frontier steps up to this many items run in one workgroup
    int32_t local_work;  // ... and only if their lists hold at most this many entries
    int32_t async_steps; // cascades as work-queue steps
    int32_t single_edge; // one edge per iteration (the sequential regime) instead of a superior edge set
    int32_t prune;       // expansion visits the neighbours of a candidate only once its CSD exceeds its
                         // core (Algorithm 3); 0 = claims them while counting the CSD
    int32_t stamp_limit; // iteration stamps restart (stamp arrays cleared) before passing this
    int32_t sublists;    // the one-pass expansion records supporter lists for the eviction
    int32_t uplists;     // long lists keep up-lists (scanned by the one-pass expansion)
    int32_t pad;
};

// Chunk items of the expansion's claim pass (pruned expansion) carry this
// flag in the chunk index.
constexpr int32_t CLAIM_CHUNK = 0x40000000;

constexpr int COOP_THREADS = 512;  // workgroup size of the cooperative kernels

struct ProgDesc;

// Outcome of one maintenance launch, written at its end by global thread 0
// into pinned host memory (one slot per launch in flight), so that the host
// can read it while the next launch already runs.
struct LaunchOut {
    int32_t epoch;     // last iteration stamp used
    int32_t iters;     // iterations run
    int32_t rem_next;  // edges left for the next iteration
    int32_t overflow;  // queue overflow code (0 = none)
    int32_t aborted;   // a grid barrier wait gave up
    int32_t pad[3];
};

// Debug log of the iterations (cm_config.debug): every selected edge of an
// edge iteration as (iteration stamp, u, v) with u < v, and every core change
// of an edge iteration as (iteration stamp, v, new core).  n[i] counts the
// entries recorded (it may pass cap: the entries beyond cap are lost).
struct DebugLog {
    int32_t *sel;              // [3 * cap] or null when the log is off
    int32_t *chg;              // [3 * cap]
    unsigned long long *n;     // [2]
    int64_t cap;
};

struct KArgs {
    DevGraph g;
    DevBatch b;
    DevQueues q;
    Tune t;
    Ctl *ctl;
    Bar *bar;
    ProgDesc *prog;      // batch program of a persistent multi-batch launch
    int32_t inserting;   // 1 = insertion batch, 0 = deletion batch
    int32_t max_iters;   // iterations this launch may run
    int32_t s;           // batch items
    int32_t bstamp;      // batch stamp (bmark values bstamp, bstamp + 1)
    int32_t cur;         // remaining list that receives the validated batch
    int32_t strict;      // packed sub-batches: drop a sub-batch with an invalid item
    LaunchOut *lout;     // maintenance launch outcome (pinned host) or null
    DebugLog dl;         // iteration log (debug mode) or all null
};

// Per-batch parameters of the validation / reservation steps.
struct BatchCtx {
    const int32_t *src;  // raw items
    const int32_t *dst;
    const int32_t *sub;  // sub-batch of each item (packed independent batches) or null
    unsigned long long *sub_bad;  // per sub-batch min of (item << 8 | -code), ~0 if none
    int32_t s;           // item count
    int32_t inserting;   // 1 = insertion batch
    int32_t cur;         // remaining list that receives the valid items
    int32_t bstamp;      // per-vertex mark values bstamp (scan) and bstamp + 1 (endpoints)
    int32_t hcap;        // hash slots used (power of two, <= allocated)
    int32_t strict;      // reject a whole (sub-)batch that has an invalid item
    int32_t n_ids;       // ids in use (range check)
};

__device__ __forceinline__ BatchCtx batch_of(const KArgs &a) {
    return BatchCtx{a.b.src_in, a.b.dst_in, a.b.sub_in, a.b.sub_bad, a.s, a.inserting, a.cur, a.bstamp,
                    a.b.hcap, a.strict, a.g.n_ids};
}

// Outcome of one batch of a batch program.
struct ProgOut {
    int32_t status;      // 0 or the error code of the first invalid item (strict)
    int32_t first_bad;
    int32_t valid;       // edges applied
    int32_t iterations;
    int32_t vdone;       // vertex batches: vertices inserted / deleted
    int32_t group;       // requests in the batch that ran this one (1 unless fused)
    int32_t ep0;         // first iteration stamp of that batch
    int32_t pad;
    unsigned long long remaining, selected, candidates, evicted, changed, scanned, rounds, steps;
    unsigned long long icand, cdeg, edeg, hdeg;
};
// Why a serving launch ended (ServeHdr.exit_reason; 0 while it runs).
enum ServeExit : int32_t { SV_RUN = 1, SV_STOP = 2, SV_IDLE = 3, SV_POOL = 4, SV_ABORT = 5, SV_TOOBIG = 6,
                           SV_RESTAMP = 7 };
// A serving launch hands back to the host after this many batches (their
// batch stamps, two per batch from the launch's first, stay below 2^29).
constexpr long long SERVE_BATCHES = 1ll << 27;

// Serving header in pinned host memory; each word on its own 128-byte line.
struct ServeHdr {
    long long tail;       // batches published by the host
    char pad0[120];
    long long head;       // batches finished by the device
    char pad1[120];
    int32_t stop;         // host: leave after the current batch
    char pad2[124];
    int32_t exit_reason;  // device: why the launch ended (0 while running)
    int32_t pad3;
    long long exit_at;    // device: first batch not finished
    char pad4[112];
};
struct ProgDesc {
    const ProgBatch *batches;
    ProgOut *out;
    const int32_t *src;
    const int32_t *dst;
    const int32_t *sub;  // sub-batch id per item (or null)
    unsigned long long *sub_bad;  // per sub-batch min of (item << 8 | -code) (or null)
    int32_t *gsrc;       // vertex deletion: gathered edges (capacity gcap)
    int32_t *gdst;
    int64_t gcap;
    int32_t *firstidx;   // [n_cap] vertex-deletion duplicate marks (INT_MAX between uses)
    ServeHdr *hdr;       // serving: request ring header (null for a fixed program)
    int32_t *bsub;       // serving: request of each item of a fused batch (capacity: batch items)
    int32_t fuse;        // serving: most requests fused into one batch (1: none)
    int32_t pad_f;
    long long sfirst;    // serving: first batch of this launch
    unsigned long long idle_ticks;  // serving: wall-clock ticks without work before leaving
    int32_t ring;        // serving: ring slots
    int32_t nb;
    int32_t first;       // first batch to run
    int32_t strict;
    int32_t bstamp0;
    int32_t stop;        // written: first batch not completed (nb when all ran)
    int32_t pool_fail;   // written: 1 when the launch stopped for a pool repack
};

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane() { return (int)__lane_id(); }
// lanes below this one
__device__ __forceinline__ unsigned long long lanes_below() { return (1ull << lane()) - 1ull; }

__device__ __forceinline__ int gwave() {
    return (int)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
}
__device__ __forceinline__ int nwaves() { return (int)((gridDim.x * blockDim.x) / WAVE); }
__device__ __forceinline__ int gtid() { return (int)(blockIdx.x * blockDim.x + threadIdx.x); }
__device__ __forceinline__ int gthreads() { return (int)(gridDim.x * blockDim.x); }

__device__ __forceinline__ int wave_sum(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Phase clock: global thread 0 reads the device wall clock before a phase
// and adds the elapsed ticks after the barrier that ends it -- in its
// workgroup's LDS, since a read-modify-write of the control block there
// would be a memory round trip right after each barrier on the wave every
// other one then waits for; ph_flush adds the sums to the control block at
// the end of a batch or launch.
// Slots after the phase ticks and counts: the cascade rounds and the grid
// and local steps of the batch (kept there for the same reason).
constexpr int PH_ROUNDS = 2 * PH_SLOTS, PH_GSTEPS = 2 * PH_SLOTS + 1, PH_LSTEPS = 2 * PH_SLOTS + 2;
constexpr int PH_WORDS = 2 * PH_SLOTS + 3;
__device__ __forceinline__ unsigned long long *ph_lds() {
    __shared__ unsigned long long acc[PH_WORDS];  // ticks, counts, steps (workgroup 0 only)
    return acc;
}
// At the start of a launch, before its first barrier (which orders the
// clearing before thread 0's first use).
__device__ __forceinline__ void ph_init() {
    if (blockIdx.x == 0 && threadIdx.x < PH_WORDS) ph_lds()[threadIdx.x] = 0ull;
}
// Count one event of slot i (PH_ROUNDS .. PH_LSTEPS); global thread 0 only.
__device__ __forceinline__ void ph_count(int i) {
    if (gtid() == 0) ph_lds()[i] += 1ull;
}
__device__ __forceinline__ unsigned long long ph_start() {
    return gtid() == 0 ? (unsigned long long)wall_clock64() : 0ull;
}
__device__ __forceinline__ void ph_stop(Ctl *, int slot, unsigned long long t0) {
    if (gtid() == 0) {
        unsigned long long *p = ph_lds();
        p[slot] += (unsigned long long)wall_clock64() - t0;
        p[PH_SLOTS + slot] += 1;
    }
}
__device__ __forceinline__ void ph_flush(Ctl *c) {
    if (gtid() == 0) {
        unsigned long long *p = ph_lds();
        for (int i = 0; i < PH_SLOTS; ++i) {
            if (p[PH_SLOTS + i]) {
                c->ph_ticks[i] += p[i];
                c->ph_count[i] += p[PH_SLOTS + i];
                p[i] = 0ull;
                p[PH_SLOTS + i] = 0ull;
            }
        }
        c->st_rounds += p[PH_ROUNDS];
        c->st_grid_steps += p[PH_GSTEPS];
        c->st_local_steps += p[PH_LSTEPS];
        p[PH_ROUNDS] = p[PH_GSTEPS] = p[PH_LSTEPS] = 0ull;
    }
}

// Coherent read of a control word.  Relaxed (no cache invalidation): the
// ordering with the data it guards comes from the grid / workgroup barrier
// the readers passed; the load itself reads the device-coherent value.
__device__ __forceinline__ int32_t ld_rlx(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_rlx64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every memory operation this wave issued has completed.
__device__ __forceinline__ void wave_drain() { __builtin_amdgcn_s_waitcnt(0); }

// Append `val` for every active lane with pred set; one atomic per wave.
// Works in divergent code: the ballot covers the active lanes only.
template <class T>
__device__ __forceinline__ void push_agg(T *q, int32_t qcap, int32_t *tail, T val, bool pred,
                                         int32_t *overflow) {
    unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    int leader = __ffsll((long long)m) - 1;
    int cnt = __popcll(m);
    int me = lane();
    int rank = __popcll(m & ((1ull << me) - 1ull));
    int base = 0;
    if (me == leader) base = atomicAdd(tail, cnt);
    base = __shfl(base, leader);
    if (pred) {
        int pos = base + rank;
        if (pos < qcap) q[pos] = val;
        else atomicOr(overflow, 1);
    }
}

// Reserve `n` consecutive entries (per lane, any n >= 0) with one atomic per
// wave; returns this lane's first position.
__device__ __forceinline__ int reserve_agg(int32_t *tail, int n) {
    unsigned long long m = __ballot(n > 0);
    if (m == 0ull) return 0;
    // exclusive prefix of n over active lanes
    int me = lane();
    int incl = n;
    for (int o = 1; o < WAVE; o <<= 1) {
        int t = __shfl_up(incl, o);
        if (me >= o) incl += t;
    }
    int total = __shfl(incl, WAVE - 1);
    int base = 0;
    int leader = __ffsll((long long)m) - 1;
    if (me == leader) base = atomicAdd(tail, total);
    base = __shfl(base, leader);
    return base + incl - n;
}

__device__ __forceinline__ int64_t chunk_item(int32_t v, int32_t c) {
    return ((int64_t)v << 32) | (uint32_t)c;
}
__device__ __forceinline__ int32_t item_v(int64_t it) { return (int32_t)(it >> 32); }
__device__ __forceinline__ int32_t item_c(int64_t it) { return (int32_t)(it & 0xffffffff); }

__device__ __forceinline__ int nchunks(int32_t len, int32_t chunk) { return (len + chunk - 1) / chunk; }

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // bijective 32-bit finaliser (xorshift-multiply)
    x ^= x >> 16; x *= 0x7feb352dU;
    x ^= x >> 15; x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ unsigned long long edge_key(int32_t a, int32_t b) {
    int32_t lo = a < b ? a : b, hi = a < b ? b : a;
    return ((unsigned long long)(uint32_t)lo << 32) | (uint32_t)hi;
}

__device__ __forceinline__ uint32_t hash_key(unsigned long long k) {
    uint32_t h = mix32((uint32_t)k ^ 0x9e3779b9U);
    return mix32(h ^ (uint32_t)(k >> 32));
}

// A team is the set of threads that shares one step: the whole grid or one
// workgroup.  Loops stride by the team size; `lead` does the team's
// bookkeeping.
struct Team {
    int rank;
    int size;
    __device__ __forceinline__ int wave() const { return rank / WAVE; }
    __device__ __forceinline__ int nwaves() const { return size / WAVE; }
    __device__ __forceinline__ bool lead() const { return rank == 0; }
};
__device__ __forceinline__ Team grid_team() { return Team{gtid(), gthreads()}; }
__device__ __forceinline__ Team block_team() { return Team{(int)threadIdx.x, (int)blockDim.x}; }

// Per-workgroup barrier state in LDS: XCC id, workgroups on that XCC,
// XCCs in use (set by gbar_setup at the start of every cooperative kernel).
__device__ __forceinline__ unsigned *bar_info() {
    __shared__ unsigned info[4];
    return info;
}

// Hardware id of the XCC (accelerator complex die) running this workgroup.
__device__ __forceinline__ unsigned xcc_id() {
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (XSLOTS - 1);  // HW_REG_XCC_ID[3:0]
}

// Wait until the generation word moves past g0, for at most wait_ticks of
// the device wall clock (the host sets it above every wait the drivers can
// create legitimately: a serving launch's idle wait, a workgroup's slice of
// local steps); a workgroup that never arrives is a bug: the barrier then
// trips the abort word instead of hanging, and the drivers stop at their
// next check.
__device__ __forceinline__ void bar_wait(Bar *b, unsigned g0) {
    unsigned polls = 0;
    unsigned long long t0 = 0;
    while (__hip_atomic_load(&b->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        if (__hip_atomic_load(&b->abort[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        __builtin_amdgcn_s_sleep(2);
        if ((++polls & 1023u) == 0u) {
            const unsigned long long now = (unsigned long long)wall_clock64();
            if (t0 == 0) {
                t0 = now;
            } else if (now - t0 > __hip_atomic_load(&b->wait_ticks[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(&b->abort[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    // one acquire for the whole workgroup after the wait (polls stay relaxed)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Grid-wide barrier of a cooperative launch (all workgroups co-resident),
// correct for any placement of workgroups: thread 0 of each workgroup
// arrives on the counter of group blockIdx % NGRP with a release (its own
// stores become visible device-wide); the last arrival of a group arrives on
// the top counter; the last group bumps the generation word that everyone
// waits on.
__device__ __forceinline__ void gbar_any(Bar *b) {
    wave_drain();  // this wave's stores and atomics have reached the cache hierarchy
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned nb = gridDim.x;
        const unsigned grp = blockIdx.x % NGRP;
        const unsigned members = nb / NGRP + (grp < nb % NGRP ? 1u : 0u);
        const unsigned ngroups = nb < (unsigned)NGRP ? nb : (unsigned)NGRP;
        const unsigned g0 = __hip_atomic_load(&b->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned a = __hip_atomic_fetch_add(&b->grp[grp * 32], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (a == members - 1u) {
            __hip_atomic_store(&b->grp[grp * 32], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned t = __hip_atomic_fetch_add(&b->top[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ngroups - 1u) {
                __hip_atomic_store(&b->top[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&b->gen[0], g0 + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        bar_wait(b, g0);
    }
    __syncthreads();
}

// Start of a cooperative kernel: every workgroup registers the XCC it runs
// on (counted under this launch's epoch, the generation word at the start,
// so nothing needs clearing between launches or graph replays), then one
// gbar_any; afterwards each workgroup knows how many workgroups share its
// XCC and how many XCCs are in use.
__device__ __forceinline__ void gbar_setup(Bar *b) {
    ph_init();
    unsigned *info = bar_info();
    unsigned long long ep = 0;
    unsigned x = 0;
    if (threadIdx.x == 0) {
        x = xcc_id();
        ep = __hip_atomic_load(&b->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long *r = &b->xreg[x * 16];
        unsigned long long old = __hip_atomic_load(r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
            const unsigned long long want = (old >> 32) == ep ? old + 1ull : ((ep << 32) | 1ull);
            const unsigned long long prev = atomicCAS(r, old, want);
            if (prev == old) break;
            old = prev;
        }
    }
    gbar_any(b);
    if (threadIdx.x == 0) {
        // XCCs with workgroups of this launch (a slot never used reads 0 in
        // both halves, so the epoch alone would not tell it apart at epoch 0)
        unsigned ng = 0;
        for (int y = 0; y < XSLOTS; ++y) {
            const unsigned long long v =
                __hip_atomic_load(&b->xreg[y * 16], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((v >> 32) == ep && (v & 0xffffffffull) != 0) ++ng;
        }
        info[0] = x;
        info[1] = (unsigned)(__hip_atomic_load(&b->xreg[x * 16], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                             0xffffffffull);
        info[2] = ng;
    }
    __syncthreads();
}

// The barrier of the step machines (after gbar_setup), grouped by XCC: the
// workgroups of one XCC share its L2, so their arrivals need no release of
// their own: the last arrival of the XCC releases once for all of them
// (their stores had reached that L2 before they arrived), then arrives on
// the top counter; the last XCC bumps the generation word.
__device__ __forceinline__ void gbar(Bar *b) {
    const unsigned *info = bar_info();
    wave_drain();  // this wave's stores and atomics have reached the cache hierarchy
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned x = info[0], members = info[1], ngroups = info[2];
        const unsigned g0 = __hip_atomic_load(&b->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned a = __hip_atomic_fetch_add(&b->grp[x * 32], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == members - 1u) {
            __hip_atomic_store(&b->grp[x * 32], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned t = __hip_atomic_fetch_add(&b->top[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ngroups - 1u) {
                __hip_atomic_store(&b->top[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&b->gen[0], g0 + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        bar_wait(b, g0);
    }
    __syncthreads();
}

// Whether the chain of local steps that workgroup 0 started at t0 (thread
// 0's clock) has used its slice: decided by thread 0, the same answer in
// every thread of the workgroup (all of them must call).
__device__ __forceinline__ bool slice_over(const Bar *b, unsigned long long t0) {
    __shared__ int over;
    if (threadIdx.x == 0)
        over = (unsigned long long)wall_clock64() - t0 >
               __hip_atomic_load(&b->slice_ticks[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const bool r = over != 0;
    __syncthreads();
    return r;
}

__device__ __forceinline__ bool bar_aborted(Bar *b) {
    return __hip_atomic_load(&b->abort[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

}  // namespace cm
