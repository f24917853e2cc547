// Device phases of batched core maintenance.  Each phase is a grid-stride
// __device__ function; the plain driver runs an iteration's phases inside one
// cooperative launch (grid barriers between phases), the persistent driver
// loops over iterations inside one launch.
//
// Notation follows the paper: core(v); SD(v) = superior degree, neighbours w
// with core(w) >= core(v) (kept in `mcd`); CSD(v) = constraint superior
// degree, neighbours w with core(w) > core(v) or core(w) == core(v) and
// SD(w) > core(v); cd = the working counter of Algorithms 3/4 and 6/7.
#pragma once
#include "cm_walk.h"

namespace cm {

// Status codes (match coremaint.h).
constexpr int32_t ST_RANGE = -2, ST_SELF = -3, ST_DUP = -4, ST_EXISTS = -5, ST_MISSING = -6,
                  ST_DEAD = -7;

__device__ __forceinline__ void flush_stat(unsigned long long *dst, long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane() == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// Per-thread statistics of a launch, kept in registers and summed into the
// control block at the end of a batch: adjacency entries read by the
// traversal phases, the list entries of the method's sets (insertion
// candidates, evicted / peeled vertices, vertices whose core moved).  Every
// thread must call flush_acc; it also flushes the phase clock and step
// counts of global thread 0.
struct Acc {
    long long scanned, cdeg, edeg, hdeg;
};
__device__ __forceinline__ void flush_acc(Ctl *c, Acc &acc) {
    flush_stat(&c->st_scanned, acc.scanned);
    flush_stat(&c->st_cdeg, acc.cdeg);
    flush_stat(&c->st_edeg, acc.edeg);
    flush_stat(&c->st_hdeg, acc.hdeg);
    ph_flush(c);
    acc = Acc{};
}

// Queue length as published by its tail, clamped to the buffer capacity
// (a tail can pass the capacity only after an overflow, which aborts the batch).
__device__ __forceinline__ int32_t qlen(const int32_t *tail, int32_t cap) {
    int32_t n = ld_rlx(tail);
    return n < cap ? n : cap;
}

// The queue tails and counts that the iteration's step machine reads at every
// step boundary sit in the control block's first 128 bytes.  One wave-wide
// load after the barrier (or workgroup barrier) that ends a step brings them
// all, lane i holding word i, instead of a chain of single agent-scope loads
// (each a round trip past the L1) in the step decision and the next step.
constexpr int SNAP_WORDS = 32;
static_assert(offsetof(Ctl, rem_count) == 0 && offsetof(Ctl, changed_count) + 4 <= 4 * SNAP_WORDS,
              "step-boundary counters must fit the snapshot");
struct Snap {
    int32_t v;  // word lane() of the control block (lanes >= SNAP_WORDS: 0)
};
// Every lane of the wave must call it.
__device__ __forceinline__ Snap take_snap(const Ctl *c) {
    const int32_t *w = reinterpret_cast<const int32_t *>(c);
    return Snap{lane() < SNAP_WORDS ? ld_rlx(w + lane()) : 0};
}
// The snapshot's value of field f (a word of the first 128 bytes of *c).
// It reads another lane's register: every lane of the wave must call it.
__device__ __forceinline__ int32_t snap_word(const Snap &s, const Ctl *c, const int32_t *f) {
    return __shfl(s.v, (int)(f - reinterpret_cast<const int32_t *>(c)));
}
__device__ __forceinline__ int32_t sqlen(const Snap &s, const Ctl *c, const int32_t *tail, int32_t cap) {
    const int32_t n = snap_word(s, c, tail);
    return n < cap ? n : cap;
}

// Debug log entry (a, b, c) for every active lane with pred set (one
// atomic per wave).
__device__ __forceinline__ void dbg_put(int32_t *buf, unsigned long long *cnt, int64_t cap, bool pred, int32_t x,
                                        int32_t y, int32_t z) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane() == leader) base = atomicAdd(cnt, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    if (pred) {
        const unsigned long long pos = base + (unsigned long long)__popcll(m & ((1ull << lane()) - 1ull));
        if (pos < (unsigned long long)cap) {
            buf[3 * pos] = x;
            buf[3 * pos + 1] = y;
            buf[3 * pos + 2] = z;
        }
    }
}

// Count the active lanes with pred set into *ctr (one atomic per wave).
__device__ __forceinline__ void count_agg(int32_t *ctr, bool pred) {
    unsigned long long m = __ballot(pred);
    unsigned long long act = __ballot(1);
    if (m && lane() == __ffsll((long long)act) - 1) atomicAdd(ctr, __popcll(m));
}

// ===========================================================================
// Batch validation (boundary convention; simple graph, Section III)
// ===========================================================================

// V1: range / dead / self-loop checks, canonical (min, max), hash insert
// (the smallest item index of each pair wins the slot).
__device__ __forceinline__ void val_canon(const KArgs &a, const BatchCtx &bc, const Team &T) {
    const int32_t n = bc.n_ids;
    const uint32_t mask = (uint32_t)bc.hcap - 1u;
    for (int32_t i = T.rank; i < bc.s; i += T.size) {
        int32_t u = bc.src[i], v = bc.dst[i];
        int32_t e = 0;
        if (u < 0 || v < 0 || u >= n || v >= n) e = ST_RANGE;
        else if (a.g.core[u] < 0 || a.g.core[v] < 0) e = ST_DEAD;
        else if (u == v) e = ST_SELF;
        int32_t lo = u < v ? u : v, hi = u < v ? v : u;
        a.b.eu[i] = lo;
        a.b.ev[i] = hi;
        a.b.su[i] = -1;
        a.b.sv[i] = -1;
        a.b.err[i] = e;
        a.b.hslot[i] = -1;
        if (e == 0) {
            unsigned long long key = edge_key(lo, hi);
            uint32_t h = hash_key(key) & mask;
            for (uint32_t probe = 0; probe <= mask; ++probe) {
                unsigned long long old = atomicCAS(&a.b.hkey[h], EMPTY_KEY, key);
                if (old == EMPTY_KEY || old == key) break;
                h = (h + 1u) & mask;
            }
            a.b.hslot[i] = (int32_t)h;
            atomicMin(&a.b.hval[h], i);
        }
    }
}

// Queue the lists of x (one per lane, x < 0 for none) for the locate scan,
// once per batch: the first lane to stamp x adds its chunk items.  Called
// by every lane of the wave; one tail atomic per wave.
__device__ __forceinline__ void mark_scan(const KArgs &a, const BatchCtx &bc, int32_t x) {
    int nch = 0;
    if (x >= 0 && atomicExch(&a.g.bmark[x], bc.bstamp) != bc.bstamp) nch = nchunks(a.g.len[x], a.t.chunk);
    const int base = reserve_agg(&a.ctl->scan_tail, nch);
    for (int c = 0; c < nch; ++c) {
        if (base + c < a.b.scap) a.b.scanq[base + c] = chunk_item(x, c);
        else atomicOr(&a.ctl->overflow, 1);
    }
}

// Lists up to this length are searched by the item itself (one or two
// cache lines); longer ones are read once by the locate scan, every entry
// probing the batch hash.
constexpr int32_t VAL_SHORT = 32;

// Absolute slot of `target` in x's list, or -1.  Eight entries are loaded
// per step before any is compared, so a lane has eight reads in flight.
__device__ __forceinline__ int64_t find_in_list(const DevGraph &g, int32_t x, int32_t target) {
    const int64_t o = g.off[x];
    const int32_t L = g.len[x];
    const int32_t *p = g.nbr + o;
    for (int32_t s = 0; s < L; s += 8) {
        int32_t e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = s + u < L ? p[s + u] : -1;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e[u] == target) return o + s + u;
    }
    return -1;
}

// V2: duplicates inside the batch; locate the valid items (insertion: the
// shorter endpoint list is enough to test existence; deletion: both lists,
// to find both slots).  A short list is searched by the item; a long one is
// queued for the locate scan.  Waves stride the batch together so that
// mark_scan is called by whole waves.
__device__ __forceinline__ void val_dup_mark(const KArgs &a, const BatchCtx &bc, const Team &T) {
    for (int32_t w0 = T.rank - lane(); w0 < bc.s; w0 += T.size) {
        const int32_t i = w0 + lane();
        int32_t x = -1, y = -1;
        if (i < bc.s && a.b.err[i] == 0) {
            if (a.b.hval[a.b.hslot[i]] != i) {
                a.b.err[i] = ST_DUP;
            } else {
                const int32_t u = a.b.eu[i], v = a.b.ev[i];
                const int32_t lu = a.g.len[u], lv = a.g.len[v];
                if (bc.inserting) {
                    const int32_t p = lu <= lv ? u : v, q = lu <= lv ? v : u;
                    if ((lu <= lv ? lu : lv) <= VAL_SHORT) {
                        if (find_in_list(a.g, p, q) >= 0) a.b.err[i] = ST_EXISTS;
                    } else {
                        x = p;
                    }
                } else {
                    if (lu <= VAL_SHORT) a.b.su[i] = find_in_list(a.g, u, v);
                    else x = u;
                    if (lv <= VAL_SHORT) a.b.sv[i] = find_in_list(a.g, v, u);
                    else y = v;
                }
            }
        }
        mark_scan(a, bc, x);
        if (!bc.inserting) mark_scan(a, bc, y);
    }
}

// V3: locate scan.  Each (vertex, chunk) item is read by one wave; every
// live neighbour probes the batch hash.  Insertion: a hit means the edge
// exists.  Deletion: a hit records the slot of the entry.  A wave loads
// SCAN_STEPS steps of its chunk, then sends their first probes, before it
// resolves any, and loads its next item with this one's length and offset.
constexpr int SCAN_STEPS = 4;
__device__ __forceinline__ void val_scan(const KArgs &a, const BatchCtx &bc, const Team &T) {
    const uint32_t mask = (uint32_t)bc.hcap - 1u;
    const int32_t n = qlen(&a.ctl->scan_tail, a.b.scap);
    const int32_t chunk = a.t.chunk;
    int32_t j = T.wave();
    if (j >= n) return;  // uniform over the wave
    int64_t item = a.b.scanq[j];
    while (j < n) {
        const int32_t jn = j + T.nwaves();
        // the next item, the length and the offset are loaded together: the
        // next item's load is unconditional (its index stays in range) and
        // the item's walk is a do-while, so that no branch puts a wait
        // between them
        const int64_t next = a.b.scanq[jn < n ? jn : j];
        const int32_t x = item_v(item);
        const int32_t L = a.g.len[x];
        const int64_t base = a.g.off[x];
        const int32_t lo = item_c(item) * chunk;
        const int32_t hi = lo + chunk < L ? lo + chunk : L;
        const int32_t *p = a.g.nbr + base;
        // every item holds slots (lo < hi); were one empty, its loads would
        // all be masked off
        int32_t s0 = lo;
        do {
            int32_t w[SCAN_STEPS];
            unsigned long long k2[SCAN_STEPS];
            uint32_t h[SCAN_STEPS];
#pragma unroll
            for (int u = 0; u < SCAN_STEPS; ++u) {
                const int32_t i = s0 + u * WAVE + lane();
                w[u] = i < hi ? p[i] : -1;
            }
#pragma unroll
            for (int u = 0; u < SCAN_STEPS; ++u) {
                h[u] = hash_key(edge_key(x, w[u])) & mask;
                k2[u] = w[u] >= 0 ? a.b.hkey[h[u]] : EMPTY_KEY;
            }
#pragma unroll
            for (int u = 0; u < SCAN_STEPS; ++u) {
                const unsigned long long key = edge_key(x, w[u]);
                uint32_t hh = h[u];
                unsigned long long kk = k2[u];
                for (uint32_t probe = 0; probe <= mask && kk != EMPTY_KEY; ++probe) {
                    if (kk == key) {
                        const int32_t i = a.b.hval[hh];
                        const int64_t slot = base + s0 + u * WAVE + lane();
                        if (bc.inserting) a.b.err[i] = ST_EXISTS;
                        else if (x == a.b.eu[i]) a.b.su[i] = slot;
                        else a.b.sv[i] = slot;
                        break;
                    }
                    hh = (hh + 1u) & mask;
                    kk = a.b.hkey[hh];
                }
            }
            s0 += SCAN_STEPS * WAVE;
        } while (s0 < hi);
        j = jn;
        item = next;
    }
}

// V4: missing edges, smallest invalid index, emit valid item indices into
// the remaining list `cur`.  For packed independent batches the smallest
// invalid item is kept per sub-batch and the emission waits for V5.
__device__ __forceinline__ void val_final(const KArgs &a, const BatchCtx &bc, const Team &T) {
    for (int32_t i = T.rank; i < bc.s; i += T.size) {
        int32_t e = a.b.err[i];
        if (!bc.inserting && e == 0 && (a.b.su[i] < 0 || a.b.sv[i] < 0)) {
            e = ST_MISSING;
            a.b.err[i] = e;
        }
        if (e != 0) {
            atomicMin(&a.ctl->first_bad, i);
            if (bc.sub)
                atomicMin(&bc.sub_bad[bc.sub[i]], ((unsigned long long)i << 8) | (unsigned long long)(-e));
        }
        push_agg<int32_t>(a.b.rem[bc.cur], a.b.cap, &a.ctl->rem_count[bc.cur], i, e == 0 && !bc.sub,
                          &a.ctl->overflow);
    }
}

// V5 (packed batches): emit the valid items; in strict mode a sub-batch with
// an invalid item is dropped whole, the others go on.
__device__ __forceinline__ void val_subfilter(const KArgs &a, const BatchCtx &bc, const Team &T) {
    for (int32_t i = T.rank; i < bc.s; i += T.size) {
        bool ok = a.b.err[i] == 0 && !(bc.strict && bc.sub_bad[bc.sub[i]] != ~0ull);
        push_agg<int32_t>(a.b.rem[bc.cur], a.b.cap, &a.ctl->rem_count[bc.cur], i, ok, &a.ctl->overflow);
    }
}

// ===========================================================================
// Capacity reservation before an insertion batch mutates anything, and
// tombstone compaction after a deletion batch.
// ===========================================================================

__device__ __forceinline__ void mark_endpoint(const KArgs &a, const BatchCtx &bc, int32_t x) {
    atomicAdd(&a.g.gain[x], 1);
    bool first = atomicExch(&a.g.bmark[x], bc.bstamp + 1) != bc.bstamp + 1;
    push_agg<int32_t>(a.b.vlist, a.g.n_cap, &a.ctl->vlist_count, x, first, &a.ctl->overflow);
}

// R1: per-vertex count of batch edges (gain) and the distinct endpoints.
__device__ __forceinline__ void res_gain(const KArgs &a, const BatchCtx &bc, const Team &T) {
    const int32_t n = qlen(&a.ctl->rem_count[bc.cur], a.b.cap);
    const int32_t *R = a.b.rem[bc.cur];
    for (int32_t idx = T.rank; idx < n; idx += T.size) {
        int32_t i = R[idx];
        mark_endpoint(a, bc, a.b.eu[i]);
        mark_endpoint(a, bc, a.b.ev[i]);
    }
}

// R2: a list that cannot take its gain moves to a spill block at the pool tail.
__device__ __forceinline__ void res_alloc(const KArgs &a, const Team &T) {
    const int32_t n = qlen(&a.ctl->vlist_count, a.g.n_cap);
    for (int32_t j = T.rank; j < n; j += T.size) {
        int32_t x = a.b.vlist[j];
        int32_t need = a.g.len[x] + a.g.gain[x];
        a.g.gain[x] = 0;
        if (need > a.g.cap[x]) {
            int32_t nc = need + (need >> 3 > 4 ? need >> 3 : 4);
            nc = (nc + 3) & ~3;
            unsigned long long pos = atomicAdd(&a.ctl->pool_tail, (unsigned long long)nc);
            if (pos + (unsigned long long)nc > (unsigned long long)a.g.pool_size) {
                atomicOr(&a.ctl->pool_fail, 1);
            } else {
                int32_t r = atomicAdd(&a.ctl->reloc_count, 1);
                a.b.reloc[r] = x;
                a.b.reloc_off[r] = (int64_t)pos;
                a.b.reloc_cap[r] = nc;
            }
        }
    }
}

// R3: copy relocated lists (one wave per list).
__device__ __forceinline__ void res_copy(const KArgs &a, const Team &T) {
    const int32_t n = qlen(&a.ctl->reloc_count, a.g.n_cap);
    for (int32_t j = T.wave(); j < n; j += T.nwaves()) {
        int32_t x = a.b.reloc[j];
        int32_t L = a.g.len[x];
        const int32_t *src = a.g.nbr + a.g.off[x];
        int32_t *dst = a.g.nbr + a.b.reloc_off[j];
        for (int32_t s = lane(); s < L; s += WAVE) dst[s] = src[s];
        if (lane() == 0) {
            atomicAdd(&a.ctl->garbage, (unsigned long long)a.g.cap[x]);
            a.g.off[x] = a.b.reloc_off[j];
            a.g.cap[x] = a.b.reloc_cap[j];
            if (a.t.uplists) a.g.ubl[x] = -1;  // the up-list stayed at the old slots
        }
    }
}

// After a deletion batch: squeeze tombstones out of the touched lists whose
// tombstone share is large (one wave per list, in place, order kept).
__device__ __forceinline__ void del_compact(const KArgs &a, const Team &T) {
    const int32_t n = qlen(&a.ctl->vlist_count, a.g.n_cap);
    for (int32_t j = T.wave(); j < n; j += T.nwaves()) {
        int32_t x = a.b.vlist[j];
        int32_t L = a.g.len[x];
        int32_t T = a.g.gain[x];
        if (lane() == 0) a.g.gain[x] = 0;
        if (!(T * 8 >= L || L <= 1024)) continue;
        int32_t *p = a.g.nbr + a.g.off[x];
        int32_t wpos = 0;
        for (int32_t s = 0; s < L; s += WAVE) {
            int32_t i = s + lane();
            int32_t w = i < L ? p[i] : -1;
            unsigned long long m = __ballot(w >= 0);
            int rank = __popcll(m & ((1ull << lane()) - 1ull));
            if (w >= 0) p[wpos + rank] = w;
            wpos += __popcll(m);
        }
        if (lane() == 0) a.g.len[x] = wpos;
    }
}


// ===========================================================================
// One iteration = one superior edge set (the loop body of Algorithms 1 and 5)
//
// An iteration is a sequence of steps: selection claim / select rounds,
// apply, cascade rounds (expansion and eviction for insertion, peel for
// deletion), core update, SD maintenance.  Every step is a team-strided
// loop; the driver runs a step on the whole grid (then a grid barrier) or,
// when it is small, inside workgroup 0 alone (then a workgroup barrier),
// continuing locally until a large step comes up.  All decisions read
// counters that were published before the last barrier, so every workgroup
// takes the same path.
// ===========================================================================

// Vertex-star iterations (see the star section below): mode 0 = ordinary
// edge iterations, 1 = insertion stars, 2 = deletion stars.
struct StarCtx {
    int32_t mode;
    int32_t v0, nv;          // insertion: new ids [v0, v0 + nv)
    int32_t s;               // insertion: batch items
    const int32_t *src;      // insertion: raw items, src = new id (runs in id order)
    const int32_t *dst;
    int32_t ng;              // deletion: gathered edges
    const int32_t *firstidx; // deletion: != INT_MAX for the ids being deleted
};

struct Iter {
    int32_t ep;    // iteration stamp
    int32_t cur;   // remaining list read by this iteration (edges, or pending stars)
    int32_t n_r;   // its length
    int32_t ins;   // 1 = insertion batch, 0 = deletion batch
    StarCtx sc;
    Snap sn;       // control counters as the last step left them
};

enum StepKind : int32_t { S_CLAIM = 0, S_SELECT, S_APPLY, S_EXPAND, S_EVICT, S_PEEL, S_CORE, S_MCD, S_DONE };

struct PC {
    int32_t step;
    int32_t r;
};


// ===========================================================================
// Asynchronous traversal steps.
//
// The expansion, eviction and peel cascades are closures: every vertex is
// claimed, evicted or peeled exactly once through an atomic (stamp exchange,
// counter crossing), so their result does not depend on the order in which
// vertices are processed.  Instead of one grid barrier per frontier round,
// an asynchronous step runs a whole cascade through one work queue: waves
// take slots from the queue head, wait for the producer to fill them, process
// the items and push the items they create.  A counter of items pushed but
// not finished (incremented before an item becomes visible, decremented after
// its children were pushed) reaching zero ends the step for every wave.
// State that waves exchange inside the step goes through agent-scope
// atomics, or through stores that complete (wave drain) before the item
// that announces them is published.  Queue 0 carries expansion items, queue
// 1 eviction / peel items (seeded by the step before).
// ===========================================================================
constexpr unsigned long long AQ_EMPTY = ~0ull;
enum AqType : int { AQ_V = 0, AQ_CNT = 1, AQ_EXP = 2, AQ_CH = 3 };

__device__ __forceinline__ unsigned long long aq_item(int type, int32_t v, int32_t c) {
    return ((unsigned long long)type << 62) | ((unsigned long long)((uint32_t)c & 0x3FFFFFFFu) << 32) |
           (unsigned long long)(uint32_t)v;
}
__device__ __forceinline__ int aq_type(unsigned long long it) { return (int)(it >> 62); }
__device__ __forceinline__ int32_t aq_v(unsigned long long it) { return (int32_t)(uint32_t)it; }
__device__ __forceinline__ int32_t aq_c(unsigned long long it) { return (int32_t)((it >> 32) & 0x3FFFFFFFu); }

// Wave-aggregated push of one item per lane with pred into queue qi.
__device__ __forceinline__ void apush(const KArgs &a, int qi, unsigned long long item, bool pred) {
    Ctl *c = a.ctl;
    wave_drain();  // stores this item announces (counter resets) are complete first
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return;
    const int leader = __ffsll((long long)m) - 1;
    const int cnt = __popcll(m);
    const int rank = __popcll(m & ((1ull << lane()) - 1ull));
    int32_t base = 0;
    if (lane() == leader) {
        atomicAdd(&c->aq_pend[qi], cnt);
        base = atomicAdd(&c->aq_tail[qi], cnt);
        wave_drain();  // the pending count is raised before any of the items is visible
    }
    base = __shfl(base, leader);
    if (pred) {
        const int32_t pos = base + rank;
        if (pos < a.q.acap) __hip_atomic_store(&a.q.aq[qi][pos], item, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else atomicOr(&c->overflow, 4);
    }
}

// Per-lane push of the nch chunk items of v (lanes with pred; any lanes).
__device__ __forceinline__ void apush_chunks(const KArgs &a, int qi, int type, int32_t v, int32_t nch, bool pred) {
    Ctl *c = a.ctl;
    wave_drain();
    int32_t base = 0;
    if (pred) {
        atomicAdd(&c->aq_pend[qi], nch);
        base = atomicAdd(&c->aq_tail[qi], nch);
    }
    wave_drain();
    if (pred) {
        for (int32_t q = 0; q < nch; ++q) {
            const int32_t pos = base + q;
            if (pos < a.q.acap)
                __hip_atomic_store(&a.q.aq[qi][pos], aq_item(type, v, q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else atomicOr(&c->overflow, 4);
        }
    }
}

// Route a vertex to queue qi: as one item, or as chunk items of `ctype` when
// its list is longer than large_deg.
__device__ __forceinline__ void apush_vertex(const KArgs &a, int qi, int ctype, int32_t w, bool pred) {
    const int32_t L = pred ? a.g.len[w] : 0;
    const bool big = pred && L > a.t.large_deg;
    apush(a, qi, aq_item(AQ_V, w, 0), pred && !big);
    if (__ballot(big)) apush_chunks(a, qi, ctype, w, nchunks(L, a.t.chunk), big);
}

// Run queue qi to exhaustion; proc(item, fresh) is called by the whole wave
// with the lanes holding a new item marked fresh.
template <class P>
__device__ __forceinline__ void aq_run(const KArgs &a, int qi, P &&proc) {
    Ctl *c = a.ctl;
    unsigned long long *Q = a.q.aq[qi];
    const int32_t cap = a.q.acap;
    constexpr int G = 16;
    unsigned polls = 0;
    unsigned long long t0 = 0;   // clock when the step last showed progress to this wave
    int32_t seen = -1;           // items handed out when last checked
    for (;;) {
        int32_t base = 0;
        if (lane() == 0) base = atomicAdd(&c->aq_head[qi], G);
        base = __shfl(base, 0);
        const int32_t idx = base + lane();
        bool waiting = lane() < G && idx < cap;
        bool done = false;
        while (__ballot(waiting) != 0ull || base >= cap) {
            unsigned long long item = AQ_EMPTY;
            bool fresh = false;
            if (waiting) {
                item = __hip_atomic_load(&Q[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (item != AQ_EMPTY) {
                    fresh = true;
                    waiting = false;
                    __hip_atomic_store(&Q[idx], AQ_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            const unsigned long long fm = __ballot(fresh);
            if (fm) {
                proc(item, fresh);
                wave_drain();  // children pushed (pending raised) before this item counts as done
                if (lane() == 0) atomicSub(&c->aq_pend[qi], __popcll(fm));
                polls = 0;
                t0 = 0;
                continue;
            }
            if (ld_rlx(&c->aq_pend[qi]) == 0 || bar_aborted(a.bar)) { done = true; break; }
            __builtin_amdgcn_s_sleep(1);
            if ((++polls & 1023u) == 0u) {
                // bounded: a wait longer than the barrier bound with no item
                // handed out anywhere is a lost item (a bug), not a hang
                const unsigned long long now = (unsigned long long)wall_clock64();
                const int32_t tail = ld_rlx(&c->aq_tail[qi]);
                if (tail != seen || t0 == 0) {
                    seen = tail;
                    t0 = now;
                } else if (now - t0 > __hip_atomic_load(&a.bar->wait_ticks[0], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)) {
                    if (lane() == 0)
                        __hip_atomic_store(&a.bar->abort[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    done = true;
                    break;
                }
            }
        }
        if (done) break;
        if (ld_rlx(&c->aq_pend[qi]) == 0) break;
    }
}

// Selection of a superior edge set from the remaining edges (Algorithms 1-2
// and 5; Definition of the k-superior edge set).  An edge <u,v> has core
// number k = min(core u, core v); the endpoints with core k are its
// constrained endpoints.  Every constrained endpoint keeps at most one
// selected edge: each edge claims its constrained endpoints with a
// pseudo-random priority and is selected when it wins all of them (further
// claim rounds fill in edges whose endpoints are still free).  A vertex is
// constrained only at its own level, so one pass builds the union of all
// k-superior edge sets.
__device__ __forceinline__ void part_claim(const KArgs &a, const Iter &it, int r, const Team &T) {
    Ctl *c = a.ctl;
    if (r == 0 && T.lead()) {
        c->sel_count = 0;
        c->rem_count[it.cur ^ 1] = 0;
        for (int j = 0; j < 3; ++j) {
            c->fq_tail[j] = 0; c->fh_tail[j] = 0;
            c->eq_tail[j] = 0; c->eh_tail[j] = 0;
        }
        c->cand_count = 0; c->chg_count = 0; c->chh_count = 0;
        c->touched_count = 0; c->changed_count = 0;
        for (int j = 0; j < 2; ++j) { c->aq_tail[j] = 0; c->aq_head[j] = 0; c->aq_pend[j] = 0; }
        c->st_iters += 1;
        c->st_remaining += (unsigned long long)it.n_r;
    }
    const int32_t *R = a.b.rem[it.cur];
    const unsigned long long hi = claim_hi(it.ep, a.t.rounds, r);
    for (int32_t idx = T.rank; idx < it.n_r; idx += T.size) {
        int32_t i = R[idx];
        if (r > 0 && a.b.esel[i] == it.ep) continue;
        int32_t u = a.b.eu[i], v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        bool fu = cu == k, fv = cv == k;
        if (r > 0 && ((fu && matched_before(a.g.matched[u], it.ep, a.t.rounds, r)) ||
                      (fv && matched_before(a.g.matched[v], it.ep, a.t.rounds, r))))
            continue;
        unsigned long long key = hi | mix32((uint32_t)i);
        if (a.t.single_edge) {
            // keys fall with the iteration, so the complemented maximum needs no reset
            atomicMax(&a.ctl->one_key, ~key);
            continue;
        }
        if (fu) atomicMin(&a.g.claim[u], key);
        if (fv) atomicMin(&a.g.claim[v], key);
    }
}

// Apply one selected edge i (Algorithm 1 / 5, the set's insertion or
// deletion), called by the select step for its winners: list append or
// tombstones, SD of its constrained endpoints, roots.  A constrained endpoint keeps at most one selected edge, so its SD
// and root status depend on this edge alone.  Every lane may call it (sel
// selects the applying lanes; pushes are wave-aggregated).
__device__ __forceinline__ void apply_edge_insert(const KArgs &a, const Iter &it, int32_t i, bool sel) {
    Ctl *c = a.ctl;
    bool ru = false, rv = false;
    int32_t u = -1, v = -1;
    if (sel) {
        u = a.b.eu[i];
        v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        int32_t pu = atomicAdd(&a.g.len[u], 1);
        if (pu < a.g.cap[u]) a.g.nbr[a.g.off[u] + pu] = v;
        else atomicOr(&c->overflow, 2);
        int32_t pv = atomicAdd(&a.g.len[v], 1);
        if (pv < a.g.cap[v]) a.g.nbr[a.g.off[v] + pv] = u;
        else atomicOr(&c->overflow, 2);
        if (cu == k) {
            int32_t m = atomicAdd(&a.g.mcd[u], 1) + 1;
            if (m > k) { a.g.stamp[u] = it.ep; a.g.cd[u] = 0; if (a.t.sublists) a.g.slen[u] = 0; ru = true; }
        }
        if (cv == k) {
            int32_t m = atomicAdd(&a.g.mcd[v], 1) + 1;
            if (m > k) { a.g.stamp[v] = it.ep; a.g.cd[v] = 0; if (a.t.sublists) a.g.slen[v] = 0; rv = true; }
        }
    }
    // Roots enter the vertex queue whatever their length: other threads may
    // still be appending to the same list in this step, so a chunk count
    // taken now could be stale.  The first expansion round splits long root
    // lists into chunks once lengths are final.
    if (a.t.async_steps) {
        apush(a, 0, aq_item(AQ_V, u, 0), ru);
        apush(a, 0, aq_item(AQ_V, v, 0), rv);
    } else {
        push_agg<int32_t>(a.q.fq[0], a.q.vcap, &c->fq_tail[0], u, ru, &c->overflow);
        push_agg<int32_t>(a.q.fq[0], a.q.vcap, &c->fq_tail[0], v, rv, &c->overflow);
    }
}

__device__ __forceinline__ void apply_edge_delete(const KArgs &a, const Iter &it, int32_t i, bool sel) {
    Ctl *c = a.ctl;
    bool pu = false, pv = false;
    int32_t u = -1, v = -1;
    if (sel) {
        u = a.b.eu[i];
        v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        a.g.nbr[a.b.su[i]] = TOMB;
        a.g.nbr[a.b.sv[i]] = TOMB;
        if (a.t.uplists) {  // an up-list may hold the deleted neighbour
            a.g.ubl[u] = -1;
            a.g.ubl[v] = -1;
        }
        if (cu == k) {
            int32_t m = atomicSub(&a.g.mcd[u], 1) - 1;
            if (m < k) { a.g.stamp[u] = it.ep; pu = true; }
        }
        if (cv == k) {
            int32_t m = atomicSub(&a.g.mcd[v], 1) - 1;
            if (m < k) { a.g.stamp[v] = it.ep; pv = true; }
        }
    }
    if (a.t.async_steps) {
        apush_vertex(a, 1, AQ_CH, u, pu);
        apush_vertex(a, 1, AQ_CH, v, pv);
    } else {
        push_vertex(a, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], u, pu);
        push_vertex(a, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], v, pv);
    }
    push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, u, pu);
    push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, v, pv);
}

__device__ __forceinline__ void part_select(const KArgs &a, const Iter &it, int r, const Team &T) {
    Ctl *c = a.ctl;
    const bool last = r == a.t.rounds - 1;
    const int32_t *R = a.b.rem[it.cur];
    const unsigned long long hi = claim_hi(it.ep, a.t.rounds, r);
    const uint32_t mstamp = matched_stamp(it.ep, a.t.rounds, r);
    for (int32_t idx = T.rank; idx < it.n_r; idx += T.size) {
        int32_t i = R[idx];
        if (r > 0 && a.b.esel[i] == it.ep) continue;  // taken in an earlier round
        int32_t u = a.b.eu[i], v = a.b.ev[i];
        int32_t cu = a.g.core[u], cv = a.g.core[v];
        int32_t k = cu < cv ? cu : cv;
        bool fu = cu == k, fv = cv == k;
        bool part = !(r > 0 && ((fu && matched_before(a.g.matched[u], it.ep, a.t.rounds, r)) ||
                                (fv && matched_before(a.g.matched[v], it.ep, a.t.rounds, r))));
        unsigned long long key = hi | mix32((uint32_t)i);
        bool win = a.t.single_edge ? ld_rlx64(&a.ctl->one_key) == ~key
                                   : part && (!fu || a.g.claim[u] == key) && (!fv || a.g.claim[v] == key);
        if (win) {
            a.b.esel[i] = it.ep;
            if (fu) a.g.matched[u] = mstamp;
            if (fv) a.g.matched[v] = mstamp;
        }
        if (a.dl.sel) dbg_put(a.dl.sel, &a.dl.n[0], a.dl.cap, win, it.ep, u, v);
        // a winner applies itself in this step (no separate apply step)
        if (it.ins) apply_edge_insert(a, it, i, win);
        else apply_edge_delete(a, it, i, win);
        const unsigned long long wm = __ballot(win);
        if (wm && lane() == __ffsll((long long)__ballot(1)) - 1)
            atomicAdd(&c->st_selected, (unsigned long long)__popcll(wm));
        push_agg<int32_t>(a.b.rem[it.cur ^ 1], a.b.cap, &c->rem_count[it.cur ^ 1], i, last && !win,
                          &c->overflow);
    }
}

// Insert the selected set into G (Algorithm 1) and update SD of the
// constrained endpoints; a constrained endpoint whose new SD exceeds its core
// is a root of the traversal (a vertex with SD <= k cannot rise).
// Positive traversal (Algorithm 3) as level-synchronous rounds over all
// levels at once.  A visited vertex v gets cd[v] = CSD(v); if CSD(v) > k it
// visits its core-k neighbours w with SD(w) > k, otherwise it is queued for
// eviction (the lemma on CSD: CSD <= k keeps v out of the (k+1)-core).  A
// candidate's counter then counts exactly its higher-core neighbours plus its
// candidate neighbours at level k, so the later peel is exact whatever the
// visiting order.
__device__ __forceinline__ bool is_support(const DevGraph &g, int32_t w, int32_t k) {
    int32_t cw = g.core[w];
    return cw > k || (cw == k && g.mcd[w] > k);
}

// ===========================================================================
// Vertex stars: a vertex insertion or deletion in few iterations.
//
// A new vertex v enters with all its edges to existing vertices at once, its
// core pre-set to hK(v) = the h-index of its neighbours' current cores (the
// largest h with at least h neighbours of core >= h).  The core numbers of a
// graph satisfy core(x) = h-index of the neighbours' cores, and inserting v
// raises no other vertex by more than one, so hK(v) <= core'(v) <= hK(v) + 1;
// an existing neighbour w is constrained by v's edge when core(w) <= hK(v)
// (only then can v support its rise), and in one iteration every existing
// vertex takes at most one constraining edge (claims, as in the superior edge
// set partition).  Then every vertex moves by at most one and the usual
// expansion / eviction rounds find who rises: roots are the constrained
// neighbours whose SD exceeds their core and v itself when SD(v) > hK(v).
// Edges between two new vertices wait for an ordinary edge pass.
//
// A deleted vertex x leaves with all its remaining edges at once: a remaining
// neighbour w is constrained when core(w) <= core(x) (the edge's constrained
// endpoint in the deletion set sense) and takes at most one constraining
// edge per iteration; two deleted vertices that are adjacent never go in the
// same iteration.  x itself is dead afterwards, so its own core is not
// maintained; every other vertex drops by at most one and the usual peel
// rounds find who drops.
// ===========================================================================
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t *p, int32_t n, int32_t key) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (p[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long star_key(const Iter &it, const KArgs &a, uint32_t id) {
    return claim_hi(it.ep, a.t.rounds, 0) | mix32(id);
}
__device__ __forceinline__ uint32_t star_mstamp(const Iter &it, const KArgs &a) {
    return matched_stamp(it.ep, a.t.rounds, 0);
}

// Insertion star i: item j of [lo, hi) is an edge of v = v0 + i to an
// existing vertex when it is valid and its other end is not new.
__device__ __forceinline__ bool star_old_edge(const KArgs &a, const StarCtx &sc, int32_t j, int32_t &w) {
    w = sc.dst[j];
    return a.b.err[j] == 0 && !(w >= sc.v0 && w < sc.v0 + sc.nv);
}

// h-index of the current cores of star v's existing neighbours (wave-wide;
// every lane returns it).
__device__ __forceinline__ int32_t star_hindex(const KArgs &a, const StarCtx &sc, int32_t lo, int32_t hi,
                                               Acc &acc) {
    int32_t deg = 0;
    for (int32_t j = lo + lane(); j < hi; j += WAVE) {
        int32_t w;
        if (star_old_edge(a, sc, j, w)) ++deg;
    }
    deg = wave_sum(deg);
    int32_t l = 0, h = deg;
    while (l < h) {  // uniform across the wave
        const int32_t mid = (l + h + 1) >> 1;
        int32_t cnt = 0;
        for (int32_t j = lo + lane(); j < hi; j += WAVE) {
            int32_t w;
            if (star_old_edge(a, sc, j, w) && a.g.core[w] >= mid) ++cnt;
        }
        cnt = wave_sum(cnt);
        if (cnt >= mid) l = mid;
        else h = mid - 1;
    }
    if (lane() == 0) acc.scanned += (long long)(hi - lo);
    return l;
}

__device__ __forceinline__ void star_run(const StarCtx &sc, int32_t i, int32_t &lo, int32_t &hi) {
    lo = lower_bound_i32(sc.src, sc.s, sc.v0 + i);
    hi = lower_bound_i32(sc.src, sc.s, sc.v0 + i + 1);
}

// Pending deletion star x and its remaining neighbour w: w is claimed when
// it is itself a pending deleted vertex or constrained by the edge.
__device__ __forceinline__ bool star_del_claims(const KArgs &a, const StarCtx &sc, int32_t x, int32_t w) {
    return sc.firstidx[w] != 0x7fffffff || a.g.core[w] <= a.g.core[x];
}

__device__ __forceinline__ void star_claim(const KArgs &a, const Iter &it, const Team &T, Acc &acc) {
    Ctl *c = a.ctl;
    const StarCtx &sc = it.sc;
    if (T.lead()) {
        c->sel_count = 0;
        c->rem_count[it.cur ^ 1] = 0;
        for (int j = 0; j < 3; ++j) {
            c->fq_tail[j] = 0; c->fh_tail[j] = 0;
            c->eq_tail[j] = 0; c->eh_tail[j] = 0;
        }
        c->cand_count = 0; c->chg_count = 0; c->chh_count = 0;
        c->touched_count = 0; c->changed_count = 0;
        for (int j = 0; j < 2; ++j) { c->aq_tail[j] = 0; c->aq_head[j] = 0; c->aq_pend[j] = 0; }
        c->st_iters += 1;
        c->st_remaining += (unsigned long long)it.n_r;
    }
    const int32_t *R = a.b.rem[it.cur];
    for (int32_t idx = T.wave(); sc.mode == 1 && idx < it.n_r; idx += T.nwaves()) {
        const int32_t id = R[idx];
        const unsigned long long key = star_key(it, a, (uint32_t)id);
        {
            const int32_t v = sc.v0 + id;
            int32_t lo, hi;
            star_run(sc, id, lo, hi);
            const int32_t hk = star_hindex(a, sc, lo, hi, acc);
            if (lane() == 0) a.g.dec[v] = hk + 1;  // kept until the star is applied
            for (int32_t j = lo + lane(); j < hi; j += WAVE) {
                int32_t w;
                if (star_old_edge(a, sc, j, w) && a.g.core[w] <= hk) atomicMin(&a.g.claim[w], key);
            }
        }
    }
    if (sc.mode == 2) {
        // deletion stars: each claims itself, and every remaining gathered
        // edge claims, for each of its pending deleted ends o, the other end
        // when that is pending too or constrained by the edge
        for (int32_t idx = T.rank; idx < it.n_r; idx += T.size) {
            const int32_t x = R[idx];
            atomicMin(&a.g.claim[x], star_key(it, a, (uint32_t)x));
            a.g.cd[x] = 0;  // lost mark of this iteration (set by the select step)
        }
        for (int32_t i = T.rank; i < sc.ng; i += T.size) {
            if (a.b.err[i] != 0) continue;
            const int32_t u = a.b.eu[i], v = a.b.ev[i];
            if (sc.firstidx[u] != 0x7fffffff && star_del_claims(a, sc, u, v))
                atomicMin(&a.g.claim[v], star_key(it, a, (uint32_t)u));
            if (sc.firstidx[v] != 0x7fffffff && star_del_claims(a, sc, v, u))
                atomicMin(&a.g.claim[u], star_key(it, a, (uint32_t)v));
        }
        if (T.lead()) acc.scanned += sc.ng;
    }
}

__device__ __forceinline__ void star_select(const KArgs &a, const Iter &it, const Team &T) {
    Ctl *c = a.ctl;
    const StarCtx &sc = it.sc;
    const int32_t *R = a.b.rem[it.cur];
    const uint32_t mstamp = star_mstamp(it, a);
    if (sc.mode == 2) {
        // a deletion star that lost any of its claims is marked (cd is free
        // during deletion iterations); the decision is taken in the apply step
        for (int32_t idx = T.rank; idx < it.n_r; idx += T.size) {
            const int32_t x = R[idx];
            if (a.g.claim[x] != star_key(it, a, (uint32_t)x)) a.g.cd[x] = it.ep;
        }
        for (int32_t i = T.rank; i < sc.ng; i += T.size) {
            if (a.b.err[i] != 0) continue;
            const int32_t u = a.b.eu[i], v = a.b.ev[i];
            if (sc.firstidx[u] != 0x7fffffff && star_del_claims(a, sc, u, v) &&
                a.g.claim[v] != star_key(it, a, (uint32_t)u))
                a.g.cd[u] = it.ep;
            if (sc.firstidx[v] != 0x7fffffff && star_del_claims(a, sc, v, u) &&
                a.g.claim[u] != star_key(it, a, (uint32_t)v))
                a.g.cd[v] = it.ep;
        }
        return;
    }
    for (int32_t idx = T.wave(); idx < it.n_r; idx += T.nwaves()) {
        const int32_t id = R[idx];
        const unsigned long long key = star_key(it, a, (uint32_t)id);
        bool lost = false;
        const int32_t vtx = sc.v0 + id;
        const int32_t hk = a.g.dec[vtx] - 1;
        int32_t lo, hi;
        star_run(sc, id, lo, hi);
        for (int32_t j = lo + lane(); j < hi; j += WAVE) {
            int32_t w;
            if (star_old_edge(a, sc, j, w) && a.g.core[w] <= hk && a.g.claim[w] != key) lost = true;
        }
        const bool win = __ballot(lost) == 0ull;
        if (win && lane() == 0) a.g.matched[vtx] = (int32_t)mstamp;
        push_agg<int32_t>(a.b.sel, a.b.cap, &c->sel_count, id, win && lane() == 0, &c->overflow);
        push_agg<int32_t>(a.b.rem[it.cur ^ 1], a.b.cap, &c->rem_count[it.cur ^ 1], id, !win && lane() == 0,
                          &c->overflow);
    }
}

// Selected insertion stars enter with all their edges to existing vertices.
__device__ __forceinline__ void star_apply_insert(const KArgs &a, const Iter &it, const Team &T) {
    Ctl *c = a.ctl;
    const StarCtx &sc = it.sc;
    const DevGraph &g = a.g;
    const int32_t n = qlen(&c->sel_count, a.b.cap);
    for (int32_t idx = T.wave(); idx < n; idx += T.nwaves()) {
        const int32_t id = a.b.sel[idx];
        const int32_t v = sc.v0 + id;
        const int32_t hk = g.dec[v] - 1;
        int32_t lo, hi;
        star_run(sc, id, lo, hi);
        int32_t sd = 0, ne = 0;
        for (int32_t j0 = lo; j0 < hi; j0 += WAVE) {
            const int32_t j = j0 + lane();
            int32_t w = -1;
            const bool e = j < hi && star_old_edge(a, sc, j, w);
            bool root = false;
            if (e) {
                const int32_t cw = g.core[w];
                int32_t pv = atomicAdd(&g.len[v], 1);
                if (pv < g.cap[v]) g.nbr[g.off[v] + pv] = w;
                else atomicOr(&c->overflow, 2);
                int32_t pw = atomicAdd(&g.len[w], 1);
                if (pw < g.cap[w]) g.nbr[g.off[w] + pw] = v;
                else atomicOr(&c->overflow, 2);
                if (cw >= hk) ++sd;
                ++ne;
                if (cw <= hk) {  // constrained: v supports w's rise
                    int32_t m = atomicAdd(&g.mcd[w], 1) + 1;
                    if (m > cw) {
                        g.stamp[w] = it.ep;
                        g.cd[w] = 0;
                        if (a.t.sublists) g.slen[w] = 0;
                        root = true;
                    }
                }
            }
            if (a.t.async_steps) apush(a, 0, aq_item(AQ_V, w, 0), root);
            else push_agg<int32_t>(a.q.fq[0], a.q.vcap, &c->fq_tail[0], w, root, &c->overflow);
        }
        sd = wave_sum(sd);
        ne = wave_sum(ne);
        const bool rv = sd > hk;
        if (lane() == 0) {
            g.core[v] = hk;
            g.mcd[v] = sd;
            g.dec[v] = 0;
            if (rv) {
                g.stamp[v] = it.ep;
                g.cd[v] = 0;
                if (a.t.sublists) g.slen[v] = 0;
            }
            atomicAdd(&c->st_selected, (unsigned long long)ne);
        }
        if (a.t.async_steps) apush(a, 0, aq_item(AQ_V, v, 0), rv && lane() == 0);
        else push_agg<int32_t>(a.q.fq[0], a.q.vcap, &c->fq_tail[0], v, rv && lane() == 0, &c->overflow);
    }
}

// Selected deletion stars lose all their remaining edges (the gathered
// edges carry both slots; err[i] = 1 marks an edge already removed).
__device__ __forceinline__ void star_apply_delete(const KArgs &a, const Iter &it, const Team &T) {
    Ctl *c = a.ctl;
    const StarCtx &sc = it.sc;
    const DevGraph &g = a.g;
    const uint32_t mstamp = star_mstamp(it, a);
    // decide: a pending star that lost no claim leaves in this iteration
    // (always on the whole grid: star steps never run inside one workgroup)
    const int32_t *R = a.b.rem[it.cur];
    for (int32_t idx = T.rank; idx < it.n_r; idx += T.size) {
        const int32_t x = R[idx];
        const bool win = g.cd[x] != it.ep;
        if (win) g.matched[x] = mstamp;
        push_agg<int32_t>(a.b.sel, a.b.cap, &c->sel_count, x, win, &c->overflow);
        push_agg<int32_t>(a.b.rem[it.cur ^ 1], a.b.cap, &c->rem_count[it.cur ^ 1], x, !win, &c->overflow);
    }
    gbar(a.bar);
    int32_t ne = 0;
    for (int32_t i = T.rank; i < sc.ng; i += T.size) {
        bool pq = false;
        int32_t q = -1;
        if (a.b.err[i] == 0) {
            const int32_t u = a.b.eu[i], v = a.b.ev[i];
            const bool su = sc.firstidx[u] != 0x7fffffff && g.matched[u] == mstamp;
            const bool sv = sc.firstidx[v] != 0x7fffffff && g.matched[v] == mstamp;
            if (su || sv) {
                g.nbr[a.b.su[i]] = TOMB;
                g.nbr[a.b.sv[i]] = TOMB;
                a.b.err[i] = 1;
                ++ne;
                const int32_t x = su ? u : v;  // the leaving star (never both: they claim each other)
                q = su ? v : u;
                if (a.t.uplists) g.ubl[q] = -1;
                const int32_t cq = g.core[q], cx = g.core[x];
                if (cq <= cx) {
                    int32_t m = atomicSub(&g.mcd[q], 1) - 1;
                    if (m < cq) { g.stamp[q] = it.ep; pq = true; }
                }
            }
        }
        if (a.t.async_steps) apush_vertex(a, 1, AQ_CH, q, pq);
        else push_vertex(a, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], q, pq);
        push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, q, pq);
    }
    ne = wave_sum(ne);
    if (lane() == 0 && ne) atomicAdd(&c->st_selected, (unsigned long long)ne);
}

// Deletion stars of this iteration are dead once their edges are gone.
__device__ __forceinline__ void star_kill(const KArgs &a, const Iter &, const Team &T) {
    const int32_t n = qlen(&a.ctl->sel_count, a.b.cap);
    for (int32_t idx = T.rank; idx < n; idx += T.size) {
        const int32_t x = a.b.sel[idx];
        a.g.core[x] = -1;
        a.g.mcd[x] = 0;
        a.g.len[x] = 0;
    }
}

// Asynchronous expansion (Algorithm 3 closure) of the roots pushed into
// queue 0 by the apply step; evictions go to queue 1.
__device__ __forceinline__ void expand_async(const KArgs &a, const Iter &it, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int32_t ep = it.ep;
    ph_count(PH_ROUNDS);
    auto claim = [&](int32_t w, int32_t k) -> bool {
        if (w < 0) return false;
        if (g.core[w] != k || g.mcd[w] <= k) return false;
        if (ld_rlx(&g.stamp[w]) == ep) return false;
        if (atomicExch(&g.stamp[w], ep) == ep) return false;
        __hip_atomic_store(&g.cd[w], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    };
    auto expand_list = [&](int32_t v, int32_t lo, int32_t hi, int32_t k) {  // whole wave
        wave_walk(g, v, lo, hi, [&](int32_t w, int32_t) { apush_vertex(a, 0, AQ_CNT, w, claim(w, k)); });
    };
    aq_run(a, 0, [&](unsigned long long item, bool fresh) {
        const int type = aq_type(item);
        const int32_t v = aq_v(item);
        const int32_t L = fresh && type == AQ_V ? g.len[v] : 0;
        // short lists: one lane each
        const bool lanev = fresh && type == AQ_V && L <= a.t.small_deg;
        int32_t k = lanev ? g.core[v] : 0;
        int32_t pcd = 0;
        if (lanev) {
            const int32_t *p = g.nbr + g.off[v];
            for (int32_t s = 0; s < L; ++s) {
                int32_t w = p[s];
                if (w >= 0 && is_support(g, w, k)) ++pcd;
            }
            __hip_atomic_store(&g.cd[v], pcd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc.scanned += L;
        }
        push_agg<int32_t>(a.q.cand, a.q.vcap, &c->cand_count, v, lanev, &c->overflow);
        apush(a, 1, aq_item(AQ_V, v, 0), lanev && pcd <= k && L <= a.t.large_deg);
        if (__ballot(lanev && pcd <= k && L > a.t.large_deg))
            apush_chunks(a, 1, AQ_CH, v, nchunks(L, a.t.chunk), lanev && pcd <= k && L > a.t.large_deg);
        if (__ballot(lanev && pcd > k)) {
            // short lists that expand: each lane pushes its claimed neighbours
            int32_t s = 0;
            const int32_t *p = lanev ? g.nbr + g.off[v] : nullptr;
            while (__ballot(lanev && pcd > k && s < L)) {
                const bool act = lanev && pcd > k && s < L;
                const int32_t w = act ? p[s] : -1;
                apush_vertex(a, 0, AQ_CNT, w, act && claim(w, k));
                ++s;
            }
            if (lanev && pcd > k) acc.scanned += L;
        }
        // everything else: one wave per item
        unsigned long long m = __ballot(fresh && !lanev);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const unsigned long long itw = __shfl(item, src);
            const int tw = aq_type(itw);
            const int32_t x = aq_v(itw);
            const int32_t cx = aq_c(itw);
            const int32_t Lx = g.len[x];
            const int32_t kx = g.core[x];
            if (tw == AQ_V) {
                if (Lx > a.t.large_deg) {
                    // a long root list: its CSD is counted chunk by chunk
                    apush_chunks(a, 0, AQ_CNT, x, nchunks(Lx, a.t.chunk), lane() == 0);
                    continue;
                }
                int32_t part = 0;
                wave_walk(g, x, 0, Lx, [&](int32_t w, int32_t) {
                    if (w >= 0 && is_support(g, w, kx)) ++part;
                });
                part = wave_sum(part);
                if (lane() == 0) {
                    __hip_atomic_store(&g.cd[x], part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    acc.scanned += Lx;
                }
                push_agg<int32_t>(a.q.cand, a.q.vcap, &c->cand_count, x, lane() == 0, &c->overflow);
                if (part > kx) {
                    if (lane() == 0) acc.scanned += Lx;
                    expand_list(x, 0, Lx, kx);
                } else {
                    apush(a, 1, aq_item(AQ_V, x, 0), lane() == 0);
                }
            } else if (tw == AQ_CNT) {
                const int32_t lo = cx * a.t.chunk, hi = lo + a.t.chunk < Lx ? lo + a.t.chunk : Lx;
                const int32_t nch = nchunks(Lx, a.t.chunk);
                int32_t part = 0;
                wave_walk(g, x, lo, hi, [&](int32_t w, int32_t) {
                    if (w >= 0 && is_support(g, w, kx)) ++part;
                });
                part = wave_sum(part);
                int last = 0;
                if (lane() == 0) {
                    acc.scanned += hi - lo;
                    atomicAdd(&g.cd[x], part);
                    wave_drain();  // the partial sum lands before this chunk counts as done
                    last = atomicAdd(&g.done[x], 1) == nch - 1;
                }
                last = __shfl(last, 0);
                if (last) {
                    int32_t tot = 0;
                    if (lane() == 0) {
                        __hip_atomic_store(&g.done[x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        tot = __hip_atomic_load(&g.cd[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    tot = __shfl(tot, 0);
                    push_agg<int32_t>(a.q.cand, a.q.vcap, &c->cand_count, x, lane() == 0, &c->overflow);
                    if (tot > kx) apush_chunks(a, 0, AQ_EXP, x, nch, lane() == 0);
                    else apush_chunks(a, 1, AQ_CH, x, nch, lane() == 0);
                }
            } else {  // AQ_EXP: claim the neighbours in one chunk
                const int32_t lo = cx * a.t.chunk, hi = lo + a.t.chunk < Lx ? lo + a.t.chunk : Lx;
                if (lane() == 0) acc.scanned += hi - lo;
                expand_list(x, lo, hi, kx);
            }
        }
    });
}

// Asynchronous eviction (Algorithm 4 cascade) of the vertices in queue 1.
__device__ __forceinline__ void evict_async(const KArgs &a, const Iter &it, Acc &acc) {
    const DevGraph &g = a.g;
    const int32_t ep = it.ep;
    ph_count(PH_ROUNDS);
    auto hit = [&](int32_t w, int32_t k) -> bool {
        if (w < 0 || g.core[w] != k || ld_rlx(&g.stamp[w]) != ep) return false;
        // a counter already at or below k has crossed once: w is evicted
        if (ld_rlx(&g.cd[w]) <= k) return false;
        return atomicSub(&g.cd[w], 1) == k + 1;
    };
    aq_run(a, 1, [&](unsigned long long item, bool fresh) {
        const int type = aq_type(item);
        const int32_t x = aq_v(item);
        const int32_t L = fresh && type == AQ_V ? g.len[x] : 0;
        const bool lanev = fresh && type == AQ_V && L <= a.t.small_deg;
        const int32_t k = lanev ? g.core[x] : 0;
        {
            int32_t s = 0;
            const int32_t *p = lanev ? g.nbr + g.off[x] : nullptr;
            while (__ballot(lanev && s < L)) {
                const bool act = lanev && s < L;
                const int32_t w = act ? p[s] : -1;
                apush_vertex(a, 1, AQ_CH, w, act && hit(w, k));
                ++s;
            }
            if (lanev) acc.scanned += L;
        }
        unsigned long long m = __ballot(fresh && !lanev);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const unsigned long long itw = __shfl(item, src);
            const int32_t xv = aq_v(itw);
            const int32_t Lx = g.len[xv];
            const int32_t kx = g.core[xv];
            int32_t lo = 0, hi = Lx;
            if (aq_type(itw) == AQ_CH) {
                lo = aq_c(itw) * a.t.chunk;
                hi = lo + a.t.chunk < Lx ? lo + a.t.chunk : Lx;
            }
            if (lane() == 0) acc.scanned += hi - lo;
            wave_walk(g, xv, lo, hi, [&](int32_t w, int32_t) { apush_vertex(a, 1, AQ_CH, w, hit(w, kx)); });
        }
    });
}

// Asynchronous peel (Algorithms 6-7 cascade) of the roots in queue 1.
__device__ __forceinline__ void peel_async(const KArgs &a, const Iter &it, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int32_t ep = it.ep;
    ph_count(PH_ROUNDS);
    auto body = [&](int32_t w, int32_t k) {
        bool first = false, fire = false;
        if (w >= 0 && g.core[w] == k && ld_rlx(&g.stamp[w]) != ep) {
            int32_t old = atomicAdd(&g.dec[w], 1);
            first = old == 0;
            fire = g.mcd[w] - old - 1 == k - 1;
            if (fire) atomicExch(&g.stamp[w], ep);
        }
        push_agg<int32_t>(a.q.touched, a.q.vcap, &c->touched_count, w, first, &c->overflow);
        push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, w, fire);
        apush_vertex(a, 1, AQ_CH, w, fire);
    };
    aq_run(a, 1, [&](unsigned long long item, bool fresh) {
        const int type = aq_type(item);
        const int32_t x = aq_v(item);
        const int32_t L = fresh && type == AQ_V ? g.len[x] : 0;
        const bool lanev = fresh && type == AQ_V && L <= a.t.small_deg;
        const int32_t k = lanev ? g.core[x] : 0;
        {
            int32_t s = 0;
            const int32_t *p = lanev ? g.nbr + g.off[x] : nullptr;
            while (__ballot(lanev && s < L)) {
                const bool act = lanev && s < L;
                body(act ? p[s] : -1, k);
                ++s;
            }
            if (lanev) acc.scanned += L;
        }
        unsigned long long m = __ballot(fresh && !lanev);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const unsigned long long itw = __shfl(item, src);
            const int32_t xv = aq_v(itw);
            const int32_t Lx = g.len[xv];
            const int32_t kx = g.core[xv];
            int32_t lo = 0, hi = Lx;
            if (aq_type(itw) == AQ_CH) {
                lo = aq_c(itw) * a.t.chunk;
                hi = lo + a.t.chunk < Lx ? lo + a.t.chunk : Lx;
            }
            if (lane() == 0) acc.scanned += hi - lo;
            wave_walk(g, xv, lo, hi, [&](int32_t w, int32_t) { body(w, kx); });
        }
    });
}

// Positive traversal with Algorithm 3's pruning: a visited vertex first
// counts its CSD, and only a vertex whose CSD exceeds k visits (claims) its
// level-k neighbours w with SD(w) > k -- in the same step for a list walked
// by one wave, and in the next round (chunk items flagged CLAIM_CHUNK) for a
// long list whose CSD is summed over chunks.  The visited set is then the
// one Algorithm 3 defines: the roots plus everything reachable from them
// through vertices with CSD > k.  It still holds every riser (a riser has
// more than k supporters, so CSD > k, and each connected piece of risers
// contains a root), and every level-k neighbour counted by an expanding
// vertex is visited, so peeling it by "cd <= k" leaves exactly the risers.
// Supporter runs longer than one wave step are walked as items of one wave
// step each.  A wave of the flattened walk takes up to 64 runs, so longer
// runs could load one wave with far more than the others; and a hub's
// supporters sit in one run, so wider items would leave a few waves walking
// it step after step while the round waits.
__device__ __forceinline__ int32_t evict_large(const KArgs &a) {
    return a.t.large_deg < WAVE ? a.t.large_deg : WAVE;
}
__device__ __forceinline__ int32_t evict_chunk(const KArgs &a) { return a.t.chunk < WAVE ? a.t.chunk : WAVE; }

__device__ __forceinline__ void expand_round_pruned(const KArgs &a, const Iter &it, int r, const Team &T,
                                                    Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = r % 3, sn = (r + 1) % 3;
    const int bc = r & 1, bn = bc ^ 1;
    const int32_t nq = sqlen(it.sn, c, &c->fq_tail[sc], a.q.vcap);
    const int32_t nh = sqlen(it.sn, c, &c->fh_tail[sc], a.q.hcap);
    const int32_t ep = it.ep;
    auto support = [&](int32_t w, int32_t k) -> bool {
        if (w < 0) return false;
        const int32_t cw = g.core[w];
        return cw > k || (cw == k && g.mcd[w] > k);
    };
    // claim w for the visited set (level k, SD > k, not yet visited)
    auto claim = [&](int32_t w, int32_t k) -> bool {
        if (w < 0 || g.core[w] != k || g.mcd[w] <= k) return false;
        if (g.stamp[w] == ep || atomicExch(&g.stamp[w], ep) == ep) return false;
        g.cd[w] = 0;
        return true;
    };
    WaveBuf bq = wave_buf(0), be = wave_buf(1), bcand = wave_buf(2);
    auto push_next = [&](int32_t w, bool p) {
        push_vertex_wb(a, bq, a.q.fq[bn], &c->fq_tail[sn], a.q.fh[bn], &c->fh_tail[sn], w, p);
    };
    auto push_evict = [&](int32_t v, bool p) {
        push_vertex_wb(a, be, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], v, p);
    };
    auto push_cand = [&](int32_t v, bool p) {
        wb_push(bcand, a.q.cand, a.q.vcap, &c->cand_count, v, p, &c->overflow);
    };
    for_batches(T, a.q.fq[bc], nq, [&](int32_t v) {
        const int32_t L = v >= 0 ? g.len[v] : 0;
        const int32_t k = v >= 0 ? g.core[v] : 0;
        const bool big = L > a.t.large_deg;
        push_chunks(a, a.q.fh[bn], &c->fh_tail[sn], v, big ? nchunks(L, a.t.chunk) : 0);
        const bool live = v >= 0 && !big;
        int32_t pcd = 0;
        flat_walk(g, v, live ? L : 0, [&](int32_t j, int32_t w, unsigned long long own) {
            const bool sup = support(j >= 0 ? w : -1, __shfl(k, j < 0 ? 0 : j));
            pcd += __popcll(__ballot(sup) & own);
        });
        if (live) { g.cd[v] = pcd; acc.scanned += L; }
        push_cand(v, live);
        push_evict(v, live && pcd <= k);
        const bool grow = live && pcd > k;
        if (__ballot(grow)) {
            flat_walk(g, v, grow ? L : 0, [&](int32_t j, int32_t w, unsigned long long) {
                const int32_t kj = __shfl(k, j < 0 ? 0 : j);
                push_next(w, j >= 0 && claim(w, kj));
            });
            if (grow) acc.scanned += L;
        }
    });
    // chunk items: CSD partial sums (the last chunk decides), or the claim
    // pass of a long list whose CSD exceeded k
    for (int32_t jx = T.wave(); jx < nh; jx += T.nwaves()) {
        const int64_t item = a.q.fh[bc][jx];
        const int32_t v = item_v(item);
        const int32_t cf = item_c(item);
        const bool claim_pass = (cf & CLAIM_CHUNK) != 0;
        const int32_t ci = cf & ~CLAIM_CHUNK;
        const int32_t L = g.len[v];
        const int32_t k = g.core[v];
        const int32_t lo = ci * a.t.chunk, hi = lo + a.t.chunk < L ? lo + a.t.chunk : L;
        const int32_t nch = nchunks(L, a.t.chunk);
        if (lane() == 0) acc.scanned += hi - lo;
        if (claim_pass) {
            wave_walk(g, v, lo, hi, [&](int32_t w, int32_t) { push_next(w, claim(w, k)); });
            continue;
        }
        int32_t part = 0;
        wave_walk(g, v, lo, hi, [&](int32_t w, int32_t) { part += support(w, k) ? 1 : 0; });
        part = wave_sum(part);
        int last = 0;
        if (lane() == 0) {
            atomicAdd(&g.cd[v], part);
            wave_drain();  // the partial sum lands before this chunk counts as done
            last = atomicAdd(&g.done[v], 1) == nch - 1;
        }
        last = __shfl(last, 0);
        if (last) {
            int32_t tot = 0;
            if (lane() == 0) {
                g.done[v] = 0;
                tot = __hip_atomic_load(&g.cd[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            tot = __shfl(tot, 0);
            push_cand(v, lane() == 0);
            push_evict(v, lane() == 0 && tot <= k);
            if (tot > k && lane() == 0) {
                const int base = atomicAdd(&c->fh_tail[sn], nch);
                for (int q = 0; q < nch; ++q) {
                    if (base + q < a.q.hcap) a.q.fh[bn][base + q] = chunk_item(v, q | CLAIM_CHUNK);
                    else atomicOr(&c->overflow, 1);
                }
            }
        }
    }
    wb_flush(bq, a.q.fq[bn], a.q.vcap, &c->fq_tail[sn], &c->overflow);
    wb_flush(be, a.q.eq[0], a.q.vcap, &c->eq_tail[0], &c->overflow);
    wb_flush(bcand, a.q.cand, a.q.vcap, &c->cand_count, &c->overflow);
}

__device__ __forceinline__ void expand_round(const KArgs &a, const Iter &it, int r, const Team &T, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = r % 3, sn = (r + 1) % 3, sx = (r + 2) % 3;
    const int bc = r & 1, bn = bc ^ 1;
    const int32_t nq = sqlen(it.sn, c, &c->fq_tail[sc], a.q.vcap);
    const int32_t nh = sqlen(it.sn, c, &c->fh_tail[sc], a.q.hcap);
    if (T.lead()) {
        c->fq_tail[sx] = 0; c->fh_tail[sx] = 0;
        ph_count(PH_ROUNDS);
    }
    const int32_t ep = it.ep;

    // One pass per list: count CSD and claim every level-k neighbour w with
    // SD(w) > k on the way, before the vertex knows whether it expands.  The
    // visited set only grows, so it still holds every vertex that rises; a
    // vertex that does not expand (CSD <= k) is evicted at once, so the
    // neighbours it counted without visiting never matter; and an expanding
    // vertex has visited every level-k neighbour its CSD counted.  Peeling
    // the visited set therefore still leaves exactly the risers.
    // Returns whether w supports a level-k vertex; *cl = w newly claimed.
    // *lk = w is a level-k supporter (core k, SD > k): a candidate this
    // iteration, so the only kind of neighbour whose counter an eviction of
    // the scanned vertex lowers.
    auto csd_claim = [&](int32_t w, int32_t k, bool &cl, bool &lk, bool *up = nullptr) -> bool {
        cl = false;
        lk = false;
        if (w < 0) return false;
        const int32_t cw = g.core[w];
        if (up) *up = cw >= k;
        if (cw > k) return true;
        if (cw != k || g.mcd[w] <= k) return false;
        lk = true;
        // already claimed: skip the atomic.  A plain load may return an
        // older stamp (then the atomic decides), never a later one.
        if (g.stamp[w] != ep && atomicExch(&g.stamp[w], ep) != ep) {
            g.cd[w] = 0;
            if (a.t.sublists) g.slen[w] = 0;
            cl = true;
        }
        return true;
    };
    const bool sl = a.t.sublists != 0;
    WaveBuf bq = wave_buf(0), be = wave_buf(1), bcand = wave_buf(2);
    auto push_next = [&](int32_t w, bool p) {
        push_vertex_wb(a, bq, a.q.fq[bn], &c->fq_tail[sn], a.q.fh[bn], &c->fh_tail[sn], w, p);
    };
    // an evicted vertex's walk is its supporter run (sublists) or its list
    auto push_evict = [&](int32_t v, bool p, int32_t nsup) {
        push_vertex_wb_len(a, be, a.q.eq[0], &c->eq_tail[0], a.q.eh[0], &c->eh_tail[0], v,
                           p ? (sl ? nsup : g.len[v]) : 0, p, sl ? evict_large(a) : a.t.large_deg,
                           sl ? evict_chunk(a) : a.t.chunk);
    };
    auto push_cand = [&](int32_t v, bool p) {
        wb_push(bcand, a.q.cand, a.q.vcap, &c->cand_count, v, p, &c->overflow);
    };

    if (a.t.prune) {
        expand_round_pruned(a, it, r, T, acc);
        return;
    }
    // Lists of up to `large` slots: flattened walks of the wave's batch;
    // longer root lists are counted chunk by chunk next round.
    for_batches(T, a.q.fq[bc], nq, [&](int32_t v) {
        const int32_t L = v >= 0 ? g.len[v] : 0;
        const int32_t k = v >= 0 ? g.core[v] : 0;
        const bool big = L > a.t.large_deg;
        push_chunks(a, a.q.fh[bn], &c->fh_tail[sn], v, big ? nchunks(L, a.t.chunk) : 0);
        const bool live = v >= 0 && !big;
        int32_t pcd = 0, nlk = 0;  // CSD; supporters written to this lane's list
        flat_walk_pos(g.nbr, g, v, live ? L : 0,
                      [&](int32_t j, int32_t w, unsigned long long own, int64_t oj, int32_t lo) {
            bool cl, lk;
            const int32_t jj = j < 0 ? 0 : j;
            const bool sup = csd_claim(j >= 0 ? w : -1, __shfl(k, jj), cl, lk);
            pcd += __popcll(__ballot(sup) & own);
            if (sl) {
                // compacted after the owner's earlier supporters and those
                // of the lanes before this one that read the same list
                const unsigned long long lkm = __ballot(lk);
                const int32_t before = __shfl(nlk, jj);
                if (lk) g.sub[oj + before + __popcll(lkm & lanes_below() & ~((1ull << lo) - 1ull))] = w;
                nlk += __popcll(lkm & own);
            }
            push_next(w, cl);
        });
        if (live) {
            g.cd[v] = pcd;
            if (sl) g.slen[v] = nlk;
            acc.scanned += L;
        }
        push_cand(v, live);
        push_evict(v, live && pcd <= k, nlk);
    });

    // Long lists, chunk by chunk; the last chunk to finish has the CSD.
    const bool ul = a.t.uplists != 0;
    for_chunks(T, a.q.fh[bc], nh, g, a.t.chunk, [&](int32_t v, int32_t lo, int32_t hi, int32_t nch) {
        int32_t k = g.core[v];
        int32_t part = 0;
        const int64_t o = g.off[v];
        // every chunk of v reads the same ubl: it changes only when the last
        // chunk of v (all others finished) completes a build
        const int32_t ub = ul ? g.ubl[v] : -1;
        int32_t seen = 0;  // entries read (uniform)
        // the chunks of v append to one supporter run: slen[v] (zero since v
        // was claimed) hands out the slots.  A chunk collects its supporters
        // in the wave's LDS buffer and reserves them with one atomic at its
        // end; a chunk longer than the buffer reserves per step.
        constexpr int SUPBUF = 256;
        __shared__ int32_t lds_sup[COOP_THREADS / WAVE][SUPBUF];
        int32_t *sbuf = lds_sup[threadIdx.x / WAVE];
        const bool bufok = a.t.chunk <= SUPBUF;
        int32_t ns = 0;  // supporters held in sbuf (uniform)
        auto body = [&](int32_t w, bool *up) {
            bool cl, lk;
            if (csd_claim(w, k, cl, lk, up)) ++part;
            if (sl) {
                const unsigned long long lkm = __ballot(lk);
                if (lkm) {
                    if (bufok) {
                        if (lk) sbuf[ns + __popcll(lkm & lanes_below())] = w;
                        ns += __popcll(lkm);
                    } else {
                        int32_t b = 0;
                        if (lane() == 0) b = atomicAdd(&g.slen[v], __popcll(lkm));
                        b = __shfl(b, 0);
                        if (lk) g.sub[o + b + __popcll(lkm & lanes_below())] = w;
                    }
                }
            }
            push_next(w, cl);
        };
        if (ub >= 0) {
            seen = walk_chunk_up(g, v, lo, hi, ub, [&](int32_t w) { body(w, nullptr); });
        } else {
            // whole chunk; with up-lists on, write this chunk's up-list
            int32_t nup = 0;
            int32_t *uw = ul ? g.upl + o + lo : nullptr;
            seen = hi - lo;
            wave_walk(g, v, lo, hi, [&](int32_t w, int32_t) {
                bool up = false;
                body(w, &up);
                if (ul) {
                    const unsigned long long um = __ballot(up);
                    if (up) uw[nup + __popcll(um & lanes_below())] = w;
                    nup += __popcll(um);
                }
            });
            if (ul && nup < hi - lo && lane() == 0) uw[nup] = -1;
        }
        if (ns > 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // other lanes' LDS writes first
            int32_t b = 0;
            if (lane() == 0) b = atomicAdd(&g.slen[v], ns);
            b = __shfl(b, 0);
            for (int32_t i = lane(); i < ns; i += WAVE) g.sub[o + b + i] = sbuf[i];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // reads done before reuse
        }
        part = wave_sum(part);
        int last = 0;
        if (lane() == 0) {
            acc.scanned += seen;
            atomicAdd(&g.cd[v], part);
            wave_drain();  // the partial sum lands before this chunk counts as done
            last = atomicAdd(&g.done[v], 1) == nch - 1;
        }
        last = __shfl(last, 0);
        if (last) {
            int32_t tot = 0, nsup = 0;
            if (lane() == 0) {
                g.done[v] = 0;
                tot = __hip_atomic_load(&g.cd[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // every chunk added its supporters (and wrote its up-list)
                // before counting itself done
                if (sl) nsup = __hip_atomic_load(&g.slen[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (ul && ub < 0) g.ubl[v] = g.len[v];
            }
            tot = __shfl(tot, 0);
            nsup = __shfl(nsup, 0);
            push_cand(v, lane() == 0);
            push_evict(v, lane() == 0 && tot <= k, nsup);
        }
    });
    wb_flush(bq, a.q.fq[bn], a.q.vcap, &c->fq_tail[sn], &c->overflow);
    wb_flush(be, a.q.eq[0], a.q.vcap, &c->eq_tail[0], &c->overflow);
    wb_flush(bcand, a.q.cand, a.q.vcap, &c->cand_count, &c->overflow);
}

// Negative traversal (Algorithm 4) as rounds: an evicted candidate lowers the
// counter of each candidate neighbour at its level; a neighbour is evicted
// exactly once, when its counter crosses from k+1 to k.
__device__ __forceinline__ void evict_round(const KArgs &a, const Iter &it, int r, const Team &T, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = r % 3, sn = (r + 1) % 3, sx = (r + 2) % 3;
    const int bc = r & 1, bn = bc ^ 1;
    const int32_t nq = sqlen(it.sn, c, &c->eq_tail[sc], a.q.vcap);
    const int32_t nh = sqlen(it.sn, c, &c->eh_tail[sc], a.q.hcap);
    if (T.lead()) {
        c->eq_tail[sx] = 0; c->eh_tail[sx] = 0;
        ph_count(PH_ROUNDS);
    }
    const int32_t ep = it.ep;
    auto hit = [&](int32_t w, int32_t k) -> bool {
        if (w < 0 || g.core[w] != k || g.stamp[w] != ep) return false;
        // a counter already at or below k has crossed once: w is evicted.
        // Counters only fall during eviction, so a plain load, which may
        // return an older value, never skips a live counter.
        if (g.cd[w] <= k) return false;
        return atomicSub(&g.cd[w], 1) == k + 1;
    };
    WaveBuf bq = wave_buf(0);
    auto push_next = [&](int32_t w, bool p) {
        push_vertex_wb(a, bq, a.q.eq[bn], &c->eq_tail[sn], a.q.eh[bn], &c->eh_tail[sn], w, p);
    };
    if (a.t.sublists) {
        // Only the evicted vertex's supporter run: every entry is a level-k
        // candidate of this iteration (the expansion scanned the evicted
        // vertex, as every candidate, before the first eviction round), so
        // the counter decrement needs no core or stamp test.  A newly
        // evicted vertex is queued by the length of its run.
        auto hit_sup = [&](int32_t w, int32_t k) -> bool {
            if (w < 0 || g.cd[w] <= k) return false;
            return atomicSub(&g.cd[w], 1) == k + 1;
        };
        auto push_ev = [&](int32_t w, bool p) {
            push_vertex_wb_len(a, bq, a.q.eq[bn], &c->eq_tail[sn], a.q.eh[bn], &c->eh_tail[sn], w,
                               p ? g.slen[w] : 0, p, evict_large(a), evict_chunk(a));
        };
        for_batches(T, a.q.eq[bc], nq, [&](int32_t v) {
            int32_t L = v >= 0 ? g.slen[v] : 0;
            const int32_t len = v >= 0 ? g.len[v] : 0;
            L = L < len ? L : len;  // never past the list, even on a count left from another iteration
            const int32_t k = v >= 0 ? g.core[v] : 0;
            acc.scanned += L;
            flat_walk_pos(g.sub, g, v, L, [&](int32_t j, int32_t w, unsigned long long, int64_t, int32_t) {
                push_ev(w, hit_sup(w, __shfl(k, j < 0 ? 0 : j)));
            });
        });
        // long supporter runs, item by item
        const int32_t ech = evict_chunk(a);
        for (int32_t jx = T.wave(); jx < nh; jx += T.nwaves()) {
            const int64_t item = a.q.eh[bc][jx];
            const int32_t x = item_v(item);
            int32_t L = g.slen[x];
            const int32_t len = g.len[x];
            L = L < len ? L : len;
            const int32_t lo = item_c(item) * ech;
            const int32_t hi = lo + ech < L ? lo + ech : L;
            const int32_t k = g.core[x];
            const int32_t *sp = g.sub + g.off[x];
            if (lane() == 0 && hi > lo) acc.scanned += hi - lo;
            for (int32_t s = lo; s < hi; s += WAVE) {
                const int32_t i = s + lane();
                const int32_t w = i < hi ? sp[i] : -1;
                push_ev(w, hit_sup(w, k));
            }
        }
    } else {
        acc.scanned += for_vertex_slots(T, a.q.eq[bc], nq, g, a.t.large_deg,
                                    [&](int32_t w, int32_t k) { push_next(w, hit(w, k)); });
        for_chunks(T, a.q.eh[bc], nh, g, a.t.chunk, [&](int32_t x, int32_t lo, int32_t hi, int32_t) {
            int32_t k = g.core[x];
            if (lane() == 0) acc.scanned += hi - lo;
            wave_walk(g, x, lo, hi, [&](int32_t w, int32_t) { push_next(w, hit(w, k)); });
        });
    }
    wb_flush(bq, a.q.eq[bn], a.q.vcap, &c->eq_tail[sn], &c->overflow);
}

// Peel cascade of the deletion (Algorithms 6-7) as rounds.  A peeled vertex
// adds one to dec[w] of each core-k neighbour w not yet peeled; w's counter
// is cd = SD(w) - dec[w] (SD on G minus the set) and w is peeled exactly
// once, when cd crosses from k to k-1.  dec is cleared after the iteration
// through the `touched` list.
__device__ __forceinline__ void peel_round(const KArgs &a, const Iter &it, int r, const Team &T, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = r % 3, sn = (r + 1) % 3, sx = (r + 2) % 3;
    const int bc = r & 1, bn = bc ^ 1;
    const int32_t nq = sqlen(it.sn, c, &c->eq_tail[sc], a.q.vcap);
    const int32_t nh = sqlen(it.sn, c, &c->eh_tail[sc], a.q.hcap);
    if (T.lead()) {
        c->eq_tail[sx] = 0; c->eh_tail[sx] = 0;
        ph_count(PH_ROUNDS);
    }
    const int32_t ep = it.ep;
    WaveBuf bq = wave_buf(0), bt = wave_buf(1), bchg = wave_buf(2);
    // cw = core[w]: cores do not change during a peel round
    auto body_c = [&](int32_t w, int32_t cw, int32_t k) {
        bool first = false, fire = false;
        if (w >= 0 && cw == k && g.stamp[w] != ep) {
            int32_t old = atomicAdd(&g.dec[w], 1);
            first = old == 0;
            fire = g.mcd[w] - old - 1 == k - 1;
            if (fire) g.stamp[w] = ep;
        }
        wb_push(bt, a.q.touched, a.q.vcap, &c->touched_count, w, first, &c->overflow);
        push_vertex_wb(a, bq, a.q.eq[bn], &c->eq_tail[sn], a.q.eh[bn], &c->eh_tail[sn], w, fire);
        push_vertex_wb(a, bchg, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, w, fire);
    };
    auto body = [&](int32_t w, int32_t k) { body_c(w, w >= 0 ? g.core[w] : -1, k); };
    acc.scanned += for_vertex_slots(T, a.q.eq[bc], nq, g, a.t.large_deg, body);
    // a long list with a valid up-list is read through it: the neighbours at
    // the peeled vertex's core are all in its up-set
    for_chunks(T, a.q.eh[bc], nh, g, a.t.chunk, [&](int32_t x, int32_t lo, int32_t hi, int32_t) {
        int32_t k = g.core[x];
        const int32_t ub = a.t.uplists ? g.ubl[x] : -1;
        int32_t seen = hi - lo;
        if (ub >= 0) seen = walk_chunk_up(g, x, lo, hi, ub, [&](int32_t w) { body(w, k); });
        else wave_walk_pre(g, x, lo, hi, [&](int32_t w) { return g.core[w]; },
                           [&](int32_t w, int32_t cw) { body_c(w, cw, k); });
        if (lane() == 0) acc.scanned += seen;
    });
    wb_flush(bq, a.q.eq[bn], a.q.vcap, &c->eq_tail[sn], &c->overflow);
    wb_flush(bt, a.q.touched, a.q.vcap, &c->touched_count, &c->overflow);
    wb_flush(bchg, a.q.chg, a.q.vcap, &c->chg_count, &c->overflow);
}

// Core update (Algorithm 1: +1 for every surviving candidate; Algorithm 5:
// -1 for every peeled vertex).  SD of a moved vertex is rebuilt next step.
__device__ __forceinline__ void apply_core(const KArgs &a, const Iter &it, const Team &T, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    long long &cdeg = acc.cdeg, &edeg = acc.edeg, &hdeg = acc.hdeg;  // list entries of the method's sets
    if (it.ins) {
        const int32_t n = sqlen(it.sn, c, &c->cand_count, a.q.vcap);
        if (T.lead()) {
            c->st_candidates += (unsigned long long)n;
            c->st_icand += (unsigned long long)n;
        }
        for (int32_t idx = T.rank; idx < n; idx += T.size) {
            int32_t v = a.q.cand[idx];
            int32_t k = g.core[v];
            bool up = g.cd[v] > k;
            const int32_t L = g.len[v];
            cdeg += L;
            if (up) hdeg += L;
            else edeg += L;
            if (up) {
                g.core[v] = k + 1;
                g.chg[v] = it.ep;
                g.mcd[v] = 0;
            }
            if (a.dl.chg) dbg_put(a.dl.chg, &a.dl.n[1], a.dl.cap, up, it.ep, v, k + 1);
            count_agg(&c->changed_count, up);
            push_vertex(a, a.q.chg, &c->chg_count, a.q.chh, &c->chh_count, v, up);
        }
    } else {
        const int32_t n = sqlen(it.sn, c, &c->chg_count, a.q.vcap);
        const int32_t nt = sqlen(it.sn, c, &c->touched_count, a.q.vcap);
        if (T.lead()) {
            atomicAdd(&c->changed_count, n);
            c->st_candidates += (unsigned long long)nt;
        }
        for (int32_t idx = T.rank; idx < n; idx += T.size) {
            int32_t v = a.q.chg[idx];
            const int32_t nc = g.core[v] - 1;
            edeg += g.len[v];
            hdeg += g.len[v];
            g.core[v] = nc;
            g.chg[v] = it.ep;
            g.mcd[v] = 0;
            if (a.t.uplists) g.ubl[v] = -1;  // neighbours at the new core join the up-set
            if (a.dl.chg) dbg_put(a.dl.chg, &a.dl.n[1], a.dl.cap, true, it.ep, v, nc);
        }
        const int32_t nh = sqlen(it.sn, c, &c->chh_count, a.q.hcap);
        for (int32_t idx = T.rank; idx < nh; idx += T.size) {
            int64_t item = a.q.chh[idx];
            bool first = item_c(item) == 0;
            int32_t v = -1, nc = 0;
            if (first) {
                v = item_v(item);
                nc = g.core[v] - 1;
                edeg += g.len[v];
                hdeg += g.len[v];
                g.core[v] = nc;
                g.chg[v] = it.ep;
                g.mcd[v] = 0;
                if (a.t.uplists) g.ubl[v] = -1;
            }
            if (a.dl.chg) dbg_put(a.dl.chg, &a.dl.n[1], a.dl.cap, first, it.ep, v, nc);
            count_agg(&c->changed_count, first);
        }
        for (int32_t idx = T.rank; idx < nt; idx += T.size) g.dec[a.q.touched[idx]] = 0;
    }
}

// SD maintenance after the core update: a moved vertex recounts SD from its
// list; an unmoved neighbour w gains (insert) or loses (delete) one when the
// moved vertex crossed w's core.
__device__ __forceinline__ void mcd_phase(const KArgs &a, const Iter &it, const Team &T, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int32_t ep = it.ep;
    const bool ins = it.ins != 0;
    // snap_word reads another lane: every lane takes part
    const unsigned long long ch = (unsigned long long)snap_word(it.sn, c, &c->changed_count);
    const unsigned long long ncand = (unsigned long long)snap_word(it.sn, c, &c->cand_count);
    if (T.lead()) {
        c->st_changed += ch;
        c->st_evicted += ins ? ncand - ch : ch;
    }
    // Only a neighbour at the level the moved vertex crossed (its new core
    // on insertion, its new core + 1 on deletion) may need a delta, so the
    // moved-this-iteration stamp is gathered for those alone.
    auto nb_c = [&](int32_t w, int32_t cw, int32_t cv) -> int32_t {
        if (w < 0) return 0;
        if (cw == (ins ? cv : cv + 1) && g.chg[w] != ep) {
            if (ins) {
                atomicAdd(&g.mcd[w], 1);
                // the moved vertex rose to w's core: it joins w's up-set
                if (a.t.uplists) g.ubl[w] = -1;
            } else {
                atomicSub(&g.mcd[w], 1);
            }
        }
        return cw >= cv ? 1 : 0;
    };
    auto nb = [&](int32_t w, int32_t cv) -> int32_t { return w < 0 ? 0 : nb_c(w, g.core[w], cv); };
    const int32_t n = sqlen(it.sn, c, &c->chg_count, a.q.vcap);
    for_batches(T, a.q.chg, n, [&](int32_t v) {
        const int32_t L = v >= 0 ? g.len[v] : 0;
        const int32_t cv = v >= 0 ? g.core[v] : 0;
        const bool big = L > a.t.large_deg;
        int32_t cnt = 0;
        flat_walk(g, v, big ? 0 : L, [&](int32_t j, int32_t w, unsigned long long own) {
            cnt += __popcll(__ballot(nb(w, __shfl(cv, j < 0 ? 0 : j)) != 0) & own);
        });
        if (v >= 0 && !big) { g.mcd[v] = cnt; acc.scanned += L; }
        unsigned long long m = __ballot(big);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const int32_t vv = __shfl(v, src);
            const int32_t cvv = __shfl(cv, src);
            const int32_t LL = __shfl(L, src);
            int32_t tot = 0;
            wave_walk(g, vv, 0, LL, [&](int32_t w, int32_t) { tot += nb(w, cvv); });
            tot = wave_sum(tot);
            if (lane() == 0) { g.mcd[vv] = tot; acc.scanned += LL; }
        }
    });
    const int32_t nh = sqlen(it.sn, c, &c->chh_count, a.q.hcap);
    for_chunks(T, a.q.chh, nh, g, a.t.chunk, [&](int32_t v, int32_t lo, int32_t hi, int32_t) {
        int32_t cv = g.core[v];
        int32_t cnt = 0;
        // cores do not change during this step
        wave_walk_pre(g, v, lo, hi, [&](int32_t w) { return g.core[w]; },
                      [&](int32_t w, int32_t cw) { cnt += nb_c(w, cw, cv); });
        cnt = wave_sum(cnt);
        if (lane() == 0) { atomicAdd(&g.mcd[v], cnt); acc.scanned += hi - lo; }
    });
}

// ---------------------------------------------------------------------------
// Step machine
// ---------------------------------------------------------------------------

// Work of a frontier step in list entries: vertex items plus chunk items
// weighted by the chunk length relative to a typical list.
__device__ __forceinline__ int64_t frontier_work(const KArgs &a, int32_t nv, int32_t nchk) {
    return (int64_t)nv + (int64_t)nchk * (a.t.chunk / 16 + 1);
}

// Sum over the threads of one workgroup (every thread of it must call).
__device__ __forceinline__ long long block_sum64(long long v) {
    __shared__ long long red[COOP_THREADS / WAVE];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    long long t = 0;
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) t += red[i];
    __syncthreads();
    return t;
}

// List entries a frontier step would walk: the lengths of its vertex items
// plus a full chunk per chunk item (computed by one workgroup).
__device__ __forceinline__ long long queue_work(const KArgs &a, const Team &T, const int32_t *q, int32_t n,
                                                int32_t nchk, int walks, const int32_t *lens) {
    long long w = 0;
    for (int32_t i = T.rank; i < n; i += T.size) w += lens[q[i]];
    w = block_sum64(w) * walks;
    return w + (long long)nchk * a.t.chunk;
}

// Whether workgroup 0 may run this step by itself: its item count already
// passed step_is_local; here the list entries it would walk are checked.
__device__ __forceinline__ bool block_local_ok(const KArgs &a, const Iter &it, const PC &pc, const Team &T) {
    Ctl *c = a.ctl;
    const int s = pc.r % 3;
    long long w = 0;
    switch (pc.step) {
    case S_EXPAND:
        w = queue_work(a, T, a.q.fq[pc.r & 1], sqlen(it.sn, c, &c->fq_tail[s], a.q.vcap), sqlen(it.sn, c, &c->fh_tail[s], a.q.hcap), 1,
                       a.g.len);
        break;
    case S_EVICT:
    case S_PEEL:
        // an eviction walks supporter runs when they are kept
        w = queue_work(a, T, a.q.eq[pc.r & 1], sqlen(it.sn, c, &c->eq_tail[s], a.q.vcap), sqlen(it.sn, c, &c->eh_tail[s], a.q.hcap), 1,
                       pc.step == S_EVICT && a.t.sublists ? a.g.slen : a.g.len);
        break;
    case S_MCD:
        w = queue_work(a, T, a.q.chg, sqlen(it.sn, c, &c->chg_count, a.q.vcap), sqlen(it.sn, c, &c->chh_count, a.q.hcap), 1, a.g.len);
        break;
    default: return true;
    }
    return w <= a.t.local_work;
}

__device__ __forceinline__ int64_t step_work(const KArgs &a, const Iter &it, const PC &pc) {
    Ctl *c = a.ctl;
    const int s = pc.r % 3;
    switch (pc.step) {
    case S_CLAIM:
    case S_SELECT: return it.n_r;
    case S_APPLY: return sqlen(it.sn, c, &c->sel_count, a.b.cap);
    case S_EXPAND:
        return frontier_work(a, sqlen(it.sn, c, &c->fq_tail[s], a.q.vcap), sqlen(it.sn, c, &c->fh_tail[s], a.q.hcap));
    case S_EVICT:
    case S_PEEL: return frontier_work(a, sqlen(it.sn, c, &c->eq_tail[s], a.q.vcap), sqlen(it.sn, c, &c->eh_tail[s], a.q.hcap));
    case S_CORE:
        // a deletion's core step also clears the peel counters of every
        // touched vertex
        return it.ins ? sqlen(it.sn, c, &c->cand_count, a.q.vcap)
                      : (int64_t)sqlen(it.sn, c, &c->chg_count, a.q.vcap) + sqlen(it.sn, c, &c->chh_count, a.q.hcap) +
                            sqlen(it.sn, c, &c->touched_count, a.q.vcap);
    case S_MCD: return frontier_work(a, sqlen(it.sn, c, &c->chg_count, a.q.vcap), sqlen(it.sn, c, &c->chh_count, a.q.hcap));
    default: return 0;
    }
}

__device__ __forceinline__ bool step_is_local(const KArgs &a, const Iter &it, const PC &pc, int64_t work) {
    if (it.sc.mode && (pc.step <= S_APPLY || pc.step == S_CORE)) return false;
    if (a.t.async_steps && (pc.step == S_EXPAND || pc.step == S_EVICT || pc.step == S_PEEL)) return false;
    if (pc.step <= S_APPLY) return work <= a.t.local_edges;
    return work <= a.t.local_items;
}

__device__ __forceinline__ bool slot_empty_f(const KArgs &a, const Iter &it, int s) {
    Ctl *c = a.ctl;
    return snap_word(it.sn, c, &c->fq_tail[s]) + snap_word(it.sn, c, &c->fh_tail[s]) == 0;
}
__device__ __forceinline__ bool slot_empty_e(const KArgs &a, const Iter &it, int s) {
    Ctl *c = a.ctl;
    return snap_word(it.sn, c, &c->eq_tail[s]) + snap_word(it.sn, c, &c->eh_tail[s]) == 0;
}

// Step that follows pc (reads the counters pc's step published).
// First cascade step once the set is applied (roots queued).
__device__ __forceinline__ PC after_apply(const KArgs &a, const Iter &it) {
    if (a.t.async_steps) {
        if (it.ins && ld_rlx(&a.ctl->aq_tail[0]) > 0) return PC{S_EXPAND, 0};
        if (ld_rlx(&a.ctl->aq_tail[1]) == 0) return PC{S_CORE, 0};
        return it.ins ? PC{S_EVICT, 0} : PC{S_PEEL, 0};
    }
    if (it.ins) {
        if (!slot_empty_f(a, it, 0)) return PC{S_EXPAND, 0};
        return slot_empty_e(a, it, 0) ? PC{S_CORE, 0} : PC{S_EVICT, 0};
    }
    return slot_empty_e(a, it, 0) ? PC{S_CORE, 0} : PC{S_PEEL, 0};
}

__device__ __forceinline__ PC next_pc(const KArgs &a, const Iter &it, const PC &pc) {
    switch (pc.step) {
    case S_CLAIM: return PC{S_SELECT, pc.r};
    case S_SELECT:
        if (it.sc.mode) return PC{S_APPLY, 0};
        // edge sets: the select steps applied their winners
        return pc.r + 1 < a.t.rounds ? PC{S_CLAIM, pc.r + 1} : after_apply(a, it);
    case S_APPLY: return after_apply(a, it);
    case S_EXPAND:
        if (a.t.async_steps) return ld_rlx(&a.ctl->aq_tail[1]) > 0 ? PC{S_EVICT, 0} : PC{S_CORE, 0};
        if (!slot_empty_f(a, it, (pc.r + 1) % 3)) return PC{S_EXPAND, pc.r + 1};
        return slot_empty_e(a, it, 0) ? PC{S_CORE, 0} : PC{S_EVICT, 0};
    case S_EVICT:
        if (a.t.async_steps) return PC{S_CORE, 0};
        return slot_empty_e(a, it, (pc.r + 1) % 3) ? PC{S_CORE, 0} : PC{S_EVICT, pc.r + 1};
    case S_PEEL:
        if (a.t.async_steps) return PC{S_CORE, 0};
        return slot_empty_e(a, it, (pc.r + 1) % 3) ? PC{S_CORE, 0} : PC{S_PEEL, pc.r + 1};
    case S_CORE: return PC{S_MCD, 0};
    default: return PC{S_DONE, 0};
    }
}

__device__ __forceinline__ void run_step(const KArgs &a, const Iter &it, const PC &pc, const Team &T,
                                         Acc &acc) {
    switch (pc.step) {
    case S_CLAIM:
        if (it.sc.mode) star_claim(a, it, T, acc);
        else part_claim(a, it, pc.r, T);
        break;
    case S_SELECT:
        if (it.sc.mode) star_select(a, it, T);
        else part_select(a, it, pc.r, T);
        break;
    case S_APPLY:  // vertex stars only: edge sets apply inside the select step
        if (it.sc.mode == 1) star_apply_insert(a, it, T);
        else star_apply_delete(a, it, T);
        break;
    case S_EXPAND:
        if (a.t.async_steps) expand_async(a, it, acc);
        else expand_round(a, it, pc.r, T, acc);
        break;
    case S_EVICT:
        if (a.t.async_steps) evict_async(a, it, acc);
        else evict_round(a, it, pc.r, T, acc);
        break;
    case S_PEEL:
        if (a.t.async_steps) peel_async(a, it, acc);
        else peel_round(a, it, pc.r, T, acc);
        break;
    case S_CORE:
        apply_core(a, it, T, acc);
        if (it.sc.mode == 2) star_kill(a, it, T);
        break;
    case S_MCD: mcd_phase(a, it, T, acc); break;
    default: break;
    }
}

// Restart the iteration stamps (whole grid, at an iteration boundary, where
// no stamp is live): every array that holds one goes back to its cleared
// value, so stamps from 1 on are fresh again (the caller keeps the stamp's
// parity, which selects the remaining-edge list).
__device__ __forceinline__ void restamp(const KArgs &a) {
    const Team G = grid_team();
    const DevGraph &g = a.g;
    for (int32_t i = G.rank; i < g.n_cap; i += G.size) {
        g.claim[i] = ~0ull;
        g.matched[i] = 0u;
        g.stamp[i] = 0;
        g.chg[i] = 0;
        g.cd[i] = 0;
    }
    for (int32_t i = G.rank; i < a.b.cap; i += G.size) a.b.esel[i] = 0;
    if (G.lead()) a.ctl->one_key = 0ull;
    gbar(a.bar);
}

// Runs up to max_iters iterations of the current batch (each one superior
// edge set).  ep is the last iteration stamp used (in/out).  Returns the
// iterations run.  Workgroup 0 publishes the step where a local run stopped
// in one of two slots (alternating), so a slow workgroup still reading the
// previous publication is never overtaken.
__device__ __forceinline__ int run_iterations(const KArgs &a, int ins, int max_iters, int32_t &ep, Acc &acc,
                              int &pubs, const StarCtx &sc = StarCtx{}) {
    Ctl *c = a.ctl;
    int it_n = 0;
    for (; it_n < max_iters; ++it_n) {
        if (ep >= a.t.stamp_limit) {
            restamp(a);
            // restart at 0 or 1, keeping ep's parity: the iteration stamped
            // ep + 1 reads the remaining list rem[(ep + 1) & 1], where the
            // previous iteration (or the batch's validation) left the edges
            ep &= 1;
        }
        Iter it;
        it.ep = ep + 1;
        it.cur = it.ep & 1;
        it.sn = take_snap(c);
        it.n_r = sqlen(it.sn, c, &c->rem_count[it.cur], a.b.cap);
        it.ins = ins;
        it.sc = sc;
        if (it.n_r == 0 || bar_aborted(a.bar)) break;
        PC pc{S_CLAIM, 0};
        bool force = false;  // published by workgroup 0: run pc on the grid
        while (pc.step != S_DONE) {
            int64_t work = step_work(a, it, pc);
            if (force || !step_is_local(a, it, pc, work)) {
                force = false;
                const unsigned long long t0 = ph_start();
                run_step(a, it, pc, grid_team(), acc);
                ph_count(PH_GSTEPS);
                gbar(a.bar);
                it.sn = take_snap(c);
                ph_stop(c, pc.step, t0);
                pc = next_pc(a, it, pc);
            } else {
                const unsigned long long t0 = ph_start();
                const int slot = pubs & 1;
                if (blockIdx.x == 0) {
                    const Team T = block_team();
                    bool fg = false;
                    const unsigned long long tl = (unsigned long long)wall_clock64();
                    for (;;) {
                        if (!block_local_ok(a, it, pc, T)) { fg = true; break; }
                        run_step(a, it, pc, T, acc);
                        ph_count(PH_LSTEPS);
                        __syncthreads();
                        it.sn = take_snap(c);
                        pc = next_pc(a, it, pc);
                        if (pc.step == S_DONE) break;
                        work = step_work(a, it, pc);
                        if (!step_is_local(a, it, pc, work)) break;
                        // a long chain (a cascade of many small rounds) hands
                        // back to the grid once per slice, so that no barrier
                        // wait outlasts its bound
                        if (slice_over(a.bar, tl)) break;
                    }
                    if (threadIdx.x == 0) {
                        c->ipub[slot][0] = pc.step;
                        c->ipub[slot][1] = pc.r;
                        c->ipub[slot][2] = fg ? 1 : 0;
                    }
                }
                gbar(a.bar);
                it.sn = take_snap(c);
                pc.step = ld_rlx(&c->ipub[slot][0]);
                pc.r = ld_rlx(&c->ipub[slot][1]);
                force = ld_rlx(&c->ipub[slot][2]) != 0;
                ++pubs;
                ph_stop(c, PH_LOCAL, t0);
            }
            if (bar_aborted(a.bar)) break;
        }
        ep = it.ep;
        if (pc.step != S_DONE) { ++it_n; break; }
    }
    return it_n;
}

// ===========================================================================
// Batch program: a sequence of batches in one persistent launch.  For each
// batch: clear the hash, validate, reserve (insertion) or count tombstones
// (deletion), run all its iterations, compact (deletion), record the
// outcome.  A strict batch with an invalid item (or a packed sub-batch with
// one) is skipped without touching the graph.  When the adjacency pool runs
// out during a reservation the launch stops before mutating anything of that
// batch and reports where (the host repacks and relaunches from there).
//
// Vertex batches follow the reduction of vertex updates to edge updates:
// an insertion activates its new ids (core 0, empty list) and inserts their
// edges (a rejected batch leaves the new ids dead); a deletion checks its
// ids, gathers their live edges (an edge between two deleted ids once),
// deletes them as one edge batch and then marks the ids dead.
// ===========================================================================
__device__ __forceinline__ int32_t hash_slots(int32_t s) {
    int32_t want = 2 * s > 1024 ? 2 * s : 1024;
    int32_t h = 1024;
    while (h < want) h <<= 1;
    return h;
}

__device__ __forceinline__ void prog_reset_ctl(const KArgs &a, const BatchCtx &bc, const Team &T) {
    Ctl *c = a.ctl;
    if (T.lead()) {
        c->rem_count[0] = 0;
        c->rem_count[1] = 0;
        c->sel_count = 0;
        for (int j = 0; j < 3; ++j) {
            c->fq_tail[j] = 0; c->fh_tail[j] = 0;
            c->eq_tail[j] = 0; c->eh_tail[j] = 0;
        }
        c->cand_count = 0; c->chg_count = 0; c->chh_count = 0;
        c->touched_count = 0; c->changed_count = 0;
        c->pool_fail = 0;
        c->first_bad = 0x7fffffff;
        c->scan_tail = 0;
        c->vlist_count = 0;
        c->reloc_count = 0;
    }
    for (int32_t i = T.rank; i < bc.hcap; i += T.size) {
        a.b.hkey[i] = EMPTY_KEY;
        a.b.hval[i] = 0x7fffffff;
    }
}

__device__ __forceinline__ void prog_clear_stats(const KArgs &a, const Team &T) {
    Ctl *c = a.ctl;
    if (T.lead()) {
        c->st_iters = 0; c->st_remaining = 0; c->st_selected = 0;
        c->st_candidates = 0; c->st_evicted = 0; c->st_changed = 0; c->st_scanned = 0;
        c->st_rounds = 0; c->st_grid_steps = 0; c->st_local_steps = 0;
        c->st_icand = 0; c->st_cdeg = 0; c->st_edeg = 0; c->st_hdeg = 0;
        c->vd_total = 0;
        c->vd_tail = 0;
        c->vd_bad = 0x7fffffff;
        c->vd_count = 0;
    }
}

__device__ __forceinline__ void prog_record(const KArgs &a, ProgOut &o, int32_t status, int32_t fb, int32_t valid,
                                           int32_t iters, int32_t vdone, int32_t ep0) {
    Ctl *c = a.ctl;
    o.group = 1;
    o.ep0 = ep0;
    o.status = status;
    o.first_bad = fb;
    o.valid = valid;
    o.iterations = iters;
    o.vdone = vdone;
    o.remaining = c->st_remaining;
    o.selected = c->st_selected;
    o.candidates = c->st_candidates;
    o.evicted = c->st_evicted;
    o.changed = c->st_changed;
    o.scanned = c->st_scanned;
    o.rounds = c->st_rounds;
    o.steps = c->st_grid_steps + c->st_local_steps;
    o.icand = c->st_icand;
    o.cdeg = c->st_cdeg;
    o.edeg = c->st_edeg;
    o.hdeg = c->st_hdeg;
}

// Validation and (insertion) capacity reservation of the edge batch bc.
// Returns 1 when the adjacency pool ran out during the reservation (nothing
// of the batch was applied), else 0; status / fb / valid describe the
// validation (the same values in every thread).  On success the valid item
// indices are in the remaining list bc.cur.
__device__ __forceinline__ int prog_prepare(const KArgs &a, const BatchCtx &bc, int32_t &status, int32_t &fb,
                                            int32_t &valid) {
    Ctl *c = a.ctl;
    const Team G = grid_team();
    unsigned long long t0 = ph_start();
    prog_reset_ctl(a, bc, G);
    gbar(a.bar);
    val_canon(a, bc, G);
    gbar(a.bar);
    val_dup_mark(a, bc, G);
    gbar(a.bar);
    val_scan(a, bc, G);
    gbar(a.bar);
    val_final(a, bc, G);
    gbar(a.bar);
    if (bc.sub) {
        val_subfilter(a, bc, G);
        gbar(a.bar);
    }
    ph_stop(c, PH_VALIDATE, t0);
    const int32_t f = ld_rlx(&c->first_bad);
    fb = f == 0x7fffffff ? -1 : f;
    valid = qlen(&c->rem_count[bc.cur], a.b.cap);
    status = 0;
    if (bc.strict && !bc.sub && f != 0x7fffffff) {
        status = a.b.err[f];
        valid = 0;
        return 0;
    }
    if (valid == 0) return 0;
    t0 = ph_start();
    res_gain(a, bc, G);
    gbar(a.bar);
    if (bc.inserting) {
        res_alloc(a, G);
        gbar(a.bar);
        if (ld_rlx(&c->pool_fail)) return 1;
        res_copy(a, G);
        gbar(a.bar);
    }
    ph_stop(c, PH_RESERVE, t0);
    return 0;
}

// After the iterations: compaction (deletion) and the scan statistic.
__device__ __forceinline__ void prog_finish(const KArgs &a, bool inserting, Acc &acc) {
    Ctl *c = a.ctl;
    if (!inserting) {
        const unsigned long long t0 = ph_start();
        del_compact(a, grid_team());
        gbar(a.bar);
        ph_stop(c, PH_COMPACT, t0);
    }
    flush_acc(c, acc);
    gbar(a.bar);
}

// Replace the remaining list of the next iteration (read by the iteration
// with stamp ep + 1) by the entries fill(i) accepts, i in [0, n).
template <class F>
__device__ __forceinline__ void prog_refill(const KArgs &a, int32_t ep, int32_t n, F &&fill) {
    Ctl *c = a.ctl;
    const int cur = (ep + 1) & 1;
    if (gtid() == 0) c->rem_count[cur] = 0;
    gbar(a.bar);
    const Team G = grid_team();
    for (int32_t i = G.rank; i < n; i += G.size) {
        int32_t val = -1;
        const bool ok = fill(i, val);
        push_agg<int32_t>(a.b.rem[cur], a.b.cap, &c->rem_count[cur], val, ok, &c->overflow);
    }
    gbar(a.bar);
}

// Vertex deletion, first part: check the ids (range, dead, repeated: the
// smallest index wins) and sum the list lengths of the valid ones.
__device__ __forceinline__ void vdel_check_ids(const KArgs &a, const ProgDesc *pd, const int32_t *ids, int32_t s,
                                               int32_t n_ids, const Team &T) {
    const DevGraph &g = a.g;
    for (int32_t i = T.rank; i < s; i += T.size) {
        int32_t x = ids[i];
        int32_t e = 0;
        if (x < 0 || x >= n_ids) e = ST_RANGE;
        else if (g.core[x] < 0) e = ST_DEAD;
        a.b.err[i] = e;
        if (e == 0) atomicMin(&pd->firstidx[x], i);
    }
}
__device__ __forceinline__ void vdel_dup_count(const KArgs &a, const ProgDesc *pd, const int32_t *ids, int32_t s,
                                               const Team &T) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    long long tot = 0;
    int32_t good = 0;
    for (int32_t i = T.rank; i < s; i += T.size) {
        if (a.b.err[i] != 0) { atomicMin(&c->vd_bad, i); continue; }
        int32_t x = ids[i];
        if (pd->firstidx[x] != i) {
            a.b.err[i] = ST_DUP;
            atomicMin(&c->vd_bad, i);
            continue;
        }
        tot += g.len[x];
        ++good;
    }
    flush_stat(&c->vd_total, tot);
    for (int o = 32; o > 0; o >>= 1) good += __shfl_xor(good, o);
    if (lane() == 0 && good) atomicAdd(&c->vd_count, good);
}
// Gather the live edges of the valid ids; an edge whose other end is also
// deleted is taken from its smaller end only.
__device__ __forceinline__ void vdel_gather_edges(const KArgs &a, const ProgDesc *pd, const int32_t *ids, int32_t s,
                                                  const Team &T) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    for (int32_t i = T.wave(); i < s; i += T.nwaves()) {
        if (a.b.err[i] != 0) continue;
        int32_t x = ids[i];
        int32_t L = g.len[x];
        wave_walk(g, x, 0, L, [&](int32_t w, int32_t) {
            bool take = w >= 0 && !(w < x && pd->firstidx[w] != 0x7fffffff);
            unsigned long long m = __ballot(take);
            int rank = __popcll(m & ((1ull << lane()) - 1ull));
            int32_t base = 0;
            if (lane() == 0 && m) base = atomicAdd(&c->vd_tail, (int32_t)__popcll(m));
            base = __shfl(base, 0);
            if (take && (int64_t)base + rank < pd->gcap) {
                pd->gsrc[base + rank] = x;
                pd->gdst[base + rank] = w;
            }
        });
    }
}
// Mark the deleted ids dead and clear their duplicate marks (also for an
// invalid batch, which only set marks).
__device__ __forceinline__ void vdel_finish_ids(const KArgs &a, const ProgDesc *pd, const int32_t *ids, int32_t s,
                                                bool apply, const Team &T) {
    const DevGraph &g = a.g;
    for (int32_t i = T.rank; i < s; i += T.size) {
        if (a.b.err[i] == ST_RANGE) continue;
        int32_t x = ids[i];
        if (apply && a.b.err[i] == 0) {
            g.core[x] = -1;
            g.mcd[x] = 0;
            g.len[x] = 0;
        }
        pd->firstidx[x] = 0x7fffffff;
    }
}

// Run batch B (index j of the launch).  Returns 1 when the launch must stop
// for a pool repack before this batch, else 0 (outcome recorded in out).
__device__ __forceinline__ int run_one_batch(const KArgs &a, const ProgDesc *pd, const ProgBatch &B, ProgOut &out,
                                             int32_t bstamp, int32_t &ep, Acc &acc, int &pubs) {
    Ctl *c = a.ctl;
    const Team G = grid_team();
    const int32_t n_ids = B.n_ids > 0 ? B.n_ids : a.g.n_ids;
    const int32_t ep_first = ep + 1;  // stamp of the batch's first iteration
    BatchCtx bc;
    bc.src = pd->src + B.off;
    bc.dst = pd->dst + B.off;
    // fused served requests carry batch-local request ids; a packed program
    // carries program-wide sub-batch ids
    bc.sub = B.nsub > 0 ? pd->bsub : (pd->sub && B.kind <= 1) ? pd->sub + B.off : nullptr;
    bc.sub_bad = pd->sub_bad;
    bc.s = B.s;
    bc.inserting = B.kind == 0 || B.kind == 2;
    bc.cur = (ep + 1) & 1;
    bc.bstamp = bstamp;
    bc.hcap = hash_slots(B.s);
    bc.strict = pd->strict;
    bc.n_ids = n_ids;
    prog_clear_stats(a, G);
    int32_t status = 0, fb = -1, valid = 0, iters = 0, vdone = 0;
    // Each kind sets up below the edge batch to validate (vb), then runs up
    // to two iteration passes and the compaction / statistics step.  One
    // call site each keeps a single inlined copy of the validation and of
    // the iteration machinery in the kernel.
    enum { P_EDGES = 1, P_STARS_IN, P_NEWNEW, P_STARS_OUT };
    BatchCtx vb = bc;
    bool validate = B.s > 0;
    int32_t vbad = 0x7fffffff;  // vertex deletion: smallest bad id index
    const int32_t *ids = pd->src + B.off;
    StarCtx sc{};
    if (B.kind == 3) {
        // vertex deletion
        if (B.s > a.b.cap) {
            if (gtid() == 0) prog_record(a, out, -9, -1, 0, 0, 0, ep_first);
            gbar(a.bar);
            return 0;
        }
        vdel_check_ids(a, pd, ids, B.s, n_ids, G);
        gbar(a.bar);
        vdel_dup_count(a, pd, ids, B.s, G);
        gbar(a.bar);
        const int32_t bad = ld_rlx(&c->vd_bad);
        const long long total = (long long)__hip_atomic_load(&c->vd_total, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
        const bool reject = (pd->strict && bad != 0x7fffffff) || total > pd->gcap;
        if (reject) {
            const int32_t code = total > pd->gcap && !(pd->strict && bad != 0x7fffffff) ? -9 : a.b.err[bad];
            gbar(a.bar);  // every thread has read the counters and err[bad]
            vdel_finish_ids(a, pd, ids, B.s, false, G);
            if (gtid() == 0) prog_record(a, out, code, bad == 0x7fffffff ? -1 : bad, 0, 0, 0, ep_first);
            gbar(a.bar);
            return 0;
        }
        vdel_gather_edges(a, pd, ids, B.s, G);
        gbar(a.bar);
        const int32_t ng = ld_rlx(&c->vd_tail);
        vdone = ld_rlx(&c->vd_count);
        vbad = bad;
        // the gathered edges are validated (slot location) and counted for
        // compaction; then the ids leave as stars
        vb.src = pd->gsrc;
        vb.dst = pd->gdst;
        vb.sub = nullptr;
        vb.s = ng;
        vb.inserting = 0;
        vb.hcap = hash_slots(ng);
        vb.strict = 1;
        validate = ng > 0;
        sc.mode = 2;
        sc.ng = ng;
        sc.firstidx = pd->firstidx;
    } else if (B.kind == 2) {
        // vertex insertion: the new ids exist (core 0, empty list) before validation
        for (int32_t i = G.rank; i < B.nv; i += G.size) {
            int32_t v = B.v0 + i;
            a.g.core[v] = 0;
            a.g.mcd[v] = 0;
            a.g.len[v] = 0;
            a.g.cap[v] = 0;
            a.g.off[v] = 0;
        }
        gbar(a.bar);
        if (B.s > 0 && pd->gsrc && B.s <= pd->gcap) {
            // device copy of the items: the star passes read them repeatedly
            for (int32_t i = G.rank; i < B.s; i += G.size) {
                pd->gsrc[i] = bc.src[i];
                pd->gdst[i] = bc.dst[i];
            }
            gbar(a.bar);
            vb.src = pd->gsrc;
            vb.dst = pd->gdst;
        }
        sc.mode = 1;
        sc.v0 = B.v0;
        sc.nv = B.nv;
        sc.s = B.s;
        sc.src = vb.src;
        sc.dst = vb.dst;
    }
    int32_t vfb = -1;
    if (validate && prog_prepare(a, vb, status, vfb, valid)) return 1;
    int pass0 = 0, pass1 = 0;  // the iteration passes, 0 = none
    if (B.kind == 3) {
        // a deletion needs no reservation, so status can only be 0 here
        if (status == 0) pass0 = P_STARS_OUT;
    } else if (status == 0 && valid > 0) {
        if (B.kind == 2) {
            pass0 = P_STARS_IN;
            pass1 = P_NEWNEW;
        } else {
            pass0 = P_EDGES;  // the valid items are already the remaining list
        }
    }
    for (int p = 0; p < 2; ++p) {
        const int kind = p == 0 ? pass0 : pass1;
        if (kind == 0) break;
        if (kind == P_STARS_IN) {
            // stars: the new vertices with at least one item
            prog_refill(a, ep, B.nv, [&](int32_t i, int32_t &x) {
                int32_t lo, hi;
                star_run(sc, i, lo, hi);
                x = i;
                return hi > lo;
            });
        } else if (kind == P_NEWNEW) {
            // edges between two new vertices: ordinary iterations
            prog_refill(a, ep, B.s, [&](int32_t j, int32_t &x) {
                const int32_t u = vb.src[j], w = vb.dst[j];
                x = j;
                return a.b.err[j] == 0 && u >= B.v0 && u < B.v0 + B.nv && w >= B.v0 && w < B.v0 + B.nv;
            });
        } else if (kind == P_STARS_OUT) {
            prog_refill(a, ep, B.s, [&](int32_t i, int32_t &x) {
                x = ids[i];
                return x >= 0 && x < n_ids && pd->firstidx[x] == i;
            });
        }
        const bool star = kind == P_STARS_IN || kind == P_STARS_OUT;
        iters += run_iterations(a, vb.inserting, 0x7fffffff, ep, acc, pubs, star ? sc : StarCtx{});
    }
    if (pass0 != 0 && validate) prog_finish(a, vb.inserting, acc);
    if (B.kind == 3) {
        vdel_finish_ids(a, pd, ids, B.s, status == 0, G);
        gbar(a.bar);
        if (gtid() == 0) prog_record(a, out, status, vbad == 0x7fffffff ? -1 : vbad, valid, iters, vdone, ep_first);
        gbar(a.bar);
        return 0;
    }
    fb = vfb;
    if (B.kind == 2) {
        vdone = status == 0 ? B.nv : 0;
        if (status != 0) {
            for (int32_t i = G.rank; i < B.nv; i += G.size) a.g.core[B.v0 + i] = -1;
        }
    }
    gbar(a.bar);  // every thread has read the counters before the next batch resets them
    if (gtid() == 0) prog_record(a, out, status, fb, valid, iters, vdone, ep_first);
    return 0;
}

__device__ __forceinline__ void run_program(const KArgs &a) {
    Ctl *c = a.ctl;
    ProgDesc *pd = a.prog;
    int32_t ep = ld_rlx(&c->epoch);
    Acc acc{};
    int pubs = 0;
    const int32_t nb = pd->nb;
    int32_t j = pd->first;
    int32_t failed = 0;
    for (; j < nb; ++j) {
        if (bar_aborted(a.bar)) break;
        const ProgBatch B = pd->batches[j];
        if (hash_slots(B.s) > a.b.hcap || B.s > a.b.cap) {  // host sized the buffers for the largest batch
            if (gtid() == 0) atomicOr(&c->overflow, 8);
            break;
        }
        if (run_one_batch(a, pd, B, pd->out[j], pd->bstamp0 + 2 * (j - pd->first), ep, acc, pubs)) {
            failed = 1;
            break;
        }
    }
    ph_flush(c);  // phases of a last batch that ended before its flush
    if (gtid() == 0) {
        c->epoch = ep;
        pd->stop = j;
        pd->pool_fail = failed;
    }
}

// Serving: the same per-batch work, with batches taken from a request ring
// that the host fills while the launch runs.  Batch j is slot j % ring.
// Global thread 0 waits for the host's published count (system-scope
// acquire on the pinned header), a stop request or the idle limit, and
// broadcasts the decision through the grid barrier; after each batch it
// publishes the finished count (system-scope release).  Every wave leaves
// when the decision is not "run".
//
// Continuous batching across sessions: when fusion is on, the edge requests
// published behind request j that have the same kind, belong to distinct
// independent sessions (disjoint graphs, no edge between them) and lie
// contiguously in the payload ring join j's batch, up to `fuse` requests:
// they are validated as one batch whose items carry their request's index
// (each request keeps its own strictness), and their iterations are shared.
// A disjoint union has no edge between its members, so every vertex's core
// moves exactly as it would with its own request alone.
__device__ __forceinline__ void run_server(const KArgs &a) {
    Ctl *c = a.ctl;
    ProgDesc *pd = a.prog;
    ServeHdr *h = pd->hdr;
    int32_t ep = ld_rlx(&c->epoch);
    Acc acc{};
    int pubs = 0;
    long long j = pd->sfirst;
    int32_t reason = SV_STOP;
    const Team G = grid_team();
    for (;;) {
        if (bar_aborted(a.bar)) { reason = SV_ABORT; break; }
        if (j - pd->sfirst >= SERVE_BATCHES) { reason = SV_RESTAMP; break; }
        if (gtid() == 0) {
            int32_t d = SV_RUN;
            long long tail = 0;
            const unsigned long long t0 = (unsigned long long)wall_clock64();
            for (;;) {
                tail = __hip_atomic_load(&h->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                if (tail > j) break;
                if (__hip_atomic_load(&h->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) { d = SV_STOP; break; }
                if ((unsigned long long)wall_clock64() - t0 > pd->idle_ticks) { d = SV_IDLE; break; }
                __builtin_amdgcn_s_sleep(16);
            }
            if (d == SV_RUN) {
                ProgBatch B = pd->batches[j % pd->ring];  // one host read, not one per thread
                int32_t gn = 1;
                c->sv_goff[0] = 0;
                c->sv_goff[1] = B.s;
                if (pd->fuse > 1 && pd->strict && B.kind <= 1 && B.session >= 0) {
                    int32_t sess[FUSE_MAX];
                    sess[0] = B.session;
                    int64_t total = B.s, end = B.off + B.s;
                    while (gn < pd->fuse && gn < FUSE_MAX && j + gn < tail) {
                        const ProgBatch X = pd->batches[(j + gn) % pd->ring];
                        if (X.kind != B.kind || X.session < 0 || X.off != end) break;
                        if (total + X.s > a.b.cap || hash_slots((int32_t)(total + X.s)) > a.b.hcap) break;
                        bool again = false;
                        for (int32_t q = 0; q < gn; ++q) again |= sess[q] == X.session;
                        if (again) break;
                        sess[gn] = X.session;
                        total += X.s;
                        end += X.s;
                        ++gn;
                        c->sv_goff[gn] = (int32_t)total;
                    }
                    B.s = (int32_t)total;
                }
                B.nsub = gn > 1 ? gn : 0;
                c->sv_batch = B;
                c->sv_gn = gn;
            }
            c->sv_decision = d;
        }
        gbar(a.bar);
        const int32_t d = ld_rlx(&c->sv_decision);
        if (d != SV_RUN) { reason = d; break; }
        const ProgBatch B = c->sv_batch;
        const int32_t gn = ld_rlx(&c->sv_gn);
        if (hash_slots(B.s) > a.b.hcap || B.s > a.b.cap) { reason = SV_TOOBIG; break; }
        if (gn > 1) {
            // request index of every item, and a clear outcome word per request
            for (int32_t i = G.rank; i < B.s; i += G.size) {
                int32_t q = 0;
                while (q + 1 < gn && ld_rlx(&c->sv_goff[q + 1]) <= i) ++q;
                pd->bsub[i] = q;
            }
            for (int32_t q = G.rank; q < gn; q += G.size) pd->sub_bad[q] = ~0ull;
            gbar(a.bar);
        }
        if (run_one_batch(a, pd, B, pd->out[j % pd->ring], pd->bstamp0 + 2 * (int32_t)(j - pd->sfirst), ep,
                          acc, pubs)) {
            reason = SV_POOL;
            break;
        }
        if (gtid() == 0 && gn > 1) {
            // each fused request gets its own outcome: status, first bad item
            // and applied count of its items, the shared batch's statistics
            const ProgOut o = pd->out[j % pd->ring];
            for (int32_t q = 0; q < gn; ++q) {
                ProgOut r = o;
                const unsigned long long sb = pd->sub_bad[q];
                const int32_t lo = c->sv_goff[q], sq = c->sv_goff[q + 1] - lo;
                r.status = sb == ~0ull ? 0 : -(int32_t)(sb & 0xffull);
                r.first_bad = sb == ~0ull ? -1 : (int32_t)(sb >> 8) - lo;
                r.valid = r.status == 0 ? sq : 0;
                r.group = gn;
                pd->out[(j + q) % pd->ring] = r;
            }
        }
        if (gtid() == 0) __hip_atomic_store(&h->head, j + gn, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        j += gn;
    }
    ph_flush(c);
    if (gtid() == 0) {
        c->epoch = ep;
        h->exit_at = j;
        __hip_atomic_store(&h->exit_reason, reason, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ===========================================================================
// Static core decomposition (initial state): level-synchronous peeling.
// Level k: every remaining vertex whose current degree is <= k gets core k
// and is removed; removing a vertex lowers its remaining neighbours'
// degrees, and a neighbour joins the level when its degree crosses from k+1
// to k (exactly once).  Empty levels are skipped by jumping k to the
// smallest remaining degree.  cd[] holds the current degree; core = -2 marks
// "not yet peeled".  Remaining lists: q.fq[0..1] (counts rm_count, rotating
// by sweep j); frontier: q.eq / q.eh (counts rotating by the frontier index
// f: a step reads slot f%3, pushes slot (f+1)%3, clears slot (f+2)%3).
// Runs as a step machine like the iterations: small sweeps and rounds run in
// workgroup 0 alone.
// ===========================================================================
enum DecStep : int32_t { D_SWEEP = 0, D_ROUND, D_DONE };

struct DState {
    int32_t step;
    int32_t k;   // level
    int32_t j;   // sweep index
    int32_t f;   // frontier slot index
};

__device__ __forceinline__ void dec_sweep(const KArgs &a, const DState &st, const Team &T) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int s0 = st.j % 3, s1 = (st.j + 1) % 3, s2 = (st.j + 2) % 3;
    const int fn = (st.f + 1) % 3, fx = (st.f + 2) % 3, fb = (st.f + 1) & 1;
    const int32_t n = qlen(&c->rm_count[s0], a.q.vcap);
    if (T.lead()) {
        c->rm_count[s2] = 0;
        c->min_deg[s2] = 0x7fffffff;
        c->eq_tail[fx] = 0; c->eh_tail[fx] = 0;
    }
    const int32_t *src = a.q.fq[st.j & 1];
    int32_t *dst = a.q.fq[(st.j + 1) & 1];
    int32_t mymin = 0x7fffffff;
    for (int32_t base = T.wave() * WAVE; base < n; base += T.nwaves() * WAVE) {
        int32_t idx = base + lane();
        int32_t v = idx < n ? src[idx] : -1;
        bool keep = false, take = false;
        if (v >= 0 && g.core[v] == -2) {
            int32_t d = g.cd[v];
            if (d <= st.k) { g.core[v] = st.k; take = true; }
            else { keep = true; mymin = d < mymin ? d : mymin; }
        }
        push_vertex(a, a.q.eq[fb], &c->eq_tail[fn], a.q.eh[fb], &c->eh_tail[fn], v, take);
        push_agg<int32_t>(dst, a.q.vcap, &c->rm_count[s1], v, keep, &c->overflow);
    }
    for (int o = 32; o > 0; o >>= 1) {
        int32_t t = __shfl_xor(mymin, o);
        mymin = t < mymin ? t : mymin;
    }
    if (lane() == 0 && mymin != 0x7fffffff) atomicMin(&c->min_deg[s1], mymin);
}

__device__ __forceinline__ void dec_round(const KArgs &a, const DState &st, const Team &T, Acc &acc) {
    Ctl *c = a.ctl;
    const DevGraph &g = a.g;
    const int sc = st.f % 3, sn = (st.f + 1) % 3, sx = (st.f + 2) % 3;
    const int bc = st.f & 1, bn = bc ^ 1;
    const int32_t nq = qlen(&c->eq_tail[sc], a.q.vcap);
    const int32_t nh = qlen(&c->eh_tail[sc], a.q.hcap);
    if (T.lead()) {
        c->eq_tail[sx] = 0; c->eh_tail[sx] = 0;
        c->dec_rounds += 1;
    }
    const int32_t k = st.k;
    auto body = [&](int32_t w) -> bool {
        if (w < 0 || g.core[w] != -2) return false;
        if (atomicSub(&g.cd[w], 1) != k + 1) return false;
        g.core[w] = k;
        return true;
    };
    WaveBuf bq = wave_buf(0);
    auto push_next = [&](int32_t w, bool p) {
        push_vertex_wb(a, bq, a.q.eq[bn], &c->eq_tail[sn], a.q.eh[bn], &c->eh_tail[sn], w, p);
    };
    acc.scanned += for_vertex_slots(T, a.q.eq[bc], nq, g, a.t.large_deg,
                                [&](int32_t w, int32_t) { push_next(w, body(w)); });
    for_chunks(T, a.q.eh[bc], nh, g, a.t.chunk, [&](int32_t x, int32_t lo, int32_t hi, int32_t) {
        if (lane() == 0) acc.scanned += hi - lo;
        wave_walk(g, x, lo, hi, [&](int32_t w, int32_t) { push_next(w, body(w)); });
    });
    wb_flush(bq, a.q.eq[bn], a.q.vcap, &c->eq_tail[sn], &c->overflow);
}

__device__ __forceinline__ bool dec_block_local_ok(const KArgs &a, const DState &st, const Team &T) {
    if (st.step != D_ROUND) return true;
    Ctl *c = a.ctl;
    const int s = st.f % 3;
    long long w = queue_work(a, T, a.q.eq[st.f & 1], qlen(&c->eq_tail[s], a.q.vcap),
                             qlen(&c->eh_tail[s], a.q.hcap), 1, a.g.len);
    return w <= a.t.local_work;
}

__device__ __forceinline__ int64_t dec_work(const KArgs &a, const DState &st) {
    Ctl *c = a.ctl;
    if (st.step == D_SWEEP) return qlen(&c->rm_count[st.j % 3], a.q.vcap);
    const int s = st.f % 3;
    return frontier_work(a, qlen(&c->eq_tail[s], a.q.vcap), qlen(&c->eh_tail[s], a.q.hcap));
}

__device__ __forceinline__ DState dec_next(const KArgs &a, const DState &st) {
    Ctl *c = a.ctl;
    DState nx = st;
    if (st.step == D_SWEEP) {
        nx.j = st.j + 1;
        nx.f = st.f + 1;
        const int fs = nx.f % 3;
        if (ld_rlx(&c->eq_tail[fs]) + ld_rlx(&c->eh_tail[fs]) != 0) {
            nx.step = D_ROUND;
            return nx;
        }
        const int s1 = nx.j % 3;
        if (ld_rlx(&c->rm_count[s1]) == 0) {
            nx.step = D_DONE;
            return nx;
        }
        int32_t md = ld_rlx(&c->min_deg[s1]);
        nx.k = md > st.k + 1 ? md : st.k + 1;
        nx.step = D_SWEEP;
        return nx;
    }
    // after a round
    nx.f = st.f + 1;
    const int fs = nx.f % 3;
    if (ld_rlx(&c->eq_tail[fs]) + ld_rlx(&c->eh_tail[fs]) != 0) {
        nx.step = D_ROUND;
        return nx;
    }
    nx.k = st.k + 1;
    nx.step = D_SWEEP;
    return nx;
}

__device__ __forceinline__ void decompose(const KArgs &a, Acc &acc) {
    Ctl *c = a.ctl;
    DState st{D_SWEEP, 0, 0, 0};
    int pubs = 0;
    int32_t kmax = 0;
    bool force = false;
    while (st.step != D_DONE) {
        if (bar_aborted(a.bar)) break;
        int64_t work = dec_work(a, st);
        if (force || work > a.t.local_items) {
            force = false;
            if (st.step == D_SWEEP) dec_sweep(a, st, grid_team());
            else { dec_round(a, st, grid_team(), acc); kmax = st.k; }
            if (gtid() == 0) c->st_grid_steps += 1;
            gbar(a.bar);
            st = dec_next(a, st);
        } else {
            const int slot = pubs & 1;
            if (blockIdx.x == 0) {
                const Team T = block_team();
                bool fg = false;
                const unsigned long long tl = (unsigned long long)wall_clock64();
                for (;;) {
                    if (!dec_block_local_ok(a, st, T)) { fg = true; break; }
                    if (st.step == D_SWEEP) dec_sweep(a, st, T);
                    else { dec_round(a, st, T, acc); kmax = st.k; }
                    if (threadIdx.x == 0) c->st_local_steps += 1;
                    __syncthreads();
                    st = dec_next(a, st);
                    if (st.step == D_DONE) break;
                    if (dec_work(a, st) > a.t.local_items) break;
                    if (slice_over(a.bar, tl)) break;
                }
                if (threadIdx.x == 0) {
                    c->dpub[slot][0] = st.step;
                    c->dpub[slot][1] = st.k;
                    c->dpub[slot][2] = st.j;
                    c->dpub[slot][3] = st.f;
                    c->dpub[slot][4] = kmax;
                    c->dpub[slot][5] = fg ? 1 : 0;
                }
            }
            gbar(a.bar);
            st.step = ld_rlx(&c->dpub[slot][0]);
            st.k = ld_rlx(&c->dpub[slot][1]);
            st.j = ld_rlx(&c->dpub[slot][2]);
            st.f = ld_rlx(&c->dpub[slot][3]);
            kmax = ld_rlx(&c->dpub[slot][4]);
            force = ld_rlx(&c->dpub[slot][5]) != 0;
            ++pubs;
        }
    }
    if (gtid() == 0) c->kmax = kmax;
}

}  // namespace cm
